"""Writes the oracle's outputs on seeded workloads (float64) for the
bench's and the tests' batch-mean error gates.  Calls only oracle/ and the
seeded input generator.

    python tests/golden/make_golden.py <name> [threads] [seed]

Walker sets (the parity walker counts of the workloads):
  * be4, ne10: the whole batch;
  * ar18, c4h6: the first 256 walkers of the batch (the oracle's cost per
    walker is about ten times the Ne-like one's);
  * c4h6_vmc: the first 256 walkers of the 8192-walker batch after the
    workload's Metropolis steps (10 moves of width 0.02 bohr, Philox keyed
    by the workload seed, counter 0, starting from the oracle's own
    log|psi|).  Walkers are independent and the draws are keyed by the
    walker index, so these are the chains of the first 256 walkers of the
    whole batch.  The moved positions and the acceptance count per walker
    are stored with the energies.

With a seed other than the workload's own, the network parameters and the
walkers are both drawn from that seed (an independent batch), and the file
is named <name>_seed<seed>_oracle.npz.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2011_07125_amd import inputs as I  # noqa: E402

PREFIX = {"ar18": 256, "c4h6": 256, "c4h6_vmc": 256}


def main(name, threads, seed=None):
    w = I.make_workload(name, seed=seed)
    t = time.time()
    pos = w["pos"][:PREFIX.get(name, w["pos"].shape[0])].astype(np.float64)
    extra = {}
    if "mcmc_steps" in w["spec"]:
        sp = w["spec"]
        r0 = O.evaluate(w["cfg"], pos, w["nuc_pos"], w["nuc_charge"], w["params"], energy=False, threads=threads)
        pos, lp, sg, acc = O.mcmc(w["cfg"], pos, w["nuc_pos"], w["params"], r0["logpsi"], r0["sign"],
                                  sp["mcmc_steps"], sp["mcmc_width"], seed=w["seed"], counter=0, threads=threads)
        extra = dict(pos=pos.astype(np.float32), logpsi0=r0["logpsi"], sign0=r0["sign"], accepted=acc,
                     mcmc_steps=sp["mcmc_steps"], mcmc_width=sp["mcmc_width"])
        pos = pos.astype(np.float32).astype(np.float64)
    r = O.evaluate(w["cfg"], pos, w["nuc_pos"], w["nuc_charge"], w["params"], threads=threads)
    amp, kappa, cond = O.amplification(w["cfg"], pos, w["nuc_pos"], w["params"], threads=threads)
    out = os.path.join(HERE, f"{name}_oracle.npz" if seed is None else f"{name}_seed{seed}_oracle.npz")
    np.savez_compressed(out, sign=r["sign"], logpsi=r["logpsi"], e_loc=r["e_loc"], e_kin=r["e_kin"],
                        e_pot=r["e_pot"], amplification=amp, kappa=kappa, cond=cond, seed=w["seed"],
                        walkers=pos.shape[0], **extra)
    print(f"{out}: {pos.shape[0]} walkers in {time.time() - t:.1f}s, mean E_L {r['e_loc'].mean():.6f}")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else os.cpu_count(),
         int(sys.argv[3]) if len(sys.argv) > 3 else None)
