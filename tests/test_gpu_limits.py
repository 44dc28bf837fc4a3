"""The largest shapes the library accepts, against the FP64 oracle.

  * 32 electrons split 17 / 15: the 17-row orbital matrices go to the
    general determinant kernel (more than 16 rows), the 15-row ones to the
    workgroup-per-matrix kernel, and the jets are 98 rows tall (padded to
    128);
  * 32 electrons of one spin (no spin-down electrons, 32 x 32 orbital
    matrices), 32 nuclei, 8 layers, 64 determinants: every configuration
    limit at once.

Both forms are checked through the local energy and the value pass; the
parameter gradient of the first shape in fp32.  Tolerances are those of
test_gpu_parity.compare and test_gpu_adjoint.check (per-walker bounds from
the oracle's rounding amplification A_w).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2011_07125_amd import ferminet as F  # noqa: E402
from paper_2011_07125_amd import inputs as I  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import compare, run_gpu, run_oracle, kappa_of, U_FORM  # noqa: E402
from test_gpu_adjoint import check, selection  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    assert torch.cuda.is_available()
    F._lib()


def localized(n_up, n_down, W, L, K, seed, orbital_bias):
    """32 unit-charge nuclei on a 4 x 4 x 2 grid of spacing 3 bohr, electron
    i within 0.3 bohr of nucleus i (spin-up electrons first), and orbital i
    of each spin given an envelope on its own electron's nucleus only
    (pi = 1 there, 0 elsewhere; Eq. (5)) plus a constant orbital bias: the
    orbital matrices are diagonally dominant, so their conditioning does not
    hide the kernels' errors.  The network weights keep their random
    initialisation."""
    g = np.arange(32)
    nuc = 3.0 * np.stack([g % 4, (g // 4) % 4, g // 16], 1).astype(np.float64)
    w = I.custom_workload(n_up, n_down, nuc, np.ones(32), W, L, 32, 8, K, seed=seed, pos_std=0.3)
    offs = I.param_offsets(w["cfg"])
    p = w["params"]
    for a, (na, base) in enumerate(((n_up, 0), (n_down, n_up))):
        if na == 0:
            continue
        o, shape = offs[f"pi{a}"]
        pi = np.zeros(shape, np.float32)
        for k in range(K):
            pi[k * na + np.arange(na), base + np.arange(na)] = 1.0
        p[o:o + pi.size] = pi.reshape(-1)
        o, shape = offs[f"g_orb{a}"]
        p[o:o + shape[0]] = orbital_bias
    return w


def split_17_15(W=6):
    return localized(17, 15, W, 2, 2, 21, 2.0)


def one_spin_all_limits(W=2):
    return localized(32, 0, W, 8, 64, 22, 8.0)


CASES = {"n32_17_15": split_17_15, "n32_one_spin": one_spin_all_limits}
_ORACLE = {}


def oracle_of(name, w):
    if name not in _ORACLE:
        _ORACLE[name] = (run_oracle(w), kappa_of(w))
    return _ORACLE[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_largest_shapes_local_energy_and_value_pass(name, form):
    say(f"case limits {name} {form}")
    w = CASES[name]()
    cfg = w["cfg"]
    assert cfg["n_elec"] == 32
    o, amp = oracle_of(name, w)
    g = run_gpu(w, form)
    if form == "fp32":
        compare(f"{name}/fp32", g, o, amp)
    else:
        compare(f"{name}/bf16", g, o, amp, form="bf16", elog_tol=1e-3, mean_tol=5e-2, walker_tol=1e-2)
    # the value pass (Metropolis and log|psi| evaluations)
    d = F.to_device(w)
    s, l = F.ferminet_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form)
    torch.cuda.synchronize()
    s, l = s.double().cpu().numpy(), l.double().cpu().numpy()
    ua = U_FORM[form] * amp
    decided = ua < 0.1
    say(f"   value pass: max |d logpsi| vs oracle {np.abs(l - o['logpsi']).max():.2e}, vs jet pass "
        f"{np.abs(l - g['logpsi']).max():.2e}")
    assert np.array_equal(s[decided], o["sign"][decided])
    assert (np.abs(l - o["logpsi"]) <= 1e-5 * np.maximum(1, np.abs(o["logpsi"])) + 64 * ua)[decided].all()
    assert (np.abs(l - g["logpsi"]) <= 1e-5 * np.maximum(1, np.abs(l)) + 64 * ua).all()


def test_largest_split_shape_parameter_gradient():
    say("case limits n32_17_15 grad_logpsi fp32")
    w = split_17_15(W=3)
    cfg = w["cfg"]
    cot = np.random.default_rng(8).normal(size=3).astype(np.float32)
    d = F.to_device(w)
    g = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                               torch.from_numpy(cot).cuda(), precision="fp32")
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    assert np.isfinite(g).all()
    sel = selection(cfg, w["seed"])
    per = O.param_grad(cfg, w["pos"], w["nuc_pos"], w["params"], sel, threads=THREADS)
    ref = (cot.astype(np.float64)[:, None] * per).sum(0)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    check("n32_17_15/fp32", g[sel], ref, amp.max(), "fp32")
