"""Throughput of the FermiNet VMC hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ne10]

One step is one pass of the whole hot path over one batch of walkers:
a Metropolis move of every walker (log|psi| of the proposal), the local
energy (sign, log|psi|, kinetic energy from the jets, Coulomb potential)
and the VMC energy gradient from the hand-written adjoint.  The headline
form runs the layer GEMMs in split bfloat16 (three bf16 MFMA passes, fp32
accumulation) with float64 determinants; the FP32 form (fp32 layer and
orbital products, float64 determinants) is timed beside it on the same
inputs, and the all-fp32 form (float32 determinants too) for context.  In
each, the local energy of the walkers of largest rounding-error scale
(determinant-sum cancellation kappa times the kinetic-energy magnitude,
and for float32 determinants the conditioning of the orbital matrices) is
re-evaluated in float64 inside the timed step, at the workload's fraction
(3% of the Ne-like batch in both forms).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

from paper_2011_07125_amd import ferminet as F  # noqa: E402
from paper_2011_07125_amd import inputs as I  # noqa: E402

PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}  # dense TFLOP/s (MFMA), MI355X
HBM_GBS = 8000.0  # MI355X HBM3E peak, GB/s
LAYER_SRC = os.path.join(ROOT, "paper_2011_07125_amd", "csrc", "layer.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "layer_gemm_ne10_traffic.md")


def layer_flops_each(cfg, W, T):
    """Algorithmic FLOPs of each of the L layer GEMMs (jet rows x [h_i,
    g^up_i, g^down_i] x d1, unpadded): [(layer, mean-field GEMM)]."""
    n, N, d1, d2, L = cfg["n_elec"], cfg["n_nuc"], cfg["width1"], cfg["width2"], cfg["n_layers"]
    out = []
    for l in range(L):
        din, ein = (4 * N, 4) if l == 0 else (d1, d2)
        out.append((2 * W * n * T * (din + 2 * ein) * d1, 2 * W * T * (2 * din) * d1))
    return out


def layer_flops(cfg, W, T):
    """Algorithmic FLOPs of the L layer GEMMs and of the L mean-field GEMMs."""
    each = layer_flops_each(cfg, W, T)
    return sum(m for m, _ in each), sum(f for _, f in each)


def walker_flops(cfg):
    """Algorithmic MFMA-shaped FLOPs per walker: (local energy, value pass).
    The local energy carries T = 3n + 2 jet rows through the one-electron
    layers (split form: per-electron part and per-walker mean-field part),
    the orbital products of both spins and the sparse 8-row two-electron
    jets; the value pass carries one row.  Padding and re-reads are not
    counted."""
    n, N, d1, d2, L, K = (cfg["n_elec"], cfg["n_nuc"], cfg["width1"], cfg["width2"], cfg["n_layers"], cfg["n_det"])
    out = []
    for T, T2 in ((3 * n + 2, 8), (1, 1)):
        main, mf = layer_flops(cfg, 1, T)
        orb = sum(2 * na * T * d1 * K * na for na in (cfg["n_up"], cfg["n_down"]))
        pair = sum(2 * T2 * n * n * (4 if l == 0 else d2) * d2 for l in range(L - 1))
        out.append(main + mf + orb + pair)
    return out[0], out[1]


def step_ceiling(cfg, mcmc_steps, grad):
    """Walkers per second of one step (mcmc_steps value passes, the local
    energy and, with grad, the adjoint at about three value passes) if every
    FLOP ran at the dense bf16 MFMA peak."""
    el, val = walker_flops(cfg)
    per_walker = el + mcmc_steps * val + (3 * val if grad else 0)
    return PEAK["bf16"] * 1e12 / per_walker


def layer_bytes_each(cfg, W, T, fused):
    """Algorithmic HBM bytes of each one-electron layer GEMM of the jet
    pass: read the jet rows of [h_i, g^up_i, g^down_i] and the per-walker
    mean-field rows P, write the new jet rows (float32), read the weights
    once (bfloat16 hi and lo planes); a launch that also forms the spin
    means of its output (fused, every layer but the last) writes the two
    per-walker mean rows as well.  The residual re-reads h_i, which is
    already counted in the input."""
    n, N, d1, d2, L = cfg["n_elec"], cfg["n_nuc"], cfg["width1"], cfg["width2"], cfg["n_layers"]
    out = []
    for l in range(L):
        din, ein = (4 * N, 4) if l == 0 else (d1, d2)
        k = din + 2 * ein
        b = 4 * W * n * T * (k + d1) + 4 * W * T * d1 + 4 * k * d1
        if fused and l + 1 < L:
            b += 4 * W * 2 * T * d1
        out.append(b)
    return out


def layer_bytes(cfg, W, T):
    """Algorithmic HBM bytes of the L one-electron layer GEMMs (no fused means)."""
    return sum(layer_bytes_each(cfg, W, T, False))


def measured_traffic():
    """HBM bytes per launch of the jet layer GEMM from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    with open(LAYER_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    vals = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("layer.hip sha256") != sha:
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes=512 << 20, reps=3):
    """A plain copy kernel of known size (y = x * 1, float32): the FETCH_SIZE
    and WRITE_SIZE counters of these launches convert counter units into
    bytes for the layer kernel's readings."""
    x = torch.rand(nbytes // 4, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del x, y


def one_step(w, d, form, state, grad, seed, counter, rescue):
    cfg = w["cfg"]
    F.vmc_mcmc_step(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], state["logpsi"], state["sign"],
                    state["mcmc_steps"], state["mcmc_width"], seed, counter, precision=form)
    if grad:
        # the local energy and the VMC gradient in one pass (the reverse
        # pass reads the jet pass's values)
        out, _, _ = F.vmc_local_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                                precision=form, parts=False, rescue=rescue)
        return out
    return F.ferminet_local_energy(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form,
                                   parts=False, rescue=rescue)


def time_form(w, form, steps, warmup, grad, rescue, mcmc_steps=1):
    d = F.to_device(w)
    cfg = w["cfg"]
    s, l = F.ferminet_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form)
    state = {"sign": s, "logpsi": l, "mcmc_steps": mcmc_steps, "mcmc_width": w["spec"].get("mcmc_width", 0.02)}
    for i in range(warmup):
        one_step(w, d, form, state, grad, 11, i, rescue)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        one_step(w, d, form, state, grad, 11, warmup + i, rescue)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # per-stage device time of two more steps (HIP events on the same stream)
    F.stage_timing(True)
    for i in range(2):
        one_step(w, d, form, state, grad, 11, warmup + steps + i, rescue)
    torch.cuda.synchronize()
    stages = F.stage_times()
    F.stage_timing(False)
    return ms, stages


def accuracy(w, form, golden, rescue):
    """Batch-mean E_L of the seeded batch against the stored oracle values
    (the oracle's walker set: the whole batch, or its first walkers), with
    and without the float64 re-evaluation, and the largest relative log|psi|
    error of the walkers that were not re-evaluated."""
    d = F.to_device(w)
    g = np.load(golden)
    n = int(g["walkers"])
    outs = {}
    for r in (rescue, 0.0):
        out = F.ferminet_local_energy(w["cfg"], d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                      precision=form, rescue=r)
        torch.cuda.synchronize()
        outs[r] = {k: v.double().cpu().numpy()[:n] for k, v in out.items()}
    o, p = outs[rescue], outs[0.0]
    e = o["e_loc"]
    ref = g["e_loc"]
    kept = np.all([o[k] == p[k] for k in ("logpsi", "e_loc", "e_kin", "e_pot")], axis=0)
    rel_l = np.abs(o["logpsi"] - g["logpsi"]) / np.maximum(1.0, np.abs(g["logpsi"]))
    res = {"walkers": n, "batch_mean_e_loc": float(e.mean()), "oracle_batch_mean_e_loc": float(ref.mean()),
           "batch_mean_error_ha": float(abs(e.mean() - ref.mean())),
           "batch_mean_error_no_reeval_ha": float(abs(p["e_loc"].mean() - ref.mean())),
           "reevaluated_walkers": int((~kept).sum()),
           "max_rel_logpsi_error_not_reevaluated": float(rel_l[kept].max())}
    # the better-conditioned half of the batch by the oracle's rounding
    # amplification (kappa times the largest orbital-matrix condition number)
    amp = g["amplification"]
    ok = amp <= np.median(amp)
    res["lower_half_amplification_walkers"] = int(ok.sum())
    res["batch_mean_error_lower_half_ha"] = float(abs(e[ok].mean() - ref[ok].mean()))
    res["sign_mismatches"] = int((o["sign"] != g["sign"]).sum())
    return res


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, budget_s=10.0):
    """The FP64 CPU oracle timed on this host on a bounded sample of the same
    workload (local energy of the first walkers)."""
    from oracle import oracle as O
    O.build(force=False)
    threads = os.cpu_count() or 1
    cfg = w["cfg"]
    n0 = max(1, min(threads, 16))
    t = time.time()
    O.evaluate(cfg, w["pos"][:n0], w["nuc_pos"], w["nuc_charge"], w["params"], threads=threads)
    dt = time.time() - t
    n = int(min(w["pos"].shape[0], max(n0, n0 * budget_s / max(dt, 1e-3))))
    n = max(n0, (n // threads) * threads) if n > threads else n
    t = time.time()
    O.evaluate(cfg, w["pos"][:n], w["nuc_pos"], w["nuc_charge"], w["params"], threads=threads)
    dt = time.time() - t
    return {"value": n / dt, "unit": "walker local-energy evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"local energy of the first {n} walkers of the {w['spec'].get('walkers')}-walker batch "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ne10")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-kfac", action="store_true", help="skip timing the KFAC statistics")
    ap.add_argument("--no-full-envelope", action="store_true",
                    help="skip timing the same step with the full-covariance envelope of Eq. (5)")
    ap.add_argument("--rescue-bf16", type=float, default=None,
                    help="fraction of walkers whose local energy is re-evaluated in float64 (bf16 form; default: "
                         "the workload's own, inputs.RESCUE)")
    ap.add_argument("--rescue-fp32", type=float, default=None, help="the same for the fp32 form")
    ap.add_argument("--no-pure-fp32", action="store_true",
                    help="skip timing the fp32 form with float32 determinants")
    ap.add_argument("--mcmc-steps", type=int, default=None,
                    help="Metropolis moves per step (default: the workload's own, else 1)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first launch a plain 512 MiB copy kernel three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (walkers are independent, so "
              "more GPUs would shard the batch)", file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "needs a GPU"
    if args.copy_calibration:
        copy_calibration()
    w = I.make_workload(args.workload)
    cfg = w["cfg"]
    if args.rescue_bf16 is None:
        args.rescue_bf16 = I.RESCUE[args.workload]["bf16"]
    if args.rescue_fp32 is None:
        args.rescue_fp32 = I.RESCUE[args.workload]["fp32_fp64det"]
    W = w["pos"].shape[0]
    T = 3 * cfg["n_elec"] + 2
    mcmc_steps = args.mcmc_steps if args.mcmc_steps is not None else w["spec"].get("mcmc_steps", 1)
    grad = True
    try:
        F.vmc_energy_gradient(cfg, *[F.to_device(dict(w, pos=w["pos"][:2]))[k]
                                     for k in ("pos", "nuc_pos", "nuc_charge", "params")],
                              torch.zeros(2, device="cuda"), precision="bf16")
    except F.FerminetError:
        grad = False  # adjoint not available in this build

    ms_bf, st_bf = time_form(w, "bf16", args.steps, args.warmup, grad, args.rescue_bf16, mcmc_steps)
    res = {}
    if not args.no_fp32:
        # the FP32 form: every layer and orbital product in float32, the
        # determinants in float64 like the bf16 form's, so that the two
        # forms differ in the layer products only
        ms_32, st_32 = time_form(w, "fp32_fp64det", args.steps, args.warmup, grad, args.rescue_fp32, mcmc_steps)
        res["fp32_form"] = {"value": W / (ms_32 * 1e-3), "ms_per_step": ms_32, "rescue_fraction": args.rescue_fp32,
                            "form": "fp32 layer and orbital GEMMs (fp32 MFMA), fp64 determinants",
                            "bf16_speedup": ms_32 / ms_bf,
                            "stage_ms": {k: round(v[0] / 2, 4) for k, v in st_32.items()}}
    if not args.no_pure_fp32:
        ms_p, _ = time_form(w, "fp32", args.steps, args.warmup, grad, args.rescue_fp32, mcmc_steps)
        res["fp32_pure_form"] = {"value": W / (ms_p * 1e-3), "ms_per_step": ms_p, "rescue_fraction": args.rescue_fp32,
                                 "form": "everything in fp32, determinants included (timing only)"}
    if not args.no_full_envelope:
        # the same step with a general 3x3 Sigma per orbital and nucleus, the
        # envelope that Section 3 replaces by the isotropic one to save time
        wf = I.full_covariance(w, noise=0.3, seed=5)
        ms_fe, st_fe = time_form(wf, "bf16", args.steps, args.warmup, grad, args.rescue_bf16, mcmc_steps)
        res["full_envelope_bf16"] = {"value": W / (ms_fe * 1e-3), "ms_per_step": ms_fe,
                                     "slowdown_vs_isotropic": ms_fe / ms_bf,
                                     "stage_ms": {k: round(v[0] / 2, 4) for k, v in st_fe.items()}}
    if grad and not args.no_kfac:
        # KFAC statistics (A and G of every dense layer) of the same batch
        d = F.to_device(w)
        c = torch.full((W,), 1.0 / W, device="cuda")
        for i in range(args.warmup):
            F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c, precision="bf16")
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for i in range(args.steps):
            F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c, precision="bf16")
        t1.record()
        torch.cuda.synchronize()
        ms_k = t0.elapsed_time(t1) / args.steps
        res["kfac_factors_bf16"] = {"ms_per_call": ms_k, "value": W / (ms_k * 1e-3), "unit": "walkers/s",
                                    "floats": F.kfac_layout(cfg)[1]}
        # the step direction from those factors (float64 Cholesky and solves)
        fac = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c,
                                      precision="bf16")
        g = torch.randn(d["params"].numel(), device="cuda")
        F.ferminet_kfac_precondition(cfg, fac, g, 1e-3)
        torch.cuda.synchronize()
        t0.record()
        for i in range(3):
            F.ferminet_kfac_precondition(cfg, fac, g, 1e-3)
        t1.record()
        torch.cuda.synchronize()
        res["kfac_precondition"] = {"ms_per_call": t0.elapsed_time(t1) / 3, "damping": 1e-3}
        # one whole VMC iteration (vmc_train_step): log|psi| refresh, 10
        # Metropolis moves, local energy, clipped-energy gradient, KFAC
        # factors, their running average, damped direction, parameter step
        d = F.to_device(w)
        fac = torch.zeros(F.kfac_layout(cfg)[1], device="cuda")
        it_args = (cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], fac, 10, 0.02, 11)
        for i in range(args.warmup):
            F.vmc_train_step(*it_args, 10 * i, 0.05, 1e-3, 1e-3, 0.0 if i == 0 else 0.95, 5.0, precision="bf16",
                             rescue=args.rescue_bf16)
        torch.cuda.synchronize()
        t0.record()
        n_it = max(1, args.steps // 2)
        for i in range(n_it):
            F.vmc_train_step(*it_args, 10 * (args.warmup + i), 0.05, 1e-3, 1e-3, 0.95, 5.0, precision="bf16",
                             rescue=args.rescue_bf16)
        t1.record()
        torch.cuda.synchronize()
        ms_it = t0.elapsed_time(t1) / n_it
        res["vmc_iteration_bf16"] = {"ms_per_iteration": ms_it, "value": W / (ms_it * 1e-3),
                                     "unit": "walker-iterations/s", "mcmc_steps": 10}
    # dominant kernel: the one-electron layer GEMM of the jet pass, a dense
    # contraction priced against the bf16 MFMA peak with its algorithmic
    # FLOPs (jet rows x [h_i, g^up_i, g^down_i] x d1, unpadded; one
    # multiply-add counted once although the split form issues three bf16
    # MFMAs for it).  Where the spin groups allow it, the launches of every
    # layer but the last also form the spin means of their output (stage
    # gemm_layer_mf, one spin group per tile): those are the dominant
    # launches and the figure is theirs; otherwise all L launches (stage
    # gemm_layer).  Its HBM rate at the bytes of its float32 jets is kept as
    # a secondary figure.
    L = cfg["n_layers"]
    fl_each = [m for m, _ in layer_flops_each(cfg, W, T)]
    fused = st_bf.get("gemm_layer_mf", (0.0, 0))[1] > 0
    by_each = layer_bytes_each(cfg, W, T, fused)
    sel = list(range(L - 1)) if fused else list(range(L))
    tot, cnt = st_bf.get("gemm_layer_mf" if fused else "gemm_layer", (0.0, 0))
    flops_per_launch = sum(fl_each[l] for l in sel) / len(sel)
    bytes_per_launch = sum(by_each[l] for l in sel) / len(sel)
    jet_launch_ms = tot / cnt if cnt else None
    tflops = flops_per_launch / (jet_launch_ms * 1e-3) / 1e12 if jet_launch_ms else None
    gbs = bytes_per_launch / (jet_launch_ms * 1e-3) / 1e9 if jet_launch_ms else None
    traffic = measured_traffic()
    value = W / (ms_bf * 1e-3)
    ceiling = step_ceiling(cfg, mcmc_steps, grad)
    roof = {"bound": "mfma", "achieved": tflops, "peak": PEAK["bf16"], "unit": "TFLOP/s",
            "frac": (tflops / PEAK["bf16"]) if tflops else None, "traffic": traffic,
            "kernel": (f"layer_gemm_kernel<MODE_BF16X3,{32 * cfg['n_up']},128,{cfg['n_up']},2,jet_mf> (one-electron "
                       f"layers 0..{L - 2}: tanh-jet epilogue and the spin means of the output)") if fused else
                      "layer_gemm_kernel<MODE_BF16X3,128,128,4,2,jet> (one-electron layer, tanh-jet epilogue)",
            "flops_per_launch": flops_per_launch, "avg_launch_ms": jet_launch_ms, "launches_timed": cnt,
            "hbm_secondary": {"achieved": gbs, "peak": HBM_GBS, "unit": "GB/s",
                              "frac": (gbs / HBM_GBS) if gbs else None, "bytes_per_launch": bytes_per_launch},
            "step": {"achieved": value, "ceiling": ceiling, "frac": value / ceiling,
                     "unit": "walker local-energy evals/s",
                     "ceiling_basis": "algorithmic MFMA FLOPs of the step (local energy, Metropolis value passes, "
                                      "adjoint as three value passes) at the 2.5 PFLOP/s dense bf16 peak"}}
    golden = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.npz")
    if os.path.exists(golden) and not args.no_accuracy and "pos" not in np.load(golden).files:
        res["accuracy_bf16"] = accuracy(w, "bf16", golden, args.rescue_bf16)
        res["accuracy_bf16"]["reeval_share_of_step"] = st_bf.get("rescue_fp64", (0.0, 1))[0] / 2 / ms_bf
        if not args.no_fp32:
            res["accuracy_fp32"] = accuracy(w, "fp32_fp64det", golden, args.rescue_fp32)
            res["accuracy_fp32"]["reeval_share_of_step"] = st_32.get("rescue_fp64", (0.0, 1))[0] / 2 / ms_32
    line = {
        "metric": "walker local-energy evals/sec (Ne-like, 16 dets) BF16+adjoint vs FP32 at <=1 mHa",
        "value": value, "unit": "walker local-energy evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_bf, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded Gaussian walkers, random-init weights)",
        "config": {"workload": f"{args.workload}: Z={w['nuc_charge'].tolist()}, {cfg['n_elec']} electrons "
                               f"({cfg['n_up']} up/{cfg['n_down']} down), {W} walkers, {cfg['n_layers']} layers "
                               f"{cfg['width1']}/{cfg['width2']}, {cfg['n_det']} dets, isotropic envelope",
                   "walkers": W, "step": f"{mcmc_steps} Metropolis move{'s' if mcmc_steps > 1 else ''} + local energy" + (" + VMC gradient" if grad else ""),
                   "form": "bf16x3 layer GEMMs (fp32 accumulation), orbital GEMM on fp32 operands split into three bf16 parts (six "
                           "bf16 MFMAs, fp32 accumulation), fp64 determinants, fp64 re-evaluation of the "
                           f"{args.rescue_bf16:.0%} walkers of largest rounding-error scale",
                   "rescue_fraction": args.rescue_bf16,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "stage_ms_bf16": {k: round(v[0] / 2, 4) for k, v in st_bf.items()},
    }
    line.update(res)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
