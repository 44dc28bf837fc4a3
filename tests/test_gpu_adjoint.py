"""The hand-written adjoint d log|psi| / d theta on the GPU against the
oracle's dual-number derivatives, on seeded parameter subsets that cover
every kind of parameter block.

Tolerance: per parameter |g_gpu - g_oracle| <= 1e-3 |g_oracle| +
(1e-5 + u A) ||g_oracle||_inf, with u the form's unit roundoff and A the
largest per-walker rounding amplification of the batch (see
test_gpu_parity.compare); errors are printed.
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
from paper_2011_07125_amd.autograd import logpsi as logpsi_fn  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)
U_FORM = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def selection(cfg, seed, n_pick=40):
    sel = list(I.fd_param_choice(cfg, n_pick, seed=seed))
    offs = I.param_offsets(cfg)
    for name, shape, kind in I.param_blocks(cfg):
        o, sh = offs[name]
        size = int(np.prod(sh))
        if size:
            sel += [o, o + size - 1]  # first and last entry of every block
    return np.array(sorted(set(sel)), dtype=np.int64)


def check(name, g_gpu, g_or, amp_max, form):
    err = np.abs(g_gpu - g_or)
    scale = np.abs(g_or).max()
    bound = 1e-3 * np.abs(g_or) + (1e-5 + U_FORM[form] * amp_max) * scale
    worst = int(np.argmax(err / np.maximum(bound, 1e-30)))
    say(f"[{name}] {g_or.size} params |g|inf={scale:.3e} max abs err={err.max():.2e} "
        f"median rel err={np.median(err / np.maximum(np.abs(g_or), 1e-30)):.2e} u*A={U_FORM[form] * amp_max:.1e} "
        f"worst idx {worst}: gpu={g_gpu[worst]:.6e} oracle={g_or[worst]:.6e}")
    assert (err <= bound).all(), f"{name}: adjoint beyond bound at {np.nonzero(err > bound)}"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    assert torch.cuda.is_available()


@pytest.mark.parametrize("name,W,form", [("be4", 32, "fp32"), ("ne10", 6, "fp32"), ("ne10", 6, "bf16"),
                                         ("c4h6", 3, "fp32")])
def test_grad_logpsi_vs_oracle(name, W, form):
    say(f"case grad_logpsi {name} W={W} {form}")
    w = I.make_workload(name, walkers=W)
    cfg = w["cfg"]
    rng = np.random.default_rng(3)
    cot = rng.normal(size=W).astype(np.float32)
    d = F.to_device(w)
    g = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                               torch.from_numpy(cot).cuda(), precision=form)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    assert np.isfinite(g).all()
    sel = selection(cfg, w["seed"])
    per = O.param_grad(cfg, w["pos"], w["nuc_pos"], w["params"], sel, threads=THREADS)  # [W][sel]
    ref = (cot.astype(np.float64)[:, None] * per).sum(0)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    check(f"{name}/{form}", g[sel], ref, amp.max(), form)


@pytest.mark.parametrize("name,W", [("ne10", 5), ("c4h6", 2)])
def test_two_electron_block_gradient_every_entry(name, W):
    """Every weight and bias of the two-electron layers (the blocks the
    pair-row backward produces, electrons grouped per workgroup) against
    the oracle's dual numbers."""
    say(f"case two-electron gradient block {name} W={W}")
    w = I.make_workload(name, walkers=W)
    cfg = w["cfg"]
    cot = np.random.default_rng(5).normal(size=W).astype(np.float32)
    d = F.to_device(w)
    g = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                               torch.from_numpy(cot).cuda(), precision="fp32")
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    offs = I.param_offsets(cfg)
    sel = []
    for bname, shape, kind in I.param_blocks(cfg):
        if bname.startswith(("W", "c")) and not bname.startswith("w_orb"):
            o, sh = offs[bname]
            sel += list(range(o, o + int(np.prod(sh))))
    sel = np.array(sorted(sel), dtype=np.int64)
    assert sel.size > 0
    per = O.param_grad(cfg, w["pos"], w["nuc_pos"], w["params"], sel, threads=THREADS)
    ref = (cot.astype(np.float64)[:, None] * per).sum(0)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    check(f"{name}/two-electron block", g[sel], ref, amp.max(), "fp32")


def test_vmc_energy_gradient_vs_oracle():
    """(1/W) sum_w (E_L,w - mean E_L) d log|psi_w| / d theta, with the
    energies from the GPU's own local energy, against the oracle's
    derivatives weighted the same way; the batch statistics in float64."""
    say("case vmc_energy_gradient be4 W=64")
    w = I.make_workload("be4", walkers=64)
    cfg = w["cfg"]
    d = F.to_device(w)
    out = F.ferminet_local_energy(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision="fp32")
    grad, stats = F.vmc_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], out["e_loc"],
                                        precision="fp32")
    torch.cuda.synchronize()
    e = out["e_loc"].double().cpu().numpy()
    st = stats.cpu().numpy()
    assert abs(st[0] - e.mean()) < 1e-12 * max(1, abs(e.mean())) * 64
    assert abs(st[1] - e.var()) < 1e-9 * max(1, e.var())
    sel = selection(cfg, 0)
    per = O.param_grad(cfg, w["pos"], w["nuc_pos"], w["params"], sel, threads=THREADS)
    c = (e - e.mean()) / e.size
    ref = (c[:, None] * per).sum(0)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    check("be4/vmc-gradient", grad.double().cpu().numpy()[sel], ref, amp.max(), "fp32")


def test_autograd_function_matches_entry_point():
    say("case autograd be4")
    w = I.make_workload("be4", walkers=16)
    cfg = w["cfg"]
    d = F.to_device(w)
    p = d["params"].clone().requires_grad_(True)
    lp, sg = logpsi_fn(p, d["pos"], d["nuc_pos"], d["nuc_charge"], cfg, "fp32")
    c = torch.linspace(-1, 1, 16, device="cuda")
    (c * lp).sum().backward()
    g = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c.contiguous())
    torch.cuda.synchronize()
    assert torch.equal(p.grad, g)
    assert not sg.requires_grad


def test_grad_chunked_equals_single_pass_and_is_deterministic():
    say("case grad chunked ne10 W=11")
    w = I.make_workload("ne10", walkers=11)
    cfg = w["cfg"]
    d = F.to_device(w)
    cot = torch.linspace(-2, 1, 11, device="cuda")
    a = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], cot)
    b = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], cot)
    F.release_workspaces()
    c = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], cot, max_chunk=4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # chunks change the order of the sums over walkers only
    assert torch.allclose(a, c, rtol=1e-4, atol=1e-6 * a.abs().max().item())


@pytest.mark.parametrize("name,W,form", [("be4", 48, "fp32"), ("ne10", 8, "fp32"), ("ne10", 8, "bf16"),
                                         ("c4h6", 3, "fp32")])
def test_per_walker_gradient_vs_oracle(name, W, form):
    """cotangent NULL: d log|psi_w| / d theta of every walker ([W][P]) on a
    seeded subset of 64 parameters plus the first and last entry of every
    block, walker by walker against the oracle's dual numbers (each walker
    against its own amplification); the cotangent-weighted sum of the rows
    equals the [P] form; a chunked call gives the same rows bit for bit."""
    say(f"case per-walker gradient {name} W={W} {form}")
    w = I.make_workload(name, walkers=W)
    cfg = w["cfg"]
    d = F.to_device(w)
    G = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], None, precision=form)
    Gc = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], None, precision=form,
                                max_chunk=max(1, W // 3))
    cot = np.random.default_rng(7).normal(size=W).astype(np.float32)
    g = F.ferminet_grad_logpsi(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                               torch.from_numpy(cot).cuda(), precision=form)
    torch.cuda.synchronize()
    assert tuple(G.shape) == (W, F.param_count(cfg))
    assert torch.equal(G, Gc)
    G = G.double().cpu().numpy()
    assert np.isfinite(G).all()
    sel = selection(cfg, w["seed"], n_pick=64)
    per = O.param_grad(cfg, w["pos"], w["nuc_pos"], w["params"], sel, threads=THREADS)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    for k in range(W):
        check(f"{name}/{form}/walker {k}", G[k, sel], per[k], amp[k], form)
    # the weighted sum of the rows against the [P] form (float32 sums in
    # another order: relative to the largest term)
    ref = cot.astype(np.float64) @ G
    gd = g.double().cpu().numpy()
    scale = (np.abs(cot)[:, None] * np.abs(G)).sum(0).max()
    err = np.abs(gd - ref).max() / scale
    say(f"   sum over walkers vs the [P] form: max error {err:.2e} of the largest term sum")
    assert err <= 1e-4


@pytest.mark.parametrize("name,W,form,rescue", [("ne10", 512, "bf16", 0.03), ("ne10", 256, "fp32_fp64det", 0.03),
                                                ("c4h6", 64, "fp32", 0.0), ("be4", 200, "fp32", 0.02)])
def test_local_energy_gradient_in_one_pass(name, W, form, rescue):
    """vmc_local_energy_gradient (the reverse pass on the values of the
    local energy's own jet pass) against ferminet_local_energy followed by
    vmc_energy_gradient: the energies and statistics bit for bit, the
    gradient to float32 rounding; with a workspace below the one-pass size
    the entry point runs the two calls in turn (bit for bit)."""
    say(f"case local energy + gradient in one pass {name} W={W} {form} rescue={rescue}")
    w = I.make_workload(name, walkers=W)
    cfg = w["cfg"]
    d = F.to_device(w)
    out, g1, st1 = F.vmc_local_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                               precision=form, rescue=rescue)
    ref = F.ferminet_local_energy(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form,
                                  rescue=rescue)
    g2, st2 = F.vmc_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], ref["e_loc"],
                                    precision=form)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(out[k], ref[k]), k
    assert torch.equal(st1, st2)
    diff = (g1 - g2).abs().max().item()
    scale = g2.abs().max().item()
    say(f"   |grad|inf {scale:.3e}, max |one pass - two calls| {diff:.3e} (bitwise equal: {torch.equal(g1, g2)})")
    assert diff <= 1e-6 * scale
    # below the one-pass workspace: the two calls in turn, in chunks (the
    # same workspace bytes give both sides the same chunks)
    ws = F.workspace(cfg, W, F.FN_ENTRY_LOCAL_ENERGY_GRADIENT, form, d["pos"].device, max(1, W // 3), rescue)
    assert ws.numel() < F.workspace_bytes(cfg, W, F.FN_ENTRY_LOCAL_ENERGY_GRADIENT, form, rescue)
    out3, g3, st3 = F.vmc_local_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                                precision=form, rescue=rescue, ws=ws)
    torch.cuda.synchronize()
    ref3 = F.ferminet_local_energy(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form,
                                   rescue=rescue, ws=ws)
    g4, st4 = F.vmc_energy_gradient(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], ref3["e_loc"],
                                    precision=form, ws=ws)
    torch.cuda.synchronize()
    for k in ref3:
        assert torch.equal(out3[k], ref3[k]), k
    assert torch.equal(g3, g4) and torch.equal(st3, st4)
