"""Statistics of the Kronecker-factored curvature (KFAC, Martens and Grosse
2015; the optimiser the paper names) on the GPU against the FP64 oracle:
for every dense layer, A = sum_w c_w sum_r a~ a~^T and G = sum_w c_w sum_r
g g^T (a~ = [layer input; 1], g = d log|psi_w| / d pre-activation, r over
the positions the layer is applied at).

Tolerance per element: |M_gpu - M_oracle| <= 1e-3 |M_oracle| + (1e-5 +
u A) max|M_oracle| with u the form's unit roundoff and A the largest
per-walker rounding amplification of the batch (as for the gradient)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2011_07125_amd import ferminet as F  # noqa: E402
from paper_2011_07125_amd import inputs as I  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)
U_FORM = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    assert torch.cuda.is_available()
    F._lib()


def two_nuclei(W=8, seed=11):
    """5 electrons (3 up, 2 down) at two nuclei, three layers, non-zero
    biases, envelope parameters away from 1 (no accidental symmetry)."""
    w = I.custom_workload(3, 2, [[0, 0, 0], [0.9, 0.4, -0.6]], [3.0, 2.0], W, 3, 32, 8, 3, seed)
    p = w["params"].astype(np.float64)
    rng = np.random.default_rng(seed)
    offs = I.param_offsets(w["cfg"])
    for name, shape, kind in I.param_blocks(w["cfg"]):
        o, sh = offs[name]
        size = int(np.prod(sh))
        if kind == "bias":
            p[o:o + size] = rng.normal(size=size) * 0.3
        elif kind in ("pi", "sigma"):
            p[o:o + size] = rng.uniform(0.5, 1.5, size=size)
    w["params"] = p.astype(np.float32)
    return w


CASES = {
    "be4": lambda: I.make_workload("be4", walkers=16),
    "two_nuclei": lambda: two_nuclei(),
    "ne10": lambda: I.make_workload("ne10", walkers=2),
}


@pytest.mark.parametrize("case,form", [("be4", "fp32"), ("be4", "bf16"), ("two_nuclei", "fp32"), ("ne10", "bf16")])
def test_kfac_factors_vs_oracle(case, form):
    say(f"case kfac factors {case} {form}")
    w = CASES[case]()
    cfg = w["cfg"]
    W = w["pos"].shape[0]
    c = (np.linspace(0.5, 1.5, W) / W).astype(np.float32)
    d = F.to_device(w)
    flat = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                   torch.from_numpy(c).cuda(), precision=form)
    torch.cuda.synchronize()
    got = {k: (A.double().cpu().numpy(), G.double().cpu().numpy()) for k, (A, G) in F.kfac_split(cfg, flat).items()}
    ref = O.kfac_factors(cfg, w["pos"], w["nuc_pos"], w["params"], c.astype(np.float64), threads=THREADS)
    amp = O.amplification(cfg, w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0].max()
    ua = U_FORM[form] * amp
    assert sorted(got) == sorted(name for name, _, _ in ref)
    for name, A, G in ref:
        for which, M, Mg in (("A", A, got[name][0]), ("G", G, got[name][1])):
            assert Mg.shape == M.shape, (name, which)
            err = np.abs(Mg - M)
            scale = np.abs(M).max()
            bound = 1e-3 * np.abs(M) + (1e-5 + ua) * scale
            say(f"   {name}.{which} {M.shape[0]}x{M.shape[1]} max|M|={scale:.3e} max err={err.max():.2e} "
                f"(u*A={ua:.1e})")
            assert (err <= bound).all(), f"{name}.{which}: beyond bound at {np.argwhere(err > bound)[:5]}"


def test_kfac_weights_scale_linearly_and_chunks_agree():
    """Doubling every weight doubles every factor; a workspace for fewer
    walkers (chunks) gives the same factors up to the order of the sums."""
    say("case kfac linearity and chunks be4 W=24")
    w = I.make_workload("be4", walkers=24)
    cfg = w["cfg"]
    d = F.to_device(w)
    c = torch.linspace(0.1, 1.0, 24, device="cuda")
    a = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c)
    b = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], 2 * c)
    F.release_workspaces()
    e = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c, max_chunk=7)
    torch.cuda.synchronize()
    tol = 1e-5 * a.abs().max().item()
    assert torch.allclose(b, 2 * a, rtol=1e-5, atol=tol)
    assert torch.allclose(e, a, rtol=1e-4, atol=tol)
    # a zero weight removes that walker
    c0 = c.clone()
    c0[5] = 0.0
    z = F.ferminet_kfac_factors(cfg, d["pos"][torch.arange(24, device="cuda") != 5], d["nuc_pos"], d["nuc_charge"],
                                d["params"], c[torch.arange(24, device="cuda") != 5])
    y = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c0)
    torch.cuda.synchronize()
    assert torch.allclose(y, z, rtol=1e-4, atol=tol)


@pytest.mark.parametrize("case", ["be4", "two_nuclei", "ne10"])
def test_kfac_precondition_vs_oracle(case):
    """The KFAC step direction (factored Tikhonov damping) on the GPU
    (float64 Cholesky and triangular solves) against the oracle's dense
    solves, both from the same float32 factors and gradient: agreement to
    the float32 rounding of the output; the envelope parameters keep their
    gradient exactly."""
    say(f"case kfac precondition {case}")
    w = CASES[case]()
    cfg = w["cfg"]
    W = w["pos"].shape[0]
    d = F.to_device(w)
    c = torch.full((W,), 1.0 / W, device="cuda")
    flat = F.ferminet_kfac_factors(cfg, d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], c)
    P = d["params"].numel()
    grad = torch.from_numpy(np.random.default_rng(7).normal(size=P).astype(np.float32)).cuda()
    lam = 1e-3
    upd = F.ferminet_kfac_precondition(cfg, flat, grad, lam)
    torch.cuda.synchronize()
    facs = [(k, A.double().cpu().numpy(), G.double().cpu().numpy()) for k, (A, G) in F.kfac_split(cfg, flat).items()]
    ref = O.kfac_precondition(cfg, facs, grad.double().cpu().numpy(), lam)
    got = upd.double().cpu().numpy()
    offs = O._kfac_param_offsets(cfg)
    covered = np.zeros(P, dtype=bool)
    for name, A, G in facs:
        off, n = offs[name], A.shape[0] * G.shape[0]
        covered[off:off + n] = True
        r, g = ref[off:off + n], got[off:off + n]
        err = np.abs(g - r)
        say(f"   {name}: max|X|={np.abs(r).max():.3e} max err={err.max():.2e}")
        assert (err <= 2e-6 * np.abs(r) + 1e-6 * np.abs(r).max()).all(), name
    assert np.array_equal(got[~covered], grad.cpu().numpy()[~covered])
