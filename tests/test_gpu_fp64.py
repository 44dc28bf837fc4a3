"""The float64 form of the HIP path and the float64 re-evaluation of the
walkers of largest error scale kappa max(1, |E_L|, |E_kin|) (1 + r cond)
(kappa: determinant-sum cancellation; cond: the largest condition number of
the walker's orbital matrices; r: unit roundoff of the determinant
arithmetic over that of the orbitals), against the FP64 CPU oracle on the
same seeded inputs.

Tolerance of the float64 form: both sides compute in float64 from the same
float32 inputs, and the library rounds its outputs to float32, so every
walker is checked against
    |d log|psi|| <= 2^-22 max(1, |log|psi||) + 1e3 u64 A_w
    |d E_L|      <= (2^-22 + 1e3 u64 A_w) max(1, |E_L|)
with u64 = 2^-53 and A_w the oracle's rounding amplification of the walker
(kappa_w times the largest 1-norm condition number of its orbital
matrices), and the sign bit-exact.
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

THREADS = min(16, os.cpu_count() or 1)
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U64 = 2.0 ** -53
KEYS = ("sign", "logpsi", "e_loc", "e_kin", "e_pot")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    assert torch.cuda.is_available()
    F._lib()


def run_gpu(w, precision, rescue=0.0, max_chunk=None):
    d = F.to_device(w)
    out = F.ferminet_local_energy(w["cfg"], d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                                  precision=precision, max_chunk=max_chunk, rescue=rescue)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in out.items()}


def check_fp64(name, g, o, amp):
    scale_l = np.maximum(1.0, np.abs(o["logpsi"]))
    # the rounding of E_L is that of its kinetic term (see test_gpu_parity.compare)
    scale_e = np.maximum(np.maximum(1.0, np.abs(o["e_loc"])), np.abs(o["e_kin"]))
    dl = np.abs(g["logpsi"] - o["logpsi"])
    de = np.abs(g["e_loc"] - o["e_loc"])
    bl = 2.0 ** -22 * scale_l + 1e3 * U64 * amp
    be = (2.0 ** -22 + 1e3 * U64 * amp) * scale_e
    say(f"[{name}] W={len(dl)} max rel dlogpsi={np.max(dl / scale_l):.2e} max rel dE_L={np.max(de / scale_e):.2e} "
        f"max u64*A={np.max(U64 * amp):.1e} |d mean E_L|={abs(g['e_loc'].mean() - o['e_loc'].mean()):.2e}")
    assert np.array_equal(g["sign"], o["sign"]), f"{name}: sign mismatch at {np.nonzero(g['sign'] != o['sign'])}"
    assert (dl <= bl).all(), f"{name}: log|psi| beyond bound at {np.nonzero(dl > bl)}"
    assert (de <= be).all(), f"{name}: E_L beyond bound at {np.nonzero(de > be)}"


@pytest.mark.parametrize("name,W", [("be4", 256), ("ne10", 48), ("c4h6", 12)])
def test_fp64_form_vs_oracle(name, W):
    say(f"case fp64 form {name} W={W}")
    w = I.make_workload(name, walkers=W)
    g = run_gpu(w, "fp64")
    o = O.evaluate(w["cfg"], w["pos"], w["nuc_pos"], w["nuc_charge"], w["params"], threads=THREADS)
    amp = O.amplification(w["cfg"], w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    check_fp64(f"{name}/fp64", g, o, amp)
    # the potential is float64 in every form
    assert np.allclose(g["e_pot"], o["e_pot"], rtol=2.0 ** -22, atol=0)


def test_fp64_form_full_ne10_vs_stored_oracle():
    """All 4096 walkers of the Ne-like batch, against the oracle's values
    stored by tests/golden/make_golden.py."""
    say("case fp64 form ne10 full batch")
    w = I.make_workload("ne10")
    gold = np.load(os.path.join(ROOT, "tests", "golden", "ne10_oracle.npz"))
    g = run_gpu(w, "fp64")
    o = {k: gold[k] for k in ("sign", "logpsi", "e_loc", "e_kin")}
    check_fp64("ne10/fp64 full", g, o, gold["amplification"])
    assert abs(g["e_loc"].mean() - o["e_loc"].mean()) < 1e-5


def test_fp64_logpsi_value_pass():
    say("case fp64 logpsi ne10 W=64")
    w = I.make_workload("ne10", walkers=64)
    d = F.to_device(w)
    s, lp = F.ferminet_logpsi(w["cfg"], d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision="fp64")
    torch.cuda.synchronize()
    o = O.evaluate(w["cfg"], w["pos"], w["nuc_pos"], w["nuc_charge"], w["params"], energy=False, threads=THREADS)
    amp = O.amplification(w["cfg"], w["pos"], w["nuc_pos"], w["params"], threads=THREADS)[0]
    lp = lp.double().cpu().numpy()
    assert np.array_equal(s.double().cpu().numpy(), o["sign"])
    assert (np.abs(lp - o["logpsi"]) <= 2.0 ** -22 * np.maximum(1, np.abs(o["logpsi"])) + 1e3 * U64 * amp).all()


@pytest.mark.parametrize("form", ["bf16", "fp32"])
def test_rescue_everything_equals_fp64_form(form):
    """rescue_fraction = 1 re-evaluates every walker: the outputs are those
    of the float64 form, bit for bit (each walker's arithmetic does not
    depend on the others in the batch)."""
    say(f"case rescue all {form} ne10 W=40")
    w = I.make_workload("ne10", walkers=40)
    g64 = run_gpu(w, "fp64")
    gr = run_gpu(w, form, rescue=1.0)
    for k in KEYS:
        assert np.array_equal(gr[k], g64[k]), f"{k}: rescued {form} differs from the fp64 form"


# unit roundoff of the determinant arithmetic over that of the orbital
# product (float32 in both forms; the bf16 form's determinants are float64)
COND_WEIGHT = {"bf16": 2.0 ** -29, "fp32": 1.0}


@pytest.mark.parametrize("form,frac", [("bf16", 0.03), ("fp32", 0.02)])
def test_rescue_selects_largest_error_scale(form, frac):
    """The re-evaluated walkers are those of largest error scale: the
    outputs of exactly k walkers change to the float64 values, and the
    walkers the oracle ranks highest by that scale (from its own kappa,
    condition numbers and energies) are among them."""
    say(f"case rescue selection ne10 W=4096 {form}")
    w = I.make_workload("ne10")
    gold = np.load(os.path.join(ROOT, "tests", "golden", "ne10_oracle.npz"))
    k = int(np.ceil(frac * 4096))
    g64 = run_gpu(w, "fp64")
    gp = run_gpu(w, form)
    gr = run_gpu(w, form, rescue=frac)
    same64 = np.all([gr[q] == g64[q] for q in KEYS], axis=0)
    sameplain = np.all([gr[q] == gp[q] for q in KEYS], axis=0)
    # every walker is either re-evaluated or untouched
    assert (same64 | sameplain).all()
    changed = np.nonzero(~sameplain)[0]
    assert len(changed) <= k
    assert same64.sum() >= k  # the k re-evaluated (plus walkers whose bf16 output is already the fp64 one)
    scale = np.maximum(np.maximum(1.0, np.abs(gold["e_loc"])), np.abs(gold["e_kin"]))
    key = gold["kappa"] * scale * (1.0 + COND_WEIGHT[form] * gold["cond"])
    top = np.argsort(-key)[: k // 2]
    say(f"   k={k} changed={len(changed)} oracle top-{k // 2} by error scale re-evaluated: {int(same64[top].sum())}")
    assert same64[top].all(), f"walkers of largest error scale not re-evaluated: {top[~same64[top]]}"


@pytest.mark.parametrize("seed", [None, 101, 202, 303, 404])
@pytest.mark.parametrize("form,frac", [("bf16", 0.03), ("fp32", 0.02)])
def test_rescue_batch_mean_within_1mha(form, frac, seed):
    """The Ne-like batch (4096 walkers), with its own seed and with four
    independent ones (other network parameters and walkers; seeds 303 and
    404 were not used to choose the forms' settings): with the float64
    re-evaluation of the default fraction the batch-mean local energy is
    within 1 mHa of the oracle's."""
    say(f"case rescue batch mean ne10 seed={seed} {form} frac={frac}")
    w = I.make_workload("ne10", seed=seed)
    name = "ne10_oracle.npz" if seed is None else f"ne10_seed{seed}_oracle.npz"
    gold = np.load(os.path.join(ROOT, "tests", "golden", name))
    gr = run_gpu(w, form, rescue=frac)
    err = abs(gr["e_loc"].mean() - gold["e_loc"].mean())
    say(f"   batch mean gpu={gr['e_loc'].mean():.6f} oracle={gold['e_loc'].mean():.6f} |d|={err * 1e3:.3f} mHa")
    assert np.array_equal(gr["sign"], gold["sign"])
    assert err <= 1e-3


@pytest.mark.parametrize("W", [8193, 9000])
def test_rescue_several_segments(W):
    """More walkers than one selection segment (8192): each segment
    re-evaluates its own ceil(f x segment) walkers of largest error scale,
    the short last segment included (1 walker of the 1-walker tail of 8193,
    9 of the 808-walker tail of 9000 at f = 0.01)."""
    say(f"case rescue segments be4 W={W}")
    w = I.make_workload("be4", walkers=W)
    frac = 0.01
    g64 = run_gpu(w, "fp64")
    gp = run_gpu(w, "fp32")
    gr = run_gpu(w, "fp32", rescue=frac)
    same64 = np.all([gr[q] == g64[q] for q in KEYS], axis=0)
    sameplain = np.all([gr[q] == gp[q] for q in KEYS], axis=0)
    assert (same64 | sameplain).all()
    for lo, hi in ((0, 8192), (8192, W)):
        k = int(np.ceil(frac * (hi - lo)))
        changed = int((~sameplain[lo:hi]).sum())
        say(f"   segment [{lo}, {hi}): changed {changed} (k {k})")
        assert changed <= k
        assert same64[lo:hi].sum() >= k


def test_rescue_chunked():
    """A workspace sized for 100 walkers: the batch runs in chunks (of at
    least 100 walkers: the library fills the workspace) and each chunk
    re-evaluates its own walkers of largest error scale, ceil(f x chunk) of
    them."""
    say("case rescue chunked ne10 W=260 chunk>=100")
    w = I.make_workload("ne10", walkers=260)
    frac = 0.1
    g64 = run_gpu(w, "fp64")
    gp = run_gpu(w, "bf16", max_chunk=100)
    gr = run_gpu(w, "bf16", rescue=frac, max_chunk=100)
    same64 = np.all([gr[q] == g64[q] for q in KEYS], axis=0)
    sameplain = np.all([gr[q] == gp[q] for q in KEYS], axis=0)
    assert (same64 | sameplain).all()
    changed = int((~sameplain).sum())
    say(f"   changed {changed}, fp64 outputs {int(same64.sum())}")
    # three chunks at most, each rounding its share up
    assert changed <= int(np.ceil(frac * 260)) + 3
    assert same64.sum() >= int(np.ceil(frac * 260))


def test_fp64_adjoint_unsupported():
    w = I.make_workload("be4", walkers=4)
    d = F.to_device(w)
    with pytest.raises(F.FerminetError) as e:
        F.ferminet_grad_logpsi(w["cfg"], d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"],
                               torch.ones(4, device="cuda"), precision="fp64")
    assert e.value.status == 5
