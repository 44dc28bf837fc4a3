"""The spin means of the mean field (Sec. 3) formed in the jet layer kernel
(FN_OPT_FUSED_MEANFIELD = 1, the default) against the separate mean-field
pass (FN_OPT_FUSED_MEANFIELD = 0): the two paths sum the same float32
values in the same order and scale them the same way, so every output of
the local energy, of the one-pass local energy and VMC gradient and of the
Metropolis moves is compared bit for bit.  The atoms with equal spin groups
of at most five electrons (be4, ne10) take the fused path; the 18-electron
atom (groups of nine) does not, and the option must not change it either.
Oracle parity of the fused path is covered by the parity and gate tests,
which run with the default."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_2011_07125_amd import ferminet as F  # noqa: E402
from paper_2011_07125_amd import inputs as I  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _restore_default():
    yield
    F.set_option(F.FN_OPT_FUSED_MEANFIELD, 1)
    F.release_workspaces()


def _run(w, d, form, fused, walkers, rescue=None):
    F.set_option(F.FN_OPT_FUSED_MEANFIELD, 1 if fused else 0)
    cfg = w["cfg"]
    pos = d["pos"][:walkers].clone()
    args = (cfg, pos, d["nuc_pos"], d["nuc_charge"], d["params"])
    res = {}
    frac = I.RESCUE[w["name"]][form] if rescue is None else rescue
    out = F.ferminet_local_energy(*args, precision=form, rescue=frac)
    res.update({"le_" + k: v for k, v in out.items()})
    out, grad, stats = F.vmc_local_energy_gradient(*args, precision=form, rescue=frac)
    res.update({"leg_" + k: v for k, v in out.items()})
    res["grad"] = grad
    res["stats"] = stats
    s, l = F.ferminet_logpsi(*args, precision=form)
    acc = F.vmc_mcmc_step(*args, l, s, 3, 0.05, 17, 0, precision=form)
    res.update({"mc_pos": pos, "mc_logpsi": l, "mc_sign": s, "mc_acc": acc})
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.mark.parametrize("form", ["bf16", "fp32_fp64det"])
@pytest.mark.parametrize("name,walkers", [("be4", 256), ("ne10", 4096), ("ne10", 777), ("ar18", 64)])
def test_fused_meanfield_same_bits(name, walkers, form):
    """777 Ne-like walkers: 1554 spin-group row tiles (padded to 1560) of
    two column tiles each, spread over the resident workgroups, so that
    the looping workgroups take unequal numbers of tiles, padding tiles
    among them."""
    say(f"case fused mean field {name} {form} W={walkers}")
    w = I.make_workload(name)
    w["name"] = name
    d = F.to_device(w)
    a = _run(w, d, form, True, walkers)
    b = _run(w, d, form, False, walkers)
    for k in a:
        same = np.array_equal(a[k], b[k], equal_nan=True)
        if not same:
            diff = np.abs(a[k].astype(np.float64) - b[k].astype(np.float64))
            say(f"   {k}: max |d| {np.nanmax(diff):.3e} at {np.unravel_index(np.nanargmax(diff), diff.shape)}")
        assert same, f"{name}/{form}: {k} differs between the fused and the separate mean-field pass"


@pytest.mark.parametrize("form", ["bf16", "fp32_fp64det"])
@pytest.mark.parametrize("n_up,n_down", [(1, 1), (3, 3), (4, 4), (3, 2)])
def test_fused_meanfield_spin_group_sizes(n_up, n_down, form):
    """Every spin-group size the fused tiles take (one to five electrons per
    spin; five is the Ne-like case above), on a two-nucleus molecule with
    128-wide one-electron layers, a ragged batch of 37 walkers and 2%
    float64 re-evaluation; 3/2 spins do not take the fused path, and the
    option must not change them either."""
    say(f"case fused mean field spins {n_up}/{n_down} {form}")
    w = I.custom_workload(n_up, n_down, [[0.0, 0.0, -0.7], [0.0, 0.0, 0.7]], [3.0, 2.0], 37, 3, 128, 16, 4,
                          seed=31 + n_up, pos_std=0.8)
    d = F.to_device(w)
    fused_launches = {}
    for fused in (True, False):
        F.set_option(F.FN_OPT_FUSED_MEANFIELD, 1 if fused else 0)
        F.stage_timing(True)
        F.ferminet_local_energy(w["cfg"], d["pos"], d["nuc_pos"], d["nuc_charge"], d["params"], precision=form)
        torch.cuda.synchronize()
        fused_launches[fused] = F.stage_times().get("gemm_layer_mf", (0.0, 0))[1]
        F.stage_timing(False)
    # the jet pass forms the means in the layer kernel for equal spins only
    assert fused_launches[True] == (2 if n_up == n_down else 0) and fused_launches[False] == 0, fused_launches
    a = _run(w, d, form, True, 37, rescue=0.02)
    b = _run(w, d, form, False, 37, rescue=0.02)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{n_up}/{n_down} {form}: {k} differs"
