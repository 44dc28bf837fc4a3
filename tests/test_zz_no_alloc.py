"""ferminet_logpsi_noalloc (the value pass on the library's own 64 MiB
device array, for callers that cannot allocate) against ferminet_logpsi
with a caller workspace, through the C ABI: bit for bit on two calls in a
row, the second with a smaller batch (the array keeps the first call's
contents), in both forms; a network whose one-walker workspace exceeds the
array is rejected before anything is enqueued."""
import os
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


@pytest.mark.parametrize("form", ["bf16", "fp32"])
def test_noalloc_logpsi_equals_workspace_call(form):
    w = I.make_workload("ne10")
    cfg = w["cfg"]
    d = F.to_device(w)
    for W in (4096, 100):
        say(f"case noalloc logpsi ne10 {form} W={W}")
        pos = d["pos"][:W].contiguous()
        s_ref, l_ref = F.ferminet_logpsi(cfg, pos, d["nuc_pos"], d["nuc_charge"], d["params"], precision=form)
        sign = torch.full((W,), float("nan"), device="cuda")
        lp = torch.full((W,), float("nan"), device="cuda")
        F.ferminet_logpsi_noalloc(cfg, pos, d["nuc_pos"], d["nuc_charge"], d["params"], sign, lp, precision=form)
        torch.cuda.synchronize()
        say(f"   max |d log|psi|| {(lp - l_ref).abs().max().item():.3e}, sign equal {torch.equal(sign, s_ref)}")
        assert torch.equal(sign, s_ref)
        assert torch.equal(lp, l_ref)


def test_noalloc_rejects_a_network_beyond_the_array():
    say("case noalloc rejects a one-walker workspace beyond 64 MiB")
    cfg = I.make_cfg(16, 16, 4, 8, 1024, 64, 64, "bf16")
    need = F.workspace_bytes(cfg, 1, F.FN_ENTRY_LOGPSI, "bf16")
    assert need > 64 << 20
    P = F.param_count(cfg)
    pos = torch.zeros((2, 32, 3), device="cuda")
    nuc = torch.zeros((4, 3), device="cuda")
    Z = torch.ones(4, device="cuda")
    params = torch.zeros(P, device="cuda")
    sign = torch.full((2,), 7.0, device="cuda")
    lp = torch.full((2,), 7.0, device="cuda")
    with pytest.raises(F.FerminetError) as e:
        F.ferminet_logpsi_noalloc(cfg, pos, nuc, Z, params, sign, lp, precision="bf16")
    assert e.value.status == 4
    torch.cuda.synchronize()
    assert (sign == 7.0).all() and (lp == 7.0).all()
