"""log|psi| as a differentiable torch function of the parameters.

forward calls ferminet_logpsi; backward calls ferminet_grad_logpsi with the
incoming gradient as the walker cotangent, so that
    torch.autograd.grad((c * logpsi).sum(), params)
is the hand-written adjoint sum_w c_w d log|psi_w| / d theta.  The sign is
not differentiable; positions receive no gradient.
"""
from __future__ import annotations

import torch

from . import ferminet as F


class FermiNetLogPsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, pos, nuc_pos, nuc_charge, cfg, precision):
        sign, logpsi = F.ferminet_logpsi(cfg, pos, nuc_pos, nuc_charge, params, precision=precision)
        ctx.save_for_backward(params, pos, nuc_pos, nuc_charge)
        ctx.cfg = cfg
        ctx.precision = precision
        ctx.mark_non_differentiable(sign)
        return logpsi, sign

    @staticmethod
    def backward(ctx, g_logpsi, g_sign):
        params, pos, nuc_pos, nuc_charge = ctx.saved_tensors
        if g_logpsi is None:
            return None, None, None, None, None, None
        grad = F.ferminet_grad_logpsi(ctx.cfg, pos, nuc_pos, nuc_charge, params, g_logpsi.contiguous().float(),
                                      precision=ctx.precision)
        return grad, None, None, None, None, None


def logpsi(params, pos, nuc_pos, nuc_charge, cfg, precision=None):
    """(log|psi| [W], sign [W]); differentiable in params."""
    return FermiNetLogPsi.apply(params, pos, nuc_pos, nuc_charge, cfg, precision)
