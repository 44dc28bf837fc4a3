"""A VMC optimisation loop over the library's one-iteration entry point
(vmc_train_step): host-side schedule only, every step of an iteration
runs in the HIP kernels.

The paper trains with KFAC and names the number of Metropolis steps per
update (10, then 20 for the second-row atoms) but no other settings; the
defaults here follow the FermiNet defaults (learning rate 0.05 / (1 + t /
10^4), damping 10^-3, norm constraint 10^-3, factor decay 0.95, energies
clipped at 5 mean absolute deviations) and are arguments.  The proposal
width is adapted every few iterations towards an acceptance rate of one
half, as random-walk Metropolis samplers commonly are.
"""
from __future__ import annotations

import math

import torch

from . import ferminet as F


def learning_rate(t: int, rate: float = 0.05, delay: float = 1e4, decay: float = 1.0) -> float:
    """rate (1 + t / delay)^-decay."""
    return rate * math.pow(1.0 + t / delay, -decay)


def adapt_width(width: float, acceptance: float, target: float = 0.5, factor: float = 1.1, lo: float = 1e-3,
                hi: float = 10.0) -> float:
    """One multiplicative step of the proposal width towards the target
    acceptance rate, kept inside [lo, hi]."""
    if acceptance > target:
        width *= factor
    elif acceptance < target:
        width /= factor
    return min(hi, max(lo, width))


def train(cfg, pos, nuc_pos, nuc_charge, params, iterations, precision="bf16", mcmc_steps=10, width=0.1,
          burn_in=100, seed=0, rate=0.05, delay=1e4, damping=1e-3, norm_constraint=1e-3, factor_decay=0.95,
          clip_scale=5.0, rescue=0.0, adapt_every=10, callback=None):
    """Optimise params (in place) for `iterations` iterations; pos is
    updated in place.  Returns the per-iteration history: dicts with the
    mean and variance of E_L, the acceptance rate, the proposal width and
    the learning rate."""
    W = pos.shape[0]
    counter = 0
    if burn_in > 0:
        s, lp = F.ferminet_logpsi(cfg, pos, nuc_pos, nuc_charge, params, precision=precision)
        chunk = adapt_every if adapt_every > 0 else burn_in
        for k in range(0, burn_in, chunk):
            n = min(chunk, burn_in - k)
            acc = F.vmc_mcmc_step(cfg, pos, nuc_pos, nuc_charge, params, lp, s, n, width, seed, counter,
                                  precision=precision)
            counter += n
            width = adapt_width(width, acc.sum().item() / (W * n))
    _, total = F.kfac_layout(cfg)
    factors = torch.zeros(total, dtype=torch.float32, device=pos.device)
    history = []
    acc_sum = 0.0
    for t in range(iterations):
        lr = learning_rate(t, rate, delay)
        _, st = F.vmc_train_step(cfg, pos, nuc_pos, nuc_charge, params, factors, mcmc_steps, width, seed, counter,
                                 lr, damping, norm_constraint, 0.0 if t == 0 else factor_decay, clip_scale,
                                 precision=precision, rescue=rescue)
        counter += mcmc_steps
        st = st.cpu().tolist()
        rec = {"t": t, "energy": st[0], "variance": st[1], "acceptance": st[2], "width": width, "lr": lr,
               "step": st[7], "left_out": int(st[8])}
        history.append(rec)
        acc_sum += st[2]
        if adapt_every and (t + 1) % adapt_every == 0:
            width = adapt_width(width, acc_sum / adapt_every)
            acc_sum = 0.0
        if callback is not None:
            callback(rec)
    return history
