"""ctypes front end of the FP64 CPU oracle (oracle/oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product path (the HIP
library and its Python binding) never imports this module.

Every array goes in as float64 (callers hand over their float32 inputs
promoted to float64, so both sides see identical values).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so with g++ (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, dbl, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        lib.orc_param_count.argtypes = [P]
        lib.orc_param_count.restype = i64
        lib.orc_param_offsets.argtypes = [P, P, i32]
        lib.orc_param_offsets.restype = i32
        lib.orc_slogdet.argtypes = [i32, P, P, P]
        lib.orc_eval.argtypes = [P, i32, P, P, P, P, i32, i32, P, P, P, P, P, P]
        lib.orc_potential.argtypes = [P, i32, P, P, P, P]
        lib.orc_param_grad.argtypes = [P, i32, P, P, P, i32, P, i32, P]
        lib.orc_det_terms.argtypes = [P, i32, P, P, P, i32, P, P]
        lib.orc_det_terms.restype = i32
        lib.orc_orbitals.argtypes = [P, i32, P, P, P, i32, P]
        lib.orc_orbitals.restype = i32
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox4x32_10.restype = None
        lib.orc_mcmc_noise.argtypes = [i32, i32, i32, u64, u64, P, P]
        lib.orc_mcmc.argtypes = [P, i32, P, P, P, i32, dbl, P, P, u64, u64, i32, P, P, P]
        lib.orc_layer_inputs.argtypes = [P, i32, P, P, P, i32, P, P, P]
        lib.orc_preact_cotangents.argtypes = [P, i32, P, P, P, i32, i32, i32, P]
        for f in ("orc_slogdet", "orc_eval", "orc_potential", "orc_param_grad", "orc_mcmc_noise", "orc_mcmc",
                  "orc_layer_inputs", "orc_preact_cotangents"):
            getattr(lib, f).restype = i32
        _lib = lib
    return _lib


def _cfg(cfg) -> np.ndarray:
    """[n, n_up, n_down, N, L, d1, d2, K, envelope]; envelope 0 isotropic
    (default), 1 full covariance."""
    env = {"isotropic": 0, "full": 1}.get(cfg.get("envelope", 0), cfg.get("envelope", 0))
    return np.array([cfg["n_elec"], cfg["n_up"], cfg["n_down"], cfg["n_nuc"], cfg["n_layers"],
                     cfg["width1"], cfg["width2"], cfg["n_det"], env], dtype=np.int32)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _threads(n):
    return int(n) if n else 0


def param_count(cfg) -> int:
    return int(_load().orc_param_count(_p(_cfg(cfg))))


def param_offsets(cfg) -> np.ndarray:
    out = np.zeros(4096, dtype=np.int64)
    c = _cfg(cfg)
    k = _load().orc_param_offsets(_p(c), _p(out), out.size)
    assert k > 0
    return out[:k].copy()


def slogdet(a):
    a = _d(a)
    n = a.shape[0]
    s = np.zeros(1)
    la = np.zeros(1)
    _load().orc_slogdet(n, _p(a), _p(s), _p(la))
    return float(s[0]), float(la[0])


def evaluate(cfg, pos, nuc_pos, nuc_charge, params, energy=True, threads=None, grad_pos=False):
    """sign, log|psi| and (energy=True) E_L, E_kin, E_pot per walker."""
    pos = _d(pos)
    W = pos.shape[0]
    nuc, Z, prm = _d(nuc_pos), _d(nuc_charge), _d(params)
    c = _cfg(cfg)
    out = {k: np.zeros(W) for k in ("sign", "logpsi", "e_loc", "e_kin", "e_pot")}
    gp = np.zeros((W, 3 * cfg["n_elec"])) if grad_pos else None
    rc = _load().orc_eval(_p(c), W, _p(pos), _p(nuc), _p(Z), _p(prm), 1 if energy else 0, _threads(threads),
                          _p(out["sign"]), _p(out["logpsi"]), _p(out["e_loc"]), _p(out["e_kin"]),
                          _p(out["e_pot"]), _p(gp) if gp is not None else None)
    assert rc == 0, rc
    if not energy:
        for k in ("e_loc", "e_kin", "e_pot"):
            del out[k]
    if gp is not None:
        out["grad_pos"] = gp
    return out


def potential(cfg, pos, nuc_pos, nuc_charge):
    """(V_ee, V_en, V_nn) per walker, [W][3]."""
    pos = _d(pos)
    W = pos.shape[0]
    out = np.zeros((W, 3))
    rc = _load().orc_potential(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(nuc_charge)), _p(out))
    assert rc == 0
    return out


def param_grad(cfg, pos, nuc_pos, params, sel, threads=None):
    """d log|psi_w| / d theta_p for p in sel: [W][len(sel)]."""
    pos = _d(pos)
    W = pos.shape[0]
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    out = np.zeros((W, sel.size))
    rc = _load().orc_param_grad(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), sel.size, _p(sel),
                                _threads(threads), _p(out))
    assert rc == 0
    return out


def det_terms(cfg, pos, nuc_pos, params, threads=None):
    """(sign_k, log|det_k^up det_k^down|) of every determinant term: [W][K] each."""
    pos = _d(pos)
    W = pos.shape[0]
    sk = np.zeros((W, cfg["n_det"]))
    lk = np.zeros((W, cfg["n_det"]))
    rc = _load().orc_det_terms(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), _threads(threads),
                               _p(sk), _p(lk))
    assert rc == 0
    return sk, lk


def node_conditioning(cfg, pos, nuc_pos, params, threads=None):
    """kappa_w = max_k |P_k| / |psi| (at least 1/K, 1 for a single
    determinant, infinite at an exact node): how strongly the signed sum of
    Eq. (4) cancels at each walker."""
    sk, lk = det_terms(cfg, pos, nuc_pos, params, threads)
    m = lk.max(axis=1, keepdims=True)
    s = (sk * np.exp(lk - m)).sum(axis=1)
    with np.errstate(divide="ignore"):
        return 1.0 / np.abs(s)


def orbital_matrices(cfg, pos, nuc_pos, params, threads=None):
    """The orbital matrices of every walker: (up [W][K][n_up][n_up],
    down [W][K][n_down][n_down]), A[i][j] = phi_i(r_j)."""
    pos = _d(pos)
    W, K, nu, nd = pos.shape[0], cfg["n_det"], cfg["n_up"], cfg["n_down"]
    out = np.zeros((W, K * (nu * nu + nd * nd)))
    rc = _load().orc_orbitals(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), _threads(threads), _p(out))
    assert rc == 0
    return out[:, :K * nu * nu].reshape(W, K, nu, nu), out[:, K * nu * nu:].reshape(W, K, nd, nd)


def amplification(cfg, pos, nuc_pos, params, threads=None):
    """Per-walker rounding amplification A_w = kappa_w * max_{k,a} cond_1(A^{ka})
    with kappa_w = max_k |P_k| / |psi_w| (cancellation of the sum of Eq. (4))
    and cond_1 the 1-norm condition number of each orbital matrix."""
    kap = node_conditioning(cfg, pos, nuc_pos, params, threads)
    up, dn = orbital_matrices(cfg, pos, nuc_pos, params, threads)
    cmax = np.ones(kap.shape)
    for M in (up, dn):
        if M.shape[-1] == 0:
            continue
        c = np.linalg.cond(M.reshape(-1, M.shape[-1], M.shape[-1]), p=1).reshape(M.shape[0], -1)
        cmax = np.maximum(cmax, c.max(axis=1))
    return kap * cmax, kap, cmax


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def mcmc_noise(W, n_elec, n_steps, seed, counter=0):
    noise = np.zeros((n_steps, W, 3 * n_elec))
    uni = np.zeros((n_steps, W))
    _load().orc_mcmc_noise(W, n_elec, n_steps, seed, counter, _p(noise), _p(uni))
    return noise, uni


def mcmc(cfg, pos, nuc_pos, params, logpsi, sign, n_steps, width, noise=None, uniforms=None, seed=0, counter=0,
         threads=None):
    """Replay n_steps Metropolis steps; returns (pos, logpsi, sign, n_accepted)."""
    pos = _d(pos).copy()
    W = pos.shape[0]
    lp = _d(logpsi).copy()
    sg = _d(sign).copy()
    acc = np.zeros(W, dtype=np.int32)
    nz = _d(noise) if noise is not None else None
    un = _d(uniforms) if uniforms is not None else None
    rc = _load().orc_mcmc(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), n_steps, float(width),
                          _p(nz) if nz is not None else None, _p(un) if un is not None else None, seed, counter,
                          _threads(threads), _p(lp), _p(sg), _p(acc))
    assert rc == 0
    return pos, lp, sg, acc


# ------------------------------------------------------------------ KFAC
# Kronecker-factored curvature statistics (Martens and Grosse 2015; the
# paper's optimiser).  For a dense layer applied at positions r of walker w
# (electrons, electron pairs, or the electrons of one spin) with inputs
# a_{w,r}, a~ = [a; 1] (the bias as a last input), and pre-activation
# cotangents g_{w,r} = d log|psi_w| / d z_{w,r}:
#     A = sum_w c_w sum_r a~ a~^T        G = sum_w c_w sum_r g g^T
# for caller weights c_w.  sum_w c_w sum_r a~ g^T is the gradient of
# sum_w c_w log|psi_w| with respect to [weights; bias].

def _din(cfg, l):
    return 4 * cfg["n_nuc"] if l == 0 else cfg["width1"]


def _ein(cfg, l):
    return 4 if l == 0 else cfg["width2"]


def layer_inputs(cfg, pos, nuc_pos, params, threads=None):
    """Inputs of the dense layers: (f1 [W][L][n][fw_max], f2 [W][L-1][n^2][ein_max],
    fo [W][n][d1]); f_i zero-padded to fw_max = 3 max(din) + 2 ein_max."""
    pos = _d(pos)
    W, n = pos.shape[0], cfg["n_elec"]
    L, d1 = cfg["n_layers"], cfg["width1"]
    ein_max = max(4, cfg["width2"])
    fw_max = 3 * max(4 * cfg["n_nuc"], d1) + 2 * ein_max
    f1 = np.zeros((W, L, n, fw_max))
    f2 = np.zeros((W, max(L - 1, 0), n * n, ein_max))
    fo = np.zeros((W, n, d1))
    rc = _load().orc_layer_inputs(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), _threads(threads),
                                  _p(f1), _p(f2), _p(fo))
    assert rc == 0
    return f1, f2, fo


def preact_cotangents(cfg, pos, nuc_pos, params, kind, layer, threads=None):
    """d log|psi_w| / d z at every (position, unit) of one dense layer,
    [W][positions][units]: kind 0 one-electron layer (n x d1), 1
    two-electron layer (n^2 pairs i n + j x d2), 2 orbitals of spin `layer`
    (n_a x K n_a)."""
    pos = _d(pos)
    W, n = pos.shape[0], cfg["n_elec"]
    if kind == 0:
        P, U = n, cfg["width1"]
    elif kind == 1:
        P, U = n * n, cfg["width2"]
    else:
        P = cfg["n_up"] if layer == 0 else cfg["n_down"]
        U = cfg["n_det"] * P
    out = np.zeros((W, P, U))
    rc = _load().orc_preact_cotangents(_p(_cfg(cfg)), W, _p(pos), _p(_d(nuc_pos)), _p(_d(params)), int(kind),
                                       int(layer), _threads(threads), _p(out))
    assert rc == 0
    return out


def kfac_blocks(cfg):
    """The dense layers in order: (name, kind, layer, d_in, d_out, positions)."""
    n, L = cfg["n_elec"], cfg["n_layers"]
    out = []
    for l in range(L):
        out.append((f"layer{l}", 0, l, 3 * _din(cfg, l) + 2 * _ein(cfg, l), cfg["width1"], n))
    for l in range(L - 1):
        out.append((f"pair{l}", 1, l, _ein(cfg, l), cfg["width2"], n * n))
    for a, na in enumerate((cfg["n_up"], cfg["n_down"])):
        if na:
            out.append((f"orbital{a}", 2, a, cfg["width1"], cfg["n_det"] * na, na))
    return out


def kfac_inputs_and_cotangents(cfg, pos, nuc_pos, params, threads=None):
    """Per block: (name, a~ [W][positions][d_in + 1], g [W][positions][d_out])."""
    f1, f2, fo = layer_inputs(cfg, pos, nuc_pos, params, threads)
    W = f1.shape[0]
    res = []
    for name, kind, l, din, dout, npos in kfac_blocks(cfg):
        if kind == 0:
            a = f1[:, l, :, :din]
        elif kind == 1:
            a = f2[:, l, :, :din]
        else:
            j0 = 0 if l == 0 else cfg["n_up"]
            a = fo[:, j0:j0 + npos, :]
        at = np.concatenate([a, np.ones((W, npos, 1))], axis=2)
        g = preact_cotangents(cfg, pos, nuc_pos, params, kind, l, threads)
        res.append((name, at, g))
    return res


def kfac_factors(cfg, pos, nuc_pos, params, weights, threads=None):
    """[(name, A, G)] with A = sum_w c_w sum_r a~ a~^T, G = sum_w c_w sum_r g g^T."""
    c = np.asarray(weights, dtype=np.float64)
    out = []
    for name, at, g in kfac_inputs_and_cotangents(cfg, pos, nuc_pos, params, threads):
        A = np.einsum("w,wri,wrj->ij", c, at, at)
        G = np.einsum("w,wri,wrj->ij", c, g, g)
        out.append((name, A, G))
    return out


def kfac_damping_pi(A, G):
    """pi of the factored Tikhonov damping (Martens and Grosse 2015, sec. 6.3):
    sqrt((tr A / dim A) / (tr G / dim G)), 1 when either trace vanishes."""
    ta, tg = np.trace(A) / A.shape[0], np.trace(G) / G.shape[0]
    return float(np.sqrt(ta / tg)) if ta > 0 and tg > 0 else 1.0


def kfac_precondition(cfg, factors, grad, damping):
    """The KFAC step direction: for every dense layer with factors (A, G) and
    gradient block M = [weights; bias] ((d_in + 1) x d_out, as stored in
    the parameter layout),
        X = (A + pi sqrt(lambda) I)^-1 M (G + sqrt(lambda) / pi I)^-1
    (factored Tikhonov damping); the envelope parameters keep their
    gradient.  factors: [(name, A, G)] as kfac_factors returns them."""
    out = np.array(grad, dtype=np.float64, copy=True)
    offs = _kfac_param_offsets(cfg)
    s = np.sqrt(damping)
    for name, A, G in factors:
        off = offs[name]
        dA, dG = A.shape[0], G.shape[0]
        M = out[off:off + dA * dG].reshape(dA, dG)
        pi = kfac_damping_pi(A, G)
        Ad = A + pi * s * np.eye(dA)
        Gd = G + (s / pi) * np.eye(dG)
        X = np.linalg.solve(Gd.T, np.linalg.solve(Ad, M).T).T
        out[off:off + dA * dG] = X.reshape(-1)
    return out


def _kfac_param_offsets(cfg):
    """Offset of each dense layer's [weights; bias] in the parameter layout
    (the weight block, immediately followed by its bias)."""
    off = param_offsets(cfg)  # V_l, b_l per layer; W_l, c_l per pair layer; w_a, g_a per spin; ...
    L = cfg["n_layers"]
    res = {}
    for name, kind, l, din, dout, npos in kfac_blocks(cfg):
        idx = 2 * l if kind == 0 else (2 * L + 2 * l if kind == 1 else 2 * L + 2 * (L - 1) + 2 * l)
        res[name] = int(off[idx])
    return res


# ------------------------------------------------------- VMC iteration
# One optimisation iteration of the variational energy E[E_L] under psi^2
# (Eq. (3); Section 2 names KFAC as the optimiser but gives no settings, so
# the following readings are stated once here):
#  * sampling: the caller's walkers take n_steps Metropolis steps from
#    log|psi| at the current parameters;
#  * walkers whose local energy is not finite (an exact node of psi, R13's
#    coincident particles) take no part in what follows; W_f counts the
#    others (the paper is silent; a single such walker would otherwise turn
#    every statistic, the gradient and the step into NaN);
#  * local energies are clipped to median +- clip_scale * mean|E_L - median|
#    (no clipping for clip_scale <= 0) and the gradient is the energy
#    gradient 2 sum_w (E~_w - mean E~) / W_f * d log|psi_w| / d theta with the
#    clipped energies E~;
#  * the KFAC factors are running averages F <- decay F + (1 - decay) F_batch
#    with batch weights 1/W_f (decay = 0 starts them from the batch);
#  * the step is theta <- theta - lr c X with X the damped KFAC direction of
#    the gradient and c = min(1, sqrt(C / (lr^2 <X, g>))) (KFAC's norm
#    constraint C; no constraint for C <= 0 or <X, g> <= 0).

def clip_energies(e, clip_scale):
    """E_L clipped to median +- clip_scale * (mean absolute deviation from
    the median); the input itself for clip_scale <= 0."""
    e = np.asarray(e, dtype=np.float64)
    if clip_scale <= 0:
        return e.copy()
    med = np.median(e)
    tv = np.mean(np.abs(e - med))
    return np.clip(e, med - clip_scale * tv, med + clip_scale * tv)


def norm_constraint_coefficient(x_dot_g, lr, norm_constraint):
    """lr * min(1, sqrt(C / (lr^2 <X, g>))): the length of the step along X."""
    if norm_constraint > 0 and x_dot_g > 0:
        return lr * min(1.0, float(np.sqrt(norm_constraint / (lr * lr * x_dot_g))))
    return lr


def vmc_train_step(cfg, pos, nuc_pos, nuc_charge, params, factors, n_steps, width, lr, damping, norm_constraint,
                   decay, clip_scale, noise=None, uniforms=None, seed=0, counter=0, threads=None):
    """One VMC iteration.  factors: [(name, A, G)] running averages from the
    previous iteration, or None (then decay is taken as 0).  Returns a dict
    with the new pos, params and factors and the intermediate results."""
    params = _d(params)
    r0 = evaluate(cfg, pos, nuc_pos, nuc_charge, params, energy=False, threads=threads)
    pos, lp, sg, acc = mcmc(cfg, pos, nuc_pos, params, r0["logpsi"], r0["sign"], n_steps, width, noise, uniforms,
                            seed, counter, threads)
    W = pos.shape[0]
    r = evaluate(cfg, pos, nuc_pos, nuc_charge, params, threads=threads)
    e = r["e_loc"]
    # walkers with a non-finite local energy (exact nodes, coincident
    # particles) take no part in the statistics, the gradient or the factors
    fin = np.isfinite(e)
    Wf = int(fin.sum())
    ec = e.copy()
    ec[fin] = clip_energies(e[fin], clip_scale)
    c = (ec[fin] - ec[fin].mean()) / Wf
    P = param_count(cfg)
    per = param_grad(cfg, pos[fin], nuc_pos, params, np.arange(P), threads=threads)
    g = 2.0 * (c @ per)
    batch = kfac_factors(cfg, pos[fin], nuc_pos, params, np.full(Wf, 1.0 / Wf), threads=threads)
    if factors is None:
        new_f = batch
    else:
        new_f = [(n, decay * A0 + (1 - decay) * A, decay * G0 + (1 - decay) * G)
                 for (n, A0, G0), (_, A, G) in zip(factors, batch)]
    X = kfac_precondition(cfg, new_f, g, damping)
    q = float(X @ g)
    coef = norm_constraint_coefficient(q, lr, norm_constraint)
    return {"pos": pos, "logpsi": lp, "sign": sg, "n_accepted": acc, "e_loc": e, "e_clip": ec, "grad": g,
            "direction": X, "x_dot_g": q, "coef": coef, "factors": new_f, "params": params - coef * X,
            "left_out": W - Wf}
