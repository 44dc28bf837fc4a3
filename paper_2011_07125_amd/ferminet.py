"""Thin ctypes binding of libferminet.so (the C ABI of include/ferminet.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory (inputs, outputs
and the workspace) and the current HIP stream.  There is no fallback: if
the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libferminet.so")

FN_PREC_FP32, FN_PREC_BF16, FN_PREC_FP32_FP64DET, FN_PREC_FP64 = 0, 1, 2, 3
FN_ENV_ISOTROPIC, FN_ENV_FULL = 0, 1
ENVELOPES = {"isotropic": FN_ENV_ISOTROPIC, "full": FN_ENV_FULL}
PRECISIONS = {"fp32": FN_PREC_FP32, "bf16": FN_PREC_BF16, "fp32_fp64det": FN_PREC_FP32_FP64DET, "fp64": FN_PREC_FP64}
FN_ENTRY_LOGPSI, FN_ENTRY_LOCAL_ENERGY, FN_ENTRY_GRAD_LOGPSI, FN_ENTRY_MCMC, FN_ENTRY_KFAC = 0, 1, 2, 3, 4
FN_ENTRY_KFAC_PRECONDITION, FN_ENTRY_TRAIN, FN_ENTRY_LOCAL_ENERGY_GRADIENT = 5, 6, 7
FN_OPT_FUSED_MEANFIELD = 1
STATUS = {0: "FN_OK", 1: "FN_ERR_NULL", 2: "FN_ERR_CONFIG", 3: "FN_ERR_SPINS", 4: "FN_ERR_WORKSPACE",
          5: "FN_ERR_UNSUPPORTED", 6: "FN_ERR_HIP", 7: "FN_ERR_ARG"}


class FerminetError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({_lib().ferminet_status_string(status).decode()})")
        self.status = status


class fn_config(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("n_elec", "n_up", "n_down", "n_nuc", "n_layers", "width1", "width2",
                                               "n_det", "precision", "envelope")] + [("rescue_fraction", ctypes.c_float)]


class fn_param_block(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("offset", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64)]


class fn_kfac_block(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("offset_A", ctypes.c_int64), ("offset_G", ctypes.c_int64),
                ("dim_A", ctypes.c_int32), ("dim_G", ctypes.c_int32), ("positions", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class fn_train_options(ctypes.Structure):
    _fields_ = [("mcmc_steps", ctypes.c_int32), ("mcmc_width", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("counter", ctypes.c_uint64), ("learning_rate", ctypes.c_float), ("damping", ctypes.c_float),
                ("norm_constraint", ctypes.c_float), ("factor_decay", ctypes.c_float),
                ("clip_scale", ctypes.c_float), ("reserved", ctypes.c_int32)]


EXPORTS = ("ferminet_status_string", "ferminet_param_count", "ferminet_param_layout", "ferminet_workspace_bytes",
           "ferminet_logpsi", "ferminet_logpsi_noalloc", "ferminet_local_energy", "ferminet_grad_logpsi", "vmc_energy_gradient",
           "vmc_local_energy_gradient", "vmc_mcmc_step", "vmc_mcmc_noise", "ferminet_kfac_factors", "ferminet_kfac_layout",
           "ferminet_kfac_precondition", "vmc_train_step",
           "ferminet_stage_timing", "ferminet_stage_times", "ferminet_stage_name", "ferminet_set_option")

_LIB = None
_LOCK = threading.Lock()


def _lib():
    global _LIB
    if _LIB is None:
        with _LOCK:
            if _LIB is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_2011_07125_amd.build)")
                lib = ctypes.CDLL(LIB_PATH)
                P, i32, i64, u64, f32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                             ctypes.c_float, ctypes.c_size_t)
                C = ctypes.POINTER(fn_config)
                lib.ferminet_status_string.argtypes = [i32]
                lib.ferminet_status_string.restype = ctypes.c_char_p
                lib.ferminet_param_count.argtypes = [C]
                lib.ferminet_param_count.restype = i64
                lib.ferminet_param_layout.argtypes = [C, P, i32, P]
                lib.ferminet_workspace_bytes.argtypes = [C, i32, i32, P]
                lib.ferminet_logpsi.argtypes = [C, i32, P, P, P, P, P, P, P, P, sz, P]
                lib.ferminet_logpsi_noalloc.argtypes = [C, i32, P, P, P, P, P, P, P, P]
                lib.ferminet_local_energy.argtypes = [C, i32, P, P, P, P, P, P, P, P, P, P, P, sz, P]
                lib.ferminet_grad_logpsi.argtypes = [C, i32, P, P, P, P, P, P, P, P, sz, P]
                lib.vmc_energy_gradient.argtypes = [C, i32, P, P, P, P, P, P, P, P, P, sz, P]
                lib.vmc_local_energy_gradient.argtypes = [C, i32, P, P, P, P, P, P, P, P, P, P, P, P, P, sz, P]
                lib.ferminet_kfac_factors.argtypes = [C, i32, P, P, P, P, P, P, P, P, sz, P]
                lib.ferminet_kfac_layout.argtypes = [C, P, i32, P, P]
                lib.ferminet_kfac_precondition.argtypes = [C, P, P, f32, P, P, sz, P]
                lib.vmc_mcmc_step.argtypes = [C, i32, P, P, P, P, P, P, P, i32, f32, u64, u64, P, P, P, P, sz, P]
                lib.vmc_mcmc_noise.argtypes = [i32, i32, i32, u64, u64, P, P, P]
                lib.vmc_train_step.argtypes = [C, i32, P, P, P, P, P, P, ctypes.POINTER(fn_train_options), P, P, P,
                                               P, P, sz, P]
                lib.ferminet_stage_timing.argtypes = [i32]
                lib.ferminet_stage_times.argtypes = [P, P, i32]
                lib.ferminet_stage_name.argtypes = [i32]
                lib.ferminet_set_option.argtypes = [i32, i32]
                for f in EXPORTS[2:]:
                    getattr(lib, f).restype = i32
                lib.ferminet_stage_name.restype = ctypes.c_char_p
                _LIB = lib
    return _LIB


def make_config(cfg: dict, precision=None, rescue: float = 0.0) -> fn_config:
    """rescue: fraction of walkers whose local energy is re-evaluated in
    float64 (those of largest determinant-sum cancellation)."""
    prec = cfg.get("precision", "fp32") if precision is None else precision
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    env = cfg.get("envelope", "isotropic")
    env = ENVELOPES[env] if isinstance(env, str) else int(env)
    return fn_config(cfg["n_elec"], cfg["n_up"], cfg["n_down"], cfg["n_nuc"], cfg["n_layers"], cfg["width1"],
                     cfg["width2"], cfg["n_det"], prec, env, float(rescue))


def _check(st: int, where: str):
    if st != 0:
        raise FerminetError(st, where)


def param_count(cfg: dict) -> int:
    c = make_config(cfg, "fp32")
    return int(_lib().ferminet_param_count(ctypes.byref(c)))


def param_layout(cfg: dict):
    c = make_config(cfg, "fp32")
    n = ctypes.c_int32(0)
    buf = (fn_param_block * 64)()
    _check(_lib().ferminet_param_layout(ctypes.byref(c), buf, 64, ctypes.byref(n)), "ferminet_param_layout")
    return [(buf[i].name.decode(), buf[i].offset, buf[i].rows, buf[i].cols) for i in range(n.value)]


def workspace_bytes(cfg: dict, chunk_walkers: int, entry: int, precision=None, rescue: float = 0.0) -> int:
    c = make_config(cfg, precision, rescue)
    out = ctypes.c_size_t(0)
    _check(_lib().ferminet_workspace_bytes(ctypes.byref(c), int(chunk_walkers), int(entry), ctypes.byref(out)),
           "ferminet_workspace_bytes")
    return int(out.value)


# workspace buffers kept per (device, entry): the caller-owned scratch of the C ABI
_WS = {}


def workspace(cfg: dict, W: int, entry: int, precision=None, device=None, max_chunk=None,
              rescue: float = 0.0) -> torch.Tensor:
    device = torch.device("cuda") if device is None else torch.device(device)
    chunk = W if max_chunk is None else max(1, min(W, max_chunk))
    nbytes = workspace_bytes(cfg, max(1, chunk), entry, precision, rescue)
    key = (device.index if device.index is not None else torch.cuda.current_device(), entry)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        # the outgrown buffer goes first, and its memory back to the device
        # (a batch of the 30-electron molecule takes about 100 GB), so that
        # the larger one is not refused for want of a contiguous block
        _WS.pop(key, None)
        del buf
        torch.cuda.empty_cache()
        try:
            buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        except torch.OutOfMemoryError:
            # the other entry points' buffers on this device give way
            for k in [k for k in _WS if k[0] == key[0]]:
                del _WS[k]
            torch.cuda.empty_cache()
            buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _WS[key] = buf
    # exactly the requested size, so that a smaller max_chunk takes effect
    return buf[:nbytes]


def release_workspaces():
    _WS.clear()
    torch.cuda.empty_cache()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _spins(cfg):
    arr = (ctypes.c_int32 * cfg["n_elec"])(*([0] * cfg["n_up"] + [1] * cfg["n_down"]))
    return arr


def _prep(x, dtype=torch.float32):
    assert x.is_cuda and x.dtype == dtype and x.is_contiguous(), "device, dtype and contiguity of inputs"
    return x


def ferminet_logpsi(cfg, pos, nuc_pos, nuc_charge, params, precision=None, ws=None, max_chunk=None):
    """sign(psi), log|psi| per walker -> (sign [W], logpsi [W]) float32."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    sign = torch.empty(W, dtype=torch.float32, device=pos.device)
    lp = torch.empty(W, dtype=torch.float32, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_LOGPSI, precision, pos.device, max_chunk) if ws is None else ws
    st = _lib().ferminet_logpsi(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(sign), _ptr(lp), _ptr(ws),
                                ws.numel(), _stream())
    _check(st, "ferminet_logpsi")
    return sign, lp


def ferminet_logpsi_noalloc(cfg, pos, nuc_pos, nuc_charge, params, sign, logpsi, precision=None):
    """ferminet_logpsi into the caller's sign [W] and logpsi [W] (float32,
    on pos's device), with the library's own device workspace: the call
    allocates no device memory (the outputs are the caller's)."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    st = _lib().ferminet_logpsi_noalloc(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                        _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(_prep(sign)),
                                        _ptr(_prep(logpsi)), _stream())
    _check(st, "ferminet_logpsi_noalloc")
    return sign, logpsi


def ferminet_local_energy(cfg, pos, nuc_pos, nuc_charge, params, precision=None, ws=None, max_chunk=None,
                          parts=True, rescue: float = 0.0):
    """-> dict(sign, logpsi, e_loc, e_kin, e_pot) float32 [W].  rescue: the
    fraction of walkers (largest determinant-sum cancellation first)
    re-evaluated in float64."""
    W = pos.shape[0]
    c = make_config(cfg, precision, rescue)
    out = {k: torch.empty(W, dtype=torch.float32, device=pos.device) for k in ("sign", "logpsi", "e_loc")}
    if parts:
        out["e_kin"] = torch.empty(W, dtype=torch.float32, device=pos.device)
        out["e_pot"] = torch.empty(W, dtype=torch.float32, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_LOCAL_ENERGY, precision, pos.device, max_chunk, rescue) if ws is None else ws
    st = _lib().ferminet_local_energy(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                      _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(out["sign"]),
                                      _ptr(out["logpsi"]), _ptr(out["e_loc"]), _ptr(out.get("e_kin")),
                                      _ptr(out.get("e_pot")), _ptr(ws), ws.numel(), _stream())
    _check(st, "ferminet_local_energy")
    return out


def ferminet_grad_logpsi(cfg, pos, nuc_pos, nuc_charge, params, cotangent, precision=None, ws=None, max_chunk=None):
    """sum_w cotangent[w] d log|psi_w| / d theta -> [P] float32; with
    cotangent None, d log|psi_w| / d theta of every walker -> [W][P]."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    shape = (params.numel(),) if cotangent is not None else (W, params.numel())
    grad = torch.empty(shape, dtype=torch.float32, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_GRAD_LOGPSI, precision, pos.device, max_chunk) if ws is None else ws
    st = _lib().ferminet_grad_logpsi(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                     _ptr(_prep(nuc_charge)), _ptr(_prep(params)),
                                     _ptr(_prep(cotangent)) if cotangent is not None else None, _ptr(grad),
                                     _ptr(ws), ws.numel(), _stream())
    _check(st, "ferminet_grad_logpsi")
    return grad


def kfac_layout(cfg):
    """[(name, offset_A, dim_A, offset_G, dim_G, positions)] and the total floats."""
    c = make_config(cfg, "fp32")
    n = ctypes.c_int32(0)
    total = ctypes.c_int64(0)
    buf = (fn_kfac_block * 32)()
    _check(_lib().ferminet_kfac_layout(ctypes.byref(c), buf, 32, ctypes.byref(n), ctypes.byref(total)),
           "ferminet_kfac_layout")
    blocks = [(buf[i].name.decode(), buf[i].offset_A, buf[i].dim_A, buf[i].offset_G, buf[i].dim_G, buf[i].positions)
              for i in range(n.value)]
    return blocks, int(total.value)


def ferminet_kfac_factors(cfg, pos, nuc_pos, nuc_charge, params, weights, precision=None, ws=None, max_chunk=None):
    """KFAC statistics of every dense layer -> flat float32 tensor in the
    layout of kfac_layout (each block's A then G)."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    _, total = kfac_layout(cfg)
    out = torch.empty(total, dtype=torch.float32, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_KFAC, precision, pos.device, max_chunk) if ws is None else ws
    st = _lib().ferminet_kfac_factors(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                      _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(_prep(weights)), _ptr(out),
                                      _ptr(ws), ws.numel(), _stream())
    _check(st, "ferminet_kfac_factors")
    return out


def ferminet_kfac_precondition(cfg, factors, grad, damping, ws=None):
    """The KFAC step direction from the factors of ferminet_kfac_factors -> [P] float32."""
    c = make_config(cfg, "fp32")
    out = torch.empty_like(grad, dtype=torch.float32)
    ws = workspace(cfg, 1, FN_ENTRY_KFAC_PRECONDITION, "fp32", grad.device) if ws is None else ws
    st = _lib().ferminet_kfac_precondition(ctypes.byref(c), _ptr(_prep(factors)), _ptr(_prep(grad)), float(damping),
                                           _ptr(out), _ptr(ws), ws.numel(), _stream())
    _check(st, "ferminet_kfac_precondition")
    return out


def kfac_split(cfg, flat):
    """{name: (A, G)} views of the output of ferminet_kfac_factors."""
    blocks, _ = kfac_layout(cfg)
    return {name: (flat[oa:oa + da * da].view(da, da), flat[og:og + dg * dg].view(dg, dg))
            for name, oa, da, og, dg, _ in blocks}


def vmc_energy_gradient(cfg, pos, nuc_pos, nuc_charge, params, e_loc, precision=None, ws=None, max_chunk=None):
    """(1/W) sum_w (E_L - mean E_L) d log|psi_w|/d theta -> (grad [P], stats [2] float64: mean, variance)."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    grad = torch.empty(params.numel(), dtype=torch.float32, device=pos.device)
    stats = torch.empty(2, dtype=torch.float64, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_GRAD_LOGPSI, precision, pos.device, max_chunk) if ws is None else ws
    st = _lib().vmc_energy_gradient(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                    _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(_prep(e_loc)), _ptr(stats),
                                    _ptr(grad), _ptr(ws), ws.numel(), _stream())
    _check(st, "vmc_energy_gradient")
    return grad, stats


def vmc_local_energy_gradient(cfg, pos, nuc_pos, nuc_charge, params, precision=None, ws=None, max_chunk=None,
                              parts=True, rescue: float = 0.0):
    """ferminet_local_energy and vmc_energy_gradient of its energies in one
    pass -> (dict(sign, logpsi, e_loc[, e_kin, e_pot]) float32 [W],
    grad [P] float32, stats [2] float64: mean and variance of e_loc)."""
    W = pos.shape[0]
    c = make_config(cfg, precision, rescue)
    out = {k: torch.empty(W, dtype=torch.float32, device=pos.device) for k in ("sign", "logpsi", "e_loc")}
    if parts:
        out["e_kin"] = torch.empty(W, dtype=torch.float32, device=pos.device)
        out["e_pot"] = torch.empty(W, dtype=torch.float32, device=pos.device)
    grad = torch.empty(params.numel(), dtype=torch.float32, device=pos.device)
    stats = torch.empty(2, dtype=torch.float64, device=pos.device)
    if ws is None:
        ws = workspace(cfg, W, FN_ENTRY_LOCAL_ENERGY_GRADIENT, precision, pos.device, max_chunk, rescue)
    st = _lib().vmc_local_energy_gradient(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                                          _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(out["sign"]),
                                          _ptr(out["logpsi"]), _ptr(out["e_loc"]), _ptr(out.get("e_kin")),
                                          _ptr(out.get("e_pot")), _ptr(stats), _ptr(grad), _ptr(ws), ws.numel(),
                                          _stream())
    _check(st, "vmc_local_energy_gradient")
    return out, grad, stats


def vmc_mcmc_step(cfg, pos, nuc_pos, nuc_charge, params, logpsi, sign, n_steps, step_width, seed, counter=0,
                  noise=None, uniforms=None, precision=None, ws=None, max_chunk=None):
    """In place on pos, logpsi, sign; returns n_accepted [W] int32."""
    W = pos.shape[0]
    c = make_config(cfg, precision)
    acc = torch.empty(W, dtype=torch.int32, device=pos.device)
    ws = workspace(cfg, W, FN_ENTRY_MCMC, precision, pos.device, max_chunk) if ws is None else ws
    st = _lib().vmc_mcmc_step(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                              _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(_prep(logpsi)), _ptr(_prep(sign)),
                              int(n_steps), float(step_width), int(seed), int(counter),
                              _ptr(_prep(noise)) if noise is not None else None,
                              _ptr(_prep(uniforms)) if uniforms is not None else None, _ptr(acc), _ptr(ws),
                              ws.numel(), _stream())
    _check(st, "vmc_mcmc_step")
    return acc


def vmc_train_step(cfg, pos, nuc_pos, nuc_charge, params, factors, mcmc_steps, mcmc_width, seed, counter,
                   learning_rate, damping=1e-3, norm_constraint=1e-3, factor_decay=0.95, clip_scale=5.0, noise=None,
                   uniforms=None, precision=None, rescue=0.0, ws=None):
    """One VMC iteration (include/ferminet.h), in place on pos, params and
    factors (the running KFAC factors, kfac_layout's total floats).
    Returns (e_loc [W] float32, stats [9] float64: mean and variance of
    e_loc, acceptance rate, median, mean |e_loc - median|, mean of the
    clipped energies, <X, g>, step length lr c, walkers left out for a
    non-finite local energy)."""
    W = pos.shape[0]
    c = make_config(cfg, precision, rescue)
    e = torch.empty(W, dtype=torch.float32, device=pos.device)
    stats = torch.empty(9, dtype=torch.float64, device=pos.device)
    o = fn_train_options(int(mcmc_steps), float(mcmc_width), int(seed), int(counter), float(learning_rate),
                         float(damping), float(norm_constraint), float(factor_decay), float(clip_scale), 0)
    ws = workspace(cfg, W, FN_ENTRY_TRAIN, precision, pos.device, rescue=rescue) if ws is None else ws
    st = _lib().vmc_train_step(ctypes.byref(c), W, _ptr(_prep(pos)), _spins(cfg), _ptr(_prep(nuc_pos)),
                               _ptr(_prep(nuc_charge)), _ptr(_prep(params)), _ptr(_prep(factors)), ctypes.byref(o),
                               _ptr(_prep(noise)) if noise is not None else None,
                               _ptr(_prep(uniforms)) if uniforms is not None else None, _ptr(e), _ptr(stats),
                               _ptr(ws), ws.numel(), _stream())
    _check(st, "vmc_train_step")
    return e, stats


def vmc_mcmc_noise(W, n_elec, n_steps, seed, counter=0, device="cuda"):
    noise = torch.empty((n_steps, W, 3 * n_elec), dtype=torch.float32, device=device)
    uni = torch.empty((n_steps, W), dtype=torch.float32, device=device)
    _check(_lib().vmc_mcmc_noise(W, n_elec, n_steps, int(seed), int(counter), _ptr(noise), _ptr(uni), _stream()),
           "vmc_mcmc_noise")
    return noise, uni


def set_option(option: int, value: int):
    """ferminet_set_option: a process-wide execution option for later calls
    (FN_OPT_FUSED_MEANFIELD: 1 forms the spin means in the layer kernel where
    the shape allows, 0 runs the separate pass; same bits)."""
    _check(_lib().ferminet_set_option(int(option), int(value)), "ferminet_set_option")


def stage_timing(enable: bool):
    """Switch the library's per-launch event timing on or off (diagnostics)."""
    _check(_lib().ferminet_stage_timing(1 if enable else 0), "ferminet_stage_timing")


def stage_times():
    """{stage name: (total ms, launches)} of the launches recorded since
    timing was switched on; clears the records."""
    cap = 64
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int32 * cap)()
    n = _lib().ferminet_stage_times(ms, cnt, cap)
    if n < 0:
        raise RuntimeError("ferminet_stage_times failed")
    return {_lib().ferminet_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n) if cnt[i] > 0}


def to_device(w: dict, device="cuda"):
    """Move a workload (paper_2011_07125_amd.inputs) to the GPU."""
    return dict(cfg=w["cfg"], pos=torch.from_numpy(w["pos"]).to(device).contiguous(),
                nuc_pos=torch.from_numpy(w["nuc_pos"]).to(device).contiguous(),
                nuc_charge=torch.from_numpy(w["nuc_charge"]).to(device).contiguous(),
                params=torch.from_numpy(w["params"]).to(device).contiguous())
