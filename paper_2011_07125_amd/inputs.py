"""Seeded synthetic workloads shaped like the paper's systems.

This module holds no arithmetic of the method: it only draws nuclei,
walkers and parameters with numpy and states the flat parameter layout
(an interface of the C ABI) as data.  It serves both the HIP path and the
CPU oracle in the tests and the bench.

Workloads (atomic units; positions in bohr):
  * be4      -- Be-like atom, Z=4, 4 electrons (2 up/2 down), 256 walkers,
                positions ~ N(0, 1 bohr^2), 2 layers of width 32/8, 4 dets.
  * ne10     -- Ne-like atom (first-row atom of Section 2), Z=10,
                10 electrons (5/5), 4096 walkers ~ N(0, 1.5 bohr^2),
                4 layers 256/32, 16 dets.
  * ar18     -- Ar-like atom (largest atom of Table 1, at its 512-unit,
                32-determinant column), Z=18, 18 electrons (9/9),
                4096 walkers ~ N(0, 2 bohr^2), 4 layers 512/32, 32 dets.
  * c4h6     -- a 30-electron molecule shaped like bicyclobutane (Table 2):
                4 carbon (Z=6) and 6 hydrogen (Z=1) nuclei at seeded
                positions in a 6-bohr box with minimum separation 1.5 bohr,
                2048 walkers Gaussian (sigma 1 bohr) around the nuclei,
                4 layers 256/32, 16 dets.
  * c4h6_vmc -- the same molecule with 8192 walkers for a full VMC
                iteration (10 Metropolis steps of width 0.02 bohr).
The real geometries of the paper's molecules are not available; the
seeded geometry stands in for them.

Random streams: numpy PCG64 with SeedSequence(seed).spawn(5):
  0 nuclei, 1 parameters (layout order), 2 walkers, 3 Metropolis, 4 choice
of parameters for finite-difference checks.
Initialisation: weights ~ N(0, 1/fan_in) (variance 1/fan_in, fan_in = the
full input width of the block), biases 0, orbital biases 0, envelope
coefficients pi = 1 and exponents sigma = 1.
"""
from __future__ import annotations

import numpy as np

SPECS = {
    "be4": dict(nuclei="atom", Z=4, n_up=2, n_down=2, walkers=256, pos_var=1.0, n_layers=2, width1=32,
                width2=8, n_det=4, seed=0, precision="fp32"),
    "ne10": dict(nuclei="atom", Z=10, n_up=5, n_down=5, walkers=4096, pos_var=1.5, n_layers=4, width1=256,
                 width2=32, n_det=16, seed=1, precision="fp32"),
    "ar18": dict(nuclei="atom", Z=18, n_up=9, n_down=9, walkers=4096, pos_var=2.0, n_layers=4, width1=512,
                 width2=32, n_det=32, seed=2, precision="bf16"),
    "c4h6": dict(nuclei="molecule", n_up=15, n_down=15, walkers=2048, pos_sigma=1.0, n_layers=4, width1=256,
                 width2=32, n_det=16, seed=3, geometry_seed=3, precision="fp32"),
    "c4h6_vmc": dict(nuclei="molecule", n_up=15, n_down=15, walkers=8192, pos_sigma=1.0, n_layers=4,
                     width1=256, width2=32, n_det=16, seed=4, geometry_seed=3, precision="bf16",
                     mcmc_steps=10, mcmc_width=0.02),
}

# Fraction of each batch whose local energy the throughput measurement and
# the accuracy gate re-evaluate in float64, per workload and form: "bf16"
# (split-bf16 layer products, fp32 orbital product, fp64 determinants) and
# "fp32_fp64det" (fp32 layer and orbital products, fp64 determinants).
# The bf16 form on the 30-electron molecule (c4h6) does not reach a 1 mHa
# batch mean at any fraction tried up to 20%; that workload's stated form is
# fp32.
RESCUE = {
    "be4": {"bf16": 0.03, "fp32_fp64det": 0.02},
    "ne10": {"bf16": 0.03, "fp32_fp64det": 0.03},
    "ar18": {"bf16": 0.05, "fp32_fp64det": 0.03},
    "c4h6": {"bf16": 0.05, "fp32_fp64det": 0.10},
    "c4h6_vmc": {"bf16": 0.03, "fp32_fp64det": 0.03},
}


def make_cfg(n_up, n_down, n_nuc, n_layers, width1, width2, n_det, precision="fp32", envelope="isotropic"):
    """envelope: 'isotropic' (one sigma per orbital and nucleus, Section 3)
    or 'full' (a 3x3 matrix Sigma per orbital and nucleus, Eq. (5))."""
    return dict(n_elec=n_up + n_down, n_up=n_up, n_down=n_down, n_nuc=n_nuc, n_layers=n_layers,
                width1=width1, width2=width2, n_det=n_det, precision=precision, envelope=envelope)


def is_full_envelope(cfg):
    return cfg.get("envelope", "isotropic") in ("full", 1)


def param_blocks(cfg):
    """The flat parameter layout, in order, as (name, shape, kind) with kind
    'weight' (init N(0, 1/shape[0])), 'bias' (0), 'pi' (1) or 'sigma' (1).

    for l in 0..L-1:  V{l} [3*din_l + 2*ein_l][d1], b{l} [d1]
    for l in 0..L-2:  W{l} [ein_l][d2],             c{l} [d2]
    for spin a:       w_orb{a} [d1][K*n_a] (column k*n_a + i), g_orb{a} [K*n_a]
    for spin a:       pi{a} [K*n_a][N]
    for spin a:       sigma{a} [K*n_a][N] (isotropic) or [K*n_a][N][3][3]
                      (full covariance, row-major, applied as Sigma (r - R))
    with din_0 = 4N, ein_0 = 4, din_l = d1 and ein_l = d2 for l > 0.
    """
    N, L, d1, d2, K = cfg["n_nuc"], cfg["n_layers"], cfg["width1"], cfg["width2"], cfg["n_det"]
    ns = (cfg["n_up"], cfg["n_down"])
    out = []
    for l in range(L):
        din, ein = (4 * N, 4) if l == 0 else (d1, d2)
        out.append((f"V{l}", (3 * din + 2 * ein, d1), "weight"))
        out.append((f"b{l}", (d1,), "bias"))
    for l in range(L - 1):
        ein = 4 if l == 0 else d2
        out.append((f"W{l}", (ein, d2), "weight"))
        out.append((f"c{l}", (d2,), "bias"))
    for a in range(2):
        out.append((f"w_orb{a}", (d1, K * ns[a]), "weight"))
        out.append((f"g_orb{a}", (K * ns[a],), "bias"))
    for a in range(2):
        out.append((f"pi{a}", (K * ns[a], N), "pi"))
    for a in range(2):
        shape = (K * ns[a], N, 3, 3) if is_full_envelope(cfg) else (K * ns[a], N)
        out.append((f"sigma{a}", shape, "sigma"))
    return out


def param_offsets(cfg):
    """{name: (offset, shape)} plus the total count under key '_total'."""
    off = 0
    res = {}
    for name, shape, _ in param_blocks(cfg):
        res[name] = (off, shape)
        off += int(np.prod(shape))
    res["_total"] = off
    return res


def init_params(cfg, rng):
    chunks = []
    for name, shape, kind in param_blocks(cfg):
        size = int(np.prod(shape))
        if kind == "weight":
            chunks.append(rng.normal(0.0, 1.0 / np.sqrt(shape[0]), size=size))
        elif kind == "bias":
            chunks.append(np.zeros(size))
        elif kind == "sigma" and len(shape) == 4:
            chunks.append(np.broadcast_to(np.eye(3), shape).reshape(-1))  # Sigma = I: sigma = 1
        else:
            chunks.append(np.ones(size))
    return np.concatenate(chunks).astype(np.float32)


def full_covariance(w, noise=0.0, seed=0):
    """The workload w with the full-covariance envelope: every isotropic
    sigma of w becomes the matrix sigma * I (the same wavefunction), plus
    noise * N(0, 1) per entry when noise > 0 (seeded)."""
    cfg = dict(w["cfg"], envelope="full")
    src = param_offsets(w["cfg"])
    dst = param_offsets(cfg)
    params = np.empty(dst["_total"], dtype=w["params"].dtype)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(5)[1]))
    for name, shape, kind in param_blocks(cfg):
        o, sh = dst[name]
        so, ssh = src[name]
        block = w["params"][so:so + int(np.prod(ssh))].astype(np.float64)
        if kind == "sigma":
            mats = block.reshape(ssh)[..., None, None] * np.eye(3)
            if noise > 0:
                mats = mats + noise * rng.normal(size=mats.shape)
            block = mats.reshape(-1)
        params[o:o + int(np.prod(sh))] = block
    return dict(w, cfg=cfg, params=params)


def molecule_geometry(seed, n_carbon=4, n_hydrogen=6, box=3.0, min_sep=1.5):
    """Nuclei placed in order (carbons first) by rejection sampling in
    [-box, box]^3 until every pairwise distance is at least min_sep."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(5)[0]))
    charges = [6.0] * n_carbon + [1.0] * n_hydrogen
    pts = []
    for _ in charges:
        while True:
            p = rng.uniform(-box, box, size=3)
            if all(np.linalg.norm(p - q) >= min_sep for q in pts):
                pts.append(p)
                break
    return np.array(pts), np.array(charges)


def make_workload(name, walkers=None, seed=None):
    """Seeded inputs of a named workload.  Returns a dict with cfg, pos
    [W][n][3] f32, nuc_pos [N][3] f32, nuc_charge [N] f32, params [P] f32,
    spins [n] int32 (0 up, 1 down; up first) and the raw spec."""
    sp = dict(SPECS[name])
    seed = sp["seed"] if seed is None else seed
    W = sp["walkers"] if walkers is None else walkers
    streams = np.random.SeedSequence(seed).spawn(5)
    rng_par = np.random.Generator(np.random.PCG64(streams[1]))
    rng_walk = np.random.Generator(np.random.PCG64(streams[2]))
    n_up, n_dn = sp["n_up"], sp["n_down"]
    n = n_up + n_dn
    if sp["nuclei"] == "atom":
        nuc = np.zeros((1, 3))
        Z = np.array([float(sp["Z"])])
        pos = rng_walk.normal(0.0, np.sqrt(sp["pos_var"]), size=(W, n, 3))
    else:
        nuc, Z = molecule_geometry(sp["geometry_seed"])
        # each nucleus receives Z_I electrons; spins alternate along that
        # list; electrons are then reordered up first
        owners = np.repeat(np.arange(len(Z)), Z.astype(int))
        spin_list = np.arange(owners.size) % 2
        order = np.concatenate([owners[spin_list == 0], owners[spin_list == 1]])
        assert order.size == n and (spin_list == 0).sum() == n_up
        pos = nuc[order][None, :, :] + rng_walk.normal(0.0, sp["pos_sigma"], size=(W, n, 3))
    cfg = make_cfg(n_up, n_dn, nuc.shape[0], sp["n_layers"], sp["width1"], sp["width2"], sp["n_det"],
                   sp.get("precision", "fp32"))
    params = init_params(cfg, rng_par)
    spins = np.array([0] * n_up + [1] * n_dn, dtype=np.int32)
    return dict(cfg=cfg, pos=pos.astype(np.float32), nuc_pos=nuc.astype(np.float32),
                nuc_charge=Z.astype(np.float32), params=params, spins=spins, spec=sp, seed=seed)


def custom_workload(n_up, n_down, nuc_pos, nuc_charge, walkers, n_layers, width1, width2, n_det, seed,
                    pos_std=1.0, precision="fp32"):
    """Small ad-hoc workload (tests): atoms or molecules of any shape."""
    streams = np.random.SeedSequence(seed).spawn(5)
    rng_par = np.random.Generator(np.random.PCG64(streams[1]))
    rng_walk = np.random.Generator(np.random.PCG64(streams[2]))
    nuc = np.asarray(nuc_pos, dtype=np.float64).reshape(-1, 3)
    Z = np.asarray(nuc_charge, dtype=np.float64).reshape(-1)
    n = n_up + n_down
    centre = nuc[np.arange(n) % nuc.shape[0]]
    pos = centre[None] + rng_walk.normal(0.0, pos_std, size=(walkers, n, 3))
    cfg = make_cfg(n_up, n_down, nuc.shape[0], n_layers, width1, width2, n_det, precision)
    params = init_params(cfg, rng_par)
    spins = np.array([0] * n_up + [1] * n_down, dtype=np.int32)
    return dict(cfg=cfg, pos=pos.astype(np.float32), nuc_pos=nuc.astype(np.float32),
                nuc_charge=Z.astype(np.float32), params=params, spins=spins, seed=seed)


def fd_param_choice(name_or_cfg, n_pick=64, seed=None):
    """The seeded set of parameter indices used for finite-difference and
    oracle-gradient checks (stream 4)."""
    if isinstance(name_or_cfg, str):
        sp = SPECS[name_or_cfg]
        seed = sp["seed"] if seed is None else seed
        w = make_workload(name_or_cfg, walkers=1, seed=seed)
        cfg = w["cfg"]
    else:
        cfg = name_or_cfg
        seed = 0 if seed is None else seed
    total = param_offsets(cfg)["_total"]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(5)[4]))
    return np.sort(rng.choice(total, size=min(n_pick, total), replace=False)).astype(np.int64)
