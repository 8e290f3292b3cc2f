"""Seeded synthetic cell states standing in for the paper's MAD snapshots.

The paper's inputs are GRMHD snapshots of a magnetically arrested disk
(384 x 300 x 64 cells, Section III.C) that are not available here; these
generators produce states of the same kind: per-cell n_e [cm^-3], T_e, T_i [K],
|B| [G] and the scale height H [cm], as FP64 NumPy arrays, with dt given in
r_g / c for a 10 M_sun black hole.  Nothing in this module evaluates a cooling
rate: it draws inputs only, and both the library tests and the oracle take
their inputs from it.

Recipes (seed = 20250513 + workload index, NumPy PCG64, draws in the order listed):
  iid     log10 n_e ~ U[10, 20]; log10 T_e ~ U[7, 11.5]; log10(T_i/T_e) ~ U[0, 2];
          log10 beta ~ U[-1, 2]; ln r ~ U[ln 2, ln 1000] (r in r_g); H/r ~ U[0.05, 0.4];
          B = sqrt(8 pi n_e k (T_e + T_i) / beta); H = (H/r) r r_g.
  sphere  spherical-polar grid, r_k = 2 * 500^((k+1/2)/n_r) r_g, theta_j = pi (j+1/2)/n_th,
          phi_l = 2 pi (l+1/2)/n_ph, phi fastest; n_e = 1e20 (r/r_g)^-1.5 LN,
          T_e = 6.3e11 (r/r_g)^-1 LN, T_i = 10 T_e LN, LN = exp(ln 1.2 z), z ~ N(0,1)
          drawn independently per field (n_e, T_e, T_i order); beta = 10^-|cos theta|;
          H = 0.3 r r_g.
  blocks  AMR-like blocks: shapes 8^3 / 16^3 / 24^3 / 32^3 / mixed with probabilities
          0.55 / 0.30 / 0.10 / 0.02 / 0.03 (mixed: each side from {8,16,24,32});
          each block is a coherent patch of the sphere profile around a seeded centre
          (r_b log-uniform in [2, 1000] r_g, theta_b ~ U(0, pi), phi_b ~ U(0, 2 pi))
          with cell spacing of the 128^3 sphere grid; per accretion state s = 0..7 the
          density is scaled n_e = 1e21 mdot_s (r/r_g)^-1.5 LN with
          mdot_s = 10^(-6 + 5.5 s / 7).
"""
import math

import numpy as np

# input-recipe constants (cgs); the recipe needs k_B for B(beta) and r_g for lengths
_K_B = 1.380649e-16
_G = 6.67430e-8
_C = 2.99792458e10
_M_SUN = 1.98847e33

BH_MASS = 10.0 * _M_SUN
R_G = _G * BH_MASS / _C ** 2            # cm
DT_DEFAULT = 1.0e-3 * R_G / _C          # s, dt = 1e-3 r_g / c

SEED_BASE = 20250513
FIELDS = ("n_e", "T_e", "T_i", "B", "H")


def _b_from_beta(n_e, T_e, T_i, beta):
    return np.sqrt(8.0 * math.pi * n_e * _K_B * (T_e + T_i) / beta)


def iid_cells(n, seed):
    """``n`` independent cells of the iid recipe."""
    rng = np.random.default_rng(seed)
    lg_n = rng.uniform(10.0, 20.0, n)
    lg_te = rng.uniform(7.0, 11.5, n)
    lg_ratio = rng.uniform(0.0, 2.0, n)
    lg_beta = rng.uniform(-1.0, 2.0, n)
    ln_r = rng.uniform(math.log(2.0), math.log(1000.0), n)
    h_over_r = rng.uniform(0.05, 0.4, n)
    n_e = 10.0 ** lg_n
    T_e = 10.0 ** lg_te
    T_i = T_e * 10.0 ** lg_ratio
    B = _b_from_beta(n_e, T_e, T_i, 10.0 ** lg_beta)
    H = h_over_r * np.exp(ln_r) * R_G
    return {"n_e": n_e, "T_e": T_e, "T_i": T_i, "B": B, "H": H}


def sphere_cells(n_r=128, n_th=128, n_ph=128, seed=SEED_BASE + 2):
    """Spherical-polar MAD-like profile, flattened with phi fastest."""
    rng = np.random.default_rng(seed)
    k = np.arange(n_r)
    j = np.arange(n_th)
    r = 2.0 * 500.0 ** ((k + 0.5) / n_r)
    th = math.pi * (j + 0.5) / n_th
    shape = (n_r, n_th, n_ph)
    rr = np.broadcast_to(r[:, None, None], shape).ravel()
    tt = np.broadcast_to(th[None, :, None], shape).ravel()
    ln12 = math.log(1.2)
    n_e = 1.0e20 * rr ** -1.5 * np.exp(ln12 * rng.standard_normal(rr.size))
    T_e = 6.3e11 / rr * np.exp(ln12 * rng.standard_normal(rr.size))
    T_i = 10.0 * T_e * np.exp(ln12 * rng.standard_normal(rr.size))
    beta = 10.0 ** (-np.abs(np.cos(tt)))
    B = _b_from_beta(n_e, T_e, T_i, beta)
    H = 0.3 * rr * R_G
    return {"n_e": n_e, "T_e": T_e, "T_i": T_i, "B": B, "H": H}


_BLOCK_SIDES = (8, 16, 24, 32)
_BLOCK_PROBS = (0.55, 0.30, 0.10, 0.02, 0.03)


def block_shapes(n_blocks, rng):
    kind = rng.choice(5, size=n_blocks, p=_BLOCK_PROBS)
    shapes = []
    for kd in kind:
        if kd < 4:
            s = _BLOCK_SIDES[kd]
            shapes.append((s, s, s))
        else:
            shapes.append(tuple(int(v) for v in rng.choice(_BLOCK_SIDES, size=3)))
    return shapes


def mdot_states(n_states=8):
    return [10.0 ** (-6.0 + 5.5 * s / 7.0) for s in range(n_states)]


def amr_blocks(n_blocks=4096, n_states=8, seed=SEED_BASE + 4, grid=128, max_cells=None):
    """Uneven AMR-like blocks times accretion-rate states.

    Returns (cells dict of flat arrays over all (state, block) pairs, blocks list of
    (first_cell, n_cells, state_id), dt per state).  Cells of one (block, state)
    are contiguous.  ``max_cells`` truncates the block list (for small tests).
    """
    rng = np.random.default_rng(seed)
    shapes = block_shapes(n_blocks, rng)
    r_c = np.exp(rng.uniform(math.log(2.0), math.log(1000.0), n_blocks))
    th_c = rng.uniform(0.0, math.pi, n_blocks)
    # cell spacing of the grid-per-axis sphere grid: dln r, dtheta, dphi
    dlnr = math.log(500.0) / grid
    dth = math.pi / grid
    ln12 = math.log(1.2)
    mdots = mdot_states(n_states)
    fields = {f: [] for f in FIELDS}
    blocks = []
    first = 0
    for s, md in enumerate(mdots):
        for b, (a0, a1, a2) in enumerate(shapes):
            if max_cells is not None and first >= max_cells:
                break
            i0 = np.arange(a0) - 0.5 * (a0 - 1)
            i1 = np.arange(a1) - 0.5 * (a1 - 1)
            r = r_c[b] * np.exp(dlnr * i0)
            th = np.clip(th_c[b] + dth * i1, 1e-3, math.pi - 1e-3)
            shp = (a0, a1, a2)
            rr = np.broadcast_to(r[:, None, None], shp).ravel()
            tt = np.broadcast_to(th[None, :, None], shp).ravel()
            m = rr.size
            n_e = 1.0e21 * md * rr ** -1.5 * np.exp(ln12 * rng.standard_normal(m))
            T_e = 6.3e11 / rr * np.exp(ln12 * rng.standard_normal(m))
            T_i = 10.0 * T_e * np.exp(ln12 * rng.standard_normal(m))
            B = _b_from_beta(n_e, T_e, T_i, 10.0 ** (-np.abs(np.cos(tt))))
            H = 0.3 * rr * R_G
            for f, v in zip(FIELDS, (n_e, T_e, T_i, B, H)):
                fields[f].append(v)
            blocks.append((first, m, s))
            first += m
    cells = {f: np.concatenate(v) for f, v in fields.items()}
    dts = np.full(n_states, DT_DEFAULT)
    return cells, blocks, dts


def workload(index, n=None):
    """Named workloads: 0 iid 32^3, 1 iid 256^3, 2 sphere 128^3, 3 iid 2^21, 4 blocks.

    ``n`` overrides the cell count of the iid workloads (for samples).
    """
    seed = SEED_BASE + index
    if index == 0:
        return iid_cells(n or 32 ** 3, seed)
    if index == 1:
        return iid_cells(n or 256 ** 3, seed)
    if index == 2:
        return sphere_cells(seed=seed)
    if index == 3:
        return iid_cells(n or 2 ** 21, seed)
    raise ValueError("workload 4 is built by amr_blocks()")
