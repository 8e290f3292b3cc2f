"""Log-spaced rate tables and multilinear interpolation (paper II.F, II.G, III.A).

The paper tabulates Q(H_th, B, n_e, T_e) on a 4-D grid and Q_cc(n_e, T_i, T_e)
on a 3-D grid, log-spaced.  Here the cooling part is held as three exact 3-D
tables over the column N = n_e H, T_e and B.  The reduction is exact, not an
approximation: from the closed forms of Section II,
  Q_brem(n_e, T)        = N^2 f(theta) / H^2,
  Q_syn(n_e, T, B, H)   = Q_syn(N, T, B, H = 1 cm) / H,
  eta(n_e, T, B, H)     = eta(N, T, B, H = 1 cm),
because x_c depends on n_e and H only through n_e H, tau_sca = 2 sigma_T N,
and the Rayleigh-Jeans and tail terms each carry one explicit 1/H.

Tables hold log2 of positive quantities (reading: values span more than sixty
decades, and power laws such as n^2 are then reproduced exactly between nodes):
  brem : log2(N^2 f_brem(theta_e))              axes (log10 N, log10 T_e, log10 B)
  synch: log2 Q_syn(N, T_e, B, H = 1)           axes (log10 N, log10 T_e, log10 B)
  eta  : log2 eta(N, T_e, B, H = 1)             axes (log10 N, log10 T_e, log10 B)
  coul : log2(Q_cc / (T_i - T_e))               axes (log10 n_e, log10 T_e, log10 T_i)
The cooling rate needs synch and eta only as the product eta Q_syn, so the
rate path reads se = synch + eta = log2(eta Q_syn) as one table.  In FP64 it is
the sum of the two; in the storage form (below) its residual is the
single-precision sum of the two stored residuals and its affine part the sum
of theirs.

Node k of an axis is u_k = lo + k (hi - lo) / (n - 1).  A query coordinate u
becomes f = (u - lo) / d with d = (hi - lo) / (n - 1), clamped to [0, n - 1];
the cell is i = min(floor f, n - 2) and the weight t = f - i.

Parity pins (tests/test_oracle_tables.py): values at nodes equal the closed
forms; interpolation reproduces any affine function of the node coordinates
exactly; it equals scipy's RegularGridInterpolator(method="linear"); clamping.
"""
from dataclasses import dataclass, field

import numpy as np

from . import physics

TABLE_NAMES = ("brem", "synch", "eta", "coul")


@dataclass(frozen=True)
class Axis:
    n: int
    lo: float
    hi: float

    @property
    def step(self):
        return (self.hi - self.lo) / (self.n - 1)

    def nodes(self):
        k = np.arange(self.n, dtype=np.float64)
        return self.lo + k * (self.hi - self.lo) / (self.n - 1)


def _default_cool(n):
    return (Axis(n, 15.0, 29.0), Axis(n, 5.95, 12.05), Axis(n, -0.5, 10.5))


def _default_coul(n):
    return (Axis(n, 9.5, 20.5), Axis(n, 5.95, 12.05), Axis(n, 5.95, 14.05))


@dataclass(frozen=True)
class TableSpec:
    """Axes of the cooling tables (log10 N, log10 T_e, log10 B) and of the
    Coulomb table (log10 n_e, log10 T_e, log10 T_i), and the readings of two
    printed formulas: ``compton`` "derived" (exponent -1 - ln P / ln A, the
    default) or "literal" (1 - ln P / ln A as printed, II.C); ``theta_i_mass``
    "m_p" (default) or "m_e" (theta_i = k T_i / m_e c^2 as printed, II.G)."""
    cool: tuple = field(default_factory=lambda: _default_cool(64))
    coul: tuple = field(default_factory=lambda: _default_coul(64))
    compton: str = "derived"
    theta_i_mass: str = "m_p"

    @staticmethod
    def default(n=64, compton="derived", theta_i_mass="m_p"):
        return TableSpec(_default_cool(n), _default_coul(n), compton, theta_i_mass)

    def axes(self, name):
        return self.coul if name == "coul" else self.cool


def _grid(axes):
    u0, u1, u2 = (a.nodes() for a in axes)
    return np.meshgrid(u0, u1, u2, indexing="ij")


def build_cooling(spec, chunk=1 << 18):
    """The three cooling tables (log2), each of shape (n_N, n_T, n_B)."""
    uN, uT, uB = _grid(spec.cool)
    N = 10.0 ** uN.ravel()
    T = 10.0 ** uT.ravel()
    B = 10.0 ** uB.ravel()
    one = np.ones_like(N)
    brem = np.empty_like(N)
    syn = np.empty_like(N)
    eta = np.empty_like(N)
    for s in range(0, N.size, chunk):
        sl = slice(s, s + chunk)
        brem[sl] = np.log2(physics.q_brem(N[sl], T[sl]))        # H = 1: n_e = N
        sy = physics.synchrotron(N[sl], T[sl], B[sl], one[sl])
        syn[sl] = np.log2(sy["q_syn"])
        if spec.compton == "literal":
            # the printed exponent: eta <= 0 wherever P A > 1, and such a node
            # has no log2 value (NaN)
            e = physics.compton_eta_printed(N[sl], T[sl], one[sl], sy["nu_c"])
            ok = (e > 0.0) & np.isfinite(e)
            eta[sl] = np.where(ok, np.log2(np.where(ok, e, 1.0)), np.nan)
        else:
            eta[sl] = np.log2(physics.compton_eta(N[sl], T[sl], one[sl], sy["nu_c"]))
    shape = uN.shape
    return {"brem": brem.reshape(shape), "synch": syn.reshape(shape), "eta": eta.reshape(shape)}


def build_coulomb(spec):
    un, ue, ui = _grid(spec.coul)
    m_ti = physics.K.M_E if spec.theta_i_mass == "m_e" else physics.K.M_P
    return np.log2(physics.coulomb_coeff(10.0 ** un, 10.0 ** ue, 10.0 ** ui, theta_i_mass=m_ti))


def build_tables(spec=None):
    """All four tables in FP64 log2 form, keyed by TABLE_NAMES."""
    spec = spec or TableSpec.default()
    out = build_cooling(spec)
    out["coul"] = build_coulomb(spec)
    return out


# ---------------------------------------------------------------------------
# FP32 storage form (precision form of the method)


def affine_fit(y):
    """Least-squares affine function of the node indices: y ~ c0 + c1 i0 + c2 i1 + c3 i2.

    On a full rectangular grid the normal equations decouple, so each slope is
    cov(y, i_a) / var(i_a) and c0 = mean(y) - sum_a c_a mean(i_a).
    """
    y = np.asarray(y, dtype=np.float64)
    coeffs = np.zeros(4)
    idx = [np.arange(n, dtype=np.float64) for n in y.shape]
    grids = np.meshgrid(*idx, indexing="ij")
    c0 = y.mean()
    for a, g in enumerate(grids):
        dg = g - g.mean()
        coeffs[a + 1] = np.sum(dg * y) / np.sum(dg * dg)
        c0 -= coeffs[a + 1] * g.mean()
    coeffs[0] = c0
    return coeffs


def affine_eval(coeffs, i0, i1, i2):
    return coeffs[0] + coeffs[1] * i0 + coeffs[2] * i1 + coeffs[3] * i2


def round_bf16(a):
    """Round float32 values to bfloat16 (the upper 16 bits of a binary32),
    round to nearest, ties to even; returned as float32.  Finite inputs."""
    bits = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32)


def quantize(y, value_dtype="f32"):
    """Storage form of one table: (coeffs FP64[4], residual FP32, stored FP64 values).

    The stored table is affine(i) + float64(r) with r = float32(y - affine(i)),
    and for the bfloat16 form r additionally rounded to bfloat16.  Multilinear
    interpolation reproduces the affine part exactly, so only the residual is
    rounded; its magnitude is what sets the storage error.
    """
    # a table with nodes that hold no value (NaN: the literal Compton reading)
    # keeps a zero affine part, so its residual is the log2 value itself
    coeffs = np.zeros(4) if np.isnan(y).any() else affine_fit(y)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in y.shape], indexing="ij")
    base = affine_eval(coeffs, *grids)
    resid = (y - base).astype(np.float32)
    if value_dtype == "bf16":
        resid = round_bf16(resid)
    elif value_dtype != "f32":
        raise ValueError("value_dtype must be 'f32' or 'bf16'")
    return coeffs, resid, base + resid.astype(np.float64)


def quantize_tables(tables, value_dtype="f32"):
    """Apply ``quantize`` to every table; returns (coeffs dict, resid dict, stored dict).

    The stored dict also holds "se", the stored form of synch + eta: affine
    part coeffs[synch] + coeffs[eta], residual the single-precision sum of the
    two stored residuals (one IEEE addition in float32, rounded to nearest)."""
    co, re, st = {}, {}, {}
    for k in TABLE_NAMES:
        co[k], re[k], st[k] = quantize(tables[k], value_dtype)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in re["synch"].shape], indexing="ij")
    r_se = np.add(re["synch"], re["eta"], dtype=np.float32)
    st["se"] = affine_eval(co["synch"] + co["eta"], *grids) + r_se.astype(np.float64)
    return co, re, st


# ---------------------------------------------------------------------------
# interpolation


def axis_coord(u, axis):
    """(i, t, clamped) for a log10 coordinate u on ``axis``."""
    u = np.asarray(u, dtype=np.float64)
    f = (u - axis.lo) / axis.step
    clamped = (f < 0.0) | (f > axis.n - 1)
    f = np.clip(f, 0.0, axis.n - 1)
    i = np.minimum(np.floor(f).astype(np.int64), axis.n - 2)
    return i, f - i, clamped


def interp3(table, axes, u0, u1, u2):
    """Trilinear interpolation of ``table`` at log10 coordinates (u0, u1, u2).

    Returns (value, clamped) where clamped is True when any coordinate was
    outside its axis range (clamp-to-edge semantics).
    """
    (i0, t0, c0), (i1, t1, c1), (i2, t2, c2) = (axis_coord(u, a) for u, a in zip((u0, u1, u2), axes))
    y = np.zeros(np.broadcast(i0, i1, i2).shape)
    for a in (0, 1):
        w0 = t0 if a else 1.0 - t0
        for b in (0, 1):
            w1 = t1 if b else 1.0 - t1
            for c in (0, 1):
                w2 = t2 if c else 1.0 - t2
                y = y + w0 * w1 * w2 * table[i0 + a, i1 + b, i2 + c]
    return y, c0 | c1 | c2
