"""The paper's own table layout (test infrastructure; only tests, the smoke
check and the benchmark's CPU baseline use this package).

Sec. II.F tabulates the total cooling Q_total(H_th, B, n_e, T_e) on a 4-D grid
of 100 log-spaced points per axis over H in [1e3, 1e12] cm, B in [1, 1e10] G,
n_e in [1e2, 1e25] cm^-3, T_e in [1e2, 1e15] K, read by linear interpolation
in each dimension (Sec. III.A, with the n_e and T_e axes flattened into one
texture axis and that one interpolated by hand).  Here the table holds log2
of the bridged Q_total (eq. total_cooling) at every node, from the closed
forms, and is read by 4-D multilinear interpolation in the log10 axes, clamped
at the edges; the flattening is a texture-memory constraint of the paper's GPU
and changes no value.  It is the comparison layout for the exact 3-D column
tables of tables.py: same closed forms, different parametrisation.
"""
import numpy as np

from . import physics
from .tables import Axis, axis_coord

AXIS_NAMES = ("H", "B", "n_e", "T_e")


def paper_axes(n=100):
    """(H, B, n_e, T_e) axes in log10 with the paper's ranges."""
    return (Axis(n, 3.0, 12.0), Axis(n, 0.0, 10.0), Axis(n, 2.0, 25.0), Axis(n, 2.0, 15.0))


def build(axes, chunk=1 << 16):
    """log2 Q_total at every node, C-ordered [H][B][n_e][T_e]."""
    shape = tuple(a.n for a in axes)
    u = np.meshgrid(*[a.nodes() for a in axes], indexing="ij")
    H, B, n_e, T_e = (10.0 ** g.ravel() for g in u)
    out = np.empty(H.size)
    for s in range(0, H.size, chunk):
        sl = slice(s, s + chunk)
        r = physics.direct_rates(n_e[sl], T_e[sl], T_e[sl], B[sl], H[sl])
        out[sl] = np.log2(r["q_rad"])
    return out.reshape(shape)


def interp4(table, axes, u):
    """Multilinear interpolation of ``table`` at log10 coordinates u = (uH, uB,
    un, uT) (arrays); returns (y, clamped)."""
    coords = [axis_coord(v, a) for v, a in zip(u, axes)]
    y = 0.0
    for corner in range(16):
        w = 1.0
        idx = []
        for d, (i, t, _) in enumerate(coords):
            bit = (corner >> (3 - d)) & 1
            w = w * (t if bit else 1.0 - t)
            idx.append(i + bit)
        y = y + w * table[tuple(idx)]
    clamped = coords[0][2] | coords[1][2] | coords[2][2] | coords[3][2]
    return y, clamped


def q_total(table, axes, n_e, T_e, B, H):
    """Q_total from the 4-D table at the given cells."""
    u = tuple(np.log10(np.asarray(v, dtype=np.float64)) for v in (H, B, n_e, T_e))
    y, _ = interp4(table, axes, u)
    return np.exp2(y)
