"""Gradients through the cooling step (test infrastructure).

For a cell the backward-Euler update defines (x, z) = (T_e', T_i') implicitly
by R(x, z; p) = (E1, E2) = 0 (see step.py), p = (n_e, T_e, T_i, B, H, table
entries).  Given cotangents g_x, g_z of the outputs, the implicit function
theorem gives the vector-Jacobian product
    J^T lam = (g_x, g_z),   J = dR/d(x, z),   gbar_p = -lam . dR/dp.
On a floor-projected cell x = T_floor is a constant, so only E2 ties z to p:
lam = (0, g_z / (dE2/dz)).  The reported input-state rates Q_rad(T_e) and
Q_cc(T_e, T_i) add their own direct derivatives with cotangents g_qrad, g_qcc.

Table entries are the log2 node values y of each table; an interpolated value
2^y depends on a corner's y through ln 2 * 2^y * (corner weight).  Every other
derivative is the exact derivative of the interpolant inside the cell the
query falls in (one-sided at nodes; zero along a clamped axis).

Pinned by tests/test_oracle_grad.py: central finite differences (relative step
1e-6, cells whose perturbation crosses a table node skipped) on the inputs and
on sampled table entries.
"""
import numpy as np

from . import constants as K
from .step import ST_FLOOR, ST_INVALID
from .tables import axis_coord

LN2 = np.log(2.0)
LN10 = np.log(10.0)


def interp_parts(table, axes, u0, u1, u2):
    """Trilinear value y, dy/du for the three log10 coordinates, and the 8 flat
    corner indices with their weights (arrays of shape (n, 8))."""
    (i0, t0, c0), (i1, t1, c1), (i2, t2, c2) = (axis_coord(u, a) for u, a in zip((u0, u1, u2), axes))
    n1, n2 = table.shape[1], table.shape[2]
    flat = table.ravel()
    y = 0.0
    dy = [0.0, 0.0, 0.0]
    idx, wts = [], []
    for a in (0, 1):
        wa, da = (t0, 1.0) if a else (1.0 - t0, -1.0)
        for b in (0, 1):
            wb, db = (t1, 1.0) if b else (1.0 - t1, -1.0)
            for c in (0, 1):
                wc, dc = (t2, 1.0) if c else (1.0 - t2, -1.0)
                k = ((i0 + a) * n1 + (i1 + b)) * n2 + (i2 + c)
                v = flat[k]
                w = wa * wb * wc
                y = y + w * v
                dy[0] = dy[0] + da * wb * wc * v
                dy[1] = dy[1] + wa * db * wc * v
                dy[2] = dy[2] + wa * wb * dc * v
                idx.append(k)
                wts.append(w)
    for k, (ax, cl) in enumerate(zip(axes, (c0, c1, c2))):
        dy[k] = np.where(cl, 0.0, dy[k] / ax.step)
    return y, dy, np.stack(idx, axis=1), np.stack(wts, axis=1)


def qrad_parts(ts, n_e, x, B, H, T_floor):
    """Bridged Q_rad at T_e' = x and its derivatives.

    Returns (q, d) with d[p] = dQ_rad/dp for p in n_e, x, B, H, and d["tab"] =
    list of (table name, corner indices, dQ_rad/dy per corner)."""
    uN = np.log10(n_e) + np.log10(H)
    ux = np.log10(x)
    uB = np.log10(B)
    yb, dyb, ib, wb = interp_parts(ts.t["brem"], ts.spec.cool, uN, ux, uB)
    # eta Q_syn through the se table (log2 of the product; synch + eta), whose
    # entries move with either table's: d se / d synch = d se / d eta = 1
    yse, dyse, ise, wse = interp_parts(ts.t["se"], ts.spec.cool, uN, ux, uB)
    vb = np.exp2(yb) / H ** 2               # Q_brem
    vse = np.exp2(yse) / H                  # eta Q_syn
    qt = vb + vse
    # dQ_thin / du_a (log10 coordinates) and the chain to physical variables
    dqt_du = [LN2 * (vb * dyb[a] + vse * dyse[a]) for a in range(3)]
    dqt = {"n_e": dqt_du[0] / (n_e * LN10),
           "x": dqt_du[1] / (x * LN10),
           "B": dqt_du[2] / (B * LN10),
           "H": dqt_du[0] / (H * LN10) - 2.0 * vb / H - vse / H}
    ts_ = 2.0 * n_e * K.SIGMA_T * H
    ta = H * qt / (4.0 * K.SIGMA_SB * x ** 4)
    D = 1.0 + K.SQRT3 * ta + 1.5 * ta * (ta + ts_)
    D_ta = K.SQRT3 + 1.5 * (2.0 * ta + ts_)
    q = qt / D
    # dQ_rad/dQ_thin including tau_abs's own dependence on Q_thin:
    # (D - tau_abs dD/dtau_abs) / D^2 = (1 - 1.5 tau_abs^2) / D^2 exactly; the
    # expanded form cancels catastrophically when scattering dominates
    fac = (1.0 - 1.5 * ta ** 2) / D ** 2
    d = {}
    for p in ("n_e", "x", "B", "H"):
        # remaining explicit dependence of tau_abs (through H, x) and tau_sca (n_e, H)
        dta = ta * ((1.0 / H if p == "H" else 0.0) - (4.0 / x if p == "x" else 0.0))
        dts = ts_ * ((1.0 / n_e if p == "n_e" else 0.0) + (1.0 / H if p == "H" else 0.0))
        d[p] = fac * dqt[p] - qt / D ** 2 * (D_ta * dta + 1.5 * ta * dts)
    d["tab"] = [("brem", ib, fac[:, None] * LN2 * vb[:, None] * wb),
                ("synch", ise, fac[:, None] * LN2 * vse[:, None] * wse),
                ("eta", ise, fac[:, None] * LN2 * vse[:, None] * wse)]
    off = x < T_floor
    q = np.where(off, 0.0, q)
    for p in ("n_e", "x", "B", "H"):
        d[p] = np.where(off, 0.0, d[p])
    d["tab"] = [(k, i, np.where(off[:, None], 0.0, v)) for k, i, v in d["tab"]]
    return q, d


def kc_parts(ts, n_e, x, z):
    """Coulomb coefficient v_c(n_e, x, z) and its derivatives (n_e, x, z, table)."""
    y, dy, idx, w = interp_parts(ts.t["coul"], ts.spec.coul, np.log10(n_e), np.log10(x), np.log10(z))
    kc = np.exp2(y)
    d = {"n_e": LN2 * kc * dy[0] / (n_e * LN10),
         "x": LN2 * kc * dy[1] / (x * LN10),
         "z": LN2 * kc * dy[2] / (z * LN10),
         "tab": [("coul", idx, LN2 * kc[:, None] * w)]}
    return kc, d


def vjp_step_be(ts, cells, out, dt, g_te, g_ti, g_qrad=None, g_qcc=None, T_floor=1.0e6):
    """Vector-Jacobian product of the backward-Euler step.

    cells: dict of input arrays (n_e, T_e, T_i, B, H); out: the oracle's step
    output (T_e_new, T_i_new, status).  Returns dict with gradients for the five
    inputs and "tables": dict of arrays shaped like the tables."""
    n_e, T_e, T_i, B, H = (np.asarray(cells[k], dtype=np.float64) for k in ("n_e", "T_e", "T_i", "B", "H"))
    n = n_e.size
    zero = np.zeros(n)
    g_te = np.broadcast_to(np.asarray(g_te, dtype=np.float64), (n,))
    g_ti = np.broadcast_to(np.asarray(g_ti, dtype=np.float64), (n,))
    g_qrad = zero if g_qrad is None else np.broadcast_to(np.asarray(g_qrad, dtype=np.float64), (n,))
    g_qcc = zero if g_qcc is None else np.broadcast_to(np.asarray(g_qcc, dtype=np.float64), (n,))
    status = np.asarray(out["status"])
    bad = (status & ST_INVALID) != 0
    floor = (status & ST_FLOOR) != 0
    x = np.where(bad, T_e, np.asarray(out["T_e_new"], dtype=np.float64))
    z = np.where(bad, T_i, np.asarray(out["T_i_new"], dtype=np.float64))
    c = K.U_PER_NKT * n_e * K.K_B
    c_n = K.U_PER_NKT * K.K_B

    qr, dq = qrad_parts(ts, n_e, x, B, H, T_floor)
    kc, dk = kc_parts(ts, n_e, x, z)
    zx = z - x
    # Jacobian of (E1, E2) with respect to (x, z)
    j11 = c + dt * dq["x"] + dt * kc - dt * zx * dk["x"]
    j12 = -dt * kc - dt * zx * dk["z"]
    j21 = -dt * kc + dt * zx * dk["x"]
    j22 = c + dt * kc + dt * zx * dk["z"]
    det = j11 * j22 - j12 * j21
    # J^T lam = g:  [j11 j21; j12 j22] lam = (g_te, g_ti)
    lam1 = np.where(floor, 0.0, (j22 * g_te - j21 * g_ti) / det)
    lam2 = np.where(floor, g_ti / j22, (j11 * g_ti - j12 * g_te) / det)
    # dE/dp
    dE1 = {"n_e": c_n * (x - T_e) + dt * dq["n_e"] - dt * zx * dk["n_e"],
           "T_e": -c, "T_i": zero, "B": dt * dq["B"], "H": dt * dq["H"]}
    dE2 = {"n_e": c_n * (z - T_i) + dt * zx * dk["n_e"],
           "T_e": zero, "T_i": -c, "B": zero, "H": zero}
    grads = {p: -(lam1 * dE1[p] + lam2 * dE2[p]) for p in ("n_e", "T_e", "T_i", "B", "H")}
    tab = {k: np.zeros(v.shape) for k, v in ts.t.items()}
    for name, idx, val in dq["tab"]:
        np.add.at(tab[name].ravel(), idx.ravel(), (-(lam1 * dt)[:, None] * val).ravel())
    for name, idx, val in dk["tab"]:
        np.add.at(tab[name].ravel(), idx.ravel(), (-(-lam1 * dt * zx + lam2 * dt * zx)[:, None] * val).ravel())

    # direct terms of the input-state rates
    qr0, dq0 = qrad_parts(ts, n_e, T_e, B, H, T_floor)
    kc0, dk0 = kc_parts(ts, n_e, T_e, T_i)
    gap = T_i - T_e
    grads["n_e"] = grads["n_e"] + g_qrad * dq0["n_e"] + g_qcc * gap * dk0["n_e"]
    grads["T_e"] = grads["T_e"] + g_qrad * dq0["x"] + g_qcc * (-kc0 + gap * dk0["x"])
    grads["T_i"] = grads["T_i"] + g_qcc * (kc0 + gap * dk0["z"])
    grads["B"] = grads["B"] + g_qrad * dq0["B"]
    grads["H"] = grads["H"] + g_qrad * dq0["H"]
    for name, idx, val in dq0["tab"]:
        np.add.at(tab[name].ravel(), idx.ravel(), (g_qrad[:, None] * val).ravel())
    for name, idx, val in dk0["tab"]:
        np.add.at(tab[name].ravel(), idx.ravel(), ((g_qcc * gap)[:, None] * val).ravel())

    for p in grads:
        grads[p] = np.where(bad, 0.0, grads[p])
    grads["tables"] = tab
    return grads


def radiated_energy_cotangents(cells):
    """Cotangents of the loss E = sum_cells c (T_e + T_i - T_e' - T_i') with
    respect to the outputs (T_e', T_i'): both -c.  The explicit part
    c (T_e + T_i) contributes dE/dT_e = dE/dT_i = c and dE/dn_e = 1.5 k (T_e + T_i - T_e' - T_i')."""
    c = K.U_PER_NKT * np.asarray(cells["n_e"], dtype=np.float64) * K.K_B
    return -c, -c
