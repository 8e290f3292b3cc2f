"""Brute-force references on tiny inputs (test infrastructure).

``scan_roots`` evaluates the two backward-Euler residuals E1, E2 of the implicit
update (paper III.B.1, reading: backward Euler) on a fine log-spaced 2-D grid of
(T_e', T_i') and returns every grid cell in which both residuals change sign
among the cell's corners, refined by a second finer grid inside each such cell.
It does not use the nested reduction that ``step.step_be`` uses, so agreement
between the two pins the solver.

``integrate_ode`` integrates du_e/dt = -Q_rad + Q_cc, du_i/dt = -Q_cc over dt
with a stiff implicit Runge-Kutta method at tight tolerance (SciPy Radau), the
"exact" step against which the time-discretisation error of the backward-Euler
and explicit updates is reported.  Reported, not a parity gate.
"""
import numpy as np
from scipy.integrate import solve_ivp

from . import constants as K
from .step import q_rad_at


def residuals(ts, cell, x, z, dt, T_floor):
    """E1, E2 of the implicit update at trial temperatures (x, z), broadcasting."""
    n_e, T_e, T_i, B, H = cell
    c = K.U_PER_NKT * n_e * K.K_B
    x, z = np.broadcast_arrays(np.asarray(x, dtype=np.float64), np.asarray(z, dtype=np.float64))
    qr = q_rad_at(ts, np.full(x.shape, n_e), x, np.full(x.shape, B), np.full(x.shape, H), T_floor)
    v_c, _ = ts.coulomb(np.full(x.shape, n_e), x, z)
    qcc = (z - x) * v_c
    return c * (x - T_e) + dt * qr - dt * qcc, c * (z - T_i) + dt * qcc


def _sign_cells(e1, e2):
    """Grid cells whose four corners show a sign change in both residuals."""
    def changes(e):
        s = np.sign(e)
        c = np.stack([s[:-1, :-1], s[1:, :-1], s[:-1, 1:], s[1:, 1:]])
        return (c.max(axis=0) > 0) & (c.min(axis=0) < 0) | (c == 0).any(axis=0)
    return np.argwhere(changes(e1) & changes(e2))


def scan_roots(ts, cell, dt, T_floor=1.0e6, n=512, refine=64):
    """Roots of (E1, E2) on a log grid over T_e' in [T_floor, Tmax], T_i' in [Tmin, Tmax].

    Returns an array of (T_e', T_i') centres of the refined sign-change cells and
    the log10 spacing of the refined grid.
    """
    n_e, T_e, T_i, B, H = (float(v) for v in cell)
    cell = (n_e, T_e, T_i, B, H)
    tmax = max(T_e, T_i)
    tmin = min(T_e, T_i, T_floor)
    lx = np.linspace(np.log10(T_floor), np.log10(tmax), n)
    lz = np.linspace(np.log10(tmin), np.log10(tmax), n)
    X, Z = np.meshgrid(10.0 ** lx, 10.0 ** lz, indexing="ij")
    e1, e2 = residuals(ts, cell, X, Z, dt, T_floor)
    hits = _sign_cells(e1, e2)
    out = []
    for a, b in hits:
        fx = np.linspace(lx[a], lx[a + 1], refine)
        fz = np.linspace(lz[b], lz[b + 1], refine)
        X2, Z2 = np.meshgrid(10.0 ** fx, 10.0 ** fz, indexing="ij")
        f1, f2 = residuals(ts, cell, X2, Z2, dt, T_floor)
        for a2, b2 in _sign_cells(f1, f2):
            out.append((10.0 ** (0.5 * (fx[a2] + fx[a2 + 1])), 10.0 ** (0.5 * (fz[b2] + fz[b2 + 1]))))
    step = max(lx[1] - lx[0], lz[1] - lz[0]) / (refine - 1)
    return np.array(out).reshape(-1, 2), step


def integrate_ode(ts, cell, dt, T_floor=1.0e6, rtol=1e-11):
    """Final (T_e, T_i) of the cooling ODE over dt (Radau, rtol ``rtol``)."""
    n_e, T_e, T_i, B, H = (float(v) for v in cell)
    c = K.U_PER_NKT * n_e * K.K_B

    def rhs(_t, y):
        te, ti = np.exp(y)
        qr = float(q_rad_at(ts, np.array([n_e]), np.array([te]), np.array([B]), np.array([H]), T_floor)[0])
        v_c, _ = ts.coulomb(np.array([n_e]), np.array([te]), np.array([ti]))
        qcc = (ti - te) * float(v_c[0])
        return [(-qr + qcc) / (c * te), -qcc / (c * ti)]

    sol = solve_ivp(rhs, (0.0, dt), [np.log(T_e), np.log(T_i)], method="Radau",
                    rtol=rtol, atol=1e-14)
    return float(np.exp(sol.y[0, -1])), float(np.exp(sol.y[1, -1]))
