"""Per-cell rates and the cooling source step (paper II.D, II.G, III.B).

Table-driven rates (``table_rates``) follow the hot path of the paper: look up
the cooling quantities at (N = n_e H, T_e, B) and the Coulomb coefficient at
(n_e, T_e, T_i), then assemble Q_brem = v_b / H^2, Q_syn = v_s / H, eta = v_eta,
Q_thin = Q_brem + eta Q_syn (eq. thin_cooling), the bridged
Q_rad = Q_thin / (1 + sqrt3 tau_abs + 1.5 tau_abs (tau_abs + tau_sca))
(eq. total_cooling multiplied through by tau_abs), and Q_cc = (T_i - T_e) v_c.
Cooling is zero below the temperature floor (III.B.2).

The implicit update (``step_be``) is backward Euler on the electron and ion
internal energies u_s = 1.5 n_e k T_s (gamma = 5/3, n_i = n_e):
  E1:  c (T_e' - T_e) + dt Q_rad(T_e') - dt Q_cc(T_e', T_i') = 0
  E2:  c (T_i' - T_i) + dt Q_cc(T_e', T_i')                 = 0,   c = 1.5 n_e k,
with n_e, B, H held fixed and every rate taken through the tables.  The paper
adapts an IMEX solver it does not spell out (III.B.1); backward Euler on the
stiff source is the reading used here.  The oracle solves it nested: for a
trial x = T_e' the ion temperature z(x) solves E2 (it lies between x and T_i),
and the outer residual is E1 + E2, g(x) = c (x + z(x) - T_e - T_i) + dt Q_rad(x).
Root choice: the first sign change of g met when moving from x = T_e in the
direction the source points, located on the T_e nodes of the cooling table and
refined by bisection.  With the floor, g jumps at T_floor; when the jump is the
sign change the answer is T_e' = T_floor exactly (floor projection).

The explicit update (``step_explicit16``) takes 16 forward-Euler substeps with
the cooling capped so that u_e drops by at most 30 % per substep (III.B.1) and
the exchange capped at 30 % of either energy and half the temperature gap.

Parity pins (tests/test_oracle_step.py): residuals of E1, E2 at the answer,
energy conservation c (dT_e + dT_i) = -dt Q_rad(T_e'), the exchange-only case
(T_e + T_i conserved, no crossing), the dt -> 0 limit, agreement with the
brute-force 2-D scan of oracle/finegrid.py, and the explicit limiter.
"""
import numpy as np

from . import constants as K
from .tables import TABLE_NAMES, interp3

# status bits, shared meaning with the library's per-cell status byte
ST_INVALID = 1
ST_CLAMP_COOL = 2
ST_CLAMP_COUL = 4
ST_FLOOR = 8
ST_MAXITER = 16
ST_MULTIROOT = 32
ST_NO_RATE = 64       # literal Compton reading: a cooling-table corner of the cell has no value


class TableSet:
    """FP64 log2 tables plus their axes; evaluates the interpolated quantities.

    ``tables`` may carry "se" (log2 of eta Q_syn; the storage form's own, see
    oracle.tables.quantize_tables); otherwise se is synch + eta."""

    def __init__(self, spec, tables):
        self.spec = spec
        self.t = {k: np.asarray(tables[k], dtype=np.float64) for k in TABLE_NAMES}
        self.t["se"] = (np.asarray(tables["se"], dtype=np.float64) if "se" in tables
                        else self.t["synch"] + self.t["eta"])

    def cooling(self, n_e, T, B, H):
        """(v_b, v_s, v_eta, v_se, clamped) at column N = n_e H; v_se = eta Q_syn(H = 1)
        from the se table (the rate path's product)."""
        uN = np.log10(n_e) + np.log10(H)
        uT = np.log10(T)
        uB = np.log10(B)
        out = []
        clamped = False
        for k in ("brem", "synch", "eta", "se"):
            y, c = interp3(self.t[k], self.spec.cool, uN, uT, uB)
            out.append(np.exp2(y))
            clamped = clamped | c
        return out[0], out[1], out[2], out[3], clamped

    def coulomb(self, n_e, T_e, T_i):
        """(v_c, clamped): the Coulomb coefficient Q_cc / (T_i - T_e)."""
        y, c = interp3(self.t["coul"], self.spec.coul, np.log10(n_e), np.log10(T_e), np.log10(T_i))
        return np.exp2(y), c


def bridge(q_thin, T, H, n_e):
    """Hubeny bridge in the form finite at tau_abs -> 0 (eq. total_cooling)."""
    tau_sca = 2.0 * n_e * K.SIGMA_T * H
    tau_abs = H * q_thin / (4.0 * K.SIGMA_SB * T ** 4)
    return q_thin / (1.0 + K.SQRT3 * tau_abs + 1.5 * tau_abs * (tau_abs + tau_sca))


def q_rad_at(ts, n_e, T, B, H, T_floor):
    """Bridged radiative cooling at electron temperature T, zero below T_floor."""
    v_b, _, _, v_se, _ = ts.cooling(n_e, T, B, H)
    q_thin = v_b / (H * H) + v_se / H
    return np.where(T < T_floor, 0.0, bridge(q_thin, T, H, n_e))


def table_rates(ts, n_e, T_e, T_i, B, H, T_floor=1.0e6):
    """All rates at the input state (dict of arrays) plus a status array."""
    n_e, T_e, T_i, B, H = (np.asarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, B, H))
    v_b, v_s, v_eta, v_se, cl_cool = ts.cooling(n_e, T_e, B, H)
    q_brem = v_b / (H * H)
    q_syn = v_s / H
    q_thin = q_brem + v_se / H
    q_rad = np.where(T_e < T_floor, 0.0, bridge(q_thin, T_e, H, n_e))
    v_c, cl_coul = ts.coulomb(n_e, T_e, T_i)
    status = (np.where(cl_cool, ST_CLAMP_COOL, 0) | np.where(cl_coul, ST_CLAMP_COUL, 0) |
              np.where(np.isnan(q_rad) & ~invalid_mask(n_e, T_e, T_i, B, H), ST_NO_RATE, 0))
    return {"q_brem": q_brem, "q_syn": q_syn, "eta": v_eta, "q_thin": q_thin,
            "q_rad": q_rad, "q_cc": (T_i - T_e) * v_c, "status": status.astype(np.uint8)}


def invalid_mask(*arrays):
    bad = np.zeros(np.shape(arrays[0]), dtype=bool)
    for a in arrays:
        bad |= ~np.isfinite(a) | (a <= 0.0)
    return bad


# ---------------------------------------------------------------------------
# backward Euler


def _bisect_log(fun, a, b, iters=80):
    """Bisection in ln x on [a, b] (a <= b elementwise) for fun(a) <= 0 <= fun(b)."""
    la, lb = np.log(a), np.log(b)
    for _ in range(iters):
        m = 0.5 * (la + lb)
        if np.all((m == la) | (m == lb)):
            break
        neg = fun(np.exp(m)) <= 0.0
        la = np.where(neg, m, la)
        lb = np.where(neg, lb, m)
    return np.exp(0.5 * (la + lb))


def ion_temperature(ts, n_e, T_i, x, c, dt):
    """z(x): the root of E2 for a trial electron temperature x.

    E2(z) = c (z - T_i) + dt (z - x) v_c(n_e, x, z) is <= 0 at z = min(x, T_i)
    and >= 0 at z = max(x, T_i); bisection in ln z between them.
    """
    lo = np.minimum(x, T_i)
    hi = np.maximum(x, T_i)

    def e2(z):
        v_c, _ = ts.coulomb(n_e, x, z)
        return c * (z - T_i) + dt * (z - x) * v_c

    z = _bisect_log(e2, lo, hi)
    return np.where(lo == hi, lo, z)


def _outer(ts, cell, x, dt, T_floor):
    """g(x) = c (x - T_e) + c (z(x) - T_i) + dt Q_rad(x) and z(x)."""
    n_e, T_e, T_i, B, H, c = cell
    z = ion_temperature(ts, n_e, T_i, x, c, dt)
    g = c * (x - T_e) + c * (z - T_i) + dt * q_rad_at(ts, n_e, x, B, H, T_floor)
    return g, z


def step_be(ts, n_e, T_e, T_i, B, H, dt, T_floor=1.0e6, diagnose=False):
    """Backward-Euler update; returns dict T_e_new, T_i_new, status (+ rates at input).

    ``diagnose`` continues the node scan past the first sign change and sets
    ST_MULTIROOT where g changes sign more than once along the path.
    """
    n_e, T_e, T_i, B, H = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (n_e, T_e, T_i, B, H))
    bad = invalid_mask(n_e, T_e, T_i, B, H)
    # placeholder state for invalid cells; their outputs are overwritten below
    n_e, T_e, T_i, B, H = (np.where(bad, 1.0e12 if k == 0 else 1.0e8, v)
                           for k, v in enumerate((n_e, T_e, T_i, B, H)))
    ncell = n_e.size
    c = K.U_PER_NKT * n_e * K.K_B
    rates = table_rates(ts, n_e, T_e, T_i, B, H, T_floor)
    status = rates["status"].copy()

    g0, z0 = _outer(ts, (n_e, T_e, T_i, B, H, c), T_e, dt, T_floor)
    down = g0 > 0.0
    # far end of the search: down to min(T_i, T_floor), up to T_i
    far = np.where(down, np.minimum(T_i, T_floor), T_i)
    # candidate points: T_e-nodes of the cooling table strictly between T_e and far,
    # T_floor if strictly between, then far; ordered away from T_e
    nodes = 10.0 ** ts.spec.cool[1].nodes()
    cand = np.concatenate([np.broadcast_to(nodes, (ncell, nodes.size)),
                           T_floor * np.ones((ncell, 1))], axis=1)
    lo_end = np.where(down, far, T_e)[:, None]
    hi_end = np.where(down, T_e, far)[:, None]
    inside = (cand > lo_end) & (cand < hi_end)
    key = np.where(inside, np.where(down[:, None], -cand, cand), np.inf)
    order = np.argsort(key, axis=1)
    cand = np.take_along_axis(cand, order, axis=1)
    count = inside.sum(axis=1)
    ncand = cand.shape[1] + 1
    cand = np.concatenate([cand, far[:, None]], axis=1)
    cand[np.arange(ncell), count] = far          # far end right after the interior points
    last = count                                  # index of the far end per cell

    x_out = T_e.copy()
    z_out = z0.copy()
    done = g0 == 0.0
    prev_x = T_e.copy()
    prev_g = g0.copy()
    brk_a = np.zeros(ncell)
    brk_b = np.zeros(ncell)
    found = np.zeros(ncell, dtype=bool)
    changes = np.zeros(ncell, dtype=np.int64)
    for j in range(ncand):
        act = (~done) & (j <= last) & ((~found) | diagnose)
        if not np.any(act):
            break
        idx = np.nonzero(act)[0]
        cell = tuple(v[idx] for v in (n_e, T_e, T_i, B, H, c))
        xj = cand[idx, j]
        gj, _ = _outer(ts, cell, xj, dt, T_floor)
        flip = (np.sign(gj) != np.sign(prev_g[idx])) | (gj == 0.0)
        changes[idx] += flip
        first = flip & ~found[idx]
        sel = idx[first]
        brk_a[sel] = np.minimum(prev_x[sel], xj[first])
        brk_b[sel] = np.maximum(prev_x[sel], xj[first])
        found[sel] = True
        prev_x[idx] = xj
        prev_g[idx] = np.where(gj == 0.0, prev_g[idx], gj)

    # refine each located sign change by bisection in ln x
    todo = np.nonzero(found & ~done)[0]
    if todo.size:
        cell = tuple(v[todo] for v in (n_e, T_e, T_i, B, H, c))
        # g <= 0 at the low end of each bracket and > 0 at its high end
        x = _bisect_log(lambda x: _outer(ts, cell, x, dt, T_floor)[0], brk_a[todo], brk_b[todo])
        x_out[todo] = x
    # floor projection: the search reached T_floor without a sign change
    floor_hit = ~found & ~done
    # the bisection can also converge onto the floor discontinuity
    near = found & (np.abs(x_out - T_floor) <= 1e-12 * T_floor)
    if np.any(near):
        idx = np.nonzero(near)[0]
        cell = tuple(v[idx] for v in (n_e, T_e, T_i, B, H, c))
        g_at, _ = _outer(ts, cell, np.full(idx.size, T_floor), dt, T_floor)
        floor_hit[idx[g_at > 0.0]] = True
    x_out = np.where(floor_hit, T_floor, x_out)
    z_out = ion_temperature(ts, n_e, T_i, x_out, c, dt)
    status = status | np.where(floor_hit, ST_FLOOR, 0).astype(np.uint8)
    if diagnose:
        status = status | np.where(changes > 1, ST_MULTIROOT, 0).astype(np.uint8)
    # invalid input: T' = T, rates NaN
    x_out = np.where(bad, np.nan, x_out)
    z_out = np.where(bad, np.nan, z_out)
    out = {"T_e_new": x_out, "T_i_new": z_out, "status": np.where(bad, ST_INVALID, status).astype(np.uint8)}
    for k in ("q_brem", "q_syn", "eta", "q_thin", "q_rad", "q_cc"):
        out[k] = np.where(bad, np.nan, rates[k])
    return out


def step_explicit16(ts, n_e, T_e, T_i, B, H, dt, T_floor=1.0e6, substeps=K.EXPLICIT_SUBSTEPS):
    """16 forward-Euler substeps with the 30 % limiter (III.B.1)."""
    n_e, T_e, T_i, B, H = (np.atleast_1d(np.asarray(v, dtype=np.float64)).copy() for v in (n_e, T_e, T_i, B, H))
    c = K.U_PER_NKT * n_e * K.K_B
    h = dt / substeps
    cap = K.EXPLICIT_CAP
    rates0 = table_rates(ts, n_e, T_e, T_i, B, H, T_floor)
    te, ti = T_e.copy(), T_i.copy()
    for _ in range(substeps):
        q_rad = q_rad_at(ts, n_e, te, B, H, T_floor)
        v_c, _ = ts.coulomb(n_e, te, ti)
        q_cc = (ti - te) * v_c
        q_r = np.minimum(q_rad, cap * c * te / h)
        lim = np.minimum(0.5 * c * np.abs(ti - te), cap * c * np.minimum(te, ti)) / h
        q_c = np.clip(q_cc, -lim, lim)
        te, ti = te + h * (q_c - q_r) / c, ti - h * q_c / c
    out = {"T_e_new": te, "T_i_new": ti, "status": rates0["status"]}
    for k in ("q_brem", "q_syn", "eta", "q_thin", "q_rad", "q_cc"):
        out[k] = rates0[k]
    return out
