"""Pins of the oracle's table-path rate assembly (paper II.D eq. thin_cooling
and eq. total_cooling, II.F, II.G, III.A).

The table path looks the cooling quantities up at the column N = n_e H and
assembles Q_brem = v_b / H^2, Q_syn = v_s / H, eta = v_eta,
Q_thin = Q_brem + eta Q_syn, the bridge with tau_sca = 2 n_e sigma_T H, and
Q_cc = (T_i - T_e) v_c.  Two pins that do not go through that code:

* at a state whose table coordinates all fall on nodes the interpolation is
  exact, so every rate must equal the closed forms of oracle.physics evaluated
  directly at the cell's own (n_e, T_e, T_i, B, H);
* between nodes the interpolated log2 values must lie within the trilinear
  error bound sum_a t_a (1 - t_a) h_a^2 max|d^2 y / du_a^2| / 2 of the exact
  log2 values.

Mutation checks plant plausible slips in a copy of oracle/step.py (a dropped
factor in tau_sca, 1/H instead of 1/H^2, the column N replaced by n_e, eta
dropped, the Coulomb sign flipped, a bridge term dropped) and require the node
pin to catch each one.
"""
import importlib.util
import os

import numpy as np
import pytest

from conftest import ROOT, rel_err
from oracle import physics as P
from oracle import step as S
from oracle import tables as T

# Small tables whose nodes are one decade (or two) apart.  The T_e axes of the
# cooling and the Coulomb tables share their nodes, and no T_e node sits on the
# synchrotron K2 switch (1e8 K) or on theta_e = 1 (10^9.773 K).
SPEC = T.TableSpec(
    cool=(T.Axis(7, 16.0, 28.0), T.Axis(7, 6.05, 12.05), T.Axis(6, 0.0, 10.0)),
    coul=(T.Axis(6, 10.0, 20.0), T.Axis(7, 6.05, 12.05), T.Axis(9, 6.05, 14.05)),
)
T_FLOOR = 10.0 ** 6.5      # between the first two T_e nodes: one layer of cells below the floor


def _node_cells():
    """One cell per cooling node (N, T_e, B), with n_e and T_i on Coulomb nodes
    drawn per cell and H = N / n_e (so that n_e H is the cooling node)."""
    rng = np.random.default_rng(20250513)
    uN, uT, uB = np.meshgrid(*(a.nodes() for a in SPEC.cool), indexing="ij")
    uN, uT, uB = uN.ravel(), uT.ravel(), uB.ravel()
    un = SPEC.coul[0].nodes()[rng.integers(0, SPEC.coul[0].n, uN.size)]
    ui = SPEC.coul[2].nodes()[rng.integers(0, SPEC.coul[2].n, uN.size)]
    n_e = 10.0 ** un
    T_e = 10.0 ** uT
    T_i = 10.0 ** ui
    B = 10.0 ** uB
    H = 10.0 ** (uN - un)
    return n_e, T_e, T_i, B, H


@pytest.fixture(scope="module")
def tabs():
    return T.build_tables(SPEC)


@pytest.fixture(scope="module")
def node_cells():
    return _node_cells()


@pytest.fixture(scope="module")
def direct(node_cells):
    return P.direct_rates(*node_cells)


def _node_errors(step_mod, tabs, cells, direct):
    """Max relative error of the table path against the closed forms at node cells."""
    ts = step_mod.TableSet(SPEC, tabs)
    n_e, T_e, T_i, B, H = cells
    got = step_mod.table_rates(ts, n_e, T_e, T_i, B, H, T_floor=T_FLOOR)
    on = T_e >= T_FLOOR
    err = {k: float(np.max(rel_err(got[k], direct[k]))) for k in ("q_brem", "q_syn", "eta", "q_thin", "q_cc")}
    err["q_rad"] = float(np.max(rel_err(got["q_rad"][on], direct["q_rad"][on])))
    err["q_rad_floor"] = float(np.max(np.abs(got["q_rad"][~on])))
    qa = step_mod.q_rad_at(ts, n_e, T_e, B, H, T_FLOOR)
    err["q_rad_at"] = float(np.max(rel_err(qa[on], direct["q_rad"][on])))
    err["q_rad_at_floor"] = float(np.max(np.abs(qa[~on])))
    return err


def test_node_cells_exercise_every_term(node_cells, direct):
    """The node cells span the regimes in which each term of the assembly matters,
    so that the comparison below can see a slip in any of them."""
    n_e, T_e, T_i, B, H = node_cells
    ta = P.tau_absorption(direct["q_thin"], T_e, H)
    ts = P.tau_scattering(n_e, H)
    D = 1.0 + P.K.SQRT3 * ta + 1.5 * ta * (ta + ts)
    assert np.any(D > 10.0) and np.any(D - 1.0 < 1e-6)          # thick and thin cells
    assert np.any(1.5 * ta * ts / D > 1e-2)                      # tau_sca visible in the bridge
    assert np.any(direct["eta"] > 1.5)                           # Compton enhancement visible
    assert np.any(direct["eta"] * direct["q_syn"] > 10.0 * direct["q_brem"])
    assert np.any(direct["q_brem"] > 10.0 * direct["eta"] * direct["q_syn"])
    assert np.ptp(np.log10(H)) > 8.0                             # powers of H visible
    assert np.any(T_e < T_FLOOR) and np.any(T_i != T_e)


def test_table_rates_equal_closed_forms_at_nodes(tabs, node_cells, direct):
    err = _node_errors(S, tabs, node_cells, direct)
    for k in ("q_brem", "q_syn", "eta", "q_thin", "q_cc", "q_rad", "q_rad_at"):
        assert err[k] < 1e-12, (k, err[k])
    assert err["q_rad_floor"] == 0.0 and err["q_rad_at_floor"] == 0.0


# (description, text in oracle/step.py, replacement)
MUTATIONS = (
    ("tau_sca without the factor 2", "tau_sca = 2.0 * n_e * K.SIGMA_T * H", "tau_sca = 1.0 * n_e * K.SIGMA_T * H"),
    ("Q_brem = v_b / H", "q_brem = v_b / (H * H)", "q_brem = v_b / H"),
    ("Q_syn = v_s", "q_syn = v_s / H", "q_syn = v_s"),
    ("column N replaced by n_e", "uN = np.log10(n_e) + np.log10(H)", "uN = np.log10(n_e)"),
    ("eta dropped from Q_thin", "q_thin = q_brem + v_se / H", "q_thin = q_brem + q_syn"),
    ("eta dropped from the se table", 'else self.t["synch"] + self.t["eta"])', 'else self.t["synch"])'),
    ("Q_syn without 1/H in q_rad_at", "q_thin = v_b / (H * H) + v_se / H", "q_thin = v_b / (H * H) + v_se"),
    ("Coulomb sign flipped", '"q_cc": (T_i - T_e) * v_c', '"q_cc": (T_e - T_i) * v_c'),
    ("bridge tau_abs^2 term dropped", "1.5 * tau_abs * (tau_abs + tau_sca)", "1.5 * tau_abs * tau_sca"),
    ("sqrt3 term dropped", "1.0 + K.SQRT3 * tau_abs + 1.5", "1.0 + 1.5"),
    ("floor test on the wrong side", "np.where(T_e < T_floor, 0.0, bridge", "np.where(T_e > T_floor, 0.0, bridge"),
)


def _mutated_step(old, new):
    path = os.path.join(ROOT, "oracle", "step.py")
    with open(path) as fh:
        src = fh.read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    spec = importlib.util.spec_from_loader("oracle._mutated_step", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), path + " (mutated)", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_node_pin_catches_planted_slip(tabs, node_cells, direct, desc, old, new):
    err = _node_errors(_mutated_step(old, new), tabs, node_cells, direct)
    worst = max(err[k] for k in ("q_brem", "q_syn", "eta", "q_thin", "q_cc", "q_rad", "q_rad_at"))
    assert worst > 1e-6 or err["q_rad_floor"] > 0.0 or err["q_rad_at_floor"] > 0.0, desc


# ---------------------------------------------------------------------------
# between nodes: the trilinear error bound

FINE = T.TableSpec(
    cool=(T.Axis(6, 21.0, 21.5), T.Axis(6, 9.0, 9.5), T.Axis(6, 4.0, 4.5)),
    coul=(T.Axis(6, 15.0, 15.5), T.Axis(6, 9.0, 9.5), T.Axis(6, 10.0, 10.5)),
)


def _exact_log2(u, which):
    """Exact log2 of a table quantity at log10 coordinates u = (u0, u1, u2)."""
    a, b, c = (10.0 ** np.asarray(v, dtype=np.float64) for v in u)
    if which == "coul":
        return np.log2(P.coulomb_coeff(a, b, c))
    one = np.ones_like(a)
    if which == "brem":
        return np.log2(P.q_brem(a, b))
    sy = P.synchrotron(a, b, c, one)
    if which == "synch":
        return np.log2(sy["q_syn"])
    return np.log2(P.compton_eta(a, b, one, sy["nu_c"]))


def _curvature_bound(cell_lo, h, which):
    """max |d^2 y / du_a^2| over a cell, per axis: second differences on a 5^3
    lattice of the cell (step h_a / 4), times 1.5 for what the lattice misses."""
    g = [cell_lo[a] + h[a] * np.linspace(0.0, 1.0, 5) for a in range(3)]
    U = np.meshgrid(*g, indexing="ij")
    y = _exact_log2(U, which)
    M = []
    for a in range(3):
        d2 = np.diff(y, n=2, axis=a) / (h[a] / 4.0) ** 2
        M.append(1.5 * np.max(np.abs(d2)))
    return np.array(M)


@pytest.mark.parametrize("which", ("brem", "synch", "eta", "coul"))
def test_off_node_within_trilinear_error_bound(which):
    axes = FINE.coul if which == "coul" else FINE.cool
    tab = T.build_coulomb(FINE) if which == "coul" else T.build_cooling(FINE)[which]
    rng = np.random.default_rng(7)
    h = np.array([a.step for a in axes])
    worst = 0.0
    for _ in range(12):
        cell = [rng.integers(0, a.n - 1) for a in axes]
        lo = np.array([axes[a].nodes()[cell[a]] for a in range(3)])
        t = rng.uniform(0.05, 0.95, size=(64, 3))
        u = [lo[a] + t[:, a] * h[a] for a in range(3)]
        y, _ = T.interp3(tab, axes, *u)
        exact = _exact_log2(u, which)
        M = _curvature_bound(lo, h, which)
        bound = np.sum(0.5 * t * (1.0 - t) * h ** 2 * M, axis=1) + 1e-13
        assert np.all(np.abs(y - exact) <= bound), which
        worst = max(worst, float(np.max(np.abs(y - exact) / bound)))
    # the bound is not vacuous: somewhere the error uses a good part of it
    assert worst > 0.05, (which, worst)
