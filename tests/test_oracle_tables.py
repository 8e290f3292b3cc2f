"""Pins of the oracle's tables and multilinear interpolation (paper II.F, II.G, III.A)."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from conftest import rel_err
from oracle import physics as P
from oracle import tables as T


def test_node_coordinates(spec64):
    for ax in spec64.cool + spec64.coul:
        u = ax.nodes()
        assert u[0] == ax.lo and u[-1] == pytest.approx(ax.hi, abs=1e-13)
        assert np.allclose(np.diff(u), ax.step, rtol=1e-12)


def test_values_at_nodes_equal_closed_forms(spec64, tables64):
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 64, size=(40, 3))
    uN, uT, uB = (spec64.cool[a].nodes()[idx[:, a]] for a in range(3))
    N, Te, B = 10.0 ** uN, 10.0 ** uT, 10.0 ** uB
    one = np.ones_like(N)
    sy = P.synchrotron(N, Te, B, one)
    want = {"brem": P.q_brem(N, Te), "synch": sy["q_syn"],
            "eta": P.compton_eta(N, Te, one, sy["nu_c"])}
    for k, v in want.items():
        got = 2.0 ** tables64[k][idx[:, 0], idx[:, 1], idx[:, 2]]
        assert np.all(rel_err(got, v) < 1e-13), k
    un, ue, ui = (spec64.coul[a].nodes()[idx[:, a]] for a in range(3))
    got = 2.0 ** tables64["coul"][idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.all(rel_err(got, P.coulomb_coeff(10.0 ** un, 10.0 ** ue, 10.0 ** ui)) < 1e-13)


def test_column_reduction_is_exact():
    """Rates depend on (n_e, H) only through N = n_e H apart from explicit powers of H."""
    rng = np.random.default_rng(4)
    n = 10 ** rng.uniform(8, 22, 200)
    H = 10 ** rng.uniform(3, 10, 200)
    Te = 10 ** rng.uniform(6, 12, 200)
    B = 10 ** rng.uniform(0, 10, 200)
    N = n * H
    one = np.ones_like(N)
    s_full = P.synchrotron(n, Te, B, H)
    s_col = P.synchrotron(N, Te, B, one)
    assert np.all(rel_err(s_full["q_syn"], s_col["q_syn"] / H) < 1e-11)
    assert np.all(rel_err(P.compton_eta(n, Te, H, s_full["nu_c"]),
                          P.compton_eta(N, Te, one, s_col["nu_c"])) < 1e-11)
    assert np.all(rel_err(P.q_brem(n, Te), P.q_brem(N, Te) / H ** 2) < 1e-13)


def test_interpolation_reproduces_affine_functions(spec64):
    rng = np.random.default_rng(5)
    axes = spec64.cool
    g = np.meshgrid(*[a.nodes() for a in axes], indexing="ij")
    coef = rng.normal(size=4)
    tab = coef[0] + coef[1] * g[0] + coef[2] * g[1] + coef[3] * g[2]
    u = [rng.uniform(a.lo, a.hi, 5000) for a in axes]
    y, clamped = T.interp3(tab, axes, *u)
    want = coef[0] + coef[1] * u[0] + coef[2] * u[1] + coef[3] * u[2]
    assert not clamped.any()
    assert np.max(np.abs(y - want)) < 1e-11


def test_interpolation_matches_scipy(spec64, tables64):
    rng = np.random.default_rng(6)
    for name in ("synch", "coul"):
        axes = spec64.axes(name)
        rgi = RegularGridInterpolator([a.nodes() for a in axes], tables64[name], method="linear")
        u = np.stack([rng.uniform(a.lo, a.hi, 5000) for a in axes], axis=1)
        y, _ = T.interp3(tables64[name], axes, u[:, 0], u[:, 1], u[:, 2])
        assert np.max(np.abs(y - rgi(u))) < 1e-11


def test_interpolation_exact_at_nodes_and_clamped(spec64, tables64):
    axes = spec64.cool
    tab = tables64["eta"]
    for k in ((0, 0, 0), (63, 63, 63), (5, 40, 63), (17, 0, 22)):
        u = [axes[a].nodes()[k[a]] for a in range(3)]
        y, cl = T.interp3(tab, axes, *u)
        assert y == pytest.approx(tab[k], abs=1e-12)
        # the last node may round one ulp past hi and then counts as clamped
        assert not cl or 63 in k
    # outside the range: clamp to the edge value, flagged
    y, cl = T.interp3(tab, axes, axes[0].lo - 3.0, axes[1].hi + 1.0, axes[2].lo)
    assert y == pytest.approx(tab[0, 63, 0], abs=1e-12) and cl


def test_affine_fit_is_least_squares(tables64):
    for name in ("synch", "coul"):
        y = tables64[name][::4, ::4, ::4]
        co = T.affine_fit(y)
        g = np.meshgrid(*[np.arange(n, dtype=float) for n in y.shape], indexing="ij")
        A = np.stack([np.ones(y.size)] + [gi.ravel() for gi in g], axis=1)
        ref, *_ = np.linalg.lstsq(A, y.ravel(), rcond=None)
        assert np.allclose(co, ref, rtol=1e-10, atol=1e-10)


def test_quantized_storage_error_bound(tables64):
    for name in T.TABLE_NAMES:
        co, resid, stored = T.quantize(tables64[name])
        err = np.abs(stored - tables64[name])
        # float32 rounding of the residual: half an ulp of |residual|
        bound = np.abs(resid.astype(np.float64)) * 2.0 ** -24 + 1e-12
        assert np.all(err <= bound), name


def test_bf16_rounding_ties_to_even_and_matches_torch():
    one = 1.0
    cases = {one: one,
             one + 2.0 ** -8: one,                              # tie, even neighbour is 1
             one + 3 * 2.0 ** -8: one + 2.0 ** -6,              # tie, rounds up to even
             one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,     # just above the tie
             -(one + 2.0 ** -8 + 2.0 ** -20): -(one + 2.0 ** -7),
             0.0: 0.0, 2.0 ** -100: 2.0 ** -100}
    got = T.round_bf16(np.array(list(cases), dtype=np.float32))
    assert np.array_equal(got, np.array(list(cases.values()), dtype=np.float32))
    torch = pytest.importorskip("torch")
    a = np.random.default_rng(9).normal(0.0, 30.0, 200000).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(T.round_bf16(a), ref)


def test_bf16_storage_error_bound(tables64):
    for name in T.TABLE_NAMES:
        co, resid, stored = T.quantize(tables64[name], "bf16")
        assert np.array_equal(resid, T.round_bf16(resid))
        err = np.abs(stored - tables64[name])
        # bfloat16 keeps 8 significant bits: half an ulp is 2^-9 relative, plus the float32 step
        bound = np.abs(resid.astype(np.float64)) * (2.0 ** -8 + 2.0 ** -24) + 1e-12
        assert np.all(err <= bound), name
