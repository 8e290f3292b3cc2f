"""The library's device source executed on the host CPU (test-only entry points
rc_selftest_*_host) against the oracle.  These catch logic errors in the
per-cell code before GPU time is spent; the parity claims themselves are made
by the GPU tests, which run the same source as gfx950 kernels."""
import numpy as np
import pytest
from scipy import special

from conftest import rel_err
from oracle import physics as P
from oracle import step as S
from oracle import tables as T
from paper_2505_08855_amd import workloads as W

R = pytest.importorskip("paper_2505_08855_amd.radcool")
DT = W.DT_DEFAULT


@pytest.fixture(scope="module")
def storage64(tables64):
    co, re, st = T.quantize_tables(tables64)
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    return resid, coeffs, st


def test_scaled_bessels():
    z = np.array([0.0053, 0.05, 0.3, 1.0, 7.0, 59.3, 300.0, 6600.0, 1e5, 1.2e7])
    for nu in (0, 1, 2):
        assert np.max(rel_err(R.selftest_special_host(nu, z), special.kve(nu, z))) < 2e-15


def test_tail_integral_and_root():
    x = np.array([1e-9, 1e-6, 1e-2, 0.7, 5.0, 80.0, 3e3, 1e5, 1e6])
    # relative error grows like z * eps in the exponential factor, z = 1.89 x^(1/3)
    assert np.max(rel_err(R.selftest_special_host(3, x), P.tail_integral(x))) < 1e-13
    lr = np.linspace(-92, 37, 40)
    assert np.max(rel_err(R.selftest_special_host(4, lr), P.solve_xc(lr))) < 1e-13


def _ulps(got, ref):
    return np.max(np.abs(got - ref) / np.spacing(np.abs(ref)))


def test_solver_elementary_functions():
    """The solver's own ln, log10, log1p, exp, exp2 against the C library:
    a few ulp over the whole double range, exact special cases."""
    rng = np.random.default_rng(11)
    x = np.concatenate([10 ** rng.uniform(-307, 308, 100000), rng.uniform(0.5, 2.0, 50000),
                        1.0 + rng.uniform(-1e-8, 1e-8, 5000), [5e-324, 2.2250738585072014e-308, 1.0, 2.0, 0.5]])
    assert _ulps(R.selftest_special_host(5, x), np.log(x)) <= 2
    assert _ulps(R.selftest_special_host(6, x), np.log10(x)) <= 4
    v = np.concatenate([rng.uniform(-0.999999, 1e3, 50000), 10 ** rng.uniform(-300, -1, 50000),
                        -(10 ** rng.uniform(-300, -1, 50000)), 10 ** rng.uniform(0, 300, 5000)])
    assert _ulps(R.selftest_special_host(7, v), np.log1p(v)) <= 4
    assert np.array_equal(R.selftest_special_host(5, np.array([1.0])), [0.0])
    assert np.array_equal(R.selftest_special_host(7, np.array([0.0, 1e-300])), [0.0, 1e-300])
    s = np.concatenate([rng.uniform(-699, 699, 100000), rng.uniform(-1e-3, 1e-3, 5000), [0.0, 1.0, -1.0]])
    assert _ulps(R.selftest_special_host(8, s), np.exp(s)) <= 2
    y = np.concatenate([rng.uniform(-1020, 1020, 100000), rng.uniform(-1.0, 1.0, 5000), [0.0, 0.5, -0.5, 1023.5]])
    assert _ulps(R.selftest_special_host(9, y), np.exp2(y)) <= 2
    # powers of two and e^0 are exact
    k = np.arange(-1000, 1001, dtype=np.float64)
    assert np.array_equal(R.selftest_special_host(9, k), np.exp2(k))
    # the ends of the range: the largest finite results, overflow, gradual
    # underflow (to within the spacing of the smallest subnormal), inf, NaN
    top = np.array([709.0, 709.5, 709.78])
    assert _ulps(R.selftest_special_host(8, top), np.exp(top)) <= 2
    e = np.array([-np.inf, np.inf, 800.0, -800.0, 709.8, 745.2, -746.0])
    with np.errstate(over="ignore"):
        assert np.array_equal(R.selftest_special_host(8, e), np.exp(e))
    sub = np.array([-710.0, -720.0, -740.0, -744.0])
    assert np.all(np.abs(R.selftest_special_host(8, sub) - np.exp(sub)) <= 5e-324)
    assert np.isnan(R.selftest_special_host(8, np.array([np.nan])))[0]


def _fastmath_generator():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(R.__file__), "csrc", "fastmath_coeffs.py")
    spec = importlib.util.spec_from_file_location("fastmath_coeffs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_polynomial_coefficients_are_the_economized_series():
    """The polynomial coefficients in rc_fastmath.hpp are the ones the
    committed generator derives, and each economized polynomial stays within
    2^-55 of its function over the reduced range (exact rational arithmetic
    against the Taylor series to degree 30, whose own remainder is below
    1e-30 there)."""
    import math
    import os
    import re
    from fractions import Fraction as F
    gen = _fastmath_generator()
    tabs = gen.tables()
    src = open(os.path.join(os.path.dirname(R.__file__), "csrc", "rc_fastmath.hpp")).read()

    def body(name):
        i = src.index(name)
        return src[i:src.index("\n}\n", i)]

    def coeffs(text):
        return [float.fromhex(h) for h in re.findall(r"(0x1\.[0-9a-f]+p[-+]\d+)", text)]

    # constants of each function, highest degree first (1.0 terms are written as literals)
    assert coeffs(body("RC_HD double fexp2(")) == [float(c) for c in tabs["exp2"][::-1][:-1]]
    assert coeffs(body("RC_HD double fexp(")) == [float(c) for c in tabs["exp"][::-1][:-2]]
    assert coeffs(body("RC_HD double flog(")) == [float(c) for c in tabs["atanh p"][::-1]]
    assert float(tabs["exp2"][0]) == 1.0 and float(tabs["exp"][0]) == float(tabs["exp"][1]) == 1.0

    def horner(c, x):
        p = F(0)
        for a in c[::-1]:
            p = p * x + F(float(a))          # the coefficients as stored
        return p

    ln2 = gen.LN2
    for k in range(-32, 33):
        f = F(k, 64)
        ref = sum(ln2 ** j * f ** j / math.factorial(j) for j in range(31))
        assert abs(horner(tabs["exp2"], f) - ref) / ref < F(1, 2 ** 55)
        r = f * ln2 * F(1002, 1000)
        ref = sum(r ** j / math.factorial(j) for j in range(31))
        assert abs(horner(tabs["exp"], r) - ref) / ref < F(1, 2 ** 55)
    smax = ((gen.SQRT2 - 1) / (gen.SQRT2 + 1)) ** 2
    for k in range(0, 33):
        sv = smax * F(k, 32)
        ref = sum(sv ** j / (2 * j + 3) for j in range(31))
        # p enters ln m = 2 f (1 + s p(s)): its error counts times s
        assert abs(horner(tabs["atanh p"], sv) - ref) * sv < F(1, 2 ** 55)


@pytest.mark.parametrize("n", [64, 128])
def test_node_values_match_oracle(n):
    spec = R.default_spec(n)
    ospec = T.TableSpec.default(n)
    rng = np.random.default_rng(n)
    idx = np.concatenate([rng.integers(0, n, size=(60, 3)),
                          np.array([[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0], [n - 1, 0, n - 1]])])
    uN, uT, uB = (ospec.cool[a].nodes()[idx[:, a]] for a in range(3))
    N, Te, B = 10.0 ** uN, 10.0 ** uT, 10.0 ** uB
    one = np.ones_like(N)
    sy = P.synchrotron(N, Te, B, one)
    want = {0: np.log2(P.q_brem(N, Te)), 1: np.log2(sy["q_syn"]),
            2: np.log2(P.compton_eta(N, Te, one, sy["nu_c"]))}
    un, ue, ui = (ospec.coul[a].nodes()[idx[:, a]] for a in range(3))
    want[3] = np.log2(P.coulomb_coeff(10.0 ** un, 10.0 ** ue, 10.0 ** ui))
    for k in range(4):
        got = np.array([R.selftest_node_host(spec, k, *[int(v) for v in row]) for row in idx])
        assert np.max(np.abs(got - want[k])) < 1e-12, k


def test_step_energy_tier_on_host(spec64, storage64, cells0_small):
    """Backward Euler on identical (oracle-built, FP32-stored) tables: 1e-9 on T'."""
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    cells = [cells0_small[f] for f in W.FIELDS]
    ref = S.step_be(ts, *cells, DT)
    got = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells0_small, DT)
    assert np.max(rel_err(got["T_e_new"], ref["T_e_new"])) < 1e-9
    assert np.max(rel_err(got["T_i_new"], ref["T_i_new"])) < 1e-9
    assert np.array_equal(got["status"], ref["status"])
    assert np.max(rel_err(got["Q_rad"], ref["q_rad"])) < 1e-12
    assert np.max(rel_err(got["Q_cc"], ref["q_cc"])) < 1e-12


def test_step_explicit16_on_host(spec64, storage64, cells0_small):
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    cells = [cells0_small[f] for f in W.FIELDS]
    ref = S.step_explicit16(ts, *cells, DT)
    got = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells0_small, DT,
                               R.default_opts(scheme="explicit16"))
    assert np.max(rel_err(got["T_e_new"], ref["T_e_new"])) < 1e-12
    assert np.max(rel_err(got["T_i_new"], ref["T_i_new"])) < 1e-12


def test_step_edge_cases_on_host(spec64, storage64):
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    cases = {  # n_e, T_e, T_i, B, H
        "floor": (1e20, 2e6, 2e6, 1e8, 1e4),
        "heating": (1e16, 1e8, 1e11, 10.0, 1e6),
        "equal_T": (1e14, 1e9, 1e9, 1e4, 1e8),
        "T_e_above_T_i": (1e15, 1e10, 1e9, 1e4, 1e8),
        "clamped_low_n": (1e3, 1e8, 1e9, 1e2, 1e8),
        "clamped_high_T": (1e12, 3e12, 1e15, 1e6, 1e8),
        "below_floor": (1e12, 5e5, 2e5, 1e3, 1e8),
        "invalid_nan": (np.nan, 1e8, 1e9, 1e3, 1e8),
        "invalid_neg": (1e12, -1e8, 1e9, 1e3, 1e8),
        "invalid_zero": (1e12, 1e8, 1e9, 0.0, 1e8),
    }
    arr = np.array(list(cases.values()), dtype=np.float64).T
    cells = dict(zip(W.FIELDS, arr))
    for dt, floor in ((DT, 1e6), (1e3 * DT, 1.5e6)):
        ref = S.step_be(ts, *arr, dt, T_floor=floor)
        got = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells, dt, R.default_opts(T_floor=floor))
        assert np.array_equal(got["status"], ref["status"]), (got["status"], ref["status"])
        ok = (ref["status"] & 1) == 0
        assert np.all(np.isnan(got["T_e_new"][~ok]))
        assert np.max(rel_err(got["T_e_new"][ok], ref["T_e_new"][ok])) < 1e-9
        assert np.max(rel_err(got["T_i_new"][ok], ref["T_i_new"][ok])) < 1e-9


@pytest.mark.parametrize("floor", [3e6, 1e7, 5e7])
def test_step_floor_branches_on_host(spec64, storage64, floor):
    """Random cells around the floor: T_e and T_i on either side of it, strong
    cooling (large dt), so that every branch of the floor handling runs."""
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    rng = np.random.default_rng(int(floor))
    n = 300
    n_e = 10 ** rng.uniform(14, 20, n)
    T_e = floor * 10 ** rng.uniform(-0.6, 0.8, n)
    T_i = T_e * 10 ** rng.uniform(-1.0, 1.5, n)
    B = np.sqrt(8 * np.pi * n_e * 1.380649e-16 * (T_e + T_i) / 10 ** rng.uniform(-1, 2, n))
    H = 10 ** rng.uniform(5, 9, n)
    dt = DT * 10 ** rng.uniform(0, 4)
    cells = {"n_e": n_e, "T_e": T_e, "T_i": T_i, "B": B, "H": H}
    ref = S.step_be(ts, n_e, T_e, T_i, B, H, dt, T_floor=floor)
    got = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells, dt, R.default_opts(T_floor=floor))
    assert (ref["status"] & S.ST_FLOOR).sum() > 0
    assert np.array_equal(got["status"], ref["status"])
    assert np.max(rel_err(got["T_e_new"], ref["T_e_new"])) < 1e-9
    assert np.max(rel_err(got["T_i_new"], ref["T_i_new"])) < 1e-9


def test_backward_matches_oracle_gradient_on_host(spec64, storage64, cells0_small):
    """The per-cell adjoint (library source on the host) against the oracle's
    implicit-function-theorem gradient on identical tables."""
    from oracle import grad as Gd
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    cells = {f: cells0_small[f][:1024] for f in W.FIELDS}
    out = S.step_be(ts, *[cells[f] for f in W.FIELDS], DT)
    rng = np.random.default_rng(5)
    cot = {k: rng.normal(size=1024) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
    ref = Gd.vjp_step_be(ts, cells, out, DT, cot["T_e_new"], cot["T_i_new"], cot["Q_rad"], cot["Q_cc"])
    fwd = {"T_e_new": out["T_e_new"], "T_i_new": out["T_i_new"], "status": out["status"]}
    g, gt = R.selftest_backward_host(R.default_spec(64), resid, coeffs, cells, fwd, cot, DT)
    # a gradient is only meaningful relative to the loss it differentiates:
    # where d L / d ln p is below ~1e-12 of the loss terms (e.g. d/dB of a
    # brem-dominated cell, flat in B up to table rounding) both sides hold noise
    mag = (np.abs(cot["T_e_new"] * out["T_e_new"]) + np.abs(cot["T_i_new"] * out["T_i_new"])
           + np.abs(cot["Q_rad"] * out["q_rad"]) + np.abs(cot["Q_cc"] * out["q_cc"]))
    for f in W.FIELDS:
        err = np.abs(g[f] - ref[f]) * cells[f]
        assert np.all(err <= 1e-9 * np.abs(ref[f] * cells[f]) + 1e-12 * mag), f
    vc = 64 ** 3
    for k, name in enumerate(T.TABLE_NAMES):
        want = ref["tables"][name].ravel()
        got = gt[k * vc:(k + 1) * vc]
        assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want)), name


@pytest.mark.parametrize("scheme", ["newton", "explicit16"])
def test_step_gas_floor_on_host(spec64, storage64, cells0_small, scheme):
    """Per-cell gas-temperature floor: cells whose input T_e + T_i lies below it
    take the step with radiative cooling off (status bit 32)."""
    from oracle import upstream as U
    resid, coeffs, stored = storage64
    ts = S.TableSet(spec64, stored)
    arr = [cells0_small[f] for f in W.FIELDS]
    floor = np.median(arr[1] + arr[2]) * np.ones_like(arr[0])
    dt = 1e3 * DT
    ref = U.step_with_gas_floor(ts, *arr, dt, floor, scheme="be" if scheme == "newton" else "ex16")
    cells = dict(cells0_small)
    cells["T_floor_gas"] = floor
    got = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells, dt, R.default_opts(scheme=scheme))
    assert np.array_equal(got["status"], ref["status"])
    off = (got["status"] & 32) != 0
    assert 0.3 < off.mean() < 0.7
    assert np.all(got["Q_rad"][off] == 0.0)
    tol = 1e-9 if scheme == "newton" else 1e-11
    for k in ("T_e_new", "T_i_new"):
        assert np.max(rel_err(got[k], ref[k])) < tol, k


def _prims(n, seed):
    rng = np.random.default_rng(seed)
    rho = 10 ** rng.uniform(-14, -2, n)
    theta = 10 ** rng.uniform(-6, 0.5, n)             # P / (rho c^2), up to relativistic
    P = theta * rho * 2.99792458e10 ** 2
    u = P / (5.0 / 3.0 - 1.0)
    r = 10 ** rng.uniform(0.2, 3, n)
    return rho, P, u, r


def test_disk_inputs_on_host():
    from oracle import upstream as U
    rho, P, u, r = _prims(4000, 5)
    prm = R.disk_params()
    H, Tf = R.selftest_disk_host(rho, P, u, r, prm)
    assert np.max(rel_err(H, U.scale_height(rho, P, u, r, prm.spin, prm.gamma, prm.r_g))) < 1e-14
    assert np.max(rel_err(Tf, U.floor_temperature(r, prm.spin, prm.h_floor))) < 1e-14
    bad = [np.array([v]) for v in (-1.0, 1.0, 1.0, 1.0)]
    assert np.isnan(R.selftest_disk_host(*bad, prm)[0][0])
    with pytest.raises(R.RadcoolError):
        R.selftest_disk_host(rho, P, u, r, R.disk_params(gamma=1.0))


def test_rad_pressure_correction_on_host():
    from oracle import upstream as U
    rng = np.random.default_rng(6)
    n = 4000
    n_e = 10 ** rng.uniform(14, 24, n)
    T_e = 10 ** rng.uniform(5, 10, n)
    H = 10 ** rng.uniform(5, 9, n)
    T, thick = R.selftest_radp_host(n_e, T_e, H)
    ref, rthick = U.rad_pressure_temperature(n_e, T_e, T_e, H)
    assert np.array_equal(thick.astype(bool), rthick)
    assert np.max(rel_err(T, ref)) < 1e-14
    assert np.isnan(R.selftest_radp_host(np.array([0.0]), np.array([1e6]), np.array([1e6]))[0][0])


def test_node4d_values_match_oracle_on_paper_ranges():
    """log2 Q_total at 4-D nodes (closed forms combined in log space) against
    the oracle's linear-space evaluation, over the paper's ranges."""
    from oracle import table4d as T4
    ax = T4.paper_axes(12)
    tab = T4.build(ax)
    g = np.meshgrid(*[10.0 ** a.nodes() for a in ax], indexing="ij")
    got = R.selftest_node4d_host(*[x.ravel() for x in g]).reshape(tab.shape)
    assert np.max(np.abs(got - tab)) < 1e-9


def test_rates4d_on_host_match_oracle_interpolation():
    from oracle import table4d as T4
    ax = T4.paper_axes(10)
    tab = T4.build(ax).astype(np.float32)
    axes = R.Axes4()
    for d, a in enumerate(ax):
        axes.n[d], axes.lo[d], axes.hi[d] = a.n, a.lo, a.hi
    cells = W.workload(0, n=3000)
    q, st = R.selftest_rates4d_host(axes, tab, cells)
    ref = T4.q_total(tab.astype(np.float64), ax, cells["n_e"], cells["T_e"], cells["B"], cells["H"])
    ref = np.where(cells["T_e"] < 1e6, 0.0, ref)
    assert np.max(rel_err(q, ref)) < 1e-12
    assert np.all(st == 0)


def test_converged_step_may_not_cross_a_table_node():
    """A cell of the 256^3 iid workload (index 10735542) whose last Newton step,
    below sqrt(tol), crossed a T_e node of the 128^3 tables: accepted without an
    evaluation on the far side it left an error first order in the slope jump
    (T_e' off by ~3e-9).  The step is now evaluated there first."""
    spec = T.TableSpec.default(128)
    co, re, st = T.quantize_tables(T.build_tables(spec))
    resid = np.concatenate([re[k].ravel() for k in T.TABLE_NAMES])
    coeffs = np.stack([co[k] for k in T.TABLE_NAMES])
    cell = dict(zip(W.FIELDS, ([3.02408923389808e+19], [308704708752.5737], [1901842603164.162],
                               [60328704.91455346], [272773157.94663656])))
    cell = {k: np.array(v) for k, v in cell.items()}
    got = R.selftest_step_host(R.default_spec(128), resid, coeffs, cell, DT)
    ref = S.step_be(S.TableSet(spec, st), *[cell[k] for k in W.FIELDS], DT)
    for k in ("T_e_new", "T_i_new"):
        assert rel_err(got[k], ref[k])[0] < 1e-12, k


def _coupling_case(n, seed):
    rng = np.random.default_rng(seed)
    ne = 10 ** rng.uniform(10, 20, n)
    te = 10 ** rng.uniform(7, 11, n)
    ti = te * 10 ** rng.uniform(0, 2, n)
    ten = te * (1 - rng.uniform(-0.5, 0.5, n))
    tin = ti * (1 - rng.uniform(-0.01, 0.01, n))
    v = rng.uniform(-0.5, 0.5, (n, 3))
    g = 1.0 / np.sqrt(1.0 - (v ** 2).sum(1))
    u = [-g] + [g * v[:, k] for k in range(3)]
    U0 = [rng.normal(size=n) * 1e3 for _ in range(4)]
    sg = rng.uniform(0.5, 2.0, n)
    return ne, te, ti, ten, tin, u, U0, sg


def test_apply_cooling_on_host():
    """The coupling's per-cell code against the oracle: lambda exactly, U to
    rounding; an invalid step (NaN temperature) keeps U; a NULL U component is
    skipped; sqrt(-g) defaults to 1."""
    from oracle import upstream as U
    ne, te, ti, ten, tin, u, U0, sg = _coupling_case(257, 3)
    ten[7] = np.nan
    dt = 4.9e-8
    for sgv in (sg, None):
        Un, lam = R.selftest_coupling_host(ne, te, ti, ten, tin, u, U0, dt, sgv)
        ref_l = U.cooling_lambda(ne, te, ti, ten, tin, dt)
        ref_U = U.apply_cooling(U0, u, ref_l, dt, sqrt_g=sgv)
        ok = np.isfinite(ref_l)
        assert not ok[7] and np.isnan(lam[7])
        assert np.max(rel_err(lam[ok], ref_l[ok])) < 1e-15
        for mu in range(4):
            assert np.max(rel_err(Un[mu], ref_U[mu])) < 1e-13
            assert Un[mu][7] == U0[mu][7]
    Un, _ = R.selftest_coupling_host(ne, te, ti, ten, tin, u, [U0[0], None, U0[2], None], dt)
    assert Un[1] is None and Un[3] is None


@pytest.mark.parametrize("floor,dt_scale", [(1e6, 1.0), (3e6, 1e3), (5e7, 1e2)])
def test_step_two_pass_identical_on_host(spec64, storage64, cells0_small, floor, dt_scale):
    """The two-pass Newton step (first round, resume record, resumed solve)
    gives bit-identical outputs to the single pass, including cells whose
    first round ends in a floor probe (stiff cells around the floor)."""
    resid, coeffs, _ = storage64
    rng = np.random.default_rng(int(floor))
    n = 400
    n_e = 10 ** rng.uniform(14, 20, n)
    T_e = floor * 10 ** rng.uniform(-0.6, 0.8, n)
    T_i = T_e * 10 ** rng.uniform(-1.0, 1.5, n)
    B = np.sqrt(8 * np.pi * n_e * 1.380649e-16 * (T_e + T_i) / 10 ** rng.uniform(-1, 2, n))
    H = 10 ** rng.uniform(5, 9, n)
    near = {"n_e": n_e, "T_e": T_e, "T_i": T_i, "B": B, "H": H}
    cells = {f: np.concatenate([cells0_small[f], near[f]]) for f in W.FIELDS}
    cells["T_e"][5] = np.nan                     # an invalid cell
    dt = DT * dt_scale
    one = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells, dt, R.default_opts(T_floor=floor, passes=1))
    two = R.selftest_step_host(R.default_spec(64), resid, coeffs, cells, dt, R.default_opts(T_floor=floor, passes=2))
    for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc", "status"):
        assert np.array_equal(one[k], two[k], equal_nan=(k != "status")), k
    if dt_scale > 1.0:
        assert (one["status"] & S.ST_FLOOR).sum() > 0
