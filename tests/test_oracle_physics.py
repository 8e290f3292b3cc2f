"""Pins of the oracle's closed-form rates (paper Section II) against values the
mathematics fixes: hand-derived numbers, limits, exact identities, independent
quadrature and brute-force sums.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from conftest import golden, rel_err
from oracle import constants as K
from oracle import physics as P


def test_fit_constants_transcription():
    g = golden("paper_fit_constants.json")
    assert K.BREM_EE_NORM == g["brem_ee_norm"]["value"]
    assert list(K.BREM_EE_LOW) == g["brem_ee_low"]["value"]
    assert list(K.BREM_EE_HIGH) == g["brem_ee_high"]["value"]
    assert K.BREM_EI_NORM == g["brem_ei_norm"]["value"]
    assert list(K.BREM_EI_LOW) == g["brem_ei_low"]["value"]
    assert list(K.BREM_EI_HIGH) == g["brem_ei_high"]["value"]
    assert K.SYN_EPS_NORM == g["syn_eps_norm"]["value"]
    assert K.IPRIME_NORM == g["iprime_norm"]["value"]
    assert K.IPRIME_C1 == g["iprime_c1"]["value"]
    assert K.IPRIME_C2 == g["iprime_c2"]["value"]
    assert K.IPRIME_A == g["iprime_a"]["value"]
    assert K.SYN_LOWT_SWITCH == g["syn_lowt_switch"]["value"]
    assert K.LN_LAMBDA == g["ln_lambda"]["value"]
    assert K.EXPLICIT_CAP == g["explicit_cap"]["value"]
    assert K.GAMMA_AD == pytest.approx(g["gamma_ad"]["value"], rel=1e-15)


# --------------------------------------------------------------------------- brem


def test_brem_branch_values_at_theta_one():
    g = golden("closed_form_values.json")
    below = np.nextafter(1.0, 0.0)
    assert P.brem_ee_shape(below) == pytest.approx(g["brem_ee_shape_theta1_low"]["value"], rel=1e-14)
    assert P.brem_ee_shape(1.0) == pytest.approx(g["brem_ee_shape_theta1_high"]["value"], rel=1e-14)
    assert P.brem_ei_shape(below) == pytest.approx(g["brem_ei_shape_theta1_low"]["value"], rel=1e-14)
    assert P.brem_ei_shape(1.0) == pytest.approx(g["brem_ei_shape_theta1_high"]["value"], rel=1e-14)
    T1 = g["T_theta_e_one_K"]["value"]
    assert P.theta_e(T1) == pytest.approx(1.0, rel=1e-15)


def test_brem_density_scaling_exact():
    T = np.array([1e6, 3e8, 1e10, 1e12])
    for n in (1e3, 1e15, 1e24):
        assert np.all(rel_err(P.q_brem(n, T), n * n * P.q_brem(1.0, T)) < 1e-15)


def test_brem_nonrelativistic_limit():
    """Q_brem -> c n^2 T^1/2 with c fixed by the printed Q_ei; slope -> 1/2."""
    g = golden("closed_form_values.json")["brem_nr_coefficient"]["value"]
    T = np.array([10.0, 100.0, 1000.0])
    ratio = P.q_brem(1.0, T) / np.sqrt(T) / g
    th = P.theta_e(T)
    # corrections are O(theta^1.34) from Q_ei and O(theta) from Q_ee / Q_ei
    assert np.all(np.abs(ratio - 1.0) < 5.0 * th)
    lnT = np.log(T)
    lnQ = np.log(P.q_brem(1.0, T))
    h = 1e-4
    slope = (np.log(P.q_brem(1.0, T * math.exp(h))) - np.log(P.q_brem(1.0, T * math.exp(-h)))) / (2 * h)
    assert np.all(np.abs(slope - 0.5) < 5.0 * th)
    del lnT, lnQ


# --------------------------------------------------------------------------- synchrotron

SYN_CASES = [  # n_e, T, B, H: cold/thin, mid, hot, strongly self-absorbed
    (1e12, 1e7, 1e3, 1e8),
    (1e14, 5e9, 1e5, 1e7),
    (1e10, 2e11, 10.0, 1e9),
    (1e20, 3e8, 1e9, 1e6),
    (1e25, 1e6, 1.0, 1e3),
]


@pytest.mark.parametrize("n_e,T,B,H", SYN_CASES)
def test_self_absorption_balance(n_e, T, B, H):
    """eq. bb_sync_aprox: H eps_s(nu_c) = 2 pi nu_c^2 k T / c^2 at the solved nu_c."""
    s = P.synchrotron(n_e, T, B, H)
    lhs = H * P.emissivity(s["nu_c"], n_e, T, B)
    rhs = 2.0 * math.pi * s["nu_c"] ** 2 * K.K_B * T / K.C_LIGHT ** 2
    assert rel_err(lhs, rhs) < 1e-12


@pytest.mark.parametrize("n_e,T,B,H", SYN_CASES)
def test_thick_limit_identity(n_e, T, B, H):
    """Exact consequence of the balance: Q_syn / Q_RJ - 1 = 3 J(x_c) / (x_c^2 I'(x_c))."""
    s = P.synchrotron(n_e, T, B, H)
    x = s["x_c"]
    lhs = s["q_syn"] / s["q_rj"] - 1.0
    rhs = 3.0 * P.tail_integral(x) / (x ** 2 * P.iprime(x))
    assert rel_err(lhs, rhs) < 1e-11


def test_rayleigh_jeans_limit():
    """Optically thick synchrotron tends to the Rayleigh-Jeans surface emission:
    Q_syn / Q_RJ - 1 ~ 9 / (1.8899 x_c^(1/3)) -> 0 as x_c grows."""
    xs = []
    excess = []
    for n_e in (1e16, 1e19, 1e22, 1e25):
        s = P.synchrotron(n_e, 1e7, 1.0, 1e8)
        xs.append(float(s["x_c"]))
        excess.append(float(s["q_syn"] / s["q_rj"] - 1.0))
    xs = np.array(xs)
    excess = np.array(excess)
    assert np.all(np.diff(xs) > 0) and np.all(np.diff(excess) < 0)
    asym = 9.0 / (K.IPRIME_A * np.cbrt(xs))
    # next order of the asymptotic series is O(x^-1/3) relative
    assert np.all(np.abs(excess / asym - 1.0) < 6.0 / np.cbrt(xs))


def test_tail_closed_form_matches_quadrature():
    for x in (1e-6, 1e-2, 0.7, 5.0, 80.0, 3e3, 1e5):
        q, _ = integrate.quad(lambda t: 3 * t ** 2 * (t ** 3) * P.iprime(t ** 3), np.cbrt(x), np.inf,
                              epsabs=0, epsrel=1e-13, limit=400)
        assert rel_err(P.tail_integral(x), q) < 1e-10


def test_tail_total_integral():
    q, _ = integrate.quad(lambda t: 3 * t ** 5 * P.iprime(t ** 3), 0, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    assert rel_err(P.tail_integral(1e-300), q) < 1e-10
    assert q == pytest.approx(26.14867923210402, rel=1e-9)


@pytest.mark.parametrize("n_e,T,B,H", SYN_CASES[:4])
def test_synchrotron_against_direct_frequency_quadrature(n_e, T, B, H):
    """eq. synchrotron integrated numerically over nu (independent of the Gamma form)."""
    s = P.synchrotron(n_e, T, B, H)
    nu_c = float(s["nu_c"])
    rj, _ = integrate.quad(lambda v: 2 * math.pi * v * v * K.K_B * T / K.C_LIGHT ** 2, 0.0, nu_c, epsrel=1e-13)
    # tail in ln nu
    tail, _ = integrate.quad(lambda l: float(P.emissivity(math.exp(l), n_e, T, B)) * math.exp(l),
                             math.log(nu_c), math.log(nu_c) + 60.0, epsabs=0, epsrel=1e-12, limit=500)
    assert rel_err(rj / H, s["q_rj"]) < 1e-12
    assert rel_err(tail, s["q_tail"]) < 1e-9


def test_balance_coefficient_against_literature():
    g = golden("closed_form_values.json")
    c = K.IPRIME_NORM * 8 * math.pi * K.C_LIGHT * K.SYN_EPS_NORM / (3 * K.E_CHARGE)
    assert c == pytest.approx(g["balance_coefficient"]["value"], rel=1e-12)
    assert c == pytest.approx(g["balance_coefficient_literature"]["value"],
                              rel=g["balance_coefficient_rel_tol"]["value"])
    # and the oracle's balance equation uses exactly that coefficient
    n_e, T, B, H = 1e14, 5e9, 1e5, 1e7
    x = float(P.synchrotron(n_e, T, B, H)["x_c"])
    th = float(P.theta_e(T))
    k2 = math.exp(float(P.ln_k2_synchrotron(T)))
    lhs = math.exp(K.IPRIME_A * x ** (1 / 3))
    rhs = c * (n_e * H / B) * (x ** (-7 / 6) + 0.4 * x ** (-17 / 12) + 0.5316 * x ** (-5 / 3)) / (th ** 3 * k2)
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_low_temperature_bessel_substitution():
    T = np.array([0.99e8, 1e8, 1.01e8])
    th = P.theta_e(T)
    k2 = np.exp(P.ln_k2_synchrotron(T))
    assert k2[0] == pytest.approx(2 * th[0] ** 2, rel=1e-14)
    assert k2[1] == pytest.approx(2 * th[1] ** 2, rel=1e-14)          # inclusive switch
    assert k2[2] == pytest.approx(special.kv(2, 1 / th[2]), rel=1e-12)  # true Bessel above


# --------------------------------------------------------------------------- Compton


def test_compton_limits():
    T = 2e9
    th = float(P.theta_e(T))
    # tau -> 0: eta -> 1 (P -> 0)
    for n_e in (1e-6, 1e-3):
        eta = P.compton_eta(n_e, T, 1.0, 1e10)
        assert 0.0 <= eta - 1.0 < 1e-20
    # E -> 3 theta from below: k -> 0, eta -> 1; E >= 3 theta: eta = 1 exactly
    nu_edge = 3 * th * K.ME_C2 / K.H_PLANCK
    for f in (1 - 1e-9, 1 - 1e-6):
        assert P.compton_eta(1e22, T, 1.0, nu_edge * f) - 1.0 < 1e-3
    assert P.compton_eta(1e22, T, 1.0, nu_edge * 1.01) == 1.0


def test_compton_geometric_series_bruteforce():
    """For an integer number k of scatterings the enhancement is the explicit sum
    1 + P (A - 1) sum_{j<k} (P A)^j (each scattering multiplies energy by A, with
    probability P)."""
    for n_e, T in ((1e24, 3e9), (1e21, 1e10), (1e23, 5e8)):
        th = float(P.theta_e(T))
        A = 1 + 4 * th + 16 * th ** 2
        Pr = -math.expm1(-2 * n_e * K.SIGMA_T * 1.0)
        for k in (1, 3, 7):
            E = 3 * th / A ** k                     # A^k = 3 theta / E
            nu = E * K.ME_C2 / K.H_PLANCK
            brute = 1 + Pr * (A - 1) * sum((Pr * A) ** j for j in range(k))
            assert P.compton_eta(n_e, T, 1.0, nu) == pytest.approx(brute, rel=1e-12)


def test_compton_removable_limit_and_bound():
    T = 5e9
    th = float(P.theta_e(T))
    A = 1 + 4 * th + 16 * th ** 2
    # choose tau so that P A == 1 up to rounding, then bracket it
    Pr = 1 / A
    tau = -math.log1p(-Pr)
    n_e = tau / (2 * K.SIGMA_T)
    nu = 1e-4 * 3 * th * K.ME_C2 / K.H_PLANCK
    k = math.log(1e4) / math.log(A)
    limit = 1 + Pr * (A - 1) * k
    for f in (1 - 1e-7, 1.0, 1 + 1e-7):
        assert P.compton_eta(n_e * f, T, 1.0, nu) == pytest.approx(limit, rel=1e-5)
    rng = np.random.default_rng(0)
    n = 10 ** rng.uniform(10, 28, 2000)
    TT = 10 ** rng.uniform(6, 12, 2000)
    nn = 10 ** rng.uniform(0, 25, 2000)
    assert np.all(P.compton_eta(n, TT, 1.0, nn) >= 1.0)


def test_printed_exponent_goes_negative():
    """The exponent exactly as printed gives eta < 0 once P A > 1; this is why the
    geometric-series form is the reading used."""
    T = 5.93e9          # theta ~ 1
    eta_lit = P.compton_eta_printed(0.5 / (2 * K.SIGMA_T), T, 1.0, 1e10)
    eta_der = P.compton_eta(0.5 / (2 * K.SIGMA_T), T, 1.0, 1e10)
    assert eta_lit < 0.0 < eta_der


# --------------------------------------------------------------------------- bridge


def test_bridge_forms_agree():
    rng = np.random.default_rng(1)
    q = 10 ** rng.uniform(-10, 30, 1000)
    T = 10 ** rng.uniform(6, 12, 1000)
    H = 10 ** rng.uniform(3, 12, 1000)
    ts = 10 ** rng.uniform(-9, 6, 1000)
    assert np.all(rel_err(P.hubeny_total(q, T, H, ts), P.hubeny_total_rewritten(q, T, H, ts)) < 1e-12)


def test_bridge_limits():
    T, H = 1e7, 1e8
    # optically thin: Q_total -> Q_thin
    q = 1e-6
    assert P.hubeny_total_rewritten(q, T, H, 1e-12) == pytest.approx(q, rel=1e-9)
    # optically thick: Q_total -> 4 sigma T^4 / H / (3 tau / 2) = 8 sigma T^4 / (3 H tau)
    for q_thick, ts in ((1e30, 1e-3), (1e20, 1e7)):
        ta = P.tau_absorption(q_thick, T, H)
        tau = ta + ts
        bb = 8 * K.SIGMA_SB * T ** 4 / (3 * H * tau)
        assert P.hubeny_total_rewritten(q_thick, T, H, ts) == pytest.approx(bb, rel=2 / tau)


# --------------------------------------------------------------------------- Coulomb


def test_coulomb_zero_at_equal_temperatures_and_sign():
    T = np.array([1e6, 1e9, 1e11, 1e13])
    assert np.all(P.q_coulomb(1e15, T, T) == 0.0)
    assert np.all(P.q_coulomb(1e15, T, 2 * T) > 0.0)
    assert np.all(P.q_coulomb(1e15, 2 * T, T) < 0.0)


def test_coulomb_nonrelativistic_limit():
    g = golden("closed_form_values.json")["coulomb_nr_limit"]["value"]
    for Te, Ti in ((1e5, 1e7), (1e6, 1e8), (1e4, 1e6)):
        te = float(P.theta_e(Te))
        ti = float(P.theta_i(Ti))
        R = float(P.coulomb_ratio(Te, Ti))
        assert R * (te + ti) ** 1.5 == pytest.approx(g, rel=5 * max(te, ti))


def test_coulomb_scaled_bessels_match_unscaled_formula():
    """Where the unscaled Bessels do not underflow, eq. coulomb_collisions evaluated
    literally with K_n equals the scaled form."""
    for Te, Ti in ((1e10, 1e12), (3e9, 5e11), (2e11, 2e13)):
        te = float(P.theta_e(Te))
        ti = float(P.theta_i(Ti))
        tm = 1 / (1 / te + 1 / ti)
        lit = ((2 * (te + ti) ** 2 + 1) / (te + ti) * special.kv(1, 1 / tm) + 2 * special.kv(0, 1 / tm)) \
            / (special.kv(2, 1 / ti) * special.kv(2, 1 / te))
        assert float(P.coulomb_ratio(Te, Ti)) == pytest.approx(lit, rel=1e-12)


def test_scaled_bessel_against_quadrature():
    """kve(nu, z) = int_0^inf exp(-z (cosh t - 1)) cosh(nu t) dt, the integral the
    library's own Bessel routine is built on."""
    for nu in (0, 1, 2):
        for z in (0.005, 0.3, 7.0, 300.0, 1e5):
            t_max = math.acosh(1.0 + 800.0 / z)      # integrand below e^-800 beyond
            q, _ = integrate.quad(lambda t: math.exp(-z * (math.cosh(t) - 1)) * math.cosh(nu * t),
                                  0, t_max, epsabs=0, epsrel=1e-13, limit=400)
            assert special.kve(nu, z) == pytest.approx(q, rel=1e-10)


def test_coulomb_prefactor_density_scaling():
    assert float(P.coulomb_coeff(1e20, 1e9, 1e11) / P.coulomb_coeff(1e10, 1e9, 1e11)) == pytest.approx(1e20, rel=1e-14)
