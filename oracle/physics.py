"""Closed-form cooling rates in plain FP64 (paper Section II).

Every function takes NumPy arrays (broadcasting) in cgs units and returns
rates in erg cm^-3 s^-1 unless stated otherwise.  Special functions come from
SciPy (``kve``, ``gammaincc``, ``gamma``); roots are found by bisection so that
nothing depends on a solver's convergence heuristics.

Readings of the paper taken here (each is listed in the design notes):
  * the sigma in the optically-thick bridge is the Stefan-Boltzmann constant
    (dimensional analysis of eq. total_cooling);
  * the Compton exponent is -1 - ln P / ln A (the geometric-series form of the
    Dermer et al. enhancement built from the printed P and A); the printed
    exponent 1 - ln P / ln A is kept as ``compton_eta_printed`` for the record;
  * E_init = h nu_c / (m_e c^2); eta = 1 when E_init >= 3 theta_e;
  * the low-temperature substitution K2 -> 2 theta^2 applies to synchrotron
    only, for T_e <= 1e8 K inclusive;
  * theta_i uses the proton mass; ln Lambda = 20; rho / m_p = n_i = n_e;
  * the brem branch at exactly theta_e = 1 is the theta >= 1 branch.

Parity pins (tests/test_oracle_physics.py): NR brem limit and n^2 scaling,
branch values at theta = 1 computed by hand, the self-absorption balance, the
exact thick-limit identity Q_syn / Q_RJ - 1 = 3 J / (x^2 I'), the tail against
direct quadrature of the emissivity, Compton limits, bridge limits, Coulomb NR
limit and zero at T_e = T_i, scaled Bessels against quadrature.
Unpinned: the physical accuracy of the printed fit coefficients.
"""
import numpy as np
from scipy import special

from . import constants as K

# ---------------------------------------------------------------------------
# dimensionless temperatures


def theta_e(T):
    """k T / m_e c^2 (Section II.A, below the bremsstrahlung equations)."""
    return K.K_B * np.asarray(T, dtype=np.float64) / K.ME_C2


def theta_i(T, ion_mass=K.M_P):
    """k T_i / m_i c^2 with m_i = m_p (reading of Section II.G)."""
    return K.K_B * np.asarray(T, dtype=np.float64) / (ion_mass * K.C_LIGHT ** 2)


# ---------------------------------------------------------------------------
# Section II.A: bremsstrahlung


def brem_ee_shape(th):
    """Bracketed factor of Q_ee (Section II.A, first case split)."""
    th = np.asarray(th, dtype=np.float64)
    a, b, c = K.BREM_EE_LOW
    low = th ** 1.5 * (1.0 + a * th + b * th ** 2 - c * th ** 2.5)
    s, g, d = K.BREM_EE_HIGH
    high = s * th * (np.log(g * th) + d)
    return np.where(th < 1.0, low, high)


def brem_ei_shape(th):
    """Bracketed factor of Q_ei (Section II.A, second case split)."""
    th = np.asarray(th, dtype=np.float64)
    a, p = K.BREM_EI_LOW
    low = 4.0 * np.sqrt(2.0 * th / np.pi ** 3) * (1.0 + a * th ** p)
    g, d, e = K.BREM_EI_HIGH
    high = 9.0 * th / (2.0 * np.pi) * (np.log(g * th + d) + e)
    return np.where(th < 1.0, low, high)


def brem_coeff(T):
    """Q_brem / n_e^2 = 2.56e-22 f_ee(theta) + 1.48e-22 f_ei(theta)."""
    th = theta_e(T)
    return K.BREM_EE_NORM * brem_ee_shape(th) + K.BREM_EI_NORM * brem_ei_shape(th)


def q_brem(n_e, T):
    """Q_brem = Q_ee + Q_ei, both proportional to n_e^2 (Section II.A)."""
    return np.asarray(n_e, dtype=np.float64) ** 2 * brem_coeff(T)


# ---------------------------------------------------------------------------
# Section II.B: synchrotron with self-absorption


def ln_iprime(x):
    """ln I'(x) for the Mahadevan fit, eq. fitting_I(xm)."""
    x = np.asarray(x, dtype=np.float64)
    return (np.log(K.IPRIME_NORM) - np.log(x) / 6.0
            + np.log1p(K.IPRIME_C1 * x ** -0.25 + K.IPRIME_C2 * x ** -0.5)
            - K.IPRIME_A * np.cbrt(x))


def iprime(x):
    return np.exp(ln_iprime(x))


def ln_k2_synchrotron(T):
    """ln K2(1/theta_e) as used in the synchrotron emissivity.

    For T_e <= 1e8 K the paper replaces K2(1/theta_e) by 2 theta_e^2
    (end of Section II.B); above it the true Bessel function is used,
    formed in log space from the exponentially scaled K2.
    """
    T = np.asarray(T, dtype=np.float64)
    th = theta_e(T)
    z = 1.0 / th
    true_ln = np.log(special.kve(2, z)) - z
    return np.where(T <= K.SYN_LOWT_SWITCH, np.log(2.0 * th ** 2), true_ln)


def nu0(T, B):
    """Frequency scale with x_M = nu / nu0: nu0 = 3 e B theta^2 / (4 pi m_e c)."""
    th = theta_e(T)
    return 3.0 * K.E_CHARGE * np.asarray(B, dtype=np.float64) * th ** 2 / (4.0 * np.pi * K.M_E * K.C_LIGHT)


def emissivity(nu, n_e, T, B):
    """eps_s(nu), eq. optically_thin_synch, erg cm^-3 s^-1 Hz^-1."""
    x = np.asarray(nu, dtype=np.float64) / nu0(T, B)
    return (K.SYN_EPS_NORM * 4.0 * np.pi * nu * n_e
            * np.exp(ln_iprime(x) - ln_k2_synchrotron(T)))


def ln_balance_rhs(n_e, T, B, H):
    """Right side of ln[I'(x_c)/x_c] = ln rhs, the self-absorption balance.

    Eq. bb_sync_aprox reads H eps_s(nu_c) = 2 pi nu_c^2 k T / c^2.  With
    nu_c = x_c nu0 and k T nu0 / c^2 = 3 e B theta^3 / (4 pi c) this becomes
    I'(x_c)/x_c = 3 e B theta^3 K2 / (8 pi c 4.43e-30 n_e H).
    """
    th = theta_e(T)
    return (np.log(3.0 * K.E_CHARGE * np.asarray(B, dtype=np.float64) * th ** 3
                   / (8.0 * np.pi * K.C_LIGHT * K.SYN_EPS_NORM))
            + ln_k2_synchrotron(T) - np.log(np.asarray(n_e, dtype=np.float64) * H))


def solve_xc(ln_rhs, lo=-80.0, hi=80.0):
    """x_c from ln I'(x)/x = ln_rhs by bisection in ln x.

    ln I'(x) - ln x is strictly decreasing in ln x (each term of
    d/dlnx ln I' is <= 0), so the root is unique.
    """
    ln_rhs = np.asarray(ln_rhs, dtype=np.float64)
    a = np.full(ln_rhs.shape, lo)
    b = np.full(ln_rhs.shape, hi)

    def phi(s):
        x = np.exp(s)
        return ln_iprime(x) - s - ln_rhs

    if np.any(phi(a) <= 0.0) or np.any(phi(b) >= 0.0):
        raise ValueError("x_c outside the bisection bracket")
    for _ in range(200):
        m = 0.5 * (a + b)
        if np.all((m == a) | (m == b)):
            break
        pos = phi(m) > 0.0
        a = np.where(pos, m, a)
        b = np.where(pos, b, m)
    return np.exp(0.5 * (a + b))


# (p, c) pairs of the tail integral J(x) = int_x^inf s I'(s) ds after s = t^3:
# s I'(s) ds = 3 * 4.0505 (t^4.5 + 0.4 t^3.75 + 0.5316 t^3) e^{-a t} dt.
_TAIL_TERMS = ((5.5, 1.0), (4.75, K.IPRIME_C1), (4.0, K.IPRIME_C2))


def tail_integral(x):
    """J(x) = int_x^inf s I'(s) ds in closed form via the upper incomplete Gamma.

    With s = t^3 each term becomes a^-p Gamma(p) Q(p, a x^(1/3)).
    """
    x = np.asarray(x, dtype=np.float64)
    z = K.IPRIME_A * np.cbrt(x)
    tot = np.zeros_like(x)
    for p, c in _TAIL_TERMS:
        tot = tot + c * K.IPRIME_A ** (-p) * special.gamma(p) * special.gammaincc(p, z)
    return 3.0 * K.IPRIME_NORM * tot


def synchrotron(n_e, T, B, H):
    """Self-absorbed synchrotron cooling, eq. synchrotron.

    Returns a dict with x_c, nu0, nu_c, the Rayleigh-Jeans part q_rj (the
    self-absorbed band radiated from the surface, divided by the volume:
    (1/H) int_0^nu_c 2 pi nu^2 k T / c^2 dnu), the optically thin tail q_tail
    (int_nu_c^inf eps_s dnu = 4.43e-30 4 pi n_e nu0^2 J(x_c) / K2) and their
    sum q_syn.
    """
    n_e, T, B, H = (np.asarray(v, dtype=np.float64) for v in (n_e, T, B, H))
    x_c = solve_xc(ln_balance_rhs(n_e, T, B, H))
    v0 = nu0(T, B)
    nu_c = v0 * x_c
    q_rj = 2.0 * np.pi * K.K_B * T * nu_c ** 3 / (3.0 * K.C_LIGHT ** 2 * H)
    q_tail = (K.SYN_EPS_NORM * 4.0 * np.pi * n_e * v0 ** 2 * tail_integral(x_c)
              * np.exp(-ln_k2_synchrotron(T)))
    return {"x_c": x_c, "nu0": v0, "nu_c": nu_c, "q_rj": q_rj,
            "q_tail": q_tail, "q_syn": q_rj + q_tail}


# ---------------------------------------------------------------------------
# Section II.C: inverse Compton enhancement at nu_c


def tau_scattering(n_e, H):
    """tau_sca = 2 n_e sigma_T H (Section II.C)."""
    return 2.0 * np.asarray(n_e, dtype=np.float64) * K.SIGMA_T * H


def compton_eta(n_e, T, H, nu_c):
    """eta_comp(nu_c) with exponent -1 - ln P / ln A.

    P = 1 - exp(-tau_sca), A = 1 + 4 theta + 16 theta^2, E = h nu_c / m_e c^2.
    For E < 3 theta write k = ln(3 theta / E) / ln A (so A^k = 3 theta / E);
    then (E / 3 theta)^(-1 - ln P/ln A) = (P A)^k and
    eta = 1 + P (A - 1) [1 - (PA)^k] / (1 - PA)
        = 1 + P (A - 1) expm1(k L) / expm1(L),  L = ln(P A),
    with the removable limit k at L = 0.  eta = 1 for E >= 3 theta.
    """
    th = theta_e(T)
    P = -np.expm1(-tau_scattering(n_e, H))
    A = 1.0 + 4.0 * th + 16.0 * th ** 2
    E = K.H_PLANCK * np.asarray(nu_c, dtype=np.float64) / K.ME_C2
    soft = E < 3.0 * th
    E_s = np.where(soft, E, 3.0 * th * 0.5)          # placeholder outside soft
    k = np.log(3.0 * th / E_s) / np.log(A)
    L = np.log(P) + np.log(A)
    L_nz = np.where(L == 0.0, 1.0, L)
    ratio = np.where(L == 0.0, k, np.expm1(k * L_nz) / np.expm1(L_nz))
    eta = 1.0 + P * (A - 1.0) * ratio
    return np.where(soft, eta, 1.0)


def compton_eta_printed(n_e, T, H, nu_c):
    """The enhancement with the exponent exactly as printed, 1 - ln P / ln A.

    Kept only to document why that reading is not used: it is negative
    whenever P A > 1.
    """
    th = theta_e(T)
    P = -np.expm1(-tau_scattering(n_e, H))
    A = 1.0 + 4.0 * th + 16.0 * th ** 2
    E = K.H_PLANCK * np.asarray(nu_c, dtype=np.float64) / K.ME_C2
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        expo = 1.0 - np.log(P) / np.log(A)
        eta = 1.0 + P * (A - 1.0) / (1.0 - P * A) * (1.0 - (E / (3.0 * th)) ** expo)
    return np.where(E < 3.0 * th, eta, 1.0)


# ---------------------------------------------------------------------------
# Sections II.C-II.D: thin total and the optically-thick bridge


def q_thin(q_brem_v, eta, q_syn):
    """eq. thin_cooling: Q_thin = Q_brem + eta(nu_c) Q_syn."""
    return q_brem_v + eta * q_syn


def tau_absorption(q_thin_v, T, H):
    """tau_abs = H Q_thin / (4 sigma T^4) with sigma = Stefan-Boltzmann."""
    return H * q_thin_v / (4.0 * K.SIGMA_SB * np.asarray(T, dtype=np.float64) ** 4)


def hubeny_total(q_thin_v, T, H, tau_sca):
    """eq. total_cooling, as printed: (4 sigma T^4 / H) / (3 tau/2 + sqrt3 + 1/tau_abs)."""
    T = np.asarray(T, dtype=np.float64)
    ta = tau_absorption(q_thin_v, T, H)
    tau = ta + tau_sca
    return (4.0 * K.SIGMA_SB * T ** 4 / H) / (1.5 * tau + K.SQRT3 + 1.0 / ta)


def hubeny_total_rewritten(q_thin_v, T, H, tau_sca):
    """Same value, multiplied through by tau_abs: Q_thin / (1 + sqrt3 ta + 1.5 ta (ta + ts)).

    Finite for tau_abs -> 0; this is the form used for table-driven rates.
    """
    ta = tau_absorption(q_thin_v, T, H)
    return q_thin_v / (1.0 + K.SQRT3 * ta + 1.5 * ta * (ta + tau_sca))


# ---------------------------------------------------------------------------
# Section II.G: Coulomb exchange


def coulomb_ratio(T_e, T_i, ion_mass=K.M_P):
    """R(theta_e, theta_i) of eq. coulomb_collisions with the e^-z factors cancelled,
    theta_i = k T_i / (ion_mass c^2).

    K2(1/th_i) K2(1/th_e) = kve2(1/th_i) kve2(1/th_e) e^{-1/th_m} and
    K_n(1/th_m) = kve_n(1/th_m) e^{-1/th_m} because 1/th_m = 1/th_e + 1/th_i,
    so the ratio is formed from scaled Bessel functions only.
    """
    te = theta_e(T_e)
    ti = theta_i(T_i, ion_mass)
    s = te + ti
    zm = 1.0 / te + 1.0 / ti
    num = (2.0 * s ** 2 + 1.0) / s * special.kve(1, zm) + 2.0 * special.kve(0, zm)
    den = special.kve(2, 1.0 / te) * special.kve(2, 1.0 / ti)
    return num / den


def coulomb_coeff(n_e, T_e, T_i, ln_lambda=K.LN_LAMBDA, ion_mass=K.M_P, theta_i_mass=None):
    """Q_cc / (T_i - T_e) > 0, eq. coulomb_collisions with rho/m_p = n_e, m_i = m_p.

    theta_i_mass is the mass in theta_i = k T_i / m c^2 (default: the ion
    mass; K.M_E gives the printed form).  The prefactor keeps m_e / m_i."""
    n_e = np.asarray(n_e, dtype=np.float64)
    pref = 1.5 * (K.M_E / ion_mass) * n_e * n_e * ln_lambda * K.C_LIGHT * K.K_B * K.SIGMA_T
    return pref * coulomb_ratio(T_e, T_i, ion_mass if theta_i_mass is None else theta_i_mass)


def q_coulomb(n_e, T_e, T_i, ln_lambda=K.LN_LAMBDA, ion_mass=K.M_P, theta_i_mass=None):
    """Q_cc, positive when ions heat electrons."""
    return (np.asarray(T_i, dtype=np.float64) - T_e) * coulomb_coeff(n_e, T_e, T_i, ln_lambda, ion_mass,
                                                                      theta_i_mass)


# ---------------------------------------------------------------------------
# direct (table-free) rates at one state


def direct_rates(n_e, T_e, T_i, B, H, compton="derived", theta_i_mass=K.M_P):
    """All rates at the state from the closed forms, no tables.

    Returns dict with q_brem, q_syn, eta, q_thin, q_rad (bridged) and q_cc.
    compton="literal" takes the printed exponent (compton_eta_printed);
    q_rad is NaN where that eta is not positive (no cooling value there).
    theta_i_mass is the mass in theta_i (K.M_E: the printed form).
    """
    n_e, T_e, T_i, B, H = (np.asarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, B, H))
    qb = q_brem(n_e, T_e)
    syn = synchrotron(n_e, T_e, B, H)
    if compton == "literal":
        eta = compton_eta_printed(n_e, T_e, H, syn["nu_c"])
    else:
        eta = compton_eta(n_e, T_e, H, syn["nu_c"])
    qt = q_thin(qb, eta, syn["q_syn"])
    ts = tau_scattering(n_e, H)
    with np.errstate(invalid="ignore"):
        q_rad = hubeny_total_rewritten(qt, T_e, H, ts)
    q_rad = np.where((eta > 0.0) & np.isfinite(eta), q_rad, np.nan)
    return {"q_brem": qb, "q_syn": syn["q_syn"], "eta": eta, "q_thin": qt,
            "q_rad": q_rad, "q_cc": q_coulomb(n_e, T_e, T_i, theta_i_mass=theta_i_mass)}
