"""Per-cell inputs upstream of the cooling step, and the post-processing
temperature correction (test infrastructure; only tests, the smoke check and
the benchmark's CPU baseline use this package).

Thermal scale height (Sec. II.F, eq. H_thermal): H_th = c_s / Omega_K with
c_s^2 = gamma P / (rho h), rho h = rho c^2 + rho eps + P the relativistic
enthalpy density, and the Keplerian frequency Omega_K = 1 / (r^(3/2) + a) in
gravitational units (r in r_g, a the dimensionless spin, Omega in c / r_g).
In cgs: H_th = (c_s / c) (r^(3/2) + a) r_g.

Temperature floor (Sec. III.B.2): T_floor = (pi/2) [h_floor Omega_K R]^2, a
gas temperature in units of c^2 (P / rho), converted to kelvin with
T_gas = T_e + T_i = (P / rho) m_p c^2 / k_B (n_i = n_e, rho = m_p n_e).  A cell
whose input gas temperature lies below it has zero radiative cooling for the
step (Coulomb exchange still acts).

Radiation-pressure correction (Sec. IV, thermal structure; eq. total_pressure):
in optically thick cells, tau_sca = n_e sigma_T H > tau_crit (4.6: fewer than 1 %
of photons escape unscattered), the pressure n_e k_B (T_e + T_i) is shared
between radiation and gas, a T^4 + n_e k_B (T + T_i) = n_e k_B (T_e + T_i), with
T_i held; the left side increases with T, so the root T in (0, T_e) is unique.

Downstream coupling (Sec. II.E, eqs. energy-momentum_eq and 4-force_calc): the
cooling enters the gas's energy-momentum equation as the 4-force density
G_mu = -lambda u_mu, lambda the radiated energy per unit volume and time; over
a step of length dt the conserved densities U_mu = sqrt(-g) T^t_mu change by
dt sqrt(-g) G_mu.  The lambda that matches a step's temperature update is the
energy it removed from the gas, 1.5 n_e k_B [(T_e - T_e') + (T_i - T_i')] / dt.
"""
import numpy as np

from . import constants as K

A_RAD = 4.0 * K.SIGMA_SB / K.C_LIGHT  # radiation constant a = 4 sigma_SB / c, erg cm^-3 K^-4
TAU_CRIT = 4.6                         # e^-tau = 0.01


def omega_k(r, a):
    """Keplerian frequency in c / r_g for radius r [r_g] and spin a."""
    return 1.0 / (np.asarray(r, dtype=np.float64) ** 1.5 + a)


def scale_height(rho, P, u, r, a, gamma, r_g):
    """H_th [cm] from rest-mass density rho [g cm^-3], gas pressure P and internal
    energy density u = rho eps [erg cm^-3], radius r [r_g]."""
    rho, P, u = (np.asarray(v, dtype=np.float64) for v in (rho, P, u))
    w = rho * K.C_LIGHT ** 2 + u + P                     # rho h, erg cm^-3
    cs = np.sqrt(gamma * P / w)                    # in units of c
    return cs / omega_k(r, a) * r_g


def floor_temperature(r, a, h_floor):
    """Gas temperature floor T_e + T_i [K] at radius r [r_g]."""
    r = np.asarray(r, dtype=np.float64)
    theta = 0.5 * np.pi * (h_floor * omega_k(r, a) * r) ** 2   # P / rho in c^2
    return theta * K.M_P * K.C_LIGHT ** 2 / K.K_B


def rad_pressure_temperature(n_e, T_e, T_i, H, tau_crit=TAU_CRIT):
    """(T_e corrected, corrected mask): T solving a T^4 + n_e k T = n_e k T_e
    where n_e sigma_T H > tau_crit, T_e elsewhere.  Bisection on ln T over
    (ln T_e - 60, ln T_e], to machine precision."""
    n_e, T_e, T_i, H = (np.asarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, H))
    tau = n_e * K.SIGMA_T * H
    thick = tau > tau_crit
    rhs = n_e * K.K_B * T_e

    def f(lt):
        t = np.exp(lt)
        return A_RAD * t ** 4 + n_e * K.K_B * t - rhs

    lo = np.log(T_e) - 60.0
    hi = np.log(T_e)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = f(mid) > 0.0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    T = np.exp(0.5 * (lo + hi))
    return np.where(thick, T, T_e), thick


ST_GAS_FLOOR = 32
NO_COOLING_FLOOR = 1.0e30      # an electron floor above every temperature: Q_rad = 0


def step_with_gas_floor(ts, n_e, T_e, T_i, B, H, dt, T_floor_gas, T_floor=1.0e6, scheme="be"):
    """The oracle's step where cells whose input gas temperature T_e + T_i lies
    below T_floor_gas have their radiative cooling switched off for the step
    (status bit ST_GAS_FLOOR); the others take the ordinary step."""
    from . import step as S
    arr = [np.asarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, B, H)]
    off = arr[1] + arr[2] < np.asarray(T_floor_gas, dtype=np.float64)
    fn = S.step_be if scheme == "be" else S.step_explicit16
    out = None
    for mask, floor in ((~off, T_floor), (off, NO_COOLING_FLOOR)):
        if not mask.any():
            continue
        part = fn(ts, *[a[mask] for a in arr], dt, T_floor=floor)
        if out is None:
            out = {k: np.zeros(arr[0].shape, dtype=np.asarray(v).dtype) for k, v in part.items()}
        for k, v in part.items():
            out[k][mask] = v
    out["status"] = np.where(off, out["status"] | ST_GAS_FLOOR, out["status"]).astype(np.uint8)
    return out


def cooling_lambda(n_e, T_e, T_i, T_e_new, T_i_new, dt):
    """Energy per unit volume and time the step removed from the gas [erg cm^-3 s^-1]."""
    n_e, T_e, T_i, T_e_new, T_i_new = (np.asarray(v, dtype=np.float64) for v in (n_e, T_e, T_i, T_e_new, T_i_new))
    return 1.5 * n_e * K.K_B * ((T_e - T_e_new) + (T_i - T_i_new)) / dt


def apply_cooling(U, u_cov, lam, dt, sqrt_g=None):
    """U_mu + dt sqrt(-g) G_mu with G_mu = -lambda u_mu; U and u_cov are
    sequences of four arrays (mu = 0..3).  Cells whose lambda is not finite keep
    U.  Returns the new list of four arrays."""
    lam = np.asarray(lam, dtype=np.float64)
    sg = np.ones_like(lam) if sqrt_g is None else np.asarray(sqrt_g, dtype=np.float64)
    ok = np.isfinite(lam)
    out = []
    for mu in range(4):
        G = -lam * np.asarray(u_cov[mu], dtype=np.float64)
        out.append(np.where(ok, np.asarray(U[mu], dtype=np.float64) + dt * sg * G, U[mu]))
    return out
