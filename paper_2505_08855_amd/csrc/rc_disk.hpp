// Per-cell inputs upstream of the cooling step, the post-processing
// radiation-pressure temperature correction and the cooling rate handed
// downstream (host and device).
//
// Thermal scale height (Sec. II.F, eq. H_thermal): H_th = c_s / Omega_K,
// c_s^2 = gamma P / (rho h) with the relativistic enthalpy density
// rho h = rho c^2 + rho eps + P, and Omega_K = 1 / (r^(3/2) + a) in
// gravitational units (r in r_g, Omega in c / r_g), so that in cgs
// H_th = (c_s / c) (r^(3/2) + a) r_g.
//
// Temperature floor (Sec. III.B.2): T_floor = (pi/2) [h_floor Omega_K R]^2 is a
// gas temperature in units of c^2 (P / rho); with n_i = n_e and rho = m_p n_e,
// P / rho = k (T_e + T_i) / m_p, so the floor on T_e + T_i in kelvin is
// T_floor m_p c^2 / k_B.
//
// Radiation-pressure correction (Sec. IV, eq. total_pressure): where
// tau_sca = n_e sigma_T H exceeds tau_crit (4.6: fewer than 1 % of photons escape
// unscattered) the pressure n_e k (T_e + T_i) is shared between radiation and
// gas with T_i held, a T^4 + n_e k T = n_e k T_e, a = 4 sigma_SB / c.  In s = ln T
// the left side minus the right is convex and increasing; Newton from a start
// at or above the root, min(ln T_e, ln (n_e k T_e / a)^(1/4)), descends
// monotonically onto it.
#pragma once

#include "rc_fastmath.hpp"
#include "rc_physics.hpp"

namespace rc {

constexpr double kARad = 4.0 * kSigmaSB / kC;   // radiation constant, erg cm^-3 K^-4

RC_HD double omega_k(double r, double a) { return 1.0 / (r * sqrt(r) + a); }

RC_HD double disk_scale_height(double rho, double P, double u, double r, double a, double gamma, double r_g) {
  const double w = rho * kC * kC + u + P;        // rho h, erg cm^-3
  const double cs = sqrt(gamma * P / w);         // units of c
  return cs / omega_k(r, a) * r_g;
}

RC_HD double floor_gas_temperature(double r, double a, double h_floor) {
  const double v = h_floor * omega_k(r, a) * r;
  return 0.5 * kPi * v * v * kMP * kC * kC / kKB;
}

// T solving a T^4 + n_e k T = n_e k T_e (T <= T_e).  Stops at the root (f no
// longer positive), or when a step no longer changes s (it is below half an
// ulp of s), or after a step below 1e-15 relative.
RC_HD double rad_pressure_temperature(double n_e, double T_e) {
  const double nk = n_e * kKB;
  const double rhs = nk * T_e;
  double s = fmin(flog(T_e), 0.25 * flog(rhs / kARad));
  for (int it = 0; it < 100; ++it) {
    const double t = fexp(s);
    const double t4 = kARad * t * t * t * t;
    const double f = t4 + nk * t - rhs;
    if (!(f > 0.0)) break;                       // at (or, by rounding, just below) the root
    const double ds = f / (4.0 * t4 + nk * t);
    const double sn = s - ds;
    if (sn == s) break;
    s = sn;
    if (ds <= 1e-15 * fabs(s)) break;
  }
  return fexp(s);
}

// energy per unit volume and time a step removed from the gas (the lambda of
// the 4-force density G_mu = -lambda u_mu, Sec. II.E)
RC_HD double cooling_lambda(double n_e, double T_e, double T_i, double T_e_new, double T_i_new, double dt) {
  return kUperNKT * n_e * kKB * ((T_e - T_e_new) + (T_i - T_i_new)) / dt;
}

}  // namespace rc
