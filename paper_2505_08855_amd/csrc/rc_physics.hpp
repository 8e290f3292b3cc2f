// Closed-form cooling physics evaluated in FP64 on the GPU (and, for the
// library's host self-tests, on the CPU from the same source).
//
// Used to build the table nodes and by the DIRECT (table-free) step variant.
// Section references are to arXiv:2505.08855:
//   II.A bremsstrahlung, II.B synchrotron with self-absorption, II.C Compton
//   enhancement, II.D optically-thick bridge, II.G Coulomb exchange.
// Special functions are this library's own: scaled modified Bessel functions
// by the trapezoidal rule on K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt
// (exponentially convergent for this analytic integrand), the upper incomplete
// Gamma function by its power series / Legendre continued fraction (evaluated
// with the modified Lentz method), and the synchrotron critical frequency by a
// bracketed Newton iteration.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define RC_HD __host__ __device__ inline

namespace rc {

// CODATA 2018, cgs
constexpr double kC = 2.99792458e10;
constexpr double kKB = 1.380649e-16;
constexpr double kH = 6.62607015e-27;
constexpr double kME = 9.1093837015e-28;
constexpr double kMP = 1.67262192369e-24;
constexpr double kE = 4.803204712570263e-10;
constexpr double kSigmaT = 6.6524587321e-25;
constexpr double kSigmaSB = 5.670374419e-5;

constexpr double kMeC2 = kME * kC * kC;
constexpr double kMpC2 = kMP * kC * kC;
constexpr double kPi = 3.14159265358979323846;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLn10 = 2.30258509299404568402;
constexpr double kLog2_10 = 3.32192809488736234787;   // log2(10)
constexpr double kSqrt3 = 1.73205080756887729353;

// fit coefficients printed in Sec. II.A and II.B
constexpr double kBremEE = 2.56e-22, kBremEI = 1.48e-22;
constexpr double kSynNorm = 4.43e-30;
constexpr double kIpNorm = 4.0505, kIpC1 = 0.4, kIpC2 = 0.5316, kIpA = 1.8899;
constexpr double kLowTSwitch = 1.0e8;
// internal energy u = n k T / (gamma - 1), gamma = 5/3 (Sec. III.C)
constexpr double kUperNKT = 1.5;

RC_HD double theta_e(double T) { return kKB * T / kMeC2; }
RC_HD double theta_p(double T) { return kKB * T / kMpC2; }

// ---------------------------------------------------------------- Sec. II.A
// Q_brem / n_e^2: the two fitted factors with their case split at theta = 1
// (theta = 1 exactly takes the theta >= 1 branch).
RC_HD double brem_coeff(double T) {
  const double th = theta_e(T);
  double ee, ei;
  if (th < 1.0) {
    const double th15 = th * sqrt(th);
    ee = th15 * (1.0 + 1.1 * th + th * th - 1.25 * th * th15);
    ei = 4.0 * sqrt(2.0 * th / (kPi * kPi * kPi)) * (1.0 + 1.781 * pow(th, 1.34));
  } else {
    ee = 1.34 * th * (log(1.123 * th) + 1.28);
    ei = 9.0 * th / (2.0 * kPi) * (log(1.123 * th + 0.48) + 1.5);
  }
  return kBremEE * ee + kBremEI * ei;
}

// ---------------------------------------------------------------- Bessel
// Exponentially scaled K_0, K_1, K_2 at z > 0:
//   kve_nu(z) = e^z K_nu(z) = int_0^inf exp(-z (cosh t - 1)) cosh(nu t) dt.
// Trapezoidal rule with step h = min(0.2, 0.7 / sqrt(z)); for this even,
// entire integrand the error decays like exp(-2 pi^2 / (h^2 z)) (large z) and
// exp(-pi^2 / h) (small z), both below 1e-16 at this h.  cosh t - 1 is formed
// as 2 sinh^2(t/2) to keep its relative accuracy at small t.
RC_HD void kve012(double z, double* k0, double* k1, double* k2) {
  const double h = fmin(0.2, 0.7 / sqrt(z));
  const double t_peak = asinh(2.0 / z);   // cosh(2t) e^{-z(cosh t - 1)} peaks here
  double s0 = 0.5, s1 = 0.5, s2 = 0.5;
  for (int k = 1; k < 20000; ++k) {
    const double t = k * h;
    const double sh = sinh(0.5 * t);
    const double e = exp(-2.0 * z * sh * sh);
    const double c1 = cosh(t);
    const double c2 = 2.0 * c1 * c1 - 1.0;
    s0 += e;
    s1 += e * c1;
    s2 += e * c2;
    if (t > t_peak && e * c2 < 1e-18 * s2) break;
  }
  *k0 = h * s0;
  *k1 = h * s1;
  *k2 = h * s2;
}

RC_HD double kve2(double z) {
  double a, b, c;
  kve012(z, &a, &b, &c);
  return c;
}

// ---------------------------------------------------------------- Sec. II.B
// ln I'(x) of the Mahadevan fit, eq. fitting_I(xm)
RC_HD double ln_iprime(double x) {
  return log(kIpNorm) - log(x) / 6.0 + log1p(kIpC1 * pow(x, -0.25) + kIpC2 / sqrt(x)) - kIpA * cbrt(x);
}

// ln K2(1/theta_e) as it enters the emissivity: 2 theta^2 at or below 1e8 K
// (end of Sec. II.B), the true Bessel function above.
RC_HD double ln_k2_synch(double T) {
  const double th = theta_e(T);
  if (T <= kLowTSwitch) return log(2.0 * th * th);
  const double z = 1.0 / th;
  return log(kve2(z)) - z;
}

// x_c solving ln(I'(x)/x) = ln_rhs: phi(s) = ln I'(e^s) - s - ln_rhs is
// strictly decreasing in s = ln x (phi' <= -7/6), so the root is unique.
// Newton in s, kept inside a bisection bracket.
RC_HD double solve_xc(double ln_rhs) {
  double lo = -80.0, hi = 80.0;      // phi(lo) > 0 > phi(hi) over the table ranges
  double s = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double q = exp(-0.25 * s);
    const double q2 = q * q;
    const double inner = 1.0 + kIpC1 * q + kIpC2 * q2;
    const double ex = exp(s / 3.0);
    const double phi = log(kIpNorm) - s / 6.0 + log(inner) - kIpA * ex - s - ln_rhs;
    const double dphi = -7.0 / 6.0 + (-0.25 * kIpC1 * q - 0.5 * kIpC2 * q2) / inner - (kIpA / 3.0) * ex;
    if (phi > 0.0) lo = s; else hi = s;
    if (phi == 0.0) return exp(s);
    double sn = s - phi / dphi;
    if (fabs(sn - s) <= 1e-15 * fmax(1.0, fabs(s))) { s = sn; break; }   // before the safeguard
    if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    s = sn;
    if (hi - lo <= 1e-15 * fmax(1.0, fabs(s))) break;
  }
  return exp(s);
}

// ln Gamma(p, z), the upper incomplete Gamma function, p > 0, z > 0.
//   z <  p + 1: Gamma(p) - gamma(p, z) with the series
//               gamma(p, z) = z^p e^-z sum_n z^n / (p (p+1) ... (p+n));
//   z >= p + 1: Legendre's continued fraction
//               Gamma(p, z) = z^p e^-z / (z+1-p - 1(1-p)/(z+3-p - 2(2-p)/(z+5-p - ...))),
//               evaluated with the modified Lentz method.
RC_HD double ln_gamma_upper(double p, double z) {
  if (z < p + 1.0) {
    double term = 1.0 / p, sum = term;
    for (int n = 1; n < 1000; ++n) {
      term *= z / (p + n);
      sum += term;
      if (term < 1e-17 * sum) break;
    }
    const double lower = exp(p * log(z) - z) * sum;
    return log(tgamma(p) - lower);
  }
  const double tiny = 1e-300;
  double b = z + 1.0 - p;
  double c = 1.0 / tiny;
  double d = 1.0 / b;
  double f = d;
  for (int i = 1; i < 1000; ++i) {
    const double an = -i * (i - p);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    f *= del;
    if (fabs(del - 1.0) < 1e-17) break;
  }
  return -z + p * log(z) + log(f);
}

// ln J(x), J(x) = int_x^inf s I'(s) ds.  With s = t^3,
// s I'(s) ds = 3 * 4.0505 (t^4.5 + 0.4 t^3.75 + 0.5316 t^3) e^{-a t} dt, so
// J = 3 * 4.0505 * sum_j c_j a^-p_j Gamma(p_j, a x^(1/3)), p = 5.5, 4.75, 4.
RC_HD double ln_tail(double x) {
  const double z = kIpA * cbrt(x);
  const double la = log(kIpA);
  const double l1 = ln_gamma_upper(5.5, z) - 5.5 * la;
  const double l2 = log(kIpC1) + ln_gamma_upper(4.75, z) - 4.75 * la;
  const double l3 = log(kIpC2) + ln_gamma_upper(4.0, z) - 4.0 * la;
  const double m = fmax(l1, fmax(l2, l3));
  return log(3.0 * kIpNorm) + m + log(exp(l1 - m) + exp(l2 - m) + exp(l3 - m));
}

struct SynchResult {
  double ln_q;    // ln Q_syn
  double nu_c;    // critical frequency, Hz
};

// Self-absorbed synchrotron cooling (eq. synchrotron) at (n_e, T, B, H):
// the self-absorption balance (eq. bb_sync_aprox) H eps_s(nu_c) =
// 2 pi nu_c^2 k T / c^2 becomes I'(x_c)/x_c = 3 e B theta^3 K2 / (8 pi c 4.43e-30 n_e H);
// the self-absorbed band radiates 2 pi k T nu_c^3 / (3 c^2 H) and the thin tail
// int_nu_c^inf eps_s dnu = 4.43e-30 4 pi n_e nu0^2 J(x_c) / K2, nu0 = 3 e B theta^2 / (4 pi m_e c).
RC_HD SynchResult synchrotron(double n_e, double T, double B, double H) {
  const double th = theta_e(T);
  const double lk2 = ln_k2_synch(T);
  const double ln_rhs = log(3.0 * kE * B * th * th * th / (8.0 * kPi * kC * kSynNorm)) + lk2 - log(n_e * H);
  const double xc = solve_xc(ln_rhs);
  const double nu0 = 3.0 * kE * B * th * th / (4.0 * kPi * kME * kC);
  const double nu_c = nu0 * xc;
  const double ln_rj = log(2.0 * kPi * kKB / (3.0 * kC * kC)) + log(T) + 3.0 * log(nu_c) - log(H);
  const double ln_tl = log(kSynNorm * 4.0 * kPi) + log(n_e) - lk2 + 2.0 * log(nu0) + ln_tail(xc);
  const double m = fmax(ln_rj, ln_tl);
  SynchResult r;
  r.ln_q = m + log1p(exp(fmin(ln_rj, ln_tl) - m));
  r.nu_c = nu_c;
  return r;
}

// ---------------------------------------------------------------- Sec. II.C
// ln eta_comp at nu_c.  P = 1 - exp(-tau_sca), tau_sca = 2 n_e sigma_T H,
// A = 1 + 4 theta + 16 theta^2, E = h nu_c / m_e c^2.  With k = ln(3 theta/E)/ln A
// the enhancement is the geometric series 1 + P (A-1) sum_{j<k} (PA)^j, i.e.
// 1 + P (A-1) expm1(k L) / expm1(L) with L = ln(P A) (limit k at L = 0);
// eta = 1 for E >= 3 theta.
RC_HD double ln_eta(double n_e, double T, double H, double nu_c) {
  const double th = theta_e(T);
  const double E = kH * nu_c / kMeC2;
  if (!(E < 3.0 * th)) return 0.0;
  const double tau = 2.0 * n_e * kSigmaT * H;
  const double P = -expm1(-tau);
  const double A = 1.0 + 4.0 * th + 16.0 * th * th;
  const double lnA = log1p(4.0 * th + 16.0 * th * th);
  const double k = log(3.0 * th / E) / lnA;
  const double L = log(P) + lnA;
  const double ratio = (L == 0.0) ? k : expm1(k * L) / expm1(L);
  return log1p(P * (A - 1.0) * ratio);
}

// eta_comp at nu_c with the exponent exactly as printed, 1 - ln P / ln A:
// 1 + P (A-1)/(1 - PA) [1 - (E/3 theta)^(1 - ln P/ln A)], 1 for E >= 3 theta.
// Negative wherever P A > 1 (the reading not taken by default).
RC_HD double eta_literal(double n_e, double T, double H, double nu_c) {
  const double th = theta_e(T);
  const double E = kH * nu_c / kMeC2;
  if (!(E < 3.0 * th)) return 1.0;
  const double tau = 2.0 * n_e * kSigmaT * H;
  const double P = -expm1(-tau);
  const double A = 1.0 + 4.0 * th + 16.0 * th * th;
  const double expo = 1.0 - log(P) / log(A);
  return 1.0 + P * (A - 1.0) / (1.0 - P * A) * (1.0 - pow(E / (3.0 * th), expo));
}

// ---------------------------------------------------------------- Sec. II.G
// Q_cc / (T_i - T_e) with rho/m_p = n_i = n_e, m_i = m_p, theta_i = k T_i / m_p c^2
// (theta_i = k T_i / m_e c^2, as printed, when theta_i_me).
// The e^-z factors of K2(1/th_i) K2(1/th_e) and K_n(1/th_m) cancel exactly
// (1/th_m = 1/th_e + 1/th_i), so only scaled Bessel functions appear.
RC_HD double ln_coulomb_coeff(double n_e, double T_e, double T_i, double ln_lambda, bool theta_i_me = false) {
  const double te = theta_e(T_e);
  const double ti = theta_i_me ? theta_e(T_i) : theta_p(T_i);
  const double s = te + ti;
  const double zm = 1.0 / te + 1.0 / ti;
  double m0, m1, m2, e0, e1, e2, i0, i1, i2;
  kve012(zm, &m0, &m1, &m2);
  kve012(1.0 / te, &e0, &e1, &e2);
  kve012(1.0 / ti, &i0, &i1, &i2);
  const double R = ((2.0 * s * s + 1.0) / s * m1 + 2.0 * m0) / (e2 * i2);
  const double pref = 1.5 * (kME / kMP) * ln_lambda * kC * kKB * kSigmaT;
  return log(pref) + 2.0 * log(n_e) + log(R);
}

// ---------------------------------------------------------------- table nodes
// log2 values stored in the tables (column form, H = 1 cm for the cooling
// tables; see the reduction note in radcool.h).
RC_HD double node_brem(double N, double T) { return (2.0 * log(N) + log(brem_coeff(T))) / kLn2; }

// With the literal Compton exponent a node whose eta is not positive has no
// log2 value: NaN.
RC_HD void node_synch_eta(double N, double T, double B, bool compton_literal, double* y_s, double* y_eta) {
  const SynchResult sr = synchrotron(N, T, B, 1.0);
  *y_s = sr.ln_q / kLn2;
  if (compton_literal) {
    const double eta = eta_literal(N, T, 1.0, sr.nu_c);
    *y_eta = (eta > 0.0 && isfinite(eta)) ? log(eta) / kLn2 : __builtin_nan("");
  } else {
    *y_eta = ln_eta(N, T, 1.0, sr.nu_c) / kLn2;
  }
}

RC_HD double node_coul(double n_e, double T_e, double T_i, double ln_lambda, bool theta_i_me) {
  return ln_coulomb_coeff(n_e, T_e, T_i, ln_lambda, theta_i_me) / kLn2;
}

}  // namespace rc
