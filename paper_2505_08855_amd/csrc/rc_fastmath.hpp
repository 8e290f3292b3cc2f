// Elementary functions for the per-cell solver (FP64, host and device).
//
// The general-purpose library versions handle every special case (NaN, inf,
// zero, negative arguments, extra-precise intermediate steps) and cost about
// 100 VALU instructions per logarithm on gfx950.  The solver only takes
// logarithms of finite positive values and exponentials of finite moderate
// ones, so these versions use textbook reductions and short polynomials:
//
//   log:  x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(f),
//         f = (m - 1) / (m + 1), |f| <= 0.1716, s = f^2:
//         2 atanh(f) = 2 f (1 + s p(s)), p(s) = 1/3 + s/5 + s^2/7 + ...
//         economized to degree 6 in s;
//         e ln 2 with ln 2 split into a 21-bit head (exact products) and tail.
//   exp2: y = k + f with k = rint(y), |f| <= 1/2; 2^f by its Taylor series in
//         f (coefficients (ln 2)^j / j!) economized to degree 11.
//   exp:  s = k ln 2 + r (Cody-Waite: k ln2_head exact), |r| <= 0.347,
//         e^r by its Taylor series economized to degree 11, scaled by 2^k.
//   log1p: u = 1 + v, log1p(v) = ln(u) v / (u - 1) (Goldberg's correction
//         for the rounding of 1 + v; exact when u == 1).
//
// The polynomials are Chebyshev economizations of the Taylor series over
// the reduced ranges (fastmath_coeffs.py next to this file derives them in
// exact arithmetic): two to three fused multiply-adds fewer than the
// truncated series of the same accuracy.  Accuracy is a few ulp over the
// whole double range; the library's host self-test compares every function
// with the C library.
#pragma once

#include "rc_physics.hpp"

namespace rc {

constexpr double kLn2Hi = 0x1.62e42p-1;             // ln 2 rounded to 21 bits
constexpr double kLn2Lo = 0x1.fdf473de6af28p-22;    // ln 2 - kLn2Hi
constexpr double kLog2E = 0x1.71547652b82fep+0;     // 1 / ln 2
constexpr double kInvLn10 = 0x1.bcb7b1526e50ep-2;   // 1 / ln 10
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;  // sqrt(1/2)

// a / b for finite a and a finite nonzero b of normal magnitude: the
// reciprocal instruction refined by one Newton step (relative error e below
// 2^-48), then the quotient q = a r with one residual correction
// q + r (a - b q), which leaves an error of order e^2 before the final
// rounding: within an ulp of a / b (a host emulation with the reciprocal off
// by up to 2^-23 rounds 2e7 random quotients correctly).  The IEEE sequence
// adds operand scaling and a fix-up step for the full range, which the
// solver's positive, moderate denominators do not need.
RC_HD double fdiv(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
#else
  return a / b;
#endif
}

// a / b for quantities that only steer an iteration (slopes, Newton steps,
// residuals whose sign and size pick the next point, not the converged
// value): the reciprocal instruction (relative error below 2^-24; measured
// 2^-24.4 at most over 4M log-uniform arguments on gfx950) refined by one
// Newton step, which squares the error (measured 2^-48.7); a Newton step
// off by that fraction moves the iterate by far less than the solve's
// tolerance.
RC_HD double fdiv_d(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
#else
  return a / b;
#endif
}

// a / b for a value rounded to single precision right after: the reciprocal
// instruction alone on the device (relative error below 2^-24)
RC_HD double fdiv_sp(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return a * __builtin_amdgcn_rcp(b);
#else
  return a / b;
#endif
}

// single-precision reciprocal (the hardware instruction on the device)
RC_HD float frcp_sp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// One Horner step p * f + c with a constant coefficient c.  On the device the
// coefficient is an operand in a scalar register pair, so the step is one
// v_fma_f64; left to itself the compiler shapes each step as a copy of c into
// the accumulator (two 32-bit immediate moves, or a 64-bit register copy)
// followed by v_fmac_f64, two to three vector instructions per term.  Same
// fused multiply-add, same result.
RC_HD double hfma(double p, double f, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(f), "s"(c));
  return r;
#else
  return fma(p, f, c);
#endif
}

// single-precision 2^y and log2 x for step proposals that need no more than
// a few digits: the hardware instructions on the device, the C library on
// the host
RC_HD float fexp2_sp(float y) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(y);
#else
  return exp2f(y);
#endif
}

RC_HD float flog2_sp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_logf(x);
#else
  return log2f(x);
#endif
}

// ln x for finite x > 0
RC_HD double flog(double x) {
  int e;
  double m = frexp(x, &e);           // [1/2, 1)
  if (m < kSqrtHalf) {
    m += m;
    --e;
  }
  const double f = fdiv(m - 1.0, m + 1.0);   // m - 1 is exact
  const double s = f * f;
  double p = 0x1.2b62ca3da2e33p-4;
  p = hfma(p, s, 0x1.39fd807189bb6p-4);
  p = hfma(p, s, 0x1.7462bba41c635p-4);
  p = hfma(p, s, 0x1.c71c62cbfea3fp-4);
  p = hfma(p, s, 0x1.2492492e0644ep-3);   // ~1/7
  p = hfma(p, s, 0x1.9999999995219p-3);   // ~1/5
  p = hfma(p, s, 0x1.5555555555558p-2);   // ~1/3
  const double f2 = f + f;
  const double lm = fma(f2 * s, p, f2);    // 2 atanh f
  const double de = (double)e;
  return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

RC_HD double flog10(double x) { return flog(x) * kInvLn10; }

// ln(1 + v) for finite v > -1
RC_HD double flog1p(double v) {
  const double u = 1.0 + v;
  if (u == 1.0) return v;
  return flog(u) * fdiv(v, u - 1.0);
}

// 2^y for finite y
RC_HD double fexp2(double y) {
  const double k = rint(y);
  const double f = y - k;             // exact
  double p = 0x1.ea044321bc0aap-32;   // ~(ln 2)^11 / 11!
  p = hfma(p, f, 0x1.e6228bff026d1p-28);
  p = hfma(p, f, 0x1.b524db38fd1f9p-24);
  p = hfma(p, f, 0x1.62bfc2c7ae40ep-20);
  p = hfma(p, f, 0x1.ffcbfc75f302dp-17);
  p = hfma(p, f, 0x1.430913112cb56p-13);
  p = hfma(p, f, 0x1.5d87fe78a2292p-10);
  p = hfma(p, f, 0x1.3b2ab6fb9f1a3p-7);
  p = hfma(p, f, 0x1.c6b08d704a0d1p-5);
  p = hfma(p, f, 0x1.ebfbdff82c5aep-3);
  p = hfma(p, f, 0x1.62e42fefa39efp-1);   // ln 2
  p = hfma(p, f, 1.0);
  return ldexp(p, (int)k);
}

// e^s.  The reduction reaches the whole double range: k up to 1024 (s below
// ln DBL_MAX = 709.78 gives p 2^1024 < DBL_MAX) and the scaling by 2^k rounds
// gradual underflow; beyond |s| = 746 e^s is +inf or 0, and inf and NaN go
// the same way (no library fallback: its constants would stay live in
// registers across the solver's loops)
RC_HD double fexp(double s) {
  if (!(fabs(s) < 746.0)) return s > 0.0 ? __builtin_inf() : (s < 0.0 ? 0.0 : s);
  const double k = rint(s * kLog2E);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, s));
  double p = 0x1.af79f6e31795fp-26;   // ~1 / 11!
  p = hfma(p, r, 0x1.28b538eba9034p-22);
  p = hfma(p, r, 0x1.71dde673efb0ep-19);
  p = hfma(p, r, 0x1.a019905f26df8p-16);
  p = hfma(p, r, 0x1.a01a01b86d2fbp-13);
  p = hfma(p, r, 0x1.6c16c18878da9p-10);
  p = hfma(p, r, 0x1.111111110da35p-7);
  p = hfma(p, r, 0x1.555555554ee74p-5);
  p = hfma(p, r, 0x1.5555555555563p-3);
  p = hfma(p, r, 0x1.0000000000011p-1);
  p = hfma(p, r, 1.0);
  p = hfma(p, r, 1.0);
  return ldexp(p, (int)k);
}

}  // namespace rc
