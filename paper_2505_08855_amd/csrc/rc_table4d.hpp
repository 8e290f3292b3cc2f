// The paper's own cooling-table layout (Sec. II.F, III.A): log2 of the bridged
// Q_total(H, B, n_e, T_e) on a 4-D grid of log-spaced nodes, read by 4-D
// multilinear interpolation in the log10 axes (clamped at the edges).  Kept as
// the comparison layout for the exact 3-D column tables: same closed forms,
// different parametrisation.  The values are stored as plain FP32 log2 values,
// as a texture would hold them.  Host and device.
#pragma once

#include "rc_fastmath.hpp"
#include "rc_physics.hpp"
#include "rc_step.hpp"

namespace rc {

// log2 of the bridged total cooling at node (H, B, n_e, T), evaluated through
// the column variables (N = n_e H, the H = 1 cm synchrotron and Compton values)
// and combined in log space, so that no intermediate overflows at the far
// corners of the paper's ranges.
RC_HD double node_total(double H, double B, double n_e, double T) {
  const double N = n_e * H;
  double ys, ye;
  node_synch_eta(N, T, B, false, &ys, &ye);
  const double lH = log2(H);
  const double lb = node_brem(N, T) - 2.0 * lH;           // log2 Q_brem
  const double ls = ys + ye - lH;                           // log2 (eta Q_syn)
  const double hi = fmax(lb, ls), lo = fmin(lb, ls);
  const double lq = hi + log2(1.0 + exp2(lo - hi));         // log2 Q_thin
  const double lta = lH + lq - log2(4.0 * kSigmaSB) - 4.0 * log2(T);   // log2 tau_abs
  const double lts = log2(2.0 * n_e * kSigmaT * H);         // log2 tau_sca
  // D = 1 + sqrt3 tau_abs + 1.5 tau_abs^2 + 1.5 tau_abs tau_sca, as a log-sum
  const double t[4] = {0.0, log2(kSqrt3) + lta, log2(1.5) + 2.0 * lta, log2(1.5) + lta + lts};
  const double m = fmax(fmax(t[0], t[1]), fmax(t[2], t[3]));
  const double lD = m + log2(exp2(t[0] - m) + exp2(t[1] - m) + exp2(t[2] - m) + exp2(t[3] - m));
  return lq - lD;
}

// the four axes (H, B, n_e, T_e) in log10
struct Axes4P {
  AxisP a[4];
};

// 4-D multilinear interpolation of the C-ordered [H][B][n_e][T_e] values at
// log10 coordinates u; *clamped is set when a coordinate left its axis
template <class Load>
RC_HD double interp4(const Load& v, const Axes4P& A, const double u[4], bool* clamped) {
  int i[4];
  double t[4];
  bool cl = false;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const Coord c = axis_coord(u[d], A.a[d]);
    i[d] = c.i;
    t[d] = c.t;
    cl = cl || c.clamped;
  }
  const long s2 = A.a[3].n, s1 = s2 * A.a[2].n, s0 = s1 * A.a[1].n;
  const long base = i[0] * s0 + i[1] * s1 + i[2] * s2 + i[3];
  double y = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int b0 = (c >> 3) & 1, b1 = (c >> 2) & 1, b2 = (c >> 1) & 1, b3 = c & 1;
    const double w = (b0 ? t[0] : 1.0 - t[0]) * (b1 ? t[1] : 1.0 - t[1]) * (b2 ? t[2] : 1.0 - t[2]) *
                     (b3 ? t[3] : 1.0 - t[3]);
    y += w * (double)v(base + b0 * s0 + b1 * s1 + b2 * s2 + b3);
  }
  *clamped = cl;
  return y;
}

}  // namespace rc
