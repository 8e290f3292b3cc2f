// Per-cell adjoint of the cooling step (host + device source).
//
// The backward-Euler update defines (x, z) = (T_e', T_i') by
//   E1 = c (x - T_e) + dt Q_rad(x) - dt (z - x) v_c(x, z) = 0,
//   E2 = c (z - T_i) + dt (z - x) v_c(x, z)               = 0,
// so for output cotangents (g_x, g_z) the vector-Jacobian product follows from
// the implicit function theorem: solve J^T lam = (g_x, g_z) with
// J = d(E1, E2)/d(x, z) (the same 2x2 Jacobian the Newton solve uses) and
// gbar_p = -lam . d(E1, E2)/dp.  A floor-projected cell has x fixed, so only E2
// ties z to the inputs.  The input-state rates Q_rad(T_e), Q_cc(T_e, T_i) add
// their direct derivatives.  Table entries are the log2 node values; a value
// 2^y depends on a corner through ln 2 * 2^y * (corner weight).  Derivatives
// are those of the interpolant inside the query's cell (zero along a clamped
// axis), as in the forward solve.
#pragma once

#include "rc_step.hpp"

namespace rc {

// trilinear point of the interleaved cooling tables: log2 of v_brem and of
// v_synch * v_eta with their gradients in the log10 coordinates, and corners
struct CoolPoint {
  double yb, yse;
  double dyb[3], dyse[3];
  long idx[8];
  double w[8];
  long cell;      // table cell (lowest corner) in cell numbering
  double t[3];    // fractional coordinates inside it
};

struct CoulPoint {
  double y;
  double dy[3];
  long idx[8];
  double w[8];
  long cell;
  double t[3];
};

template <class Tab>
RC_HD CoolPoint cool_point(const Tab& tab, const StepParams& P, double u0, double u1, double u2, int n1, int n2) {
  const Coord c0 = axis_coord(u0, P.g->ax[0]), c1 = axis_coord(u1, P.g->ax[1]), c2 = axis_coord(u2, P.g->ax[2]);
  CoolPoint r;
  double yb = 0.0, yse = 0.0;
  double gb[3] = {0.0, 0.0, 0.0}, gse[3] = {0.0, 0.0, 0.0};
  float2 v[8];                           // the solver's {brem, se} pairs, corner (a, b, m) at 4a + 2b + m
  tab.cool8(c0.i, c1.i, c2.i, v);
  int k = 0;
  for (int a = 0; a < 2; ++a) {
    const double wa = a ? c0.t : 1.0 - c0.t, da = a ? 1.0 : -1.0;
    for (int b = 0; b < 2; ++b) {
      const double wb = b ? c1.t : 1.0 - c1.t, db = b ? 1.0 : -1.0;
      for (int m = 0; m < 2; ++m, ++k) {
        const double wm = m ? c2.t : 1.0 - c2.t, dm = m ? 1.0 : -1.0;
        const double w = wa * wb * wm;
        const double vb = v[k].x, vse = v[k].y;
        yb += w * vb;
        yse += w * vse;
        const double g0 = da * wb * wm, g1 = wa * db * wm, g2 = wa * wb * dm;
        gb[0] += g0 * vb; gb[1] += g1 * vb; gb[2] += g2 * vb;
        gse[0] += g0 * vse; gse[1] += g1 * vse; gse[2] += g2 * vse;
        r.idx[k] = ((long)(c0.i + a) * n1 + (c1.i + b)) * n2 + (c2.i + m);
        r.w[k] = w;
      }
    }
  }
  r.cell = ((long)c0.i * (n1 - 1) + c1.i) * (n2 - 1) + c2.i;
  r.t[0] = c0.t; r.t[1] = c1.t; r.t[2] = c2.t;
  const double f0 = c0.i + c0.t, f1 = c1.i + c1.t, f2 = c2.i + c2.t;
  const double* cb = P.g->coef[0];
  const double* cs = P.g->coef[1];
  const double* ce = P.g->coef[2];
  r.yb = cb[0] + cb[1] * f0 + cb[2] * f1 + cb[3] * f2 + yb;
  r.yse = (cs[0] + ce[0]) + (cs[1] + ce[1]) * f0 + (cs[2] + ce[2]) * f1 + (cs[3] + ce[3]) * f2 + yse;
  const double dfdu[3] = {c0.dfdu, c1.dfdu, c2.dfdu};
  for (int q = 0; q < 3; ++q) {
    r.dyb[q] = (cb[q + 1] + gb[q]) * dfdu[q];
    r.dyse[q] = (cs[q + 1] + ce[q + 1] + gse[q]) * dfdu[q];
  }
  return r;
}

template <class Tab>
RC_HD CoulPoint coul_point(const Tab& tab, const StepParams& P, double u0, double u1, double u2, int n1, int n2) {
  const Coord c0 = axis_coord(u0, P.g->ax[3]), c1 = axis_coord(u1, P.g->ax[4]), c2 = axis_coord(u2, P.g->ax[5]);
  CoulPoint r;
  double y = 0.0, g[3] = {0.0, 0.0, 0.0};
  float cv[8];
  tab.coul8(c0.i, c1.i, c2.i, cv);
  int k = 0;
  for (int a = 0; a < 2; ++a) {
    const double wa = a ? c0.t : 1.0 - c0.t, da = a ? 1.0 : -1.0;
    for (int b = 0; b < 2; ++b) {
      const double wb = b ? c1.t : 1.0 - c1.t, db = b ? 1.0 : -1.0;
      for (int m = 0; m < 2; ++m, ++k) {
        const double wm = m ? c2.t : 1.0 - c2.t, dm = m ? 1.0 : -1.0;
        const double v = cv[k];
        const double w = wa * wb * wm;
        y += w * v;
        g[0] += da * wb * wm * v; g[1] += wa * db * wm * v; g[2] += wa * wb * dm * v;
        r.idx[k] = ((long)(c0.i + a) * n1 + (c1.i + b)) * n2 + (c2.i + m);
        r.w[k] = w;
      }
    }
  }
  r.cell = ((long)c0.i * (n1 - 1) + c1.i) * (n2 - 1) + c2.i;
  r.t[0] = c0.t; r.t[1] = c1.t; r.t[2] = c2.t;
  const double* co = P.g->coef[3];
  r.y = co[0] + co[1] * (c0.i + c0.t) + co[2] * (c1.i + c1.t) + co[3] * (c2.i + c2.t) + y;
  const double dfdu[3] = {c0.dfdu, c1.dfdu, c2.dfdu};
  for (int q = 0; q < 3; ++q) r.dy[q] = (co[q + 1] + g[q]) * dfdu[q];
  return r;
}

// Q_rad at T_e' = x and its partial derivatives (n_e, x, B, H), plus dQ_rad/dy
// per unit corner weight for the brem table (sb) and for the synch and eta
// tables (sse, the same for both since they enter as a product).
struct QradPartials {
  double q, dn, dx, dB, dH, sb, sse;
};

RC_HD QradPartials qrad_partials(const CoolPoint& cp, double n_e, double x, double B, double H, bool on) {
  QradPartials r = {0, 0, 0, 0, 0, 0, 0};
  if (!on) return r;
  const double vb = fexp2(cp.yb) / (H * H);
  const double vse = fexp2(cp.yse) / H;
  const double qt = vb + vse;
  double du[3];
  for (int a = 0; a < 3; ++a) du[a] = kLn2 * (vb * cp.dyb[a] + vse * cp.dyse[a]);
  const double dqt_n = du[0] / (n_e * kLn10);
  const double dqt_x = du[1] / (x * kLn10);
  const double dqt_B = du[2] / (B * kLn10);
  const double dqt_H = du[0] / (H * kLn10) - 2.0 * vb / H - vse / H;
  const double ts = 2.0 * n_e * kSigmaT * H;
  const double x2 = x * x;
  const double ta = H * qt / (4.0 * kSigmaSB * x2 * x2);
  const double D = 1.0 + kSqrt3 * ta + 1.5 * ta * (ta + ts);
  const double Dta = kSqrt3 + 1.5 * (2.0 * ta + ts);
  const double q = qt / D;
  const double iD = 1.0 / D, qD2 = qt * iD * iD;
  // dQ_rad/dQ_thin with tau_abs's own dependence on Q_thin:
  // (D - ta dD/dta) / D^2 = (1 - 1.5 ta^2) / D^2 exactly (the expanded form
  // cancels when scattering dominates); the rest is the explicit dependence of
  // ta on H and x and of ts on n_e and H
  const double fac = (1.0 - 1.5 * ta * ta) * iD * iD;
  r.q = q;
  r.dn = fac * dqt_n - qD2 * 1.5 * ta * ts / n_e;
  r.dx = fac * dqt_x + qD2 * Dta * 4.0 * ta / x;
  r.dB = fac * dqt_B;
  r.dH = fac * dqt_H - qD2 * (Dta * ta + 1.5 * ta * ts) / H;
  r.sb = fac * kLn2 * vb;
  r.sse = fac * kLn2 * vse;
  return r;
}

struct CellGrad {
  double n_e, T_e, T_i, B, H;
};

// Adjoint of one cell.  (x, z, status) are the forward outputs.  Table-entry
// contributions go to sc.cool(idx[8], brem[8], synch_eta[8]) and
// sc.coul(idx[8], coul[8]): the synchrotron and Compton tables enter only as
// the product v_synch v_eta, so their log2 entries receive identical
// gradients and are scattered once; when the solution and the input state
// fall in the same table cell their corner contributions are merged first.
// A scatter with kRecords set receives instead one record per evaluation
// point (sc.cool_rec / sc.coul_rec: table cell, coefficients, fractional
// coordinates) for a later reduction by table cell.
template <class Tab, class Scatter>
RC_HD void cell_vjp(const Tab& tab, const StepParams& P, int c1, int c2, int k1, int k2, double n_e, double T_e,
                    double T_i, double B, double H, double floor_gas, double x, double z, unsigned char status,
                    double g_x, double g_z, double g_qr, double g_qc, bool newton, bool want_tables, CellGrad* out,
                    Scatter& sc) {
  // radiative cooling switched off for the step by the gas-temperature floor
  const bool cool_off = T_e + T_i < floor_gas;
  out->n_e = out->T_e = out->T_i = out->B = out->H = 0.0;
  if (status & ST_INVALID) return;
  const double dt = P.dt;
  const double c = kUperNKT * n_e * kKB;
  const double c_n = kUperNKT * kKB;
  const double lne = flog10(n_e), lH = flog10(H), lB = flog10(B);
  double gn = 0.0, gTe = 0.0, gTi = 0.0, gB = 0.0, gH = 0.0;
  // corner coefficients of the two evaluation points (solution, input)
  double cb[2] = {0.0, 0.0}, cse[2] = {0.0, 0.0}, cc[2] = {0.0, 0.0};
  CoolPoint cp[2];
  CoulPoint kp[2];
  bool have[2] = {false, false};
  if (newton) {
    const bool floor = (status & ST_FLOOR) != 0;
    const double lx = flog10(x), lz = flog10(z);
    cp[0] = cool_point(tab, P, lne + lH, lx, lB, c1, c2);
    kp[0] = coul_point(tab, P, lne, lx, lz, k1, k2);
    have[0] = true;
    const QradPartials qp = qrad_partials(cp[0], n_e, x, B, H, !cool_off && x >= P.T_floor);
    const double kc = fexp2(kp[0].y);
    const double kn = kLn2 * kc * kp[0].dy[0] / (n_e * kLn10);
    const double kx = kLn2 * kc * kp[0].dy[1] / (x * kLn10);
    const double kz = kLn2 * kc * kp[0].dy[2] / (z * kLn10);
    const double zx = z - x;
    const double j11 = c + dt * qp.dx + dt * kc - dt * zx * kx;
    const double j12 = -dt * kc - dt * zx * kz;
    const double j21 = -dt * kc + dt * zx * kx;
    const double j22 = c + dt * kc + dt * zx * kz;
    double l1, l2;
    if (floor) {
      l1 = 0.0;
      l2 = g_z / j22;
    } else {
      const double det = j11 * j22 - j12 * j21;
      l1 = (j22 * g_x - j21 * g_z) / det;
      l2 = (j11 * g_z - j12 * g_x) / det;
    }
    gn = -(l1 * (c_n * (x - T_e) + dt * qp.dn - dt * zx * kn) + l2 * (c_n * (z - T_i) + dt * zx * kn));
    gTe = l1 * c;
    gTi = l2 * c;
    gB = -l1 * dt * qp.dB;
    gH = -l1 * dt * qp.dH;
    cb[0] = -l1 * dt * qp.sb;
    cse[0] = -l1 * dt * qp.sse;
    cc[0] = (l1 - l2) * dt * zx * kLn2 * kc;
  } else {
    gTe = g_x;    // rates only: T' = T
    gTi = g_z;
  }
  if (g_qr != 0.0 || g_qc != 0.0) {
    const double lte = flog10(T_e), lti = flog10(T_i);
    cp[1] = cool_point(tab, P, lne + lH, lte, lB, c1, c2);
    kp[1] = coul_point(tab, P, lne, lte, lti, k1, k2);
    have[1] = true;
    const QradPartials qp = qrad_partials(cp[1], n_e, T_e, B, H, !cool_off && T_e >= P.T_floor);
    const double kc = fexp2(kp[1].y);
    const double kn = kLn2 * kc * kp[1].dy[0] / (n_e * kLn10);
    const double kx = kLn2 * kc * kp[1].dy[1] / (T_e * kLn10);
    const double kz = kLn2 * kc * kp[1].dy[2] / (T_i * kLn10);
    const double gap = T_i - T_e;
    gn += g_qr * qp.dn + g_qc * gap * kn;
    gTe += g_qr * qp.dx + g_qc * (-kc + gap * kx);
    gTi += g_qc * (kc + gap * kz);
    gB += g_qr * qp.dB;
    gH += g_qr * qp.dH;
    cb[1] = g_qr * qp.sb;
    cse[1] = g_qr * qp.sse;
    cc[1] = g_qc * gap * kLn2 * kc;
  }
  out->n_e = gn;
  out->T_e = gTe;
  out->T_i = gTi;
  out->B = gB;
  out->H = gH;
  if (!want_tables) return;
  if constexpr (Scatter::kRecords != 0) {
    // one record per evaluation point: its table cell, coefficients and
    // fractional coordinates (the corner weights are rebuilt from them)
    for (int p = 0; p < 2; ++p) {
      if (have[p] && (cb[p] != 0.0 || cse[p] != 0.0)) sc.cool_rec(p, cp[p].cell, cb[p], cse[p], cp[p].t);
      if (have[p] && cc[p] != 0.0) sc.coul_rec(p, kp[p].cell, cc[p], kp[p].t);
    }
  } else {
    // cooling tables
    {
      double vb[8], vse[8];
      if (have[0] && have[1] && cp[0].idx[0] == cp[1].idx[0]) {
        if (cb[0] != 0.0 || cse[0] != 0.0 || cb[1] != 0.0 || cse[1] != 0.0) {
          for (int k = 0; k < 8; ++k) {
            vb[k] = cb[0] * cp[0].w[k] + cb[1] * cp[1].w[k];
            vse[k] = cse[0] * cp[0].w[k] + cse[1] * cp[1].w[k];
          }
          sc.cool(cp[0].idx, vb, vse);
        }
      } else {
        for (int p = 0; p < 2; ++p) {
          if (!have[p] || (cb[p] == 0.0 && cse[p] == 0.0)) continue;
          for (int k = 0; k < 8; ++k) {
            vb[k] = cb[p] * cp[p].w[k];
            vse[k] = cse[p] * cp[p].w[k];
          }
          sc.cool(cp[p].idx, vb, vse);
        }
      }
    }
    // Coulomb table
    {
      double vc[8];
      if (have[0] && have[1] && kp[0].idx[0] == kp[1].idx[0]) {
        if (cc[0] != 0.0 || cc[1] != 0.0) {
          for (int k = 0; k < 8; ++k) vc[k] = cc[0] * kp[0].w[k] + cc[1] * kp[1].w[k];
          sc.coul(kp[0].idx, vc);
        }
      } else {
        for (int p = 0; p < 2; ++p) {
          if (!have[p] || cc[p] == 0.0) continue;
          for (int k = 0; k < 8; ++k) vc[k] = cc[p] * kp[p].w[k];
          sc.coul(kp[p].idx, vc);
        }
      }
    }
  }
}

}  // namespace rc
