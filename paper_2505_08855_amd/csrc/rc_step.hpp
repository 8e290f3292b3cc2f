// Per-cell cooling source step, compiled for gfx950 and (for the library's
// host self-tests) for the host CPU from the same source.
//
// Method (arXiv:2505.08855): rates from log2 tables by multilinear
// interpolation (Sec. III.A), thin total Q_thin = Q_brem + eta Q_syn
// (eq. thin_cooling), the Hubeny bridge (eq. total_cooling) written as
// Q_rad = Q_thin / (1 + sqrt3 ta + 1.5 ta (ta + ts)), Coulomb exchange
// Q_cc = (T_i - T_e) v_c (eq. coulomb_collisions), then the energy update of
// Sec. III.B.1 with the floor of Sec. III.B.2:
//
//   backward Euler, u_s = 1.5 n_e k T_s, c = 1.5 n_e k:
//     E1 = c (x - T_e) + dt Q_rad(x) - dt (z - x) v_c(x, z) = 0
//     E2 = c (z - T_i) + dt (z - x) v_c(x, z)               = 0
//   solved as a 2x2 Newton reduced by its Schur complement: for a trial
//   x = T_e' the ion temperature z(x) solves E2 (Newton in z inside the
//   bracket [min(x, T_i), max(x, T_i)]), and the outer residual E1 + E2 is
//   driven to zero by Newton in s = ln x on
//     G(s) = log1p([c (x - T_e) + c (z - T_i) + dt Q_rad(x)] / (c (T_e + T_i))),
//   whose slope uses dz/dx = -(dE2/dx)/(dE2/dz) (the off-diagonal Jacobian
//   blocks).  Every derivative is the exact derivative of the interpolant
//   inside the current table cell.  The iteration starts at x = T_e, moves in
//   the direction the source points and keeps a sign bracket, so it lands on
//   the first root met from the initial state; when the step would cross the
//   temperature floor it probes G at the floor and projects onto it if the
//   cooling is still too strong there.
//
//   explicit: 16 forward-Euler substeps, cooling capped at 30 % of u_e per
//   substep, exchange capped at 30 % of either energy and half the gap.
//
// Corner values are gathered once per table cell: the cooling tables are
// pre-reduced along (N, B), which stay fixed during the solve, to a linear
// function of the T_e weight, and the Coulomb table along n_e to a bilinear
// function of the (T_e, T_i) weights; a new gather happens only when an
// iterate leaves the cached cell.
#pragma once

#include "rc_physics.hpp"

namespace rc {

enum : unsigned char {
  ST_INVALID = 1, ST_CLAMP_COOL = 2, ST_CLAMP_COUL = 4, ST_FLOOR = 8, ST_MAXITER = 16
};
enum { SCHEME_NEWTON = 0, SCHEME_EXPLICIT16 = 1, SCHEME_RATES = 2 };

struct AxisP {
  double lo;
  double inv_d;   // (n - 1) / (hi - lo)
  int n;
};

// Everything a step kernel needs besides the table memory.
struct StepParams {
  AxisP ax[6];          // cooling (N, T_e, B), Coulomb (n_e, T_e, T_i)
  double coef[4][4];    // affine part of each log2 table in node-index space
  double dt, T_floor, tol, ln_lambda;
  int max_iter, scheme;
};

struct Coord {
  int i;
  double t;
  double dfdu;          // df/du, 0 when clamped
  bool clamped;
};

// f = (u - lo) / d, clamped to [0, n-1]; cell i = min(floor f, n - 2), t = f - i
RC_HD Coord axis_coord(double u, const AxisP& a) {
  double f = (u - a.lo) * a.inv_d;
  Coord c;
  c.clamped = !(f >= 0.0 && f <= (double)(a.n - 1));
  c.dfdu = c.clamped ? 0.0 : a.inv_d;
  f = fmin(fmax(f, 0.0), (double)(a.n - 1));
  int i = (int)floor(f);
  if (i > a.n - 2) i = a.n - 2;
  c.i = i;
  c.t = f - (double)i;
  return c;
}

// Table memory in global memory: cooling tables interleaved per node as
// {brem, synch, eta, 0} (one 16-byte load per corner serves all three), the
// Coulomb table planar; both C-ordered [i0][i1][i2].
struct GlobalTab {
  const float4* cool;
  const float* coul;
  int c1, c2;           // cooling n1, n2
  int k1, k2;           // Coulomb n1, n2
  RC_HD float4 cool_at(int i0, int i1, int i2) const { return cool[((long)i0 * c1 + i1) * c2 + i2]; }
  RC_HD float coul_at(int i0, int i1, int i2) const { return coul[((long)i0 * k1 + i1) * k2 + i2]; }
};

struct CellOut {
  double T_e_new, T_i_new, q_rad, q_cc, q_brem, q_syn, eta;
  unsigned char status;
};

template <class Tab>
struct CellSolver {
  const Tab& tab;
  const StepParams& P;
  double n_e, T_e, T_i, B, H;
  double c, S, tau_sca, invH, invH2, dt;
  // cooling: fixed (N, B) coordinates, cached T cell
  Coord cN, cB;
  int iT;
  double A[3], Sl[3];    // y_k(t) = A_k + Sl_k t inside cell iT
  // Coulomb: fixed n_e coordinate, cached (T_e, T_i) cell
  Coord cn;
  int ie, ii;
  double K0, v00, v10, v01, v11;
  // work counters: outer evaluations, inner Newton iterations, table-cell gathers
  int n_outer = 0, n_inner = 0, n_gather = 0;

  RC_HD CellSolver(const Tab& t, const StepParams& p) : tab(t), P(p), iT(-1), ie(-1), ii(-1) {}

  RC_HD void setup(double ne, double te, double ti, double b, double h) {
    n_e = ne; T_e = te; T_i = ti; B = b; H = h;
    dt = P.dt;
    c = kUperNKT * n_e * kKB;
    S = T_e + T_i;
    tau_sca = 2.0 * n_e * kSigmaT * H;
    invH = 1.0 / H;
    invH2 = invH * invH;
    const double lne = log10(n_e);
    cN = axis_coord(lne + log10(H), P.ax[0]);
    cB = axis_coord(log10(B), P.ax[2]);
    cn = axis_coord(lne, P.ax[3]);
    iT = -1;
    ie = -1;
    ii = -1;
  }

  // gather the 8 cooling corners of T cell i and reduce them along (N, B)
  RC_HD void load_cool(int i) {
    iT = i;
    ++n_gather;
    const double wN[2] = {1.0 - cN.t, cN.t};
    const double wB[2] = {1.0 - cB.t, cB.t};
    double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double w = wN[a] * wB[b];
        const float4 p = tab.cool_at(cN.i + a, i, cB.i + b);
        const float4 q = tab.cool_at(cN.i + a, i + 1, cB.i + b);
        lo[0] += w * (double)p.x; lo[1] += w * (double)p.y; lo[2] += w * (double)p.z;
        hi[0] += w * (double)q.x; hi[1] += w * (double)q.y; hi[2] += w * (double)q.z;
      }
    }
    const double fN = cN.i + cN.t, fB = cB.i + cB.t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double* co = P.coef[k];
      A[k] = co[0] + co[1] * fN + co[2] * (double)i + co[3] * fB + lo[k];
      Sl[k] = co[2] + hi[k] - lo[k];
    }
  }

  RC_HD void load_coul(int je, int ji) {
    ++n_gather;
    ie = je;
    ii = ji;
    const double w0 = 1.0 - cn.t, w1 = cn.t;
    v00 = w0 * tab.coul_at(cn.i, je, ji) + w1 * tab.coul_at(cn.i + 1, je, ji);
    v10 = w0 * tab.coul_at(cn.i, je + 1, ji) + w1 * tab.coul_at(cn.i + 1, je + 1, ji);
    v01 = w0 * tab.coul_at(cn.i, je, ji + 1) + w1 * tab.coul_at(cn.i + 1, je, ji + 1);
    v11 = w0 * tab.coul_at(cn.i, je + 1, ji + 1) + w1 * tab.coul_at(cn.i + 1, je + 1, ji + 1);
    const double* co = P.coef[3];
    K0 = co[0] + co[1] * (cn.i + cn.t) + co[2] * (double)je + co[3] * (double)ji;
  }

  // cooling-table log2 values at T = exp(lnx): brem, synch + eta (summed),
  // plus d/dln x of each
  RC_HD void cool_y(double lnx, double* yb, double* yse, double* db, double* dse, Coord* cT) {
    *cT = axis_coord(lnx * (1.0 / kLn10), P.ax[1]);
    if (cT->i != iT) load_cool(cT->i);
    const double t = cT->t;
    *yb = A[0] + Sl[0] * t;
    *yse = A[1] + A[2] + (Sl[1] + Sl[2]) * t;
    const double g = cT->dfdu * (1.0 / kLn10);
    *db = Sl[0] * g;
    *dse = (Sl[1] + Sl[2]) * g;
  }

  // bridged Q_rad at T = x (zero when cooling is off) and dQ_rad/dln x
  RC_HD void q_rad(double x, double lnx, bool on, double* q, double* dq) {
    if (!on) { *q = 0.0; *dq = 0.0; return; }
    double yb, yse, db, dse;
    Coord cT;
    cool_y(lnx, &yb, &yse, &db, &dse, &cT);
    const double vb = exp2(yb) * invH2;
    const double vs = exp2(yse) * invH;
    const double qthin = vb + vs;
    const double dlq = kLn2 * (vb * db + vs * dse) / qthin;
    const double x2 = x * x;
    const double ta = H * qthin / (4.0 * kSigmaSB * x2 * x2);
    const double D = 1.0 + kSqrt3 * ta + 1.5 * ta * (ta + tau_sca);
    *q = qthin / D;
    const double dta = ta * (dlq - 4.0);
    const double dD = (kSqrt3 + 1.5 * (2.0 * ta + tau_sca)) * dta;
    *dq = *q * (dlq - dD / D);
  }

  // Coulomb coefficient v_c(x, z) and its partial derivatives d ln v_c / d ln x, d ln v_c / d ln z
  RC_HD double kcoul(double x, double z, double* dlx, double* dlz, Coord* ce, Coord* ci) {
    *ce = axis_coord(log10(x), P.ax[4]);
    *ci = axis_coord(log10(z), P.ax[5]);
    if (ce->i != ie || ci->i != ii) load_coul(ce->i, ci->i);
    const double te = ce->t, ti = ci->t;
    const double c2 = P.coef[3][2], c3 = P.coef[3][3];
    const double y = K0 + c2 * te + c3 * ti + (1.0 - te) * (1.0 - ti) * v00 + te * (1.0 - ti) * v10 +
                     (1.0 - te) * ti * v01 + te * ti * v11;
    const double dye = c2 + (1.0 - ti) * (v10 - v00) + ti * (v11 - v01);
    const double dyi = c3 + (1.0 - te) * (v01 - v00) + te * (v11 - v10);
    *dlx = kLn2 * dye * ce->dfdu * (1.0 / kLn10);
    *dlz = kLn2 * dyi * ci->dfdu * (1.0 / kLn10);
    return exp2(y);
  }

  // z(x) solving E2; returns z and dz/dx
  RC_HD double solve_z(double x, double zg, double* dzdx, int* iters) {
    double lo = fmin(x, T_i), hi = fmax(x, T_i);
    if (!(hi > lo)) { *dzdx = 1.0; return lo; }
    double z = fmin(fmax(zg, lo), hi);
    double dlx, dlz, K;
    Coord ce, ci;
    for (int it = 0; it < 60; ++it) {
      K = kcoul(x, z, &dlx, &dlz, &ce, &ci);
      const double E = c * (z - T_i) + dt * (z - x) * K;
      if (E == 0.0) break;                  // z is an exact root
      if (E < 0.0) lo = z; else hi = z;
      const double dE = c + dt * K + dt * (z - x) * K * dlz / z;
      const double dz = -E / dE;
      ++*iters;
      ++n_inner;
      // converged: Newton converges quadratically, so after a step below
      // 1e-8 z the remaining error is ~1e-16 z.  Tested before the bracket
      // safeguard, which would reject a step below the bracket end's ulp.
      if (fabs(dz) <= 1e-8 * z) { z += dz; break; }
      double zn = z + dz;
      if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
      z = zn;
      if (hi - lo <= 1e-15 * z) break;
    }
    K = kcoul(x, z, &dlx, &dlz, &ce, &ci);
    const double dEz = c + dt * K + dt * (z - x) * K * dlz / z;
    const double dEx = -dt * K + dt * (z - x) * K * dlx / x;
    *dzdx = -dEx / dEz;
    return z;
  }

  // outer residual G(s) and dG/ds at x = exp(s); z is updated in place
  RC_HD double outer(double s, bool on, double* z, double* dG, int* iters) {
    ++n_outer;
    const double x = exp(s);
    double q, dq, dzdx;
    q_rad(x, s, on, &q, &dq);
    *z = solve_z(x, *z, &dzdx, iters);
    const double numer = c * ((x - T_e) + (*z - T_i)) + dt * q;
    const double P_ = c * S + numer;
    *dG = (c * x * (1.0 + dzdx) + dt * dq) / P_;
    return log1p(numer / (c * S));
  }

  // rates at the input state
  RC_HD void rates(CellOut* o) {
    double yb, yse, db, dse;
    Coord cT;
    cool_y(log(T_e), &yb, &yse, &db, &dse, &cT);
    const double t = cT.t;
    const double yb_ = A[0] + Sl[0] * t, ys_ = A[1] + Sl[1] * t, ye_ = A[2] + Sl[2] * t;
    o->q_brem = exp2(yb_) * invH2;
    o->q_syn = exp2(ys_) * invH;
    o->eta = exp2(ye_);
    const double qthin = o->q_brem + o->eta * o->q_syn;
    const double T2 = T_e * T_e;
    const double ta = H * qthin / (4.0 * kSigmaSB * T2 * T2);
    o->q_rad = (T_e < P.T_floor) ? 0.0 : qthin / (1.0 + kSqrt3 * ta + 1.5 * ta * (ta + tau_sca));
    double dlx, dlz;
    Coord ce, ci;
    const double K = kcoul(T_e, T_i, &dlx, &dlz, &ce, &ci);
    o->q_cc = (T_i - T_e) * K;
    unsigned char st = 0;
    if (cN.clamped || cT.clamped || cB.clamped) st |= ST_CLAMP_COOL;
    if (cn.clamped || ce.clamped || ci.clamped) st |= ST_CLAMP_COUL;
    o->status = st;
  }

  RC_HD void newton(CellOut* o) {
    const double s0 = log(T_e);
    const double sf = log(P.T_floor);
    const double tol = P.tol;
    const double step_tol = sqrt(tol);
    int iters = 0;
    double z = T_i, dG;
    bool on = T_e >= P.T_floor;
    double G = outer(s0, on, &z, &dG, &iters);
    double s = s0;
    unsigned char st = 0;
    if (G == 0.0) { o->T_e_new = T_e; o->T_i_new = z; return; }
    double lo, hi;           // bracket in s with G(lo) < 0 < G(hi)
    bool lo_known, hi_known;
    bool floor_pending = false;
    if (G > 0.0) {
      hi = s0; hi_known = true;
      lo = log(fmin(T_i, P.T_floor)); lo_known = false;
      floor_pending = on && (P.T_floor <= T_i);   // the floor, not T_i, bounds the descent
      if (!floor_pending) lo_known = true;       // G(T_i) < 0 when everything is below the floor
    } else {
      lo = s0; lo_known = true;
      hi = log(T_i); hi_known = true;
      if (T_e < P.T_floor && P.T_floor < T_i) {
        // the floor lies inside the bracket: decide which side holds the root
        double zf = z, dGf;
        const double Gm = outer(sf, false, &zf, &dGf, &iters);
        if (Gm >= 0.0) {
          hi = sf;                              // root below the floor, cooling off
        } else {
          zf = z;
          const double Gp = outer(sf, true, &zf, &dGf, &iters);
          if (Gp >= 0.0) {
            o->T_e_new = P.T_floor; o->T_i_new = zf; o->status |= ST_FLOOR; return;
          }
          lo = sf; s = sf; G = Gp; dG = dGf; z = zf;
        }
      }
    }
    bool done = false;
    for (int it = 0; it < P.max_iter; ++it) {
      double sn = s - G / dG;
      const bool newton_ok = (dG > 0.0) && (sn == sn);
      if (newton_ok && fabs(sn - s) <= step_tol && !(floor_pending && sn < sf)) {
        // converged: Newton converges quadratically, so once the step is below
        // sqrt(tol) the error left after taking it is O(tol).  Tested before
        // the bracket safeguard, which could reject a step below an end's ulp.
        s = sn;
        double dzdx;
        z = solve_z(exp(s), z, &dzdx, &iters);
        done = true;
        break;
      }
      if (floor_pending && newton_ok && sn < sf) {
        // the step would cross the floor: probe G just above it
        floor_pending = false;
        double zf = z, dGf;
        const double Gf = outer(sf, true, &zf, &dGf, &iters);
        if (Gf >= 0.0) {
          o->T_e_new = P.T_floor; o->T_i_new = zf; o->status |= ST_FLOOR; return;
        }
        lo = sf; lo_known = true;
        s = sf; G = Gf; dG = dGf; z = zf;
        continue;
      }
      if (!newton_ok || sn >= hi || sn <= lo || (!lo_known && sn < lo)) {
        sn = lo_known ? 0.5 * (lo + hi) : 0.5 * (lo + s);
      }
      s = sn;
      on = exp(s) >= P.T_floor;
      G = outer(s, on, &z, &dG, &iters);
      if (G > 0.0) { hi = s; hi_known = true; }
      else if (G < 0.0) { lo = s; lo_known = true; }
      else { done = true; break; }
      if (lo_known && hi_known && (hi - lo) <= tol) {
        done = true;
        break;
      }
    }
    if (!done) st |= ST_MAXITER;
    o->T_e_new = exp(s);
    o->T_i_new = z;
    o->status |= st;
  }

  RC_HD void explicit16(CellOut* o) {
    const double h = dt / 16.0;
    double te = T_e, ti = T_i;
    for (int k = 0; k < 16; ++k) {
      double q, dq, dlx, dlz;
      Coord ce, ci;
      q_rad(te, log(te), te >= P.T_floor, &q, &dq);
      const double K = kcoul(te, ti, &dlx, &dlz, &ce, &ci);
      const double qcc = (ti - te) * K;
      const double qr = fmin(q, 0.3 * c * te / h);
      const double lim = fmin(0.5 * c * fabs(ti - te), 0.3 * c * fmin(te, ti)) / h;
      const double qc = fmin(fmax(qcc, -lim), lim);
      const double dte = h * (qc - qr) / c;
      const double dti = -h * qc / c;
      te += dte;
      ti += dti;
    }
    o->T_e_new = te;
    o->T_i_new = ti;
  }
};

RC_HD bool bad_input(double v) { return !(v > 0.0) || !isfinite(v); }

template <class Tab>
RC_HD void cool_cell(const Tab& tab, const StepParams& P, double n_e, double T_e, double T_i, double B,
                     double H, CellOut* o) {
  if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
    const double nan = __builtin_nan("");
    o->T_e_new = o->T_i_new = o->q_rad = o->q_cc = o->q_brem = o->q_syn = o->eta = nan;
    o->status = ST_INVALID;
    return;
  }
  CellSolver<Tab> cs(tab, P);
  cs.setup(n_e, T_e, T_i, B, H);
  cs.rates(o);
  if (P.scheme == SCHEME_NEWTON) {
    cs.newton(o);
  } else if (P.scheme == SCHEME_EXPLICIT16) {
    cs.explicit16(o);
  } else {
    o->T_e_new = T_e;
    o->T_i_new = T_i;
  }
}

// Table-free rates at the input state from the closed forms (DIRECT variant).
RC_HD void direct_rates(const StepParams& P, double n_e, double T_e, double T_i, double B, double H,
                        CellOut* o) {
  if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
    const double nan = __builtin_nan("");
    o->T_e_new = o->T_i_new = o->q_rad = o->q_cc = o->q_brem = o->q_syn = o->eta = nan;
    o->status = ST_INVALID;
    return;
  }
  o->q_brem = n_e * n_e * brem_coeff(T_e);
  const SynchResult sr = synchrotron(n_e, T_e, B, H);
  o->q_syn = exp(sr.ln_q);
  o->eta = exp(ln_eta(n_e, T_e, H, sr.nu_c));
  const double qthin = o->q_brem + o->eta * o->q_syn;
  const double T2 = T_e * T_e;
  const double ta = H * qthin / (4.0 * kSigmaSB * T2 * T2);
  const double ts = 2.0 * n_e * kSigmaT * H;
  o->q_rad = (T_e < P.T_floor) ? 0.0 : qthin / (1.0 + kSqrt3 * ta + 1.5 * ta * (ta + ts));
  o->q_cc = (T_i - T_e) * exp(ln_coulomb_coeff(n_e, T_e, T_i, P.ln_lambda));
  o->T_e_new = T_e;
  o->T_i_new = T_i;
  o->status = 0;
}

}  // namespace rc
