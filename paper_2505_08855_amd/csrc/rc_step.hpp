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
//   blocks).  Each iterate also takes Newton's step on the log-ratio form
//   ln(energy gained) - ln(energy lost) of the electron-ion pair, which has
//   the sign of G, and of the two steps the one that overshoots less is taken
//   (cooling residuals are convex in s, heating ones concave); a long first
//   step goes to the root of a model of the cell instead.  Every derivative is
//   the exact derivative of the interpolant inside the current table cell.  A
//   step below sqrt(tol) that stays in the current cells ends the solve, T_i'
//   following by first-order extrapolation along z(x).  The iteration starts
//   at x = T_e, moves in
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

#include "rc_fastmath.hpp"
#include "rc_physics.hpp"

namespace rc {

enum : unsigned char {
  ST_INVALID = 1, ST_CLAMP_COOL = 2, ST_CLAMP_COUL = 4, ST_FLOOR = 8, ST_MAXITER = 16, ST_GAS_FLOOR = 32,
  ST_NO_RATE = 64
};

// Electron floor of a cell whose cooling is switched off for the step (its
// input gas temperature lies below the gas-temperature floor): above every
// temperature, so Q_rad is zero along the whole solve.
constexpr double kNoCoolingFloor = 1e300;
constexpr double kLnNoCoolingFloor = 690.7755278982137;    // ln 1e300
enum { SCHEME_NEWTON = 0, SCHEME_EXPLICIT16 = 1, SCHEME_RATES = 2 };

struct AxisP {
  double lo;
  double inv_d;   // (n - 1) / (hi - lo)
  int n;
};

// Geometry of a table set: fixed per table handle, kept in device memory (a
// host copy serves the host self-tests) so that kernels read it through the
// scalar cache instead of holding it in registers.
struct TableGeom {
  AxisP ax[6];          // cooling (N, T_e, B), Coulomb (n_e, T_e, T_i)
  double coef[4][4];    // affine part of each log2 table in node-index space
  double coef_se[4];    // coef[1] + coef[2]: the synchrotron and eta tables enter as a sum
  int same_te;          // the cooling and Coulomb T_e axes coincide (one coordinate serves both)
};

// Everything a step kernel needs besides the table memory.
struct StepParams {
  const TableGeom* g;
  double dt, T_floor, tol, ln_lambda;
  double ln_T_floor, sqrt_tol;   // log(T_floor), sqrt(tol)
  int max_iter, scheme;
  int compton_literal, theta_i_me;   // readings of the table set (used by the closed forms)
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
//
// The solver reads the cooling tables as two quantities per corner: brem and
// se = log2(Q_syn eta), the synchrotron and Compton tables summed (they enter
// the rates only as a product).  se's stored residual is the single-precision
// sum of the two stored residuals (one IEEE addition, rounded to nearest), its
// affine part the sum of theirs; every accessor forms it the same way, and
// the cell-blocked copy stores it.
RC_HD float2 brem_se(const float4& p) { return make_float2(p.x, p.y + p.z); }

// the 8 corners of the table cell with lowest corner (i0, i1, i2) through an
// accessor's single-node reads, corner (a, b, c) at a * 4 + b * 2 + c
template <class T>
RC_HD void corners8(const T& t, int i0, int i1, int i2, float4 (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = t.cool_at(i0 + (k >> 2), i1 + ((k >> 1) & 1), i2 + (k & 1));
}

// the same as {brem, se} pairs
template <class T>
RC_HD void corners8se(const T& t, int i0, int i1, int i2, float2 (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = brem_se(t.cool_at(i0 + (k >> 2), i1 + ((k >> 1) & 1), i2 + (k & 1)));
}

template <class T>
RC_HD void corners8c(const T& t, int i0, int i1, int i2, float (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = t.coul_at(i0 + (k >> 2), i1 + ((k >> 1) & 1), i2 + (k & 1));
}

struct GlobalTab {
  const float4* cool;
  const float* coul;
  int c1, c2;           // cooling n1, n2
  int k1, k2;           // Coulomb n1, n2
  RC_HD float4 cool_at(int i0, int i1, int i2) const { return cool[((long)i0 * c1 + i1) * c2 + i2]; }
  RC_HD float coul_at(int i0, int i1, int i2) const { return coul[((long)i0 * k1 + i1) * k2 + i2]; }
  RC_HD void cool8(int i0, int i1, int i2, float2 (&v)[8]) const { corners8se(*this, i0, i1, i2, v); }
  RC_HD void coul8(int i0, int i1, int i2, float (&v)[8]) const { corners8c(*this, i0, i1, i2, v); }
};

// bfloat16 bits -> float (exact: bfloat16 is the upper half of a binary32)
RC_HD float bf16_to_float(unsigned v) { return __builtin_bit_cast(float, v << 16); }

// The same tables stored as bfloat16 residuals (storage-precision
// experiment): 8 bytes per cooling node {brem, synch, eta, 0}, 2 bytes per
// Coulomb node.  Widened to float on load; the arithmetic after that is the
// FP32-storage path's.
struct GlobalTabBF16 {
  const uint2* cool;
  const unsigned short* coul;
  int c1, c2;
  int k1, k2;
  RC_HD float4 cool_at(int i0, int i1, int i2) const {
    const uint2 p = cool[((long)i0 * c1 + i1) * c2 + i2];
    return make_float4(bf16_to_float(p.x & 0xffffu), bf16_to_float(p.x >> 16), bf16_to_float(p.y & 0xffffu), 0.0f);
  }
  RC_HD float coul_at(int i0, int i1, int i2) const { return bf16_to_float(coul[((long)i0 * k1 + i1) * k2 + i2]); }
  RC_HD void cool8(int i0, int i1, int i2, float2 (&v)[8]) const { corners8se(*this, i0, i1, i2, v); }
  RC_HD void coul8(int i0, int i1, int i2, float (&v)[8]) const { corners8c(*this, i0, i1, i2, v); }
};

// The FP32 tables with a cell-blocked copy: the 8 corners of every table cell
// stored together, corner (a, b, c) at a * 4 + b * 2 + c (cooling: 8 {brem,
// se} pairs, 64 bytes, one aligned 64-byte block; Coulomb: 8 floats, 32
// bytes).  A corner gather then touches one block instead of four pairs of
// nodes, for 4 times the cooling and 8 times the Coulomb table memory.  The
// node layout stays for the single-corner reads.
struct CellTab {
  const float4* cool;
  const float* coul;
  const float2* cool_cells;
  const float* coul_cells;
  int c1, c2;
  int k1, k2;
  RC_HD float4 cool_at(int i0, int i1, int i2) const { return cool[((long)i0 * c1 + i1) * c2 + i2]; }
  RC_HD float coul_at(int i0, int i1, int i2) const { return coul[((long)i0 * k1 + i1) * k2 + i2]; }
  RC_HD void cool8(int i0, int i1, int i2, float2 (&v)[8]) const {
    const float2* p = cool_cells + (((long)i0 * (c1 - 1) + i1) * (c2 - 1) + i2) * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[k];
  }
  RC_HD void coul8(int i0, int i1, int i2, float (&v)[8]) const {
    const float* p = coul_cells + (((long)i0 * (k1 - 1) + i1) * (k2 - 1) + i2) * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[k];
  }
};

struct CellOut {
  double T_e_new, T_i_new, q_rad, q_cc, q_brem, q_syn, eta;
  unsigned char status;
};

// Iteration state of the backward-Euler Newton solve: current iterate s =
// ln T_e' with its residual G and slope dG, the ion temperature z solved
// there, the sign bracket [lo, hi] in s, the pending evaluation point
// (kind, se, xe) and flags.
struct NewtonState {
  double s, G, dG, z, lo, hi, se, xe, z_floor;
  int kind, iters, flags;
};

// The part of NewtonState a cell still needs after its first round when that
// round did not finish it: the first round leaves the iterate at s0 = ln T_e,
// z_floor at T_i and the round count at 0, and the pending point's
// temperature follows from se and the kind, so 56 bytes resume the solve
// exactly where it stopped.
struct NewtonResume {
  double G, dG, z, lo, hi, se;
  int kind_flags;       // kind | flags << 3
  int pad;
};

// Number of difficulty classes of unfinished cells (see CellSolver::resume_class).
constexpr int kResumeClasses = 16;

// the table coordinates that stay fixed during a cell's solve: N and B of the
// cooling tables, n_e of the Coulomb table
struct FixedCoords {
  Coord N, B, n;
};

RC_HD FixedCoords fixed_coords(const StepParams& P, double n_e, double b, double h, double* lh10 = nullptr) {
  const double lne = flog10(n_e);
  const double lh = flog10(h);
  if (lh10) *lh10 = lh;
  return {axis_coord(lne + lh, P.g->ax[0]), axis_coord(flog10(b), P.g->ax[2]), axis_coord(lne, P.g->ax[3])};
}

// The inner solve's last evaluation point: its T_i coordinate t (with the
// clamp flag) and 1 / z there.
struct ZLast {
  double t, iz;
  bool clamped;
};

template <class Tab>
struct CellSolver {
  const Tab& tab;
  const StepParams& P;
  // per-cell constants (dt is per cell so that batched work items can carry their own);
  // lH = log2 H, folded into the cached cooling exponents (Q_brem = v_b / H^2,
  // Q_syn = v_s / H)
  double T_e, T_i, H, c, tau_sca, lH, dt;
  // gather coordinates that stay fixed during the solve
  int iN, iB, in_;
  double tN, tB, tn;
  // cooling cache inside T cell iT: log2 v_brem = Ab + Sb t, log2(v_synch v_eta) = Ase + Sse t
  int iT;
  double Ab, Ase, Sb, Sse;
  // Coulomb cache inside cell (ie, ii): log2 v_c = C0 + C1 te + C2 ti + C3 te ti
  // (the affine part plus the bilinear interpolant, expanded in te and ti)
  int ie, ii;
  double C0, C1, C2, C3;
  unsigned char clamp;
  bool cool_off;        // radiative cooling switched off for this cell (gas-temperature floor)
  double lnTi;          // ln T_i; read only where the solve starts (newton_begin)

  RC_HD CellSolver(const Tab& t, const StepParams& p) : tab(t), P(p) {}

  // electron temperature floor of this cell and its logarithm
  RC_HD double Tf() const { return cool_off ? kNoCoolingFloor : P.T_floor; }
  RC_HD double lnTf() const { return cool_off ? kLnNoCoolingFloor : P.ln_T_floor; }

  // per-cell constants and fixed coordinates; returns s0 = ln T_e.  A cell
  // whose gas temperature T_e + T_i lies below floor_gas (0 = none) has no
  // radiative cooling this step.
  RC_HD double setup(double n_e, double te, double ti, double b, double h, double dt_, double floor_gas = 0.0) {
    dt = dt_;
    cool_off = te + ti < floor_gas;
    T_e = te;
    T_i = ti;
    H = h;
    c = kUperNKT * n_e * kKB;
    tau_sca = 2.0 * n_e * kSigmaT * h;
    double lh10;
    const FixedCoords f = fixed_coords(P, n_e, b, h, &lh10);
    lH = lh10 * kLog2_10;
    const Coord &cN = f.N, &cB = f.B, &cn = f.n;
    iN = cN.i; tN = cN.t;
    iB = cB.i; tB = cB.t;
    in_ = cn.i; tn = cn.t;
    const double s0 = flog(te);
    const double lte = s0 * (1.0 / kLn10);
    lnTi = flog(ti);
    clamp = cool_off ? ST_GAS_FLOOR : 0;
    if (cN.clamped || cB.clamped || axis_coord(lte, P.g->ax[1]).clamped) clamp |= ST_CLAMP_COOL;
    if (cn.clamped || axis_coord(lte, P.g->ax[4]).clamped || axis_coord(lnTi * kInvLn10, P.g->ax[5]).clamped)
      clamp |= ST_CLAMP_COUL;
    iT = ie = ii = -1;
    return s0;
  }

  // gather the 8 cooling corners of T cell i and reduce them along (N, B)
  RC_HD void load_cool(int i) {
    iT = i;
    const double wN[2] = {1.0 - tN, tN};
    const double wB[2] = {1.0 - tB, tB};
    double lb = 0.0, lse = 0.0, hb = 0.0, hse = 0.0;
    float2 v[8];
    tab.cool8(iN, i, iB, v);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double w = wN[a] * wB[b];
        const float2 p = v[a * 4 + b];
        const float2 q = v[a * 4 + 2 + b];
        lb += w * (double)p.x;
        lse += w * (double)p.y;
        hb += w * (double)q.x;
        hse += w * (double)q.y;
      }
    }
    const double fN = iN + tN, fB = iB + tB;
    const double* cb = P.g->coef[0];
    const double* cse = P.g->coef_se;
    Ab = cb[0] + cb[1] * fN + cb[2] * (double)i + cb[3] * fB + lb - 2.0 * lH;
    Sb = cb[2] + hb - lb;
    Ase = cse[0] + cse[1] * fN + cse[2] * (double)i + cse[3] * fB + lse - lH;
    Sse = cse[2] + hse - lse;
  }

  RC_HD void load_coul(int je, int ji) {
    ie = je;
    ii = ji;
    const double w0 = 1.0 - tn, w1 = tn;
    float v[8];
    tab.coul8(in_, je, ji, v);
    const double v00 = w0 * v[0] + w1 * v[4];
    const double v10 = w0 * v[2] + w1 * v[6];
    const double v01 = w0 * v[1] + w1 * v[5];
    const double v11 = w0 * v[3] + w1 * v[7];
    const double* co = P.g->coef[3];
    C0 = co[0] + co[1] * (in_ + tn) + co[2] * (double)je + co[3] * (double)ji + v00;
    C1 = co[2] + (v10 - v00);
    C2 = co[3] + (v01 - v00);
    C3 = (v11 - v10) - (v01 - v00);
  }

  // Corner gathers of one evaluation at T_e = x (cooling coordinate cT,
  // Coulomb coordinate ce) and T_i = z (coordinate ci).  When either cached
  // cell no longer contains the point both tables are re-read in one block,
  // so that all their loads are in flight together and a re-gather costs one
  // memory latency, not two; the table whose cell did not change re-reads
  // lines that are already cached.  With the default axes the two T_e axes
  // coincide and both cells change together anyway.
  RC_HD void gather(const Coord& cT, const Coord& ce, const Coord& ci, bool cool_needed) {
    if ((cool_needed && cT.i != iT) || ce.i != ie || ci.i != ii) {
      load_cool(cT.i);
      load_coul(ce.i, ci.i);
    }
  }

  // bridged Q_rad at T = x (cooling coordinate cT, its cell gathered; zero
  // when cooling is off) and dQ_rad/dln x
  RC_HD void q_rad(double x, const Coord& cT, bool on, double* q, double* dq) {
    if (!on) { *q = 0.0; *dq = 0.0; return; }
    const double t = cT.t;
    const double g = cT.dfdu * (1.0 / kLn10);       // d t / d ln x
    const double vb = fexp2(Ab + Sb * t);            // Q_brem
    const double vs = fexp2(Ase + Sse * t);          // eta Q_syn
    const double qthin = vb + vs;
    const double dlq = kLn2 * g * fdiv_d(vb * Sb + vs * Sse, qthin);
    const double x2 = x * x;
    const double ta = fdiv(H * qthin, 4.0 * kSigmaSB * x2 * x2);
    const double D = 1.0 + kSqrt3 * ta + 1.5 * ta * (ta + tau_sca);
    const double iD = fdiv(1.0, D);
    *q = qthin * iD;
    const double dD = (kSqrt3 + 1.5 * (2.0 * ta + tau_sca)) * ta * (dlq - 4.0);
    *dq = *q * (dlq - dD * iD);
  }

  // Coulomb coefficient v_c at (T_e coordinate ce, T_i coordinate ci, cell
  // gathered) and the partial derivatives d ln v_c / d ln T_e, d ln v_c / d ln T_i
  RC_HD double kcoul_at(const Coord& ce, const Coord& ci, double* dlx, double* dlz) const {
    const double te = ce.t, ti = ci.t;
    const double dye = C1 + C3 * ti;          // d log2 v_c / d te
    const double dyi = C2 + C3 * te;          // d log2 v_c / d ti
    const double y = C0 + C1 * te + dyi * ti;
    *dlx = kLn2 * dye * ce.dfdu * (1.0 / kLn10);
    *dlz = kLn2 * dyi * ci.dfdu * (1.0 / kLn10);
    return fexp2(y);
  }

  // the same at T_i = z, gathering the Coulomb cell if z left the cached one
  RC_HD double kcoul(const Coord& ce, double z, double* dlx, double* dlz, Coord* ci_out) {
    const Coord ci = axis_coord(flog10(z), P.g->ax[5]);
    if (ce.i != ie || ci.i != ii) load_coul(ce.i, ci.i);
    *ci_out = ci;
    return kcoul_at(ce, ci, dlx, dlz);
  }

  // z(x) solving E2 = c (z - T_i) + dt (z - x) v_c(x, z) = 0 inside
  // [min(x, T_i), max(x, T_i)], where E2 changes sign; returns z and dz/dx.
  // z0 is the first trial z, already inside that interval, with its Coulomb
  // coordinate ci0 (cell gathered); *K_first receives v_c there.  *zl
  // receives the last evaluation point's T_i coordinate and 1 / z there
  // (the Coulomb cell cached on return is that point's).
  RC_HD double solve_z(double x, const Coord& ce, double z0, const Coord& ci0, double* dzdx, double* K_first,
                       ZLast* zl) {
    double lo = fmin(x, T_i), hi = fmax(x, T_i);
    double z = z0;
    double K = 0.0, dlx = 0.0, dlz = 0.0;
    Coord cz = ci0;
    if (!(hi > lo)) {
      // x == T_i: z = T_i solves E2; implicit derivative dz/dx = dt K / (c + dt K)
      K = kcoul_at(ce, ci0, &dlx, &dlz);
      if (K_first) *K_first = K;
      *dzdx = fdiv_d(dt * K, c + dt * K);
      zl->t = ci0.t; zl->iz = fdiv_d(1.0, lo); zl->clamped = ci0.clamped;
      return lo;
    }
    double dEz = c, iz = 0.0;
    for (int it = 0; it < 60; ++it) {
      K = it == 0 ? kcoul_at(ce, ci0, &dlx, &dlz) : kcoul(ce, z, &dlx, &dlz, &cz);
      if (it == 0 && K_first) *K_first = K;
      const double E = c * (z - T_i) + dt * (z - x) * K;
      iz = fdiv_d(1.0, z);
      const double Kz = K * dlz * iz;         // d v_c / dz
      dEz = c + dt * K + dt * (z - x) * Kz;
      if (E == 0.0) break;                  // z is an exact root
      if (E < 0.0) lo = z; else hi = z;
      // Chebyshev's third-order step.  Inside one Coulomb cell ln v_c is
      // linear in ln z (the interpolant is bilinear in the log coordinates),
      // so v_c'' = v_c' (dlz - 1) / z and E2'' = dt (2 v_c' + (z - x) v_c'')
      // exactly; with the Newton step -r, r = E2 / E2', the step is
      // -r (1 + r E2'' / (2 E2')), kept as Newton's where that correction
      // exceeds one half (strong curvature: the bracket then decides).
      // (Halley's form, -r / (1 - r E2'' / (2 E2')), takes the same number
      // of passes and one division more.)
      const double iE = fdiv_d(1.0, dEz);
      const double r = E * iE;
      const double d2E = dt * Kz * (2.0 + (z - x) * (dlz - 1.0) * iz);
      const double a = 0.5 * r * d2E * iE;
      const double dz = fabs(a) < 0.5 ? -r * (1.0 + a) : -r;
      // converged: the iteration converges cubically, so after a step below
      // 1e-4 z the remaining error is of order 1e-12 z (a host count over
      // 262,144 iid cells against Newton's iteration stopped at 1e-6 z:
      // 8.01 instead of 9.53 inner passes per wavefront, T_e' moving by at
      // most 1.5e-12 and T_i' by 2e-14, the largest distance from the
      // oracle's solution unchanged at 1.2e-11).  A last step that crosses
      // into another Coulomb cell leaves z outside the cell the solve
      // evaluated, which the outer convergence test rejects.  Tested before
      // the bracket safeguard, which would reject a step below the bracket
      // end's ulp.
      if (fabs(dz) <= 1e-4 * z) { z += dz; break; }
      double zn = z + dz;
      if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
      z = zn;
      if (hi - lo <= 1e-15 * z) break;
    }
    const double dEx = -dt * K + dt * (z - x) * K * fdiv_d(dlx, x);
    *dzdx = -fdiv_d(dEx, dEz);
    zl->t = cz.t; zl->iz = iz; zl->clamped = cz.clamped;
    return z;
  }

  // Outer residual G = log1p([c (x - T_e) + c (z - T_i) + dt Q_rad(x)] / (c (T_e + T_i)))
  // at x = exp(s), with its slope dG/ds, Q_rad(x), v_c at the warm start and
  // dz/dx; *ds3 receives a second step proposal, or NaN:
  //  * mode 1 (an iterate): the Newton step of the log-ratio form
  //      G3 = ln Pg - ln Ng,
  //    Pg = dt Q_rad + c (x - T_e)+ + c (z - T_i)+,  Ng = c (T_e - x)+ + c (T_i - z)+,
  //    the energy gained and lost by the electron-ion pair; G3 has the sign
  //    of G.  Why: where numer / cS is small G is close to numer / cS, a steep
  //    exponential of s when radiation dominates, and Newton on G creeps; ln Pg
  //    and ln Ng are close to linear in s away from x = T_e.
  //  * mode 2 (the first evaluation): the root of a model of the cell.  A
  //    cooling cell (G > 0): power-law cooling of the slope at T_e against
  //    the exchange terms linear in x,
  //      ln(dt q) + p d = ln(A (1 - e^d) + R0),  d = s' - s,
  //    A = c T_e (1 + dz/dx), R0 = c (T_i - z).  A heating cell (G < 0): the
  //    electrons' gain against a power law in x of the ion transfer (below).
  //    Solved in single precision by kHeatSteps / kCoolSteps Newton steps on
  //    the model from the Newton step of G: it is only a proposal, and the
  //    safeguards of the driver still apply.  (A host count over 262,144 iid
  //    cells and over the spherical profile: 5 and 4 model steps give the same
  //    round counts as 1 and 2, so the model's own root need not be reached.)
  static constexpr int kHeatSteps = 1, kCoolSteps = 2;
  RC_HD double outer(double s, double x, bool on, int mode, double lnTi_first, double* z, double* dG,
                     double* q_out, double* K_first, double* dzdx_out, double* ds3, ZLast* zl) {
    const double lx = s * (1.0 / kLn10);
    double q, dq, dzdx;
    const Coord cT = axis_coord(lx, P.g->ax[1]);
    const Coord ce = P.g->same_te ? cT : axis_coord(lx, P.g->ax[4]);
    const double z0 = fmin(fmax(*z, fmin(x, T_i)), fmax(x, T_i));
    // the first evaluation (x = T_e) starts the inner solve at z0 = T_i,
    // whose logarithm the caller passes
    double lz0;
    if (mode == 2) lz0 = lnTi_first * kInvLn10;
    else lz0 = flog10(z0);
    const Coord ci = axis_coord(lz0, P.g->ax[5]);
    gather(cT, ce, ci, on);
    q_rad(x, cT, on, &q, &dq);
    *z = solve_z(x, ce, z0, ci, &dzdx, K_first, zl);
    const double numer = c * ((x - T_e) + (*z - T_i)) + dt * q;
    const double cx = c * x * (1.0 + dzdx);
    const double cS = c * (T_e + T_i);
    *dG = fdiv_d(cx + dt * dq, cS + numer);
    *q_out = q;
    *dzdx_out = dzdx;
    *ds3 = __builtin_nan("");
    const double G = flog1p(fdiv_d(numer, cS));
    if (mode == 1) {
      const double cxz = c * x * dzdx;
      double Pg = dt * q, Ng = 0.0, dP = dt * dq, dN = 0.0;
      if (x > T_e) { Pg += c * (x - T_e); dP += c * x; } else { Ng += c * (T_e - x); dN -= c * x; }
      if (*z > T_i) { Pg += c * (*z - T_i); dP += cxz; } else { Ng += c * (T_i - *z); dN -= cxz; }
      if (Pg > 0.0 && Ng > 0.0) {
        // 1 / Ng to full precision: near the root Pg / Ng is close to 1 and
        // its logarithm is the step
        const double iP = fdiv_d(1.0, Pg), iN = fdiv(1.0, Ng);
        const double dG3 = dP * iP - dN * iN;
        if (dG3 > 0.0) *ds3 = -fdiv_d(flog(Pg * iN), dG3);
      }
    } else if (mode == 2 && numer < 0.0 && *dG > 0.0 && *z < T_i) {
      // first step of a heating cell: the electrons' gain
      //   c T_e (e^d - 1) + dt q e^(p d)
      // against the ion transfer N0 e^(b0 d), both slopes taken at T_e; in
      // base 2 and relative to N0 = c (T_i - z):
      //   f(u) = log2(a (2^u - 1) + r 2^(p u)) - b0 u
      const double N0 = c * (T_i - *z);
      const double iN0 = fdiv_sp(1.0, N0);
      const float a = (float)(c * x * iN0), r = (float)(dt * q * iN0);
      const float p = q > 0.0 ? (float)fdiv_sp(dq, q) : 0.0f;
      const float b0 = (float)(-c * x * dzdx * iN0);
      float u = (float)fdiv_sp(-G, *dG * kLn2);
      for (int k = 0; k < kHeatSteps; ++k) {
        const float e = fexp2_sp(u), eq = fexp2_sp(p * u);
        const float Pn = a * (e - 1.0f) + r * eq;
        const float un = u - (flog2_sp(Pn) - b0 * u) * frcp_sp((a * e + p * r * eq) * frcp_sp(Pn) - b0);
        u = un > 0.0f ? un : 0.5f * u;
      }
      *ds3 = (double)u * kLn2;
    } else if (mode == 2 && numer > 0.0 && q > 0.0 && *dG > 0.0) {
      // in base 2: u = d / ln 2, f(u) = L + p u - log2(1 - 2^u + r0),
      // L = log2(dt q / A), r0 = R0 / A
      const double icx = fdiv_sp(1.0, cx);
      const float p = (float)fdiv_sp(dq, q);
      const float L = flog2_sp((float)(dt * q * icx));
      const float r0 = (float)(c * (T_i - *z) * icx);
      float u = (float)fdiv_sp(-G, *dG * kLn2);
      for (int k = 0; k < kCoolSteps; ++k) {
        const float e = fexp2_sp(u);
        const float R = (1.0f - e) + r0;
        const float un = u - (L + p * u - flog2_sp(R)) * frcp_sp(p + e * frcp_sp(R));
        u = un < 0.0f ? un : 0.5f * u;
      }
      *ds3 = (double)u * kLn2;
    }
    return G;
  }

  // Newton driver.  Every evaluation of the outer residual goes through one
  // call site (newton_round: evaluate at the pending point, then choose the
  // next one), so the inlined rate code exists once in the kernel; the whole
  // iteration state lives in NewtonState, separate from the cell's constants.
  enum { FIRST = 0, ITER = 1, PROBE_ON = 2, PROBE_OFF = 3, DONE = 4 };
  static constexpr double kModelMinStep = 0.01;   // in ln T_e
  enum { F_LO_KNOWN = 1, F_FLOOR_PENDING = 2, F_HEATING = 4, F_ON = 8 };

  RC_HD void newton_begin(double s0, NewtonState& ns) const {
    ns.s = s0; ns.G = 0.0; ns.dG = 1.0; ns.z = T_i;
    // until the first round sets the bracket, hi carries ln T_i: the first
    // inner solve starts at z = T_i and the bracket ends are logarithms of
    // T_i (or of the floor), so one logarithm serves all three
    ns.lo = 0.0; ns.hi = lnTi;
    ns.z_floor = T_i;
    ns.kind = FIRST; ns.iters = 0;
    ns.se = s0; ns.xe = T_e;
    ns.flags = (T_e >= Tf()) ? F_ON : 0;
  }

  // one evaluation at the pending point; returns true when the cell is done
  // (T_e_new, T_i_new and the FLOOR / MAXITER bits are then in o)
  RC_HD bool newton_round(NewtonState& ns, CellOut* o) {
    const double T_floor = Tf();
    const double sf = lnTf();
    const double tol = P.tol;
    // The loop runs once per evaluation; a converged step loops back to the
    // DONE exit so that every exit of a converging cell shares one path.
    for (;;) {
    const int kind = ns.kind;
    if (kind == DONE) {
      o->T_e_new = ns.xe;
      o->T_i_new = ns.z;
      return true;
    }
    const int mode = kind == ITER ? 1 : kind == FIRST ? 2 : 0;
    double ze = ns.z, dGe, q, Kf, dzdx_e, ds3;
    ZLast zl;
    const double Ge = outer(ns.se, ns.xe, (ns.flags & F_ON) != 0, mode, ns.hi, &ze, &dGe, &q, &Kf, &dzdx_e, &ds3, &zl);
    bool propose = false;
    // dz/dx at the iterate when this round's evaluation became the iterate;
    // 0 otherwise (the next inner solve then starts from z unchanged)
    double dzdx = 0.0;
    if (kind == FIRST) {
      o->q_rad = q;
      o->q_cc = (T_i - T_e) * Kf;
      ns.G = Ge; ns.dG = dGe; ns.z = ze; dzdx = dzdx_e;
      if (ns.G == 0.0) { o->T_e_new = T_e; o->T_i_new = ze; return true; }
      const bool on0 = (ns.flags & F_ON) != 0;
      if (ns.G > 0.0) {
        ns.lo = fmin(ns.hi, sf);               // ln min(T_i, T_floor)
        ns.hi = ns.s;
        if (on0) ns.flags |= F_FLOOR_PENDING;
        else ns.flags |= F_LO_KNOWN;          // below the floor G(T_i) < 0 is guaranteed
        propose = true;
      } else {
        ns.flags |= F_HEATING | F_LO_KNOWN;
        ns.lo = ns.s;                          // hi = ln T_i: G(T_i) >= 0
        if (T_e < T_floor && T_floor < T_i) {
          // the floor lies inside the bracket: probe it with cooling off first
          ns.kind = PROBE_OFF; ns.se = sf; ns.xe = T_floor; ns.flags &= ~F_ON;
        } else {
          propose = true;
        }
      }
    } else if (kind == PROBE_ON) {
      ns.z_floor = ze;
      if (Ge < 0.0) {                          // root above the floor
        ns.lo = sf; ns.flags |= F_LO_KNOWN;
        ns.s = sf; ns.G = Ge; ns.dG = dGe; ns.z = ze; dzdx = dzdx_e;
        propose = true;
      } else if (!(ns.flags & F_HEATING) && T_i < T_floor) {
        // the root can also lie under the floor, where cooling is off
        ns.kind = PROBE_OFF; ns.se = sf; ns.xe = T_floor; ns.flags &= ~F_ON;
      } else {
        o->T_e_new = T_floor; o->T_i_new = ze; o->status |= ST_FLOOR;
        return true;
      }
    } else if (kind == PROBE_OFF) {
      if (ns.flags & F_HEATING) {
        if (Ge >= 0.0) {                       // root below the floor, cooling off
          ns.hi = sf;
          propose = true;
        } else {
          ns.kind = PROBE_ON; ns.se = sf; ns.xe = T_floor; ns.flags |= F_ON;
        }
      } else if (Ge > 0.0) {                   // descent continues under the floor
        ns.hi = sf; ns.lo = flog(T_i); ns.flags |= F_LO_KNOWN;
        ns.s = sf; ns.G = Ge; ns.dG = dGe; ns.z = ze; dzdx = dzdx_e;
        propose = true;
      } else {
        o->T_e_new = T_floor; o->T_i_new = ns.z_floor; o->status |= ST_FLOOR;
        return true;
      }
    } else {  // ITER
      ns.s = ns.se; ns.G = Ge; ns.dG = dGe; ns.z = ze; dzdx = dzdx_e;
      if (ns.G > 0.0) ns.hi = ns.s;
      else if (ns.G < 0.0) { ns.lo = ns.s; ns.flags |= F_LO_KNOWN; }
      if (ns.G == 0.0 || ((ns.flags & F_LO_KNOWN) && (ns.hi - ns.lo) <= tol)) {
        o->T_e_new = ns.xe; o->T_i_new = ze;
        return true;
      }
      if (++ns.iters >= P.max_iter) {
        o->status |= ST_MAXITER;
        o->T_e_new = ns.xe; o->T_i_new = ze;
        return true;
      }
      propose = true;
    }
    if (!propose) return false;
    {
      const double s = ns.s, lo = ns.lo, hi = ns.hi;
      const bool lo_known = (ns.flags & F_LO_KNOWN) != 0;
      const bool floor_pending = (ns.flags & F_FLOOR_PENDING) != 0;
      // Choice between the two proposals.  A long first step takes the model
      // root.  On an iterate both Newton steps point at the
      // root; G and G3 are convex in s on a cooling cell (radiative loss grows
      // faster than exponentially in s near the root) and concave on a heating
      // cell (the Coulomb gain falls with T_e), so of two Newton steps the one
      // that overshoots less -- the longer on the convex side above the root,
      // the shorter below it, and the reverse for concave -- is the closer.
      const bool use3 = (ds3 == ds3);
      const double dsG = -fdiv_d(ns.G, ns.dG);
      double sn = s + dsG;
      if (use3) {
        // the model root is a single-precision estimate: taken only for a
        // long first step, never as the converged one
        if (kind == FIRST) sn = fabs(dsG) > kModelMinStep ? s + ds3 : sn;
        else if (!(ns.dG > 0.0)) sn = s + ds3;
        else sn = s + ((ns.flags & F_HEATING) ? fmax(ds3, dsG) : fmin(ds3, dsG));
      }
      const bool newton_ok = (use3 || ns.dG > 0.0) && (sn == sn);
      const bool small = newton_ok && fabs(sn - s) <= P.sqrt_tol && !(floor_pending && sn < sf);
      // bracket safeguard: a step outside the bracket, or no usable step,
      // becomes the bisection point (a small step is tested for convergence
      // before the safeguard, which could reject a step below an end's ulp)
      const bool bad = !newton_ok || sn >= hi || (lo_known ? sn <= lo : sn < lo);
      const double s_mid = lo_known ? 0.5 * (lo + hi) : 0.5 * (lo + s);
      double s_next = (small || !bad) ? sn : s_mid;
      // the next iterate's temperature, computed once for every lane
      double xn = fexp(s_next);
      if (small) {
        // converged: Newton converges quadratically, so once the step is
        // below sqrt(tol) the error left after taking it is O(tol) -- provided
        // the step stays inside the table cells of the current iterate (the
        // interpolant is smooth inside a cell; across a node its slope jumps
        // and the step's error is first order in the jump).  T_i' is the
        // first-order extrapolation z + dz/dx (x' - x) along the solution
        // curve z(x) of the ion equation, whose error is second order in
        // x' - x, so O(tol) too, under the same condition on the Coulomb
        // cells.
        const double zn = ns.z + dzdx * (xn - ns.xe);
        const double lxn = sn * (1.0 / kLn10);
        const int jT = axis_coord(lxn, P.g->ax[1]).i;
        const int je = P.g->same_te ? jT : axis_coord(lxn, P.g->ax[4]).i;
        // T_i cell of zn against the cached one, from the last inner
        // evaluation's coordinate t at z_l: with u = zn / z_l - 1 the new
        // coordinate is t + (dt/d ln z) ln(1 + u), and u (1 + 2|u|) <=
        // ln(1 + u) <= u for |u| <= 1/2, so the test is conservative (a
        // point next to a cell edge may take one more round).  A clamped
        // coordinate takes the exact test.
        bool same_ti;
        if (zl.clamped) {
          same_ti = axis_coord(flog10(zn), P.g->ax[5]).i == ii;
        } else {
          const double u = fma(zn, zl.iz, -1.0);
          const double au = fabs(u), dtdl = P.g->ax[5].inv_d * kInvLn10;
          same_ti = au < 0.25 && zl.t + dtdl * fmin(u, 0.0) * (1.0 + 2.0 * au) >= 0.0 &&
                    zl.t + dtdl * fmax(u, 0.0) < 1.0;
        }
        const bool same_cells = (!(ns.flags & F_ON) || jT == iT) && je == ie && same_ti;
        if (same_cells) {
          ns.z = zn;
          ns.kind = DONE; ns.xe = xn;
          continue;
        }
        if (bad) {                             // not finished after all: the safeguard applies
          s_next = s_mid;
          xn = fexp(s_next);
        }
      }
      if (!small && floor_pending && (!newton_ok || sn < sf)) {
        // the descent would cross the floor (decided on the raw Newton step:
        // the safeguard only halves towards it): probe G just above it
        ns.flags &= ~F_FLOOR_PENDING;
        ns.kind = PROBE_ON; ns.se = sf; ns.xe = T_floor; ns.flags |= F_ON;
        return false;
      }
      ns.z += dzdx * (xn - ns.xe);             // first-order warm start of the next inner solve
      ns.kind = ITER; ns.se = s_next; ns.xe = xn;
      if (ns.xe >= T_floor) ns.flags |= F_ON; else ns.flags &= ~F_ON;
    }
    return false;
    }
  }

  RC_HD void newton(double s0, CellOut* o) {
    NewtonState ns;
    newton_begin(s0, ns);
    while (!newton_round(ns, o)) {
    }
  }

  // state of a cell that its first round left unfinished
  RC_HD static void save_resume(const NewtonState& ns, NewtonResume* r) {
    r->G = ns.G; r->dG = ns.dG; r->z = ns.z; r->lo = ns.lo; r->hi = ns.hi; r->se = ns.se;
    r->kind_flags = ns.kind | (ns.flags << 3);
    r->pad = 0;
  }

  // the NewtonState save_resume came from (setup() of the same cell has run)
  RC_HD void load_resume(double s0, const NewtonResume& r, NewtonState& ns) const {
    ns.s = s0; ns.G = r.G; ns.dG = r.dG; ns.z = r.z; ns.lo = r.lo; ns.hi = r.hi; ns.se = r.se;
    ns.kind = r.kind_flags & 7;
    ns.flags = r.kind_flags >> 3;
    ns.iters = 0;
    ns.z_floor = T_i;
    // the pending point: exp(se) for an iterate (computed the same way when
    // it was proposed), the floor for a floor probe
    ns.xe = ns.kind == ITER ? fexp(ns.se) : Tf();
  }

  // Difficulty class of a cell after an unfinished first round, for grouping
  // cells that need similar numbers of further rounds: half-decade bins of
  // the first proposed step |se - s0| in ln T_e, from below 1e-6 (class 0) to
  // above 10^0.5 (class 14); class 15 for a floor probe.  The further round
  // count grows with that step (Newton from a model root: a short first step
  // converges in one more round, a step of order one takes three).
  RC_HD static int resume_class(const NewtonState& ns) {
    if (ns.kind != ITER) return kResumeClasses - 1;
    const float d = (float)fabs(ns.se - ns.s);
    const float l = flog2_sp(d > 1e-30f ? d : 1e-30f) * 0.30103f;   // log10
    const int k = (int)floorf(2.0f * (l + 6.0f));
    return k < 0 ? 0 : (k > kResumeClasses - 2 ? kResumeClasses - 2 : k);
  }

  RC_HD void explicit16(double s0, CellOut* o) {
    const double h = dt / 16.0;
    double te = T_e, ti = T_i, lte = s0 * (1.0 / kLn10);
    for (int k = 0; k < 16; ++k) {
      double q, dq, dlx, dlz;
      const bool on = te >= Tf();
      const Coord cT = axis_coord(lte, P.g->ax[1]);
      const Coord ce = axis_coord(lte, P.g->ax[4]);
      const Coord ci = axis_coord(flog10(ti), P.g->ax[5]);
      gather(cT, ce, ci, on);
      q_rad(te, cT, on, &q, &dq);
      const double K = kcoul_at(ce, ci, &dlx, &dlz);
      const double qcc = (ti - te) * K;
      if (k == 0) { o->q_rad = q; o->q_cc = qcc; }
      const double qr = fmin(q, 0.3 * c * te / h);
      const double lim = fmin(0.5 * c * fabs(ti - te), 0.3 * c * fmin(te, ti)) / h;
      const double qc = fmin(fmax(qcc, -lim), lim);
      te += h * (qc - qr) / c;
      ti -= h * qc / c;
      lte = flog10(te);
    }
    o->T_e_new = te;
    o->T_i_new = ti;
  }

  RC_HD void rates(double s0, CellOut* o) {
    const double lte = s0 * (1.0 / kLn10);
    double q, dq, dlx, dlz;
    const bool on = T_e >= Tf();
    const Coord cT = axis_coord(lte, P.g->ax[1]);
    const Coord ce = axis_coord(lte, P.g->ax[4]);
    const Coord ci = axis_coord(flog10(T_i), P.g->ax[5]);
    gather(cT, ce, ci, on);
    q_rad(T_e, cT, on, &q, &dq);
    o->q_rad = q;
    // a cooling-table corner without a value (literal Compton reading)
    if (!(q == q)) o->status |= ST_NO_RATE;
    o->q_cc = (T_i - T_e) * kcoul_at(ce, ci, &dlx, &dlz);
    o->T_e_new = T_e;
    o->T_i_new = T_i;
  }

  // the three cooling quantities separately at the input state (diagnostic outputs)
  RC_HD void diagnostics(double s0, CellOut* o) {
    const Coord cT = axis_coord(s0 * (1.0 / kLn10), P.g->ax[1]);
    const double wN[2] = {1.0 - tN, tN};
    const double wB[2] = {1.0 - tB, tB};
    const double wT[2] = {1.0 - cT.t, cT.t};
    double y[3] = {0.0, 0.0, 0.0};
    float4 v[8];
    corners8(tab, iN, cT.i, iB, v);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const double w = wN[a] * wT[m] * wB[b];
          const float4 p = v[a * 4 + m * 2 + b];
          y[0] += w * (double)p.x;
          y[1] += w * (double)p.y;
          y[2] += w * (double)p.z;
        }
    const double fN = iN + tN, fT = cT.i + cT.t, fB = iB + tB;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double* co = P.g->coef[k];
      y[k] += co[0] + co[1] * fN + co[2] * fT + co[3] * fB;
    }
    const double invH = 1.0 / H;
    o->q_brem = fexp2(y[0]) * invH * invH;
    o->q_syn = fexp2(y[1]) * invH;
    o->eta = fexp2(y[2]);
  }
};

RC_HD bool bad_input(double v) { return !(v > 0.0) || !isfinite(v); }

template <int SCHEME, class Tab>
RC_HD void cool_cell(const Tab& tab, const StepParams& P, double dt, double n_e, double T_e, double T_i, double B,
                     double H, double floor_gas, bool diag, CellOut* o) {
  if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
    const double nan = __builtin_nan("");
    o->T_e_new = o->T_i_new = o->q_rad = o->q_cc = o->q_brem = o->q_syn = o->eta = nan;
    o->status = ST_INVALID;
    return;
  }
  CellSolver<Tab> cs(tab, P);
  const double s0 = cs.setup(n_e, T_e, T_i, B, H, dt, floor_gas);
  o->status = cs.clamp;
  if (SCHEME == SCHEME_NEWTON) {
    cs.newton(s0, o);
  } else if (SCHEME == SCHEME_EXPLICIT16) {
    cs.explicit16(s0, o);
  } else {
    cs.rates(s0, o);
  }
  if (diag) cs.diagnostics(s0, o);
}

// runtime scheme selection (host self-test path)
template <class Tab>
RC_HD void cool_cell_any(const Tab& tab, const StepParams& P, double n_e, double T_e, double T_i, double B,
                         double H, double floor_gas, bool diag, CellOut* o) {
  if (P.scheme == SCHEME_NEWTON) cool_cell<SCHEME_NEWTON>(tab, P, P.dt, n_e, T_e, T_i, B, H, floor_gas, diag, o);
  else if (P.scheme == SCHEME_EXPLICIT16)
    cool_cell<SCHEME_EXPLICIT16>(tab, P, P.dt, n_e, T_e, T_i, B, H, floor_gas, diag, o);
  else cool_cell<SCHEME_RATES>(tab, P, P.dt, n_e, T_e, T_i, B, H, floor_gas, diag, o);
}

// Table-free rates at the input state from the closed forms (DIRECT variant).
RC_HD void direct_rates(const StepParams& P, double n_e, double T_e, double T_i, double B, double H,
                        double floor_gas, CellOut* o) {
  if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
    const double nan = __builtin_nan("");
    o->T_e_new = o->T_i_new = o->q_rad = o->q_cc = o->q_brem = o->q_syn = o->eta = nan;
    o->status = ST_INVALID;
    return;
  }
  o->q_brem = n_e * n_e * brem_coeff(T_e);
  const SynchResult sr = synchrotron(n_e, T_e, B, H);
  o->q_syn = exp(sr.ln_q);
  o->eta = P.compton_literal ? eta_literal(n_e, T_e, H, sr.nu_c) : exp(ln_eta(n_e, T_e, H, sr.nu_c));
  const double qthin = o->q_brem + o->eta * o->q_syn;
  const double T2 = T_e * T_e;
  const double ta = H * qthin / (4.0 * kSigmaSB * T2 * T2);
  const double ts = 2.0 * n_e * kSigmaT * H;
  const bool off = T_e + T_i < floor_gas;
  const bool cooling = !off && T_e >= P.T_floor;
  const bool no_rate = cooling && !(o->eta > 0.0 && isfinite(o->eta));
  o->q_rad = !cooling ? 0.0 : no_rate ? __builtin_nan("") : qthin / (1.0 + kSqrt3 * ta + 1.5 * ta * (ta + ts));
  o->q_cc = (T_i - T_e) * exp(ln_coulomb_coeff(n_e, T_e, T_i, P.ln_lambda, P.theta_i_me != 0));
  o->T_e_new = T_e;
  o->T_i_new = T_i;
  o->status = (off ? ST_GAS_FLOOR : 0) | (no_rate ? ST_NO_RATE : 0);
}

}  // namespace rc
