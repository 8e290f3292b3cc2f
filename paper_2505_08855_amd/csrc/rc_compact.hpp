// In-workgroup compaction of the Newton solve.
//
// Cells of one tile (up to kTile = 256 cells, one per thread) need very
// different numbers of Newton rounds: most converge after one or two residual
// evaluations, stiff cells need up to ten.  Run as plain threads, every wave
// would take as long as its slowest lane.  Here every round performs one
// evaluation per still-active cell, after which the survivors' complete solver
// state is written compactly to LDS (structure of arrays, consecutive slots,
// no bank conflicts) and re-read by the first n threads; waves whose threads
// have no cell left retire, so late rounds run on dense waves.  The per-cell
// arithmetic is exactly that of CellSolver::newton, so results are identical.
#pragma once

#include "rc_kernels.hpp"

namespace rc {

constexpr int kTile = 256;

// parked per-cell state, 25 doubles + 8 ints per slot (59 KB for 256 slots)
struct ParkedTile {
  double d[25][kTile];
  int i[8][kTile];
  int count[2];
};

template <class Tab>
__device__ inline void park(ParkedTile& L, int slot, const CellSolver<Tab>& c, double n_e, const NewtonState& ns,
                            int cell, int status) {
  L.d[0][slot] = c.T_e; L.d[1][slot] = c.T_i; L.d[2][slot] = c.H; L.d[3][slot] = n_e;
  L.d[4][slot] = c.tN; L.d[5][slot] = c.tB; L.d[6][slot] = c.tn;
  L.d[7][slot] = c.Ab; L.d[8][slot] = c.Ase; L.d[9][slot] = c.Sb; L.d[10][slot] = c.Sse;
  L.d[11][slot] = c.K0; L.d[12][slot] = c.v00; L.d[13][slot] = c.v10; L.d[14][slot] = c.v01;
  L.d[15][slot] = c.v11;
  L.d[16][slot] = ns.s; L.d[17][slot] = ns.G; L.d[18][slot] = ns.dG; L.d[19][slot] = ns.z;
  L.d[20][slot] = ns.lo; L.d[21][slot] = ns.hi; L.d[22][slot] = ns.se; L.d[23][slot] = ns.xe;
  L.d[24][slot] = ns.z_floor;
  L.i[0][slot] = c.iN; L.i[1][slot] = c.iB; L.i[2][slot] = c.in_;
  L.i[3][slot] = c.iT; L.i[4][slot] = c.ie; L.i[5][slot] = c.ii;
  L.i[6][slot] = cell | (ns.kind << 8) | (ns.flags << 11) | (status << 16);   // 8 | 3 | 4 | 8 bits
  L.i[7][slot] = ns.iters;
}

// restore a parked cell: the CellSolver members exactly as setup() and the
// gathers left them (the derived constants are recomputed with the same
// expressions), the Newton state, the tile-local cell index, the status and n_e
template <class Tab>
__device__ inline void unpark(const ParkedTile& L, int slot, CellSolver<Tab>& c, double dt, NewtonState& ns,
                              int* cell, int* status, double* n_e_out) {
  const double n_e = L.d[3][slot];
  *n_e_out = n_e;
  c.dt = dt;
  c.T_e = L.d[0][slot];
  c.T_i = L.d[1][slot];
  c.H = L.d[2][slot];
  c.c = kUperNKT * n_e * kKB;
  c.cS = c.c * (c.T_e + c.T_i);
  c.tau_sca = 2.0 * n_e * kSigmaT * c.H;
  c.invH = 1.0 / c.H;
  c.invH2 = c.invH * c.invH;
  c.tN = L.d[4][slot]; c.tB = L.d[5][slot]; c.tn = L.d[6][slot];
  c.Ab = L.d[7][slot]; c.Ase = L.d[8][slot]; c.Sb = L.d[9][slot]; c.Sse = L.d[10][slot];
  c.K0 = L.d[11][slot]; c.v00 = L.d[12][slot]; c.v10 = L.d[13][slot]; c.v01 = L.d[14][slot];
  c.v11 = L.d[15][slot];
  ns.s = L.d[16][slot]; ns.G = L.d[17][slot]; ns.dG = L.d[18][slot]; ns.z = L.d[19][slot];
  ns.lo = L.d[20][slot]; ns.hi = L.d[21][slot]; ns.se = L.d[22][slot]; ns.xe = L.d[23][slot];
  ns.z_floor = L.d[24][slot];
  c.iN = L.i[0][slot]; c.iB = L.i[1][slot]; c.in_ = L.i[2][slot];
  c.iT = L.i[3][slot]; c.ie = L.i[4][slot]; c.ii = L.i[5][slot];
  const int p = L.i[6][slot];
  *cell = p & 0xff;
  ns.kind = (p >> 8) & 0x7;
  ns.flags = (p >> 11) & 0xf;
  *status = (p >> 16) & 0xff;
  ns.iters = L.i[7][slot];
}

// Backward-Euler Newton over cells first .. first + count - 1 (count <=
// blockDim.x == kTile), one cell per thread in the first round, compacted
// afterwards.  Every thread of the workgroup must call it (it synchronises).
template <class Tab>
__device__ void newton_tile(const Tab& tab, const StepParams& P, double dt, int64_t first, int count,
                            const StateArgs& s, const OutArgs& o, bool diag, ParkedTile& L) {
  const int tid = threadIdx.x;
  if (tid == 0) { L.count[0] = 0; L.count[1] = 0; }
  __syncthreads();
  if (tid < count) {
    const int64_t i = first + tid;
    const double n_e = s.n_e[i], T_e = s.T_e[i], T_i = s.T_i[i], B = s.B[i], H = s.H[i];
    CellOut r;
    if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
      const double nan = __builtin_nan("");
      r.T_e_new = r.T_i_new = r.q_rad = r.q_cc = r.q_brem = r.q_syn = r.eta = nan;
      r.status = ST_INVALID;
      store(o, i, r);
    } else {
      CellSolver<Tab> cs(tab, P);
      const double s0 = cs.setup(n_e, T_e, T_i, B, H, dt);
      r.status = cs.clamp;
      if (diag) {
        cs.diagnostics(s0, &r);
        if (o.Q_brem) o.Q_brem[i] = r.q_brem;
        if (o.Q_syn) o.Q_syn[i] = r.q_syn;
        if (o.eta) o.eta[i] = r.eta;
      }
      NewtonState ns;
      cs.newton_begin(s0, ns);
      const bool done = cs.newton_round(ns, &r);      // the first evaluation gives the input-state rates
      if (o.Q_rad) o.Q_rad[i] = r.q_rad;
      if (o.Q_cc) o.Q_cc[i] = r.q_cc;
      if (done) {
        if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
        if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
        if (o.status) o.status[i] = r.status;
      } else {
        const int slot = atomicAdd(&L.count[0], 1);
        park(L, slot, cs, n_e, ns, tid, r.status);
      }
    }
  }
  __syncthreads();
  int n = L.count[0];
  for (int round = 0; n > 0; ++round) {
    const int cur = round & 1, nxt = cur ^ 1;
    if (tid == 0) L.count[nxt] = 0;    // last read at the previous round's start; visible after the barrier below
    CellSolver<Tab> cs(tab, P);
    NewtonState ns;
    int cell = 0, status = 0;
    double n_e = 0.0;
    const bool mine = tid < n;
    if (mine) unpark(L, tid, cs, dt, ns, &cell, &status, &n_e);
    __syncthreads();                   // every slot read before any is rewritten
    if (mine) {
      CellOut r;
      r.status = (unsigned char)status;
      const bool done = cs.newton_round(ns, &r);
      const int64_t i = first + cell;
      if (done) {
        if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
        if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
        if (o.status) o.status[i] = r.status;
      } else {
        const int slot = atomicAdd(&L.count[nxt], 1);
        park(L, slot, cs, n_e, ns, cell, r.status);
      }
    }
    __syncthreads();
    n = L.count[nxt];
  }
}

}  // namespace rc
