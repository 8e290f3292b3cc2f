// Backward-Euler Newton with straggler deferral.
//
// The number of outer evaluations differs widely between cells: most need one
// to three, strongly cooling or heating cells up to seven.  A wave runs as many
// rounds as its slowest lane, so with independent cells most lanes idle in the
// late rounds.  Here a wave iterates only while at least kDeferBelow of its 64
// lanes are still active; then it appends the remaining cells' solver states to
// a queue (one wave-aggregated atomic reserves the slots) and moves on.  The
// next launch takes the queue 64 entries per wave, so the stragglers run on
// dense waves, under the same rule; the last launch runs every remaining cell
// to completion.  Each launch performs at least one round per item before it
// may defer it again, so every launch makes progress.
//
// A wave defers at most kDeferBelow - 1 of its 64 items, so a queue fed by at
// most n items never holds more than (kDeferBelow - 1) * ceil(n / 64) entries.
// The per-cell arithmetic is that of CellSolver::newton, so the results are the
// same as the plain kernel's up to floating-point contraction differences.
#pragma once

#include "rc_kernels.hpp"

namespace rc {

constexpr int kDeferBelow = 32;
constexpr int kPhases = 6;       // launches; the last one runs to completion
constexpr int kQueueDoubles = 9;

__host__ __device__ inline int64_t defer_capacity(int64_t n) { return (kDeferBelow - 1) * ((n + 63) / 64); }

// One queue, structure of arrays over cap entries: cell index, the nine
// doubles of NewtonState and its packed integers.
struct DeferQueue {
  int64_t* cell;
  double* v;           // v[k * cap + slot], k = s, G, dG, z, lo, hi, se, xe, z_floor
  unsigned* packed;    // kind | flags << 4 | iters << 8
  int64_t cap;
};

struct PhaseArgs {
  DeferQueue in, out;
  unsigned long long* count;   // count[p] = entries phase p appended to its output queue
  int phase;
};

__device__ inline void queue_put(const DeferQueue& q, int64_t slot, int64_t cell, const NewtonState& ns) {
  const double v[kQueueDoubles] = {ns.s, ns.G, ns.dG, ns.z, ns.lo, ns.hi, ns.se, ns.xe, ns.z_floor};
#pragma unroll
  for (int k = 0; k < kQueueDoubles; ++k) q.v[k * q.cap + slot] = v[k];
  q.cell[slot] = cell;
  q.packed[slot] = (unsigned)ns.kind | ((unsigned)ns.flags << 4) | ((unsigned)ns.iters << 8);
}

__device__ inline int64_t queue_get(const DeferQueue& q, int64_t slot, NewtonState& ns) {
  double v[kQueueDoubles];
#pragma unroll
  for (int k = 0; k < kQueueDoubles; ++k) v[k] = q.v[k * q.cap + slot];
  ns.s = v[0]; ns.G = v[1]; ns.dG = v[2]; ns.z = v[3]; ns.lo = v[4]; ns.hi = v[5];
  ns.se = v[6]; ns.xe = v[7]; ns.z_floor = v[8];
  const unsigned p = q.packed[slot];
  ns.kind = (int)(p & 0xfu);
  ns.flags = (int)((p >> 4) & 0xfu);
  ns.iters = (int)(p >> 8);
  return q.cell[slot];
}

// Number of set bits of mask below this lane.
__device__ inline int lanes_below(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// One wave's share of a phase: items chunk*64 .. chunk*64+63 of the phase's
// input (cells when FRESH, else entries of the input queue).  Every lane of
// the wave must call it (it votes).
template <class Tab, bool FRESH, bool LAST>
__device__ void newton_phase_chunk(const Tab& tab, const StepParams& P, const StateArgs& s, const OutArgs& o,
                                   const PhaseArgs& q, int64_t items, int64_t chunk, bool diag) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t item = chunk * 64 + lane;
  bool active = item < items;
  CellSolver<Tab> cs(tab, P);
  NewtonState ns;
  CellOut r;
  int64_t cell = 0;
  if (active) {
    if (FRESH) {
      cell = item;
    } else {
      cell = queue_get(q.in, item, ns);
    }
    const double n_e = s.n_e[cell], T_e = s.T_e[cell], T_i = s.T_i[cell], B = s.B[cell], H = s.H[cell];
    if (FRESH && (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H))) {
      const double nan = __builtin_nan("");
      r.T_e_new = r.T_i_new = r.q_rad = r.q_cc = r.q_brem = r.q_syn = r.eta = nan;
      r.status = ST_INVALID;
      store(o, cell, r);
      active = false;
    } else {
      const double s0 = cs.setup(n_e, T_e, T_i, B, H, P.dt, floor_gas_at(s, cell));
      r.status = cs.clamp;
      if (FRESH) {
        if (diag) {
          cs.diagnostics(s0, &r);
          if (o.Q_brem) o.Q_brem[cell] = r.q_brem;
          if (o.Q_syn) o.Q_syn[cell] = r.q_syn;
          if (o.eta) o.eta[cell] = r.eta;
        }
        cs.newton_begin(s0, ns);
      }
    }
  }
  for (int round = 0;; ++round) {
    const unsigned long long act = __ballot(active);
    if (act == 0) break;
    if (!LAST && round > 0 && __popcll(act) < kDeferBelow) {
      const int leader = __ffsll((long long)act) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(&q.count[q.phase], (unsigned long long)__popcll(act));
      base = __shfl(base, leader);
      if (active) queue_put(q.out, (int64_t)base + lanes_below(act), cell, ns);
      break;
    }
    if (active) {
      const bool first = ns.kind == CellSolver<Tab>::FIRST;
      const bool done = cs.newton_round(ns, &r);
      if (first) {
        if (o.Q_rad) o.Q_rad[cell] = r.q_rad;
        if (o.Q_cc) o.Q_cc[cell] = r.q_cc;
      }
      if (done) {
        if (o.T_e_new) o.T_e_new[cell] = r.T_e_new;
        if (o.T_i_new) o.T_i_new[cell] = r.T_i_new;
        if (o.status) o.status[cell] = r.status;
        active = false;
      }
    }
  }
}

}  // namespace rc
