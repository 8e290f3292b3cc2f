// Adjoint kernel and the rc_cool_step_backward entry point.
//
// One thread per cell: recompute the interpolant pieces at the forward
// solution and at the input state, solve the transposed 2x2 system and write
// the five input gradients (coalesced).  Table-entry gradients, when asked
// for, take no floating-point atomics: every cell writes one record per
// evaluation point (its table cell, coefficients and fractional coordinates),
// a counting sort groups the records by table cell (integer atomics on the
// counts and placement cursors, aggregated per wavefront), one thread per
// table cell (one workgroup for a crowded one) adds up its records' corner
// contributions into cell-blocked scratch, and a last pass folds the cells
// onto the table nodes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>
#include <vector>

#include "radcool.h"
#include "rc_grad.hpp"
#include "rc_internal.hpp"

namespace rc {

struct BwdArgs {
  const double *n_e, *T_e, *T_i, *B, *H;
  const double* T_floor_gas;   // optional per-cell gas-temperature floor
  const double *x, *z;
  const uint8_t* status;
  const double *g_x, *g_z, *g_qr, *g_qc;
  double *o_n, *o_Te, *o_Ti, *o_B, *o_H, *o_tab;
  double* g_cool_cells;   // scratch, cell-blocked: {brem, synch * eta} per corner of each cooling cell
  double* g_coul_cells;   // scratch, cell-blocked: one value per corner of each Coulomb cell
  unsigned *key_cool, *key_coul, *cnt_cool, *cnt_coul;   // gradient records (see RecordScatter)
  double *rec_cool, *rec_coul;
  int c1, c2, k1, k2;
  long vc;
  int newton;
};

// The adjoint without table gradients: cell_vjp is called with want_tables
// false, so nothing reaches the scatter.
struct NoScatter {
  enum { kRecords = 0 };
  __device__ void cool(const long*, const double*, const double*) const {}
  __device__ void coul(const long*, const double*) const {}
};

// Table-gradient records: the adjoint writes, per cell and evaluation point,
// the table cell it fell in, its coefficients and fractional coordinates
// (cooling: cb, cse, t0, t1, t2; Coulomb: cc, t0, t1, t2) and counts the
// records of each table cell; a counting sort by table cell then lets one
// thread per table cell add up its records' corner contributions without
// atomics on the gradients.  Record r = 2 i + p of cell i and point p; its key
// is ~0u when the point contributes nothing.
// Add 1 to cnt[key] for every active lane.  Neighbouring cells of coherent
// inputs share table cells, and one atomic per lane on one counter serializes;
// so the first kPeel distinct keys among the active lanes of the wavefront
// take one atomic each, and the lanes left (independent inputs) one each.
// The peel loop is uniform over the active lanes.
constexpr int kPeel = 4;

__device__ inline void wave_count(unsigned* cnt, unsigned key) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t todo = __ballot(1);
  for (int it = 0; it < kPeel && todo; ++it) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const unsigned lk = __shfl(key, leader);
    const uint64_t same = __ballot(key == lk) & todo;
    if (lane == leader) atomicAdd(cnt + lk, (unsigned)__popcll(same));
    todo &= ~same;
  }
  if ((todo >> lane) & 1ull) atomicAdd(cnt + key, 1u);
}

struct RecordScatter {
  enum { kRecords = 1 };
  unsigned* key_cool;
  double* rec_cool;
  unsigned* cnt_cool;
  unsigned* key_coul;
  double* rec_coul;
  unsigned* cnt_coul;
  long r0;
  __device__ void cool_rec(int p, long cell, double cb, double cse, const double* t) const {
    const long r = r0 + p;
    double* q = rec_cool + r * 5;
    q[0] = cb; q[1] = cse; q[2] = t[0]; q[3] = t[1]; q[4] = t[2];
    key_cool[r] = (unsigned)cell;
    wave_count(cnt_cool, (unsigned)cell);
  }
  __device__ void coul_rec(int p, long cell, double cc, const double* t) const {
    const long r = r0 + p;
    double* q = rec_coul + r * 4;
    q[0] = cc; q[1] = t[0]; q[2] = t[1]; q[3] = t[2];
    key_coul[r] = (unsigned)cell;
    wave_count(cnt_coul, (unsigned)cell);
  }
};

template <class Tab, bool CELLS>
__global__ __launch_bounds__(256, 2) void k_backward(Tab tab, StepParams P, BwdArgs a, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  using Scatter = typename std::conditional<CELLS, RecordScatter, NoScatter>::type;
  Scatter sc;
  if constexpr (CELLS) {
    sc = RecordScatter{a.key_cool, a.rec_cool, a.cnt_cool, a.key_coul, a.rec_coul, a.cnt_coul, 2 * i};
    a.key_cool[2 * i] = a.key_cool[2 * i + 1] = ~0u;
    a.key_coul[2 * i] = a.key_coul[2 * i + 1] = ~0u;
  }
  CellGrad g;
  const double x = a.newton ? a.x[i] : a.T_e[i];
  const double z = a.newton ? a.z[i] : a.T_i[i];
  const uint8_t st = a.status ? a.status[i] : (uint8_t)0;
  cell_vjp(tab, P, a.c1, a.c2, a.k1, a.k2, a.n_e[i], a.T_e[i], a.T_i[i], a.B[i], a.H[i],
           a.T_floor_gas ? a.T_floor_gas[i] : 0.0, x, z, st,
           a.g_x ? a.g_x[i] : 0.0, a.g_z ? a.g_z[i] : 0.0, a.g_qr ? a.g_qr[i] : 0.0, a.g_qc ? a.g_qc[i] : 0.0,
           a.newton != 0, a.o_tab != nullptr, &g, sc);
  if (a.o_n) a.o_n[i] = g.n_e;
  if (a.o_Te) a.o_Te[i] = g.T_e;
  if (a.o_Ti) a.o_Ti[i] = g.T_i;
  if (a.o_B) a.o_B[i] = g.B;
  if (a.o_H) a.o_H[i] = g.H;
}

__global__ void k_zero_u32(unsigned* p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0u;
}

// exclusive scan of 1024-element chunks (one workgroup each); chunk totals to sums
__global__ __launch_bounds__(1024) void k_scan_chunks(const unsigned* in, unsigned* out, unsigned* sums, long n) {
  __shared__ unsigned buf[1024];
  const long i = blockIdx.x * 1024L + threadIdx.x;
  const unsigned v = i < n ? in[i] : 0u;
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const unsigned add = threadIdx.x >= (unsigned)d ? buf[threadIdx.x - d] : 0u;
    __syncthreads();
    buf[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < n) out[i] = buf[threadIdx.x] - v;
  if (threadIdx.x == 1023) sums[blockIdx.x] = buf[1023];
}

__global__ void k_scan_add(unsigned* out, const unsigned* offs, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] += offs[i / 1024];
}

// place record indices by table cell (cursor starts as the exclusive scan);
// lanes of a wavefront with the same key take consecutive places from one atomic
__global__ __launch_bounds__(256) void k_order(const unsigned* key, unsigned* cursor, unsigned* order, long nrec) {
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // whole wavefronts step through the records so that every ballot is uniform
  const long stride = (long)gridDim.x * blockDim.x;
  for (long base = blockIdx.x * (long)blockDim.x; base < nrec; base += stride) {
    const long r = base + threadIdx.x;
    const unsigned k = r < nrec ? key[r] : ~0u;
    uint64_t todo = __ballot(k != ~0u);
    for (int it = 0; it < kPeel && todo; ++it) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const unsigned lk = __shfl(k, leader);
      const uint64_t same = __ballot(k == lk) & todo;
      unsigned pos0 = 0;
      if (lane == leader) pos0 = atomicAdd(cursor + lk, (unsigned)__popcll(same));
      pos0 = __shfl(pos0, leader);
      if ((same >> lane) & 1ull) order[pos0 + __popcll(same & below)] = (unsigned)r;
      todo &= ~same;
    }
    if ((todo >> lane) & 1ull) order[atomicAdd(cursor + k, 1u)] = (unsigned)r;
  }
}

// table cells with more records than this are summed by k_gather_heavy
constexpr unsigned kHeavy = 128;

// one thread per table cell: the corner contributions of its records, written
// to the cell-blocked gradient scratch (zero for a cell without records, and
// for a heavy cell, which k_gather_heavy then adds to)
template <bool COOL>
__global__ void k_gather_records(const unsigned* start, const unsigned* cnt, const unsigned* order,
                                 const double* rec, double* cells, long ncell, unsigned* heavy, unsigned* nheavy) {
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < ncell; c += (long)gridDim.x * blockDim.x) {
    double acc0[8], acc1[8];
    for (int k = 0; k < 8; ++k) acc0[k] = acc1[k] = 0.0;
    const bool is_heavy = cnt[c] > kHeavy;
    if (is_heavy) heavy[atomicAdd(nheavy, 1u)] = (unsigned)c;
    const unsigned b = start[c], m = is_heavy ? 0u : cnt[c];   // heavy cells: k_gather_heavy
    for (unsigned j = 0; j < m; ++j) {
      const double* q = rec + (long)order[b + j] * (COOL ? 5 : 4);
      const double c0 = q[0], c1 = COOL ? q[1] : 0.0;
      const double t0 = q[COOL ? 2 : 1], t1 = q[COOL ? 3 : 2], t2 = q[COOL ? 4 : 3];
      for (int k = 0; k < 8; ++k) {
        const double w = ((k >> 2) ? t0 : 1.0 - t0) * (((k >> 1) & 1) ? t1 : 1.0 - t1) * ((k & 1) ? t2 : 1.0 - t2);
        acc0[k] += c0 * w;
        if (COOL) acc1[k] += c1 * w;
      }
    }
    if (COOL) {
      for (int k = 0; k < 8; ++k) {
        cells[c * 16 + 2 * k] = acc0[k];
        cells[c * 16 + 2 * k + 1] = acc1[k];
      }
    } else {
      for (int k = 0; k < 8; ++k) cells[c * 8 + k] = acc0[k];
    }
  }
}

// heavy table cells (coherent inputs put many cells into one table cell):
// one workgroup per heavy cell, its threads striding over the cell's records,
// then a workgroup reduction and plain stores (no floating-point atomics)
template <bool COOL>
__global__ __launch_bounds__(256) void k_gather_heavy(const unsigned* start, const unsigned* cnt, const unsigned* order,
                                                      const double* rec, double* cells, const unsigned* heavy,
                                                      const unsigned* nheavy) {
  constexpr int V = COOL ? 16 : 8;
  __shared__ double red[V][256];
  const unsigned nh = *nheavy;
  for (unsigned h = blockIdx.x; h < nh; h += gridDim.x) {
    const unsigned c = heavy[h];
    const unsigned b = start[c], m = cnt[c];
    double acc[V];
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    for (unsigned j = threadIdx.x; j < m; j += blockDim.x) {
      const double* q = rec + (long)order[b + j] * (COOL ? 5 : 4);
      const double c0 = q[0], c1 = COOL ? q[1] : 0.0;
      const double t0 = q[COOL ? 2 : 1], t1 = q[COOL ? 3 : 2], t2 = q[COOL ? 4 : 3];
      for (int k = 0; k < 8; ++k) {
        const double w = ((k >> 2) ? t0 : 1.0 - t0) * (((k >> 1) & 1) ? t1 : 1.0 - t1) * ((k & 1) ? t2 : 1.0 - t2);
        if (COOL) {
          acc[2 * k] += c0 * w;
          acc[2 * k + 1] += c1 * w;
        } else {
          acc[k] += c0 * w;
        }
      }
    }
    for (int v = 0; v < V; ++v) red[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
      if ((int)threadIdx.x < d)
        for (int v = 0; v < V; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + d];
      __syncthreads();
    }
    if ((int)threadIdx.x < V) cells[(long)c * V + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// fold cell-blocked gradients onto the nodes: node (i0, i1, i2) is corner
// (a, b, m) of cell (i0 - a, i1 - b, i2 - m) wherever that cell exists; the
// synch * eta gradient goes to both tables' slots
__global__ void k_finish_cells(double* g_tab, const double* cool_cells, const double* coul_cells, int n0, int n1,
                               int n2, int m0, int m1, int m2) {
  const long vc = (long)n0 * n1 * n2, vk = (long)m0 * m1 * m2;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < vc + vk; j += (long)gridDim.x * blockDim.x) {
    const bool cl = j < vc;
    const long v = cl ? j : j - vc;
    const int d0 = cl ? n0 : m0, d1 = cl ? n1 : m1, d2 = cl ? n2 : m2;
    const int i2 = (int)(v % d2), i1 = (int)((v / d2) % d1), i0 = (int)(v / ((long)d1 * d2));
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < 8; ++k) {
      const int a = k >> 2, b = (k >> 1) & 1, m = k & 1;
      const int c0 = i0 - a, c1 = i1 - b, c2 = i2 - m;
      if (c0 < 0 || c1 < 0 || c2 < 0 || c0 > d0 - 2 || c1 > d1 - 2 || c2 > d2 - 2) continue;
      const long cell = ((long)c0 * (d1 - 1) + c1) * (d2 - 1) + c2;
      if (cl) {
        s0 += cool_cells[cell * 16 + 2 * k];
        s1 += cool_cells[cell * 16 + 2 * k + 1];
      } else {
        s0 += coul_cells[cell * 8 + k];
      }
    }
    if (cl) {
      g_tab[v] += s0;
      g_tab[vc + v] += s1;
      g_tab[2 * vc + v] += s1;
    } else {
      g_tab[3 * vc + v] += s0;
    }
  }
}

// exclusive scan of m counts into out; tmp holds the chunk sums of every
// level (at most 2 ceil(m / 1024) + 2 entries)
void scan_counts(const unsigned* in, unsigned* out, long m, unsigned* tmp, hipStream_t hs) {
  const long nb = (m + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nb), dim3(1024), 0, hs, in, out, tmp, m);
  if (nb > 1) {
    scan_counts(tmp, tmp, nb, tmp + nb, hs);
    hipLaunchKernelGGL(k_scan_add, dim3(4096), dim3(256), 0, hs, out, (const unsigned*)tmp, m);
  }
}

}  // namespace rc

using namespace rc;

extern "C" rc_status rc_cool_step_backward(rc_tables t, const rc_state* state, int64_t n, double dt,
                                           const rc_step_opts* opts, const rc_fwd* fwd, const rc_cotangent* cot,
                                           const rc_grad* grad, void* stream) {
  if (!handle_ok(t)) return set_error(RC_ESTATE, "rc_cool_step_backward: invalid table handle");
  if (!state || !grad) return set_error(RC_EINVAL, "rc_cool_step_backward: state or grad is NULL");
  if (n < 0) return set_error(RC_EINVAL, "rc_cool_step_backward: n < 0");
  StepParams P;
  rc_status st = make_params(t, dt, opts, &P);
  if (st != RC_OK) return st;
  if (opts->scheme == RC_SCHEME_EXPLICIT16)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step_backward: the explicit scheme has no adjoint");
  if (opts->variant == RC_VARIANT_DIRECT)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step_backward: the DIRECT variant has no table adjoint");
  if (t->spec.compton_exponent == RC_COMPTON_LITERAL)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step_backward: tables of the literal Compton exponent have no adjoint");
  const bool newton = opts->scheme == RC_SCHEME_NEWTON;
  if (n > 0 && (!state->n_e || !state->T_e || !state->T_i || !state->B || !state->H))
    return set_error(RC_EINVAL, "rc_cool_step_backward: a state pointer is NULL");
  if (n > 0 && newton && (!fwd || !fwd->T_e_new || !fwd->T_i_new || !fwd->status))
    return set_error(RC_EINVAL, "rc_cool_step_backward: the Newton scheme needs the forward T_e_new, T_i_new, status");
  if (n == 0) return RC_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return set_error(RC_ESTATE, "rc_cool_step_backward: tables live on another device than the current one");
  BwdArgs a;
  a.n_e = state->n_e; a.T_e = state->T_e; a.T_i = state->T_i; a.B = state->B; a.H = state->H;
  a.T_floor_gas = state->T_floor_gas;
  a.x = fwd ? fwd->T_e_new : nullptr;
  a.z = fwd ? fwd->T_i_new : nullptr;
  a.status = fwd ? fwd->status : nullptr;
  a.g_x = cot ? cot->T_e_new : nullptr;
  a.g_z = cot ? cot->T_i_new : nullptr;
  a.g_qr = cot ? cot->Q_rad : nullptr;
  a.g_qc = cot ? cot->Q_cc : nullptr;
  a.o_n = grad->n_e; a.o_Te = grad->T_e; a.o_Ti = grad->T_i; a.o_B = grad->B; a.o_H = grad->H;
  a.o_tab = grad->tables;
  a.c1 = t->spec.cool.n[1]; a.c2 = t->spec.cool.n[2];
  a.k1 = t->spec.coul.n[1]; a.k2 = t->spec.coul.n[2];
  a.vc = (long)volume(t->spec.cool);
  a.newton = newton ? 1 : 0;
  const int block = opts->block ? opts->block : 256;
  const int64_t grid = (n + block - 1) / block;
  if (grid > 0x7fffffffLL) return set_error(RC_EINVAL, "rc_cool_step_backward: n too large for one launch");
  hipStream_t hs = (hipStream_t)stream;
  // table reads: AUTO takes FP32 tables through the cell-blocked copy, as the
  // forward step does (built here if no call has built it yet), CELL requires
  // it; the other variants read the node layout
  const bool cells = opts->variant == RC_VARIANT_CELL ||
                     (opts->variant == RC_VARIANT_AUTO && t->spec.value_dtype == RC_VALUE_F32);
  if (cells && (st = ensure_cells(t, hs)) != RC_OK) return st;
  const auto with_bwd_tab = [&](auto&& f) {
    if (cells) return f(cell_tab(t));
    return with_tab(t, f);
  };
  a.g_cool_cells = a.g_coul_cells = nullptr;
  a.key_cool = a.key_coul = a.cnt_cool = a.cnt_coul = nullptr;
  a.rec_cool = a.rec_coul = nullptr;
  const rc_axes &ca = t->spec.cool, &ka = t->spec.coul;
  const long mc = (long)(ca.n[0] - 1) * (ca.n[1] - 1) * (ca.n[2] - 1);   // table cells
  const long mk = (long)(ka.n[0] - 1) * (ka.n[1] - 1) * (ka.n[2] - 1);
  const long nrec = 2 * n;                                               // records per table kind
  if (nrec > 0xfffffffeLL) return set_error(RC_EINVAL, "rc_cool_step_backward: n too large for the gradient records");
  // scratch: [cooling cells x 16][Coulomb cells x 8][cooling records x 5][Coulomb records x 4] doubles, then
  // uint32: keys, orders (2 x nrec each), counts, starts, cursors (3 x (mc + mk)), scan sums
  const long sc_c = 2 * ((mc + 1023) / 1024) + 2, sc_k = 2 * ((mk + 1023) / 1024) + 2;
  const size_t dbl = sizeof(double) * (size_t)(16 * mc + 8 * mk + 9 * nrec);
  const size_t u32 = sizeof(unsigned) * (size_t)(4 * nrec + 4 * (mc + mk) + sc_c + sc_k + 2);
  if (a.o_tab) {
    if (t->gscratch_bytes < dbl + u32) {
      if (t->d_gscratch) (void)hipFree(t->d_gscratch);
      t->d_gscratch = nullptr;
      t->gscratch_bytes = 0;
      const hipError_t ae = hipMalloc(&t->d_gscratch, dbl + u32);
      if (ae != hipSuccess) return hip_fail(ae, "hipMalloc(table-gradient scratch)");
      t->gscratch_bytes = dbl + u32;
    }
    double* d = (double*)t->d_gscratch;
    a.g_cool_cells = d;
    a.g_coul_cells = d + 16 * mc;
    a.rec_cool = d + 16 * mc + 8 * mk;
    a.rec_coul = a.rec_cool + 5 * nrec;
    unsigned* u = (unsigned*)((char*)t->d_gscratch + dbl);
    a.key_cool = u;
    a.key_coul = u + nrec;
    unsigned* order_cool = u + 2 * nrec;
    unsigned* order_coul = u + 3 * nrec;
    a.cnt_cool = u + 4 * nrec;
    a.cnt_coul = a.cnt_cool + mc;
    unsigned* start_cool = a.cnt_coul + mk;
    unsigned* start_coul = start_cool + mc;
    unsigned* cur_cool = start_coul + mk;
    unsigned* cur_coul = cur_cool + mc;
    unsigned* tmp_c = cur_coul + mk;
    unsigned* tmp_k = tmp_c + sc_c;
    unsigned* heavy_cool = tmp_k + sc_k;
    unsigned* heavy_coul = heavy_cool + mc;
    unsigned* nheavy = heavy_coul + mk;   // [cooling, Coulomb]
    hipLaunchKernelGGL(k_zero_u32, dim3(4096), dim3(256), 0, hs, a.cnt_cool, mc + mk);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, hs, nheavy, 2L);
    with_bwd_tab([&](auto tab) {
      hipLaunchKernelGGL((k_backward<decltype(tab), true>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, a, n);
      return 0;
    });
    scan_counts(a.cnt_cool, start_cool, mc, tmp_c, hs);
    scan_counts(a.cnt_coul, start_coul, mk, tmp_k, hs);
    hipError_t ce = hipMemcpyAsync(cur_cool, start_cool, sizeof(unsigned) * (mc + mk), hipMemcpyDeviceToDevice, hs);
    if (ce != hipSuccess) return hip_fail(ce, "rc_cool_step_backward: cursor copy");
    hipLaunchKernelGGL(k_order, dim3(4096), dim3(256), 0, hs, (const unsigned*)a.key_cool, cur_cool, order_cool, nrec);
    hipLaunchKernelGGL(k_order, dim3(4096), dim3(256), 0, hs, (const unsigned*)a.key_coul, cur_coul, order_coul, nrec);
    hipLaunchKernelGGL(k_gather_records<true>, dim3(4096), dim3(256), 0, hs, (const unsigned*)start_cool,
                       (const unsigned*)a.cnt_cool, (const unsigned*)order_cool, (const double*)a.rec_cool,
                       a.g_cool_cells, mc, heavy_cool, nheavy);
    hipLaunchKernelGGL(k_gather_records<false>, dim3(4096), dim3(256), 0, hs, (const unsigned*)start_coul,
                       (const unsigned*)a.cnt_coul, (const unsigned*)order_coul, (const double*)a.rec_coul,
                       a.g_coul_cells, mk, heavy_coul, nheavy + 1);
    hipLaunchKernelGGL(k_gather_heavy<true>, dim3(1024), dim3(256), 0, hs, (const unsigned*)start_cool,
                       (const unsigned*)a.cnt_cool, (const unsigned*)order_cool, (const double*)a.rec_cool,
                       a.g_cool_cells, (const unsigned*)heavy_cool, (const unsigned*)nheavy);
    hipLaunchKernelGGL(k_gather_heavy<false>, dim3(1024), dim3(256), 0, hs, (const unsigned*)start_coul,
                       (const unsigned*)a.cnt_coul, (const unsigned*)order_coul, (const double*)a.rec_coul,
                       a.g_coul_cells, (const unsigned*)heavy_coul, (const unsigned*)(nheavy + 1));
    hipLaunchKernelGGL(k_finish_cells, dim3(4096), dim3(256), 0, hs, a.o_tab, (const double*)a.g_cool_cells,
                       (const double*)a.g_coul_cells, ca.n[0], ca.n[1], ca.n[2], ka.n[0], ka.n[1], ka.n[2]);
  } else {
    with_bwd_tab([&](auto tab) {
      hipLaunchKernelGGL((k_backward<decltype(tab), false>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, a, n);
      return 0;
    });
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rc_cool_step_backward launch");
  return RC_OK;
}

extern "C" rc_status rc_selftest_backward_host(const rc_table_spec* spec, const float* resid, const double* coeffs,
                                               const double* n_e, const double* T_e, const double* T_i,
                                               const double* B, const double* H, const double* T_e_new,
                                               const double* T_i_new, const uint8_t* status,
                                               const double* cot_T_e_new, const double* cot_T_i_new,
                                               const double* cot_Q_rad, const double* cot_Q_cc, int64_t n,
                                               double dt, const rc_step_opts* opts, double* g_n_e, double* g_T_e,
                                               double* g_T_i, double* g_B, double* g_H, double* g_tables) {
  if (!spec_ok(spec) || !resid || !coeffs) return set_error(RC_EINVAL, "rc_selftest_backward_host: bad table arguments");
  if (!n_e || !T_e || !T_i || !B || !H || !opts || n < 0)
    return set_error(RC_EINVAL, "rc_selftest_backward_host: bad argument");
  rc_tables_s host;
  host.spec = *spec;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) host.coef[k][j] = coeffs[4 * k + j];
  StepParams P;
  rc_status st = make_params(&host, dt, opts, &P, true);
  if (st != RC_OK) return st;
  const bool newton = opts->scheme == RC_SCHEME_NEWTON;
  if (opts->scheme == RC_SCHEME_EXPLICIT16) return set_error(RC_EUNSUPPORTED, "explicit scheme has no adjoint");
  if (newton && (!T_e_new || !T_i_new || !status)) return set_error(RC_EINVAL, "forward outputs required");
  const long vc = (long)volume(spec->cool);
  const std::vector<float> stored = storage_values(*spec, resid);
  std::vector<float4> cool((size_t)vc);
  for (long i = 0; i < vc; ++i) cool[i] = make_float4(stored[i], stored[vc + i], stored[2 * vc + i], 0.0f);
  GlobalTab tab{cool.data(), stored.data() + 3 * vc, spec->cool.n[1], spec->cool.n[2], spec->coul.n[1],
                spec->coul.n[2]};
  struct HostScatter {
    enum { kRecords = 0 };
    double* g;
    long vc;
    void cool(const long* idx, const double* vb, const double* vse) const {
      for (int k = 0; k < 8; ++k) {
        g[idx[k]] += vb[k];
        g[vc + idx[k]] += vse[k];
        g[2 * vc + idx[k]] += vse[k];
      }
    }
    void coul(const long* idx, const double* vc_) const {
      for (int k = 0; k < 8; ++k) g[3 * vc + idx[k]] += vc_[k];
    }
  } sc{g_tables, vc};
  for (int64_t i = 0; i < n; ++i) {
    CellGrad g;
    cell_vjp(tab, P, spec->cool.n[1], spec->cool.n[2], spec->coul.n[1], spec->coul.n[2], n_e[i], T_e[i], T_i[i],
             B[i], H[i], 0.0, newton ? T_e_new[i] : T_e[i], newton ? T_i_new[i] : T_i[i], status ? status[i] : 0,
             cot_T_e_new ? cot_T_e_new[i] : 0.0, cot_T_i_new ? cot_T_i_new[i] : 0.0,
             cot_Q_rad ? cot_Q_rad[i] : 0.0, cot_Q_cc ? cot_Q_cc[i] : 0.0, newton, g_tables != nullptr, &g, sc);
    if (g_n_e) g_n_e[i] = g.n_e;
    if (g_T_e) g_T_e[i] = g.T_e;
    if (g_T_i) g_T_i[i] = g.T_i;
    if (g_B) g_B[i] = g.B;
    if (g_H) g_H[i] = g.H;
  }
  return RC_OK;
}
