// Adjoint kernel and the rc_cool_step_backward entry point.
//
// One thread per cell: recompute the interpolant pieces at the forward
// solution and at the input state, solve the transposed 2x2 system and write
// the five input gradients (coalesced).  Table-entry gradients, when asked
// for, take no per-cell floating-point atomics in global memory: every cell
// writes one record per evaluation point (its table cell, coefficients and
// fractional coordinates); the records are grouped by bucket of consecutive
// table cells (LDS histograms, a scan, LDS cursors), each bucket's corner
// contributions are summed in LDS, and a last pass folds the cell-blocked
// sums onto the table nodes.
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
  double* g_cool_cells;   // scratch, per cooling cell and corner k: brem at plane 2k, synch * eta at 2k + 1
  double* g_coul_cells;   // scratch, per Coulomb cell and corner k at plane k (planes of one value per cell)
  unsigned *key_cool, *key_coul;   // gradient records (see RecordScatter)
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
// the table cell it fell in (its key), its coefficients and fractional
// coordinates (cooling: cb, cse, t0, t1, t2; Coulomb: cc, t0, t1, t2).
// Record r = 2 i + p of cell i and point p; its key is ~0u when the point
// contributes nothing.
struct RecordScatter {
  enum { kRecords = 1 };
  unsigned* key_cool;
  double* rec_cool;
  unsigned* key_coul;
  double* rec_coul;
  long r0;
  __device__ void cool_rec(int p, long cell, double cb, double cse, const double* t) const {
    const long r = r0 + p;
    double* q = rec_cool + r * 5;
    q[0] = cb; q[1] = cse; q[2] = t[0]; q[3] = t[1]; q[4] = t[2];
    key_cool[r] = (unsigned)cell;
  }
  __device__ void coul_rec(int p, long cell, double cc, const double* t) const {
    const long r = r0 + p;
    double* q = rec_coul + r * 4;
    q[0] = cc; q[1] = t[0]; q[2] = t[1]; q[3] = t[2];
    key_coul[r] = (unsigned)cell;
  }
};

template <class Tab, bool CELLS>
__global__ __launch_bounds__(256, 2) void k_backward(Tab tab, StepParams P, BwdArgs a, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  using Scatter = typename std::conditional<CELLS, RecordScatter, NoScatter>::type;
  Scatter sc;
  if constexpr (CELLS) {
    sc = RecordScatter{a.key_cool, a.rec_cool, a.key_coul, a.rec_coul, 2 * i};
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

// fold the per-cell gradients onto the nodes: node (i0, i1, i2) is corner
// (a, b, m) of cell (i0 - a, i1 - b, i2 - m) wherever that cell exists; the
// synch * eta gradient goes to both tables' slots.  The cell gradients are
// stored corner-plane by corner-plane (plane p holds one value per table
// cell), so consecutive nodes read consecutive cells of each plane.
__global__ void k_finish_cells(double* g_tab, const double* cool_cells, const double* coul_cells, int n0, int n1,
                               int n2, int m0, int m1, int m2) {
  const long vc = (long)n0 * n1 * n2, vk = (long)m0 * m1 * m2;
  const long mc = (long)(n0 - 1) * (n1 - 1) * (n2 - 1), mk = (long)(m0 - 1) * (m1 - 1) * (m2 - 1);
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
        s0 += cool_cells[(2 * k) * mc + cell];
        s1 += cool_cells[(2 * k + 1) * mc + cell];
      } else {
        s0 += coul_cells[k * mk + cell];
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

// ------------------------------------------------------------------ bucketed table gradients
//
// The records of one table kind are grouped by bucket: cpb consecutive table
// cells, a whole number of LDS windows of kW cells (a window's cell-blocked
// gradients fill 32 KiB), with as few windows per bucket as keep the bucket
// count within kMaxBuckets (one window per bucket up to about 3 million table
// cells).  A count pass builds, per workgroup of kPlaceChunk records, an LDS
// histogram of their buckets and writes it as one column of a bucket-major
// count matrix; an exclusive scan of the matrix gives every (bucket,
// workgroup) pair its first position; a placement pass recounts with LDS
// cursors seeded from the scan and writes each record's index and its table
// cell inside the bucket there (no global atomics).  Then one workgroup per
// slice of at most kSlice records of a bucket adds, window by window, the
// slice's corner contributions into LDS (FP64 atomic adds in LDS) and writes
// the window out: plain stores when the bucket has one slice, global FP64
// atomic adds of the nonzero entries when it has several (crowded table cells
// of coherent inputs; the gradient scratch is zeroed first).  Sums in LDS and
// across slices are taken in a run-dependent order.

constexpr int kWindowBytes = 32768;          // a window's cell-blocked sums (plus one pad double per cell)
constexpr long kMaxBuckets = 12288;          // LDS histogram of 48 KiB
constexpr long kPlaceChunk = 16384;          // records per workgroup of the count and placement passes
constexpr unsigned kSlice = 16384;           // records per workgroup of the accumulation
constexpr int kUnroll = 8;                   // keys in flight per thread (count, placement)
constexpr int kAccUnroll = 4;                // records in flight per thread (accumulation)

template <bool COOL> constexpr int kV = COOL ? 16 : 8;                   // doubles per table cell
template <bool COOL> constexpr int kW = kWindowBytes / (kV<COOL> * 8);   // table cells per LDS window

// table cells per bucket for m table cells: the fewest whole windows that
// keep the number of buckets within kMaxBuckets
template <bool COOL>
long cells_per_bucket(long m) {
  const long per = kW<COOL> * kMaxBuckets;
  return kW<COOL> * ((m + per - 1) / per);
}

__global__ __launch_bounds__(256) void k_bucket_count(const unsigned* key, long nrec, unsigned cpb, int nb,
                                                      unsigned* hist) {
  extern __shared__ unsigned lh[];
  const int tid = (int)threadIdx.x;
  const long g = blockIdx.x, G = gridDim.x;
  for (int b = tid; b < nb; b += blockDim.x) lh[b] = 0u;
  __syncthreads();
  const long r1 = nrec < (g + 1) * kPlaceChunk ? nrec : (g + 1) * kPlaceChunk;
  // kUnroll keys in flight per thread
  for (long rb = g * kPlaceChunk + tid; rb < r1; rb += kUnroll * (long)blockDim.x) {
    unsigned k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = rb + u * (long)blockDim.x < r1 ? key[rb + u * (long)blockDim.x] : ~0u;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (k[u] != ~0u) atomicAdd(&lh[k[u] / cpb], 1u);
  }
  __syncthreads();
  for (int b = tid; b < nb; b += blockDim.x) hist[(long)b * G + g] = lh[b];
}

__global__ __launch_bounds__(256) void k_bucket_place(const unsigned* key, long nrec, unsigned cpb, int nb,
                                                      const unsigned* offs, uint2* order) {
  extern __shared__ unsigned lc[];
  const int tid = (int)threadIdx.x;
  const long g = blockIdx.x, G = gridDim.x;
  for (int b = tid; b < nb; b += blockDim.x) lc[b] = offs[(long)b * G + g];
  __syncthreads();
  const long r1 = nrec < (g + 1) * kPlaceChunk ? nrec : (g + 1) * kPlaceChunk;
  for (long rb = g * kPlaceChunk + tid; rb < r1; rb += kUnroll * (long)blockDim.x) {
    unsigned k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = rb + u * (long)blockDim.x < r1 ? key[rb + u * (long)blockDim.x] : ~0u;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (k[u] == ~0u) continue;
      const unsigned b = k[u] / cpb;
      order[atomicAdd(&lc[b], 1u)] = make_uint2((unsigned)(rb + u * (long)blockDim.x), k[u] - b * cpb);
    }
  }
}

// slices per bucket; the records of bucket b are [offs[b G], offs[(b + 1) G])
// (the last bucket ends at the number of records placed)
__global__ void k_bucket_slices(const unsigned* hist, const unsigned* offs, long G, int nb, unsigned* ns) {
  const unsigned total = offs[(long)nb * G - 1] + hist[(long)nb * G - 1];
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    const unsigned lo = offs[(long)b * G], hi = b + 1 < nb ? offs[(long)(b + 1) * G] : total;
    ns[b] = (hi - lo + kSlice - 1) / kSlice;
  }
}

template <bool COOL>
__global__ __launch_bounds__(256) void k_bucket_accum(const uint2* order, const double* rec, const unsigned* hist,
                                                      const unsigned* offs, long G, unsigned cpb, int nb,
                                                      const unsigned* ns, const unsigned* sstart, double* cells,
                                                      long m) {
  // a window's cell-blocked sums in LDS, V + 1 doubles per cell: the odd
  // stride spreads the lanes' random cells over the LDS banks (with a stride
  // of V doubles every cell starts in the same two banks)
  constexpr int V = kV<COOL>, W = kW<COOL>, RW = COOL ? 5 : 4, VP = V + 1;
  __shared__ double acc[W * VP];
  const unsigned w = blockIdx.x;
  if (w >= sstart[nb - 1] + ns[nb - 1]) return;           // past the last slice (uniform)
  // the slice's bucket: the last b with sstart[b] <= w (buckets without
  // records have no slice and share their successor's start)
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sstart[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  const int b = lo;
  const int tid = (int)threadIdx.x;
  const unsigned total = offs[(long)nb * G - 1] + hist[(long)nb * G - 1];
  const unsigned bend = b + 1 < nb ? offs[(long)(b + 1) * G] : total;
  const unsigned j0 = offs[(long)b * G] + (w - sstart[b]) * kSlice;
  const unsigned j1 = bend - j0 < kSlice ? bend : j0 + kSlice;
  const bool single = ns[b] == 1;
  for (unsigned w0 = 0; w0 < cpb; w0 += W) {
    const long first = (long)b * cpb + w0;                 // first table cell of the window
    if (first >= m) break;                                 // uniform
    for (int i = tid; i < W * VP; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    // kAccUnroll records in flight per thread: their placements, then their records
    for (unsigned jb = j0 + tid; jb < j1; jb += kAccUnroll * blockDim.x) {
      unsigned lc[kAccUnroll], ri[kAccUnroll];
      double q[kAccUnroll][RW];
#pragma unroll
      for (int u = 0; u < kAccUnroll; ++u) {
        const unsigned j = jb + u * blockDim.x;
        const uint2 o = j < j1 ? order[j] : make_uint2(0u, ~0u);
        ri[u] = o.x;
        lc[u] = o.y - w0;                                 // ~0u: past the slice
        if (o.y == ~0u || lc[u] >= (unsigned)W) lc[u] = ~0u;   // or another window's cell
      }
#pragma unroll
      for (int u = 0; u < kAccUnroll; ++u)
        if (lc[u] != ~0u) {
          const double* r = rec + (long)ri[u] * RW;
#pragma unroll
          for (int v = 0; v < RW; ++v) q[u][v] = r[v];
        }
#pragma unroll
      for (int u = 0; u < kAccUnroll; ++u) {
        if (lc[u] == ~0u) continue;
        const double c0 = q[u][0], c1 = COOL ? q[u][1] : 0.0;
        const double t0 = q[u][COOL ? 2 : 1], t1 = q[u][COOL ? 3 : 2], t2 = q[u][COOL ? 4 : 3];
        double* a = acc + lc[u] * VP;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const double wk = ((k >> 2) ? t0 : 1.0 - t0) * (((k >> 1) & 1) ? t1 : 1.0 - t1) * ((k & 1) ? t2 : 1.0 - t2);
          if (COOL) {
            atomicAdd(a + 2 * k, c0 * wk);
            atomicAdd(a + 2 * k + 1, c1 * wk);
          } else {
            atomicAdd(a + k, c0 * wk);
          }
        }
      }
    }
    __syncthreads();
    // out to the corner planes: the window's cells are consecutive in each plane
    const long n_here = m - first < W ? m - first : W;
    for (long i = tid; i < n_here * V; i += blockDim.x) {
      const long p = i / n_here, c = i - p * n_here;
      const double v = acc[c * VP + p];
      double* out = cells + p * m + first + c;
      if (single) *out = v;
      else if (v != 0.0) atomicAdd(out, v);
    }
    __syncthreads();                                       // before the next window clears acc
  }
}

__global__ void k_zero_f64(double* p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
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
  a.key_cool = a.key_coul = nullptr;
  a.rec_cool = a.rec_coul = nullptr;
  const rc_axes &ca = t->spec.cool, &ka = t->spec.coul;
  const long mc = (long)(ca.n[0] - 1) * (ca.n[1] - 1) * (ca.n[2] - 1);   // table cells
  const long mk = (long)(ka.n[0] - 1) * (ka.n[1] - 1) * (ka.n[2] - 1);
  const long nrec = 2 * n;                                               // records per table kind
  if (a.o_tab) {
    // record positions are 32-bit
    if (nrec > 0xfffffffeLL)
      return set_error(RC_EINVAL, "rc_cool_step_backward: n too large for the table-gradient records");
    // buckets of each kind (cells per bucket, bucket count), workgroups of the count and placement passes
    const long cpb_c = cells_per_bucket<true>(mc), cpb_k = cells_per_bucket<false>(mk);
    const long nbc = (mc + cpb_c - 1) / cpb_c, nbk = (mk + cpb_k - 1) / cpb_k;
    const long Gr = (nrec + kPlaceChunk - 1) / kPlaceChunk;
    // scratch: [cooling cells x 16][Coulomb cells x 8][cooling records x 5][Coulomb records x 4] doubles,
    // then uint32: keys (2 x nrec), placed records (2 x nrec uint2), count matrices and their scans
    // (2 x (nbc + nbk) x Gr), slices per bucket and their scans (2 x (nbc + nbk)), scan sums
    const long mat = (nbc + nbk) * Gr;
    const long tmpn = 2 * (((nbc > nbk ? nbc : nbk) * Gr + 1023) / 1024) + 2;   // the largest scan's sums
    if (mat > 0x7fffffffL) return set_error(RC_EINVAL, "rc_cool_step_backward: n too large for the gradient buckets");
    const size_t dbl = sizeof(double) * (size_t)(16 * mc + 8 * mk + 9 * nrec);
    const size_t u32 = sizeof(unsigned) * (size_t)(2 * nrec + 4 * nrec + 2 * mat + 2 * (nbc + nbk) + tmpn);
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
    uint2* order_cool = (uint2*)(u + 2 * nrec);
    uint2* order_coul = order_cool + nrec;
    unsigned* hist_c = u + 6 * nrec;
    unsigned* offs_c = hist_c + nbc * Gr;
    unsigned* hist_k = offs_c + nbc * Gr;
    unsigned* offs_k = hist_k + nbk * Gr;
    unsigned* ns_c = offs_k + nbk * Gr;
    unsigned* ss_c = ns_c + nbc;
    unsigned* ns_k = ss_c + nbc;
    unsigned* ss_k = ns_k + nbk;
    unsigned* tmp = ss_k + nbk;
    hipLaunchKernelGGL(k_zero_f64, dim3(4096), dim3(256), 0, hs, a.g_cool_cells, 16 * mc + 8 * mk);
    with_bwd_tab([&](auto tab) {
      hipLaunchKernelGGL((k_backward<decltype(tab), true>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, a, n);
      return 0;
    });
    // per kind: bucket counts, their scan, placement, slices per bucket and their scan, accumulation
    const auto group = [&](auto cool, const unsigned* key, const double* rec, long m, long cpb, long nb,
                           unsigned* hist, unsigned* offs, uint2* order, unsigned* ns, unsigned* ss, double* cells) {
      constexpr bool C = decltype(cool)::value;
      const size_t lds = sizeof(unsigned) * (size_t)nb;
      hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)Gr), dim3(256), lds, hs, key, nrec, (unsigned)cpb, (int)nb,
                         hist);
      scan_counts(hist, offs, nb * Gr, tmp, hs);
      hipLaunchKernelGGL(k_bucket_place, dim3((unsigned)Gr), dim3(256), lds, hs, key, nrec, (unsigned)cpb, (int)nb,
                         (const unsigned*)offs, order);
      hipLaunchKernelGGL(k_bucket_slices, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, hs, (const unsigned*)hist,
                         (const unsigned*)offs, Gr, (int)nb, ns);
      scan_counts(ns, ss, nb, tmp, hs);
      // at most one slice per bucket plus one per kSlice records
      const unsigned slices = (unsigned)(nb + (nrec + kSlice - 1) / kSlice);
      hipLaunchKernelGGL((k_bucket_accum<C>), dim3(slices), dim3(256), 0, hs, (const uint2*)order, rec,
                         (const unsigned*)hist, (const unsigned*)offs, Gr, (unsigned)cpb, (int)nb,
                         (const unsigned*)ns, (const unsigned*)ss, cells, m);
    };
    group(std::true_type{}, (const unsigned*)a.key_cool, (const double*)a.rec_cool, mc, cpb_c, nbc, hist_c, offs_c,
          order_cool, ns_c, ss_c, a.g_cool_cells);
    group(std::false_type{}, (const unsigned*)a.key_coul, (const double*)a.rec_coul, mk, cpb_k, nbk, hist_k, offs_k,
          order_coul, ns_k, ss_k, a.g_coul_cells);
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
