// Step kernels and the rc_cool_step entry point.
//
// One thread per cell.  State arrays are read once, coalesced (FP64 SoA);
// table corners are gathered per table cell by the accessor of the variant;
// outputs are written once, coalesced.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "radcool.h"
#include "rc_internal.hpp"
#include "rc_kernels.hpp"
#include "rc_lds.hpp"

namespace rc {

// Occupancy target (waves per SIMD) the register allocator works to for
// each scheme; the Newton solve trades a little spilling for latency hiding.
// Measured on the 256^3 iid step (128^3 tables): the one-kernel solve at 3
// waves per SIMD (168 VGPRs, 6 spilled) 2.18 ms against 2.67 ms at 2 (182
// VGPRs, none spilled) and 2.84 ms at 4 (128 VGPRs, 52 spilled); the
// two-pass step keeps its first pass at 2 and its resumed pass at 3.  Three
// waves hide the table-gather and transcendental latencies well enough; a
// fourth costs more in spill traffic than it hides.
#ifndef RC_NEWTON_WAVES
#define RC_NEWTON_WAVES 3
#endif
#ifndef RC_FIRST_WAVES
#define RC_FIRST_WAVES 2
#endif
#ifndef RC_RESUME_WAVES
#define RC_RESUME_WAVES 3
#endif
template <int SCHEME>
constexpr int kStepWaves = SCHEME == SCHEME_NEWTON ? RC_NEWTON_WAVES : SCHEME == SCHEME_EXPLICIT16 ? 3 : 1;

template <int SCHEME, class Tab>
__global__ __launch_bounds__(256, kStepWaves<SCHEME>) void k_step(Tab tab, StepParams P, StateArgs s, OutArgs o,
                                                                 int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CellOut r;
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  cool_cell<SCHEME>(tab, P, P.dt, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], floor_gas_at(s, i), diag, &r);
  store(o, i, r);
}

// LDS-tiled variant: the fixed table coordinates of every cell, their range
// over the workgroup (a min / max reduction across the lanes of each
// wavefront, then across its wavefronts), staging of the box into LDS, then
// the scheme (every thread of the workgroup reaches both barriers).
// LDS per workgroup: 256 bytes per cell (64 KiB at 256 cells), so that
// residency is set by registers, not LDS, at every workgroup size
constexpr int kLdsPerCell = 256;

template <int SCHEME, class Base>
__global__ __launch_bounds__(256, kStepWaves<SCHEME>) void k_step_lds(Base base, StepParams P, StateArgs s, OutArgs o,
                                                                     int64_t n) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int wred[4][6];        // per wavefront: min and max of the three fixed indices
  const int tid = (int)threadIdx.x;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + tid;
  // fixed table indices of this cell (N, B cooling cells, n_e Coulomb cell);
  // invalid cells and cells past n read no table
  int cl[3] = {INT_MAX, INT_MAX, INT_MAX}, ch[3] = {INT_MIN, INT_MIN, INT_MIN};
  if (i < n) {
    const double n_e = s.n_e[i], B = s.B[i], H = s.H[i];
    if (!(bad_input(n_e) || bad_input(s.T_e[i]) || bad_input(s.T_i[i]) || bad_input(B) || bad_input(H))) {
      const FixedCoords f = fixed_coords(P, n_e, B, H);
      cl[0] = ch[0] = f.N.i;
      cl[1] = ch[1] = f.B.i;
      cl[2] = ch[2] = f.n.i;
    }
  }
  // range of the workgroup's cells: a min / max reduction inside each
  // wavefront, then over the (at most four) wavefronts through LDS
  const int wave = tid >> 6;
  for (int d = 0; d < 3; ++d) {
    cl[d] = wave_min(cl[d]);
    ch[d] = wave_max(ch[d]);
  }
  if ((tid & 63) == 0)
    for (int d = 0; d < 3; ++d) {
      wred[wave][d] = cl[d];
      wred[wave][3 + d] = ch[d];
    }
  __syncthreads();
  const int nw = ((int)blockDim.x + 63) >> 6;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int a = wred[0][d], b = wred[0][3 + d];
    for (int w = 1; w < nw; ++w) {
      a = min(a, wred[w][d]);
      b = max(b, wred[w][3 + d]);
    }
    // uniform over the workgroup: keep it in scalar registers
    lo[d] = __builtin_amdgcn_readfirstlane(a);
    hi[d] = __builtin_amdgcn_readfirstlane(b);
  }
  // the box extent is the cells' index range plus the upper corner of the
  // highest cell; cooling nodes hold the solver's {brem, se} pair (8 bytes)
  const int c1 = base.c1, k1 = base.k1, k2 = base.k2;
  const long budget = (long)kLdsPerCell * blockDim.x;
  int dN = 0, dB = 0, dn = 0;
  if (hi[0] >= lo[0]) {
    dN = hi[0] - lo[0] + 2;
    dB = hi[1] - lo[1] + 2;
    if ((long)dN * c1 * dB * (long)sizeof(float2) > budget) dN = dB = 0;
    dn = hi[2] - lo[2] + 2;
    // the Coulomb box is staged only beside a staged cooling box
    if (dN == 0 || (long)dN * c1 * dB * (long)sizeof(float2) + (long)dn * k1 * k2 * (long)sizeof(float) > budget)
      dn = 0;
  }
  float2* cool_l = (float2*)lds;
  float* coul_l = (float*)(lds + (size_t)dN * c1 * dB * sizeof(float2));
  const int vcool = dN * c1 * dB;
  for (int k = tid; k < vcool; k += (int)blockDim.x) {
    const int b = k % dB, t = (k / dB) % c1, a = k / (dB * c1);
    cool_l[k] = brem_se(base.cool_at(lo[0] + a, t, lo[1] + b));
  }
  const int vcoul = dn * k1 * k2;
  for (int k = tid; k < vcoul; k += (int)blockDim.x) {
    const int c = k % k2, t = (k / k2) % k1, a = k / (k2 * k1);
    coul_l[k] = base.coul_at(lo[2] + a, t, c);
  }
  __syncthreads();
  if (i >= n) return;
  CellOut r;
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  const double n_e = s.n_e[i], T_e = s.T_e[i], T_i = s.T_i[i], B = s.B[i], H = s.H[i], fg = floor_gas_at(s, i);
  if (dN == 0) {
    cool_cell<SCHEME>(base, P, P.dt, n_e, T_e, T_i, B, H, fg, diag, &r);
  } else if (dn == 0) {
    const LdsTab<Base, false> tab{base, cool_l, coul_l, lo[0], lo[1], dB, lo[2]};
    cool_cell<SCHEME>(tab, P, P.dt, n_e, T_e, T_i, B, H, fg, diag, &r);
  } else {
    const LdsTab<Base, true> tab{base, cool_l, coul_l, lo[0], lo[1], dB, lo[2]};
    cool_cell<SCHEME>(tab, P, P.dt, n_e, T_e, T_i, B, H, fg, diag, &r);
  }
  store(o, i, r);
}

// ------------------------------------------------------------------ two-pass Newton step
//
// A wavefront runs as many Newton rounds as its slowest lane, and on
// independent cells the per-cell round count spreads from 1 to 5 (mean 2.3,
// wavefront maximum 4.6 on the iid workload).  The two-pass step regroups the
// work: pass 1 runs every cell's first round (the rates at the input state,
// the first residual, the first proposed step) in cell order and writes out
// the cells it finished; the others leave a 56-byte resume record and a
// difficulty class (the length of the proposed step, which predicts the
// further round count).  A counting sort per tile of kTile cells orders each
// tile's unfinished cells by class, and pass 2 resumes them in that order, so
// that the lanes of a wavefront need similar numbers of further rounds.  The
// per-cell arithmetic is the single-pass kernel's: results are identical.

constexpr int kTile = 4096;                 // cells per sort tile
constexpr uint8_t kClassDone = 0xff;        // class of a cell finished in pass 1

struct ResumeArgs {
  NewtonResume* rec;    // per cell: resume record (unfinished cells only)
  uint8_t* cls;         // per cell: difficulty class, kClassDone when finished
  uint16_t* list;       // per tile: tile-local indices of unfinished cells, by class
  unsigned* count;      // per tile: number of unfinished cells
  int64_t ntiles;
};

template <class Tab>
__global__ __launch_bounds__(256, RC_FIRST_WAVES) void k_newton_first(Tab tab, StepParams P, StateArgs s, OutArgs o,
                                                                     ResumeArgs ra, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double n_e = s.n_e[i], T_e = s.T_e[i], T_i = s.T_i[i], B = s.B[i], H = s.H[i];
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  CellOut r;
  if (bad_input(n_e) || bad_input(T_e) || bad_input(T_i) || bad_input(B) || bad_input(H)) {
    const double nan = __builtin_nan("");
    r.T_e_new = r.T_i_new = r.q_rad = r.q_cc = r.q_brem = r.q_syn = r.eta = nan;
    r.status = ST_INVALID;
    store(o, i, r);
    ra.cls[i] = kClassDone;
    return;
  }
  CellSolver<Tab> cs(tab, P);
  const double s0 = cs.setup(n_e, T_e, T_i, B, H, P.dt, floor_gas_at(s, i));
  r.status = cs.clamp;
  NewtonState ns;
  cs.newton_begin(s0, ns);
  const bool done = cs.newton_round(ns, &r);
  if (diag) cs.diagnostics(s0, &r);
  if (o.Q_rad) put_rate(o.Q_rad, o.rates_f32, i, r.q_rad);
  if (o.Q_cc) put_rate(o.Q_cc, o.rates_f32, i, r.q_cc);
  if (o.Q_brem) o.Q_brem[i] = r.q_brem;
  if (o.Q_syn) o.Q_syn[i] = r.q_syn;
  if (o.eta) o.eta[i] = r.eta;
  if (done) {
    if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
    if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
    if (o.status) o.status[i] = r.status;
    ra.cls[i] = kClassDone;
  } else {
    CellSolver<Tab>::save_resume(ns, &ra.rec[i]);
    ra.cls[i] = (uint8_t)CellSolver<Tab>::resume_class(ns);
  }
}

// one workgroup per tile: counting sort of the tile's unfinished cells by class
__global__ __launch_bounds__(256) void k_tile_sort(ResumeArgs ra, int64_t n) {
  __shared__ unsigned hist[kResumeClasses];
  constexpr int kPer = kTile / 256;
  const int tid = (int)threadIdx.x;
  const int64_t base = blockIdx.x * (int64_t)kTile;
  const int m = (int)(n - base < kTile ? n - base : kTile);
  if (tid < kResumeClasses) hist[tid] = 0u;
  __syncthreads();
  uint8_t c[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int j = tid + 256 * k;
    c[k] = j < m ? ra.cls[base + j] : kClassDone;
    if (c[k] != kClassDone) atomicAdd(&hist[c[k]], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    unsigned acc = 0;
    for (int k = 0; k < kResumeClasses; ++k) {
      const unsigned h = hist[k];
      hist[k] = acc;
      acc += h;
    }
    ra.count[blockIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (c[k] != kClassDone) ra.list[base + atomicAdd(&hist[c[k]], 1u)] = (uint16_t)(tid + 256 * k);
}

// Pass 2: one wavefront per 64 sorted cells of a tile.  Workgroups are dealt
// to the 8 XCDs round-robin, so the mapping below puts all chunks of a tile on
// one XCD, consecutively: the tile's state and records are fetched into one L2.
template <class Tab>
__global__ __launch_bounds__(64, RC_RESUME_WAVES) void k_newton_resume(Tab tab, StepParams P, StateArgs s, OutArgs o,
                                                                     ResumeArgs ra) {
  const int64_t b = blockIdx.x;
  const int64_t slot = b >> 3;
  const int64_t tile = (slot / (kTile / 64)) * 8 + (b & 7);
  const unsigned chunk = (unsigned)(slot % (kTile / 64));
  if (tile >= ra.ntiles) return;
  const unsigned j = chunk * 64u + threadIdx.x;
  if (j >= ra.count[tile]) return;
  const int64_t i = tile * kTile + ra.list[tile * kTile + j];
  CellSolver<Tab> cs(tab, P);
  const double s0 = cs.setup(s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], P.dt, floor_gas_at(s, i));
  CellOut r;
  r.status = cs.clamp;
  NewtonState ns;
  cs.load_resume(s0, ra.rec[i], ns);
  while (!cs.newton_round(ns, &r)) {
  }
  if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
  if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
  if (o.status) o.status[i] = r.status;
}

__global__ __launch_bounds__(256) void k_direct(StepParams P, StateArgs s, OutArgs o, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CellOut r;
  direct_rates(P, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], floor_gas_at(s, i), &r);
  store(o, i, r);
}

// the two-pass step's scratch in the table handle, grown to hold n cells
rc_status step_scratch(rc_tables_s* t, int64_t n, ResumeArgs* ra) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_rec = up(sizeof(NewtonResume) * (size_t)n);
  const size_t b_cls = up((size_t)n);
  const size_t b_list = up(sizeof(uint16_t) * (size_t)ntiles * kTile);
  const size_t b_cnt = up(sizeof(unsigned) * (size_t)ntiles);
  const size_t need = b_rec + b_cls + b_list + b_cnt;
  if (t->step_scratch_bytes < need) {
    if (t->d_step_scratch) (void)hipFree(t->d_step_scratch);
    t->d_step_scratch = nullptr;
    t->step_scratch_bytes = 0;
    const hipError_t e = hipMalloc(&t->d_step_scratch, need);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(two-pass step scratch)");
    t->step_scratch_bytes = need;
  }
  char* p = (char*)t->d_step_scratch;
  ra->rec = (NewtonResume*)p;
  ra->cls = (uint8_t*)(p + b_rec);
  ra->list = (uint16_t*)(p + b_rec + b_cls);
  ra->count = (unsigned*)(p + b_rec + b_cls + b_list);
  ra->ntiles = ntiles;
  return RC_OK;
}

// ------------------------------------------------------------------ allocation-free step
//
// The two-pass step of rc_cool_step_noalloc takes its scratch from this
// file-scope array instead of the table handle.  Sized for kNoAllocMaxCells
// cells: resume records, classes, tile lists and tile counts, each part
// 256-byte aligned, at offsets fixed for the maximum size.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns on each device (every device holds its own copy).
constexpr int64_t kNoAllocMaxCells = RC_NOALLOC_MAX_CELLS;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr int64_t kNoAllocTiles = (kNoAllocMaxCells + kTile - 1) / kTile;
constexpr size_t kNaRec = 0;
constexpr size_t kNaCls = kNaRec + align256(sizeof(NewtonResume) * (size_t)kNoAllocMaxCells);
constexpr size_t kNaList = kNaCls + align256((size_t)kNoAllocMaxCells);
constexpr size_t kNaCount = kNaList + align256(sizeof(uint16_t) * (size_t)kNoAllocTiles * kTile);
constexpr size_t kNaBytes = kNaCount + align256(sizeof(unsigned) * (size_t)kNoAllocTiles);

__device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kMaxDevices = 64;

// the device address of `scratch` on device dev, looked up once per device
// (with dev current) and kept for the life of the process
rc_status noalloc_scratch(int dev, int64_t n, ResumeArgs* ra) {
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return set_error(RC_EDEVICE, "rc_cool_step_noalloc: device index out of range");
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
      const hipError_t e = hipGetSymbolAddress(&ptr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        ptr[dev] = nullptr;
        return hip_fail(e, "rc_cool_step_noalloc: hipGetSymbolAddress(scratch)");
      }
    }
    p = ptr[dev];
  }
  char* b = (char*)p;
  ra->rec = (NewtonResume*)(b + kNaRec);
  ra->cls = (uint8_t*)(b + kNaCls);
  ra->list = (uint16_t*)(b + kNaList);
  ra->count = (unsigned*)(b + kNaCount);
  ra->ntiles = (n + kTile - 1) / kTile;
  return RC_OK;
}

rc_status make_params(rc_tables t, double dt, const rc_step_opts* o, StepParams* P, bool host) {
  if (!o) return set_error(RC_EINVAL, "step options are NULL");
  if (o->scheme < RC_SCHEME_NEWTON || o->scheme > RC_SCHEME_RATES) return set_error(RC_EINVAL, "unknown scheme");
  if (o->variant < RC_VARIANT_AUTO || o->variant > RC_VARIANT_CELL) return set_error(RC_EINVAL, "unknown variant");
  if (o->max_iter < 1 || o->max_iter > 1000) return set_error(RC_EINVAL, "max_iter outside [1, 1000]");
  if (!(o->T_floor >= 0.0) || !std::isfinite(o->T_floor)) return set_error(RC_EINVAL, "T_floor must be finite and >= 0");
  if (!(o->tol > 0.0) || !(o->tol < 1.0)) return set_error(RC_EINVAL, "tol must lie in (0, 1)");
  if (o->block != 0 && (o->block < 64 || o->block > 256 || (o->block % 64) != 0))
    return set_error(RC_EINVAL, "block must be 0 or a multiple of 64 in [64, 256]");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(RC_EINVAL, "dt must be finite and > 0");
  if (o->passes < 0 || o->passes > 2) return set_error(RC_EINVAL, "passes must be 0, 1 or 2");
  if (o->grid < 0 || o->grid > RC_MAX_GRID) return set_error(RC_EINVAL, "grid must lie in [0, RC_MAX_GRID]");
  if (o->rate_dtype != RC_RATE_F64 && o->rate_dtype != RC_RATE_F32)
    return set_error(RC_EINVAL, "rate_dtype must be RC_RATE_F64 or RC_RATE_F32");
  if (o->reserved != 0) return set_error(RC_EINVAL, "reserved option field must be 0");
  if (t->spec.compton_exponent == RC_COMPTON_LITERAL && o->scheme != RC_SCHEME_RATES)
    return set_error(RC_EUNSUPPORTED, "tables of the literal Compton exponent serve the rates scheme only: "
                                      "eta has no value wherever P A > 1, so no energy update is defined there");
  if (host) {
    fill_geom(t);
    P->g = &t->geom;
  } else {
    if (!t->d_geom) return set_error(RC_ESTATE, "table geometry is not on the device");
    P->g = t->d_geom;
  }
  P->dt = dt;
  P->T_floor = o->T_floor;
  P->tol = o->tol;
  P->ln_T_floor = std::log(o->T_floor);
  P->sqrt_tol = std::sqrt(o->tol);
  P->ln_lambda = t->spec.ln_lambda;
  P->max_iter = o->max_iter;
  P->scheme = o->scheme;
  P->compton_literal = t->spec.compton_exponent == RC_COMPTON_LITERAL ? 1 : 0;
  P->theta_i_me = t->spec.theta_i_mass == RC_THETA_I_ME ? 1 : 0;
  return RC_OK;
}


}  // namespace rc

using namespace rc;

namespace {

// rc_cool_step, and with noalloc set rc_cool_step_noalloc: the two-pass
// scratch comes from the static array and the cell-blocked table copy is used
// only if it already exists (AUTO then falls back to the node layout, whose
// results are identical; CELL without it is an error)
rc_status cool_step_impl(rc_tables t, const rc_state* state, int64_t n, double dt, const rc_step_opts* opts,
                         const rc_out* out, void* stream, bool noalloc) {
  if (!handle_ok(t)) return set_error(RC_ESTATE, "rc_cool_step: invalid table handle");
  if (!state || !out) return set_error(RC_EINVAL, "rc_cool_step: state or out is NULL");
  if (n < 0) return set_error(RC_EINVAL, "rc_cool_step: n < 0");
  StepParams P;
  rc_status st = make_params(t, dt, opts, &P);
  if (st != RC_OK) return st;
  if (n > 0 && (!state->n_e || !state->T_e || !state->T_i || !state->B || !state->H))
    return set_error(RC_EINVAL, "rc_cool_step: a state pointer is NULL");
  // AUTO: the cell-blocked copy for FP32 tables (one cache line per cooling
  // corner gather; measured fastest for every scheme), plain global reads for
  // bfloat16 tables
  int variant = opts->variant != RC_VARIANT_AUTO ? opts->variant
              : t->spec.value_dtype == RC_VALUE_F32 ? RC_VARIANT_CELL : RC_VARIANT_GLOBAL;
  if (noalloc) {
    if (n > kNoAllocMaxCells)
      return set_error(RC_EINVAL, "rc_cool_step_noalloc: n exceeds RC_NOALLOC_MAX_CELLS (the static scratch)");
    const bool have_cells = t->d_cool_cells && t->d_coul_cells;
    if (variant == RC_VARIANT_CELL && !have_cells) {
      if (opts->variant == RC_VARIANT_CELL)
        return set_error(RC_ESTATE, "rc_cool_step_noalloc: the cell-blocked table copy does not exist yet (it is "
                                    "built by the first rc_cool_step that reads it)");
      variant = RC_VARIANT_GLOBAL;
    }
  }
  if (variant == RC_VARIANT_DIRECT && opts->scheme != RC_SCHEME_RATES)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step: the DIRECT variant evaluates rates only (scheme RC_SCHEME_RATES)");
  if (variant == RC_VARIANT_TEX)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step: gfx950 exposes no texture sampling to HIP; plain global "
                                      "loads already go through the vector L1 cache (use RC_VARIANT_GLOBAL)");
  if (n == 0) return RC_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return set_error(RC_ESTATE, "rc_cool_step: tables live on another device than the current one");
  StateArgs s{state->n_e, state->T_e, state->T_i, state->B, state->H, state->T_floor_gas};
  const OutArgs o = out_args(out, opts);
  // library choice: one-wavefront workgroups for the Newton solve (measured
  // fastest: a workgroup retires as soon as its slowest cell is done), 256
  // threads for the single-evaluation schemes
  const int block = opts->block ? opts->block : (opts->scheme == RC_SCHEME_NEWTON ? 64 : 256);
  const int64_t grid = (n + block - 1) / block;
  if (grid > 0x7fffffffLL) return set_error(RC_EINVAL, "rc_cool_step: n too large for one launch");
  hipStream_t hs = (hipStream_t)stream;
  // the same launches for every table accessor
  const auto launch = [&](auto tab) -> rc_status {
      using Tab = decltype(tab);
      if (opts->scheme == RC_SCHEME_NEWTON)
        hipLaunchKernelGGL((k_step<SCHEME_NEWTON, Tab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
      else if (opts->scheme == RC_SCHEME_EXPLICIT16)
        hipLaunchKernelGGL((k_step<SCHEME_EXPLICIT16, Tab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
      else
        hipLaunchKernelGGL((k_step<SCHEME_RATES, Tab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
      return RC_OK;
  };
  // two-pass Newton step (identical results; see k_newton_first)
  const bool two_pass = opts->scheme == RC_SCHEME_NEWTON && opts->passes == 2 &&
                        (variant == RC_VARIANT_CELL || variant == RC_VARIANT_GLOBAL);
  const auto launch2 = [&](auto tab) -> rc_status {
      using Tab = decltype(tab);
      ResumeArgs ra;
      rc_status rs = noalloc ? noalloc_scratch(dev, n, &ra) : step_scratch(t, n, &ra);
      if (rs != RC_OK) return rs;
      hipLaunchKernelGGL((k_newton_first<Tab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, ra, n);
      hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)ra.ntiles), dim3(256), 0, hs, ra, n);
      const int64_t g2 = (ra.ntiles + 7) / 8 * 8 * (kTile / 64);
      hipLaunchKernelGGL((k_newton_resume<Tab>), dim3((unsigned)g2), dim3(64), 0, hs, tab, P, s, o, ra);
      return RC_OK;
  };
  if (two_pass && variant == RC_VARIANT_CELL) {
    st = noalloc ? RC_OK : ensure_cells(t, hs);
    if (st != RC_OK) return st;
    st = launch2(cell_tab(t));
    if (st != RC_OK) return st;
  } else if (two_pass) {
    st = with_tab(t, launch2);
    if (st != RC_OK) return st;
  } else if (variant == RC_VARIANT_DIRECT) {
    hipLaunchKernelGGL(k_direct, dim3((unsigned)grid), dim3(block), 0, hs, P, s, o, n);
  } else if (variant == RC_VARIANT_CELL) {
    st = noalloc ? RC_OK : ensure_cells(t, hs);
    if (st != RC_OK) return st;
    st = launch(cell_tab(t));
    if (st != RC_OK) return st;
  } else if (variant == RC_VARIANT_LDS) {
    // workgroups of 256 cells (or opts.block) share one staged box
    const int lb = opts->block ? opts->block : 256;
    const unsigned lg = (unsigned)((n + lb - 1) / lb);
    st = with_tab(t, [&](auto base) -> rc_status {
      using Base = decltype(base);
      if (opts->scheme == RC_SCHEME_NEWTON)
        hipLaunchKernelGGL((k_step_lds<SCHEME_NEWTON, Base>), dim3(lg), dim3(lb), (size_t)kLdsPerCell * lb, hs, base, P, s, o, n);
      else if (opts->scheme == RC_SCHEME_EXPLICIT16)
        hipLaunchKernelGGL((k_step_lds<SCHEME_EXPLICIT16, Base>), dim3(lg), dim3(lb), (size_t)kLdsPerCell * lb, hs, base, P, s, o, n);
      else
        hipLaunchKernelGGL((k_step_lds<SCHEME_RATES, Base>), dim3(lg), dim3(lb), (size_t)kLdsPerCell * lb, hs, base, P, s, o, n);
      return RC_OK;
    });
    if (st != RC_OK) return st;
  } else {
    st = with_tab(t, launch);
    if (st != RC_OK) return st;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rc_cool_step launch");
  return RC_OK;
}

}  // namespace

extern "C" rc_status rc_cool_step(rc_tables t, const rc_state* state, int64_t n, double dt,
                                  const rc_step_opts* opts, const rc_out* out, void* stream) {
  return cool_step_impl(t, state, n, dt, opts, out, stream, false);
}

extern "C" rc_status rc_cool_step_noalloc(rc_tables t, const rc_state* state, int64_t n, double dt,
                                          const rc_step_opts* opts, const rc_out* out, void* stream) {
  return cool_step_impl(t, state, n, dt, opts, out, stream, true);
}
