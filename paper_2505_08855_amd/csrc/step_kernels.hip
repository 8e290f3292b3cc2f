// Step kernels and the rc_cool_step entry point.
//
// One thread per cell.  State arrays are read once, coalesced (FP64 SoA);
// table corners are gathered per table cell by the accessor of the variant;
// outputs are written once, coalesced.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "radcool.h"
#include "rc_internal.hpp"
#include "rc_kernels.hpp"
#include "rc_lds.hpp"

namespace rc {

// Occupancy target (waves per SIMD) the register allocator works to for
// each scheme; the Newton solve trades a little spilling for latency hiding.
#ifndef RC_NEWTON_WAVES
#define RC_NEWTON_WAVES 2
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

// LDS-tiled variant: the fixed table coordinates of every cell, a workgroup
// reduction of their range, staging of the box into LDS, then the scheme
// (every thread of the workgroup reaches both barriers).
// LDS per workgroup: 256 bytes per cell (64 KiB at 256 cells), so that
// residency is set by registers, not LDS, at every workgroup size
constexpr int kLdsPerCell = 256;

template <int SCHEME, class Base>
__global__ __launch_bounds__(256, kStepWaves<SCHEME>) void k_step_lds(Base base, StepParams P, StateArgs s, OutArgs o,
                                                                     int64_t n) {
  extern __shared__ __align__(16) char lds[];
  __shared__ LdsBox box;
  const int tid = (int)threadIdx.x;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + tid;
  if (tid < 3) {
    box.lo[tid] = INT_MAX;
    box.hi[tid] = INT_MIN;
  }
  __syncthreads();
  if (i < n) {
    const double n_e = s.n_e[i], B = s.B[i], H = s.H[i];
    // invalid cells read no table
    if (!(bad_input(n_e) || bad_input(s.T_e[i]) || bad_input(s.T_i[i]) || bad_input(B) || bad_input(H))) {
      const FixedCoords f = fixed_coords(P, n_e, B, H);
      atomicMin(&box.lo[0], f.N.i); atomicMax(&box.hi[0], f.N.i);
      atomicMin(&box.lo[1], f.B.i); atomicMax(&box.hi[1], f.B.i);
      atomicMin(&box.lo[2], f.n.i); atomicMax(&box.hi[2], f.n.i);
    }
  }
  __syncthreads();
  // the box is uniform over the workgroup: keep it in scalar registers; its
  // extent is the cells' index range plus the upper corner of the highest cell
  const int c1 = base.c1, k1 = base.k1, k2 = base.k2;
  const long budget = (long)kLdsPerCell * blockDim.x;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = __builtin_amdgcn_readfirstlane(box.lo[d]);
    hi[d] = __builtin_amdgcn_readfirstlane(box.hi[d]);
  }
  int dN = 0, dB = 0, dn = 0;
  if (hi[0] >= lo[0]) {
    dN = hi[0] - lo[0] + 2;
    dB = hi[1] - lo[1] + 2;
    if ((long)dN * c1 * dB * (long)sizeof(float4) > budget) dN = dB = 0;
    dn = hi[2] - lo[2] + 2;
    // the Coulomb box is staged only beside a staged cooling box
    if (dN == 0 || (long)dN * c1 * dB * (long)sizeof(float4) + (long)dn * k1 * k2 * (long)sizeof(float) > budget)
      dn = 0;
  }
  float4* cool_l = (float4*)lds;
  float* coul_l = (float*)(lds + (size_t)dN * c1 * dB * sizeof(float4));
  const int vcool = dN * c1 * dB;
  for (int k = tid; k < vcool; k += (int)blockDim.x) {
    const int b = k % dB, t = (k / dB) % c1, a = k / (dB * c1);
    cool_l[k] = base.cool_at(lo[0] + a, t, lo[1] + b);
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

__global__ __launch_bounds__(256) void k_direct(StepParams P, StateArgs s, OutArgs o, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CellOut r;
  direct_rates(P, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], floor_gas_at(s, i), &r);
  store(o, i, r);
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
  return RC_OK;
}


}  // namespace rc

using namespace rc;

extern "C" rc_status rc_cool_step(rc_tables t, const rc_state* state, int64_t n, double dt,
                                  const rc_step_opts* opts, const rc_out* out, void* stream) {
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
  OutArgs o{out->T_e_new, out->T_i_new, out->Q_rad, out->Q_cc, out->Q_brem, out->Q_syn, out->eta, out->status};
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
  if (variant == RC_VARIANT_DIRECT) {
    hipLaunchKernelGGL(k_direct, dim3((unsigned)grid), dim3(block), 0, hs, P, s, o, n);
  } else if (variant == RC_VARIANT_CELL) {
    st = ensure_cells(t, hs);
    if (st != RC_OK) return st;
    const rc_table_spec& sp = t->spec;
    st = launch(CellTab{(const float4*)t->d_cool, (const float*)t->d_coul, (const float4*)t->d_cool_cells,
                        (const float*)t->d_coul_cells, sp.cool.n[1], sp.cool.n[2], sp.coul.n[1], sp.coul.n[2]});
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
