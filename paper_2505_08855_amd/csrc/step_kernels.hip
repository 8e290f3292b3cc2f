// Step kernels and the rc_cool_step entry point.
//
// One thread per cell.  State arrays are read once, coalesced (FP64 SoA);
// table corners are gathered per table cell by the accessor of the variant;
// outputs are written once, coalesced.
#include <hip/hip_runtime.h>

#include <cmath>

#include "radcool.h"
#include "rc_internal.hpp"
#include "rc_compact.hpp"
#include "rc_kernels.hpp"

namespace rc {

template <int SCHEME, class Tab>
__global__ __launch_bounds__(256) void k_step(Tab tab, StepParams P, StateArgs s, OutArgs o, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CellOut r;
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  cool_cell<SCHEME>(tab, P, P.dt, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], diag, &r);
  store(o, i, r);
}

// Newton with in-workgroup compaction: one tile of kTile cells per workgroup
template <class Tab>
__global__ __launch_bounds__(kTile) void k_newton_compact(Tab tab, StepParams P, StateArgs s, OutArgs o, int64_t n) {
  __shared__ ParkedTile L;
  const int64_t first = (int64_t)blockIdx.x * kTile;
  const int64_t left = n - first;
  const int count = left < kTile ? (int)left : kTile;
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  newton_tile(tab, P, P.dt, first, count, s, o, diag, L);
}

__global__ __launch_bounds__(256) void k_direct(StepParams P, StateArgs s, OutArgs o, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CellOut r;
  direct_rates(P, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], &r);
  store(o, i, r);
}

rc_status make_params(rc_tables t, double dt, const rc_step_opts* o, StepParams* P) {
  if (!o) return set_error(RC_EINVAL, "step options are NULL");
  if (o->scheme < RC_SCHEME_NEWTON || o->scheme > RC_SCHEME_RATES) return set_error(RC_EINVAL, "unknown scheme");
  if (o->variant < RC_VARIANT_AUTO || o->variant > RC_VARIANT_DIRECT) return set_error(RC_EINVAL, "unknown variant");
  if (o->max_iter < 1 || o->max_iter > 1000) return set_error(RC_EINVAL, "max_iter outside [1, 1000]");
  if (!(o->T_floor >= 0.0) || !std::isfinite(o->T_floor)) return set_error(RC_EINVAL, "T_floor must be finite and >= 0");
  if (!(o->tol > 0.0) || !(o->tol < 1.0)) return set_error(RC_EINVAL, "tol must lie in (0, 1)");
  if (o->block != 0 && (o->block < 64 || o->block > 256 || (o->block % 64) != 0))
    return set_error(RC_EINVAL, "block must be 0 or a multiple of 64 in [64, 256]");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(RC_EINVAL, "dt must be finite and > 0");
  fill_axes(t->spec, P->ax);
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) P->coef[k][j] = t->coef[k][j];
  P->dt = dt;
  P->T_floor = o->T_floor;
  P->tol = o->tol;
  P->ln_lambda = t->spec.ln_lambda;
  P->max_iter = o->max_iter;
  P->scheme = o->scheme;
  return RC_OK;
}

void release_textures(rc_tables_s* t) {
  for (int k = 0; k < 4; ++k) {
    if (t->tex[k]) (void)hipDestroyTextureObject(t->tex[k]);
    if (t->tex_arr[k]) (void)hipFreeArray(t->tex_arr[k]);
    t->tex[k] = 0;
    t->tex_arr[k] = nullptr;
  }
  t->tex_ready = false;
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
  int variant = opts->variant == RC_VARIANT_AUTO ? RC_VARIANT_GLOBAL : opts->variant;
  if (variant == RC_VARIANT_DIRECT && opts->scheme != RC_SCHEME_RATES)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step: the DIRECT variant evaluates rates only (scheme RC_SCHEME_RATES)");
  if (variant == RC_VARIANT_LDS || variant == RC_VARIANT_TEX)
    return set_error(RC_EUNSUPPORTED, "rc_cool_step: variant not available in this build");
  if (n == 0) return RC_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return set_error(RC_ESTATE, "rc_cool_step: tables live on another device than the current one");
  StateArgs s{state->n_e, state->T_e, state->T_i, state->B, state->H};
  OutArgs o{out->T_e_new, out->T_i_new, out->Q_rad, out->Q_cc, out->Q_brem, out->Q_syn, out->eta, out->status};
  const int block = opts->block ? opts->block : 256;
  const int64_t grid = (n + block - 1) / block;
  if (grid > 0x7fffffffLL) return set_error(RC_EINVAL, "rc_cool_step: n too large for one launch");
  hipStream_t hs = (hipStream_t)stream;
  if (variant == RC_VARIANT_DIRECT) {
    hipLaunchKernelGGL(k_direct, dim3((unsigned)grid), dim3(block), 0, hs, P, s, o, n);
  } else {
    GlobalTab tab{t->d_cool, t->d_coul, t->spec.cool.n[1], t->spec.cool.n[2], t->spec.coul.n[1], t->spec.coul.n[2]};
    if (opts->scheme == RC_SCHEME_NEWTON && opts->block == 0)
      hipLaunchKernelGGL(k_newton_compact<GlobalTab>, dim3((unsigned)((n + kTile - 1) / kTile)), dim3(kTile), 0, hs,
                         tab, P, s, o, n);
    else if (opts->scheme == RC_SCHEME_NEWTON)
      hipLaunchKernelGGL((k_step<SCHEME_NEWTON, GlobalTab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
    else if (opts->scheme == RC_SCHEME_EXPLICIT16)
      hipLaunchKernelGGL((k_step<SCHEME_EXPLICIT16, GlobalTab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
    else
      hipLaunchKernelGGL((k_step<SCHEME_RATES, GlobalTab>), dim3((unsigned)grid), dim3(block), 0, hs, tab, P, s, o, n);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rc_cool_step launch");
  return RC_OK;
}
