// The paper-layout 4-D cooling table: GPU build, import / export, and the
// rates kernel that reads it (Sec. II.F, III.A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>

#include "radcool.h"
#include "rc_internal.hpp"
#include "rc_kernels.hpp"
#include "rc_table4d.hpp"

namespace rc {
namespace {

constexpr uint32_t kTable4Magic = 0x52433434u;   // "RC44"

bool axes4_ok(const rc_axes4* a) {
  if (!a) return false;
  int64_t v = 1;
  for (int d = 0; d < 4; ++d) {
    if (a->n[d] < 2 || a->n[d] > 4096 || !std::isfinite(a->lo[d]) || !std::isfinite(a->hi[d]) || !(a->hi[d] > a->lo[d]))
      return false;
    v *= a->n[d];
  }
  return v <= ((int64_t)1 << 31);
}

RC_HD int64_t volume4(const rc_axes4& a) { return (int64_t)a.n[0] * a.n[1] * a.n[2] * a.n[3]; }

Axes4P axes4p(const rc_axes4& a) {
  Axes4P p;
  for (int d = 0; d < 4; ++d) {
    p.a[d].lo = a.lo[d];
    p.a[d].inv_d = (double)(a.n[d] - 1) / (a.hi[d] - a.lo[d]);
    p.a[d].n = a.n[d];
  }
  return p;
}

struct FloatLoad {
  const float* v;
  RC_HD float operator()(long i) const { return v[i]; }
};

__global__ void k_nodes4d(rc_axes4 a, float* out) {
  const int64_t n = volume4(a);
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx;
    double x[4];
    for (int d = 3; d >= 0; --d) {
      const int k = (int)(r % a.n[d]);
      r /= a.n[d];
      x[d] = exp10(a.lo[d] + k * (a.hi[d] - a.lo[d]) / (a.n[d] - 1));
    }
    out[idx] = (float)node_total(x[0], x[1], x[2], x[3]);
  }
}

// Q_rad of one cell from the 4-D table; status: RC_ST_INVALID or the
// cooling-clamp bit
RC_HD void rates4d_cell(const float* v, const Axes4P& A, double T_floor, double n_e, double T_e, double B, double H,
                        double* q, uint8_t* st) {
  if (bad_input(n_e) || bad_input(T_e) || bad_input(B) || bad_input(H)) {
    *q = __builtin_nan("");
    *st = ST_INVALID;
    return;
  }
  const double u[4] = {flog10(H), flog10(B), flog10(n_e), flog10(T_e)};
  bool clamped;
  const double y = interp4(FloatLoad{v}, A, u, &clamped);
  *q = T_e < T_floor ? 0.0 : fexp2(y);
  *st = clamped ? ST_CLAMP_COOL : 0;
}

__global__ __launch_bounds__(256) void k_rates4d(const float* v, Axes4P A, StateArgs s, double T_floor, double* q,
                                                 uint8_t* st, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double qi;
  uint8_t si;
  rates4d_cell(v, A, T_floor, s.n_e[i], s.T_e[i], s.B[i], s.H[i], &qi, &si);
  if (q) q[i] = qi;
  if (st) st[i] = si;
}

}  // namespace
}  // namespace rc

struct rc_table4d_s {
  uint32_t magic = 0;
  int device = -1;
  rc_axes4 axes{};
  float* d_v = nullptr;
};

using namespace rc;

namespace {

bool t4_ok(rc_table4d t) { return t && t->magic == kTable4Magic; }

rc_status new_table4(const rc_axes4* a, rc_table4d_s** out) {
  rc_table4d_s* t = new (std::nothrow) rc_table4d_s();
  if (!t) return set_error(RC_ENOMEM, "host allocation of the 4-D table handle failed");
  t->axes = *a;
  t->magic = kTable4Magic;
  if (hipGetDevice(&t->device) != hipSuccess) t->device = -1;
  const hipError_t e = hipMalloc(&t->d_v, sizeof(float) * volume4(*a));
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "hipMalloc(4-D table)");
  }
  *out = t;
  return RC_OK;
}

void free_table4(rc_table4d_s* t) {
  if (!t) return;
  if (t->d_v) (void)hipFree(t->d_v);
  t->magic = 0;
  delete t;
}

}  // namespace

extern "C" rc_status rc_paper_axes4(rc_axes4* a, int32_t n) {
  if (!a || n < 2 || n > 4096) return set_error(RC_EINVAL, "rc_paper_axes4: axes is NULL or n outside [2, 4096]");
  const double lo[4] = {3.0, 0.0, 2.0, 2.0}, hi[4] = {12.0, 10.0, 25.0, 15.0};
  for (int d = 0; d < 4; ++d) {
    a->n[d] = n;
    a->lo[d] = lo[d];
    a->hi[d] = hi[d];
  }
  return RC_OK;
}

extern "C" rc_status rc_build_table4d(const rc_axes4* axes, void* stream, rc_table4d* out) {
  if (!out) return set_error(RC_EINVAL, "rc_build_table4d: out is NULL");
  *out = nullptr;
  if (!axes4_ok(axes)) return set_error(RC_EINVAL, "rc_build_table4d: invalid axes");
  rc_table4d_s* t = nullptr;
  rc_status st = new_table4(axes, &t);
  if (st != RC_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  const int64_t v = volume4(*axes);
  const unsigned grid = (unsigned)std::min<int64_t>((v + 255) / 256, 65535);
  hipLaunchKernelGGL(k_nodes4d, dim3(grid), dim3(256), 0, hs, *axes, t->d_v);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) {
    free_table4(t);
    return hip_fail(e, "rc_build_table4d: node evaluation");
  }
  *out = t;
  return RC_OK;
}

extern "C" rc_status rc_table4d_import(const rc_axes4* axes, const float* values, void* stream, rc_table4d* out) {
  if (!out) return set_error(RC_EINVAL, "rc_table4d_import: out is NULL");
  *out = nullptr;
  if (!axes4_ok(axes) || !values) return set_error(RC_EINVAL, "rc_table4d_import: invalid axes or values NULL");
  const int64_t v = volume4(*axes);
  for (int64_t i = 0; i < v; ++i)
    if (!std::isfinite(values[i])) return set_error(RC_EINVAL, "rc_table4d_import: non-finite value");
  rc_table4d_s* t = nullptr;
  rc_status st = new_table4(axes, &t);
  if (st != RC_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(t->d_v, values, sizeof(float) * v, hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) {
    free_table4(t);
    return hip_fail(e, "rc_table4d_import: upload");
  }
  *out = t;
  return RC_OK;
}

extern "C" rc_status rc_table4d_export(rc_table4d t, rc_axes4* axes, float* values) {
  if (!t4_ok(t)) return set_error(RC_ESTATE, "rc_table4d_export: invalid handle");
  if (axes) *axes = t->axes;
  if (values) {
    const hipError_t e = hipMemcpy(values, t->d_v, sizeof(float) * volume4(t->axes), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rc_table4d_export: download");
  }
  return RC_OK;
}

extern "C" rc_status rc_table4d_destroy(rc_table4d t) {
  if (!t) return RC_OK;
  if (!t4_ok(t)) return set_error(RC_ESTATE, "rc_table4d_destroy: invalid handle");
  free_table4(t);
  return RC_OK;
}

extern "C" rc_status rc_rates4d(rc_table4d t, const rc_state* state, int64_t n, double T_floor, double* Q_rad,
                                uint8_t* status, void* stream) {
  if (!t4_ok(t)) return set_error(RC_ESTATE, "rc_rates4d: invalid handle");
  if (!state || n < 0) return set_error(RC_EINVAL, "rc_rates4d: state is NULL or n < 0");
  if (!(T_floor >= 0.0) || !std::isfinite(T_floor)) return set_error(RC_EINVAL, "rc_rates4d: T_floor must be finite and >= 0");
  if (n > 0 && (!state->n_e || !state->T_e || !state->B || !state->H))
    return set_error(RC_EINVAL, "rc_rates4d: a state pointer is NULL");
  if (n == 0) return RC_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return set_error(RC_ESTATE, "rc_rates4d: the table lives on another device than the current one");
  if ((n + 255) / 256 > 0x7fffffffLL) return set_error(RC_EINVAL, "rc_rates4d: n too large for one launch");
  StateArgs s{state->n_e, state->T_e, state->T_i, state->B, state->H, nullptr};
  hipLaunchKernelGGL(k_rates4d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, t->d_v,
                     axes4p(t->axes), s, T_floor, Q_rad, status, n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RC_OK : hip_fail(e, "rc_rates4d launch");
}

extern "C" rc_status rc_selftest_node4d_host(const double* H, const double* B, const double* n_e, const double* T,
                                             int64_t n, double* log2_q) {
  if (!H || !B || !n_e || !T || !log2_q || n < 0) return set_error(RC_EINVAL, "rc_selftest_node4d_host: bad argument");
  for (int64_t i = 0; i < n; ++i) log2_q[i] = node_total(H[i], B[i], n_e[i], T[i]);
  return RC_OK;
}

extern "C" rc_status rc_selftest_rates4d_host(const rc_axes4* axes, const float* values, const double* n_e,
                                              const double* T_e, const double* B, const double* H, int64_t n,
                                              double T_floor, double* Q_rad, uint8_t* status) {
  if (!axes4_ok(axes) || !values || !n_e || !T_e || !B || !H || !Q_rad || !status || n < 0 || !(T_floor >= 0.0))
    return set_error(RC_EINVAL, "rc_selftest_rates4d_host: bad argument");
  const Axes4P A = axes4p(*axes);
  for (int64_t i = 0; i < n; ++i) rates4d_cell(values, A, T_floor, n_e[i], T_e[i], B[i], H[i], &Q_rad[i], &status[i]);
  return RC_OK;
}
