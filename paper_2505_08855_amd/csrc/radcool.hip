// C-ABI front end of the cooling library (include/radcool.h): argument
// validation, error reporting, table build / import / export / file I/O and
// the launch of the per-cell step kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "radcool.h"
#include "rc_internal.hpp"

namespace {

thread_local std::string g_err;

rc_status fail(rc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

namespace rc {

rc_status set_error(rc_status s, const char* msg) { return fail(s, msg); }

rc_status hip_fail(hipError_t e, const char* what) {
  return fail(RC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool axes_ok(const rc_axes& a) {
  for (int k = 0; k < 3; ++k) {
    if (a.n[k] < 2 || a.n[k] > 4096) return false;
    if (!std::isfinite(a.lo[k]) || !std::isfinite(a.hi[k]) || !(a.lo[k] < a.hi[k])) return false;
  }
  const double vol = (double)a.n[0] * a.n[1] * a.n[2];
  return vol <= (double)(1LL << 31);
}

bool spec_ok(const rc_table_spec* s) {
  return s && axes_ok(s->cool) && axes_ok(s->coul) && std::isfinite(s->ln_lambda) && s->ln_lambda > 0.0 &&
         (s->value_dtype == RC_VALUE_F32 || s->value_dtype == RC_VALUE_BF16) &&
         (s->compton_exponent == RC_COMPTON_DERIVED || s->compton_exponent == RC_COMPTON_LITERAL) &&
         (s->theta_i_mass == RC_THETA_I_MP || s->theta_i_mass == RC_THETA_I_ME) && s->reserved == 0 &&
         (s->external_storage != nullptr || s->external_bytes == 0);
}

StorageLayout storage_layout(const rc_table_spec& s) {
  const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const bool bf = s.value_dtype == RC_VALUE_BF16;
  const size_t vc = (size_t)volume(s.cool), vk = (size_t)volume(s.coul);
  const size_t mc = (size_t)(s.cool.n[0] - 1) * (s.cool.n[1] - 1) * (s.cool.n[2] - 1);
  const size_t mk = (size_t)(s.coul.n[0] - 1) * (s.coul.n[1] - 1) * (s.coul.n[2] - 1);
  StorageLayout L;
  L.cells = !bf;
  L.geom = 0;
  L.cool = up(sizeof(TableGeom));
  L.coul = L.cool + up((bf ? 8 : 16) * vc);
  L.cool_cells = L.coul + up((bf ? 2 : 4) * vk);
  L.coul_cells = L.cool_cells + (L.cells ? up(8 * sizeof(float2) * mc) : 0);
  L.total = L.coul_cells + (L.cells ? up(8 * sizeof(float) * mk) : 0);
  return L;
}

int64_t volume(const rc_axes& a) { return (int64_t)a.n[0] * a.n[1] * a.n[2]; }

void fill_axes(const rc_table_spec& s, AxisP ax[6]) {
  for (int k = 0; k < 3; ++k) {
    ax[k].lo = s.cool.lo[k];
    ax[k].inv_d = (double)(s.cool.n[k] - 1) / (s.cool.hi[k] - s.cool.lo[k]);
    ax[k].n = s.cool.n[k];
    ax[3 + k].lo = s.coul.lo[k];
    ax[3 + k].inv_d = (double)(s.coul.n[k] - 1) / (s.coul.hi[k] - s.coul.lo[k]);
    ax[3 + k].n = s.coul.n[k];
  }
}

double node_u(const rc_axes& a, int axis, int k) {
  return a.lo[axis] + k * (a.hi[axis] - a.lo[axis]) / (a.n[axis] - 1);
}

}  // namespace rc

using namespace rc;

// ------------------------------------------------------------------ defaults

extern "C" rc_status rc_default_spec(rc_table_spec* spec, int32_t n) {
  if (!spec || n < 2 || n > 4096) return fail(RC_EINVAL, "rc_default_spec: spec is NULL or n outside [2, 4096]");
  const double cl[3] = {15.0, 5.95, -0.5}, ch[3] = {29.0, 12.05, 10.5};
  const double kl[3] = {9.5, 5.95, 5.95}, kh[3] = {20.5, 12.05, 14.05};
  for (int k = 0; k < 3; ++k) {
    spec->cool.n[k] = n; spec->cool.lo[k] = cl[k]; spec->cool.hi[k] = ch[k];
    spec->coul.n[k] = n; spec->coul.lo[k] = kl[k]; spec->coul.hi[k] = kh[k];
  }
  spec->ln_lambda = 20.0;
  spec->value_dtype = RC_VALUE_F32;
  spec->compton_exponent = RC_COMPTON_DERIVED;
  spec->theta_i_mass = RC_THETA_I_MP;
  spec->reserved = 0;
  spec->external_storage = nullptr;
  spec->external_bytes = 0;
  return RC_OK;
}

extern "C" rc_status rc_tables_storage_bytes(const rc_table_spec* spec, uint64_t* bytes) {
  if (!bytes) return fail(RC_EINVAL, "rc_tables_storage_bytes: bytes is NULL");
  if (!spec) return fail(RC_EINVAL, "rc_tables_storage_bytes: spec is NULL");
  rc_table_spec s = *spec;
  s.external_storage = nullptr;
  s.external_bytes = 0;
  if (!spec_ok(&s)) return fail(RC_EINVAL, "rc_tables_storage_bytes: invalid table spec");
  *bytes = (uint64_t)storage_layout(s).total;
  return RC_OK;
}

extern "C" rc_status rc_default_opts(rc_step_opts* o) {
  if (!o) return fail(RC_EINVAL, "rc_default_opts: opts is NULL");
  o->scheme = RC_SCHEME_NEWTON;
  o->variant = RC_VARIANT_AUTO;
  o->max_iter = 60;
  o->block = 0;
  o->T_floor = 1.0e6;
  o->tol = 1.0e-12;
  o->passes = 0;
  o->grid = 0;
  o->rate_dtype = RC_RATE_F64;
  o->reserved = 0;
  return RC_OK;
}

extern "C" const char* rc_last_error(void) { return g_err.c_str(); }

extern "C" int32_t rc_constants(double* out, int32_t n) {
  const double v[8] = {kC, kKB, kH, kME, kMP, kE, kSigmaT, kSigmaSB};
  if (!out || n <= 0) return 0;
  const int32_t m = n < 8 ? n : 8;
  for (int32_t k = 0; k < m; ++k) out[k] = v[k];
  return m;
}

// ------------------------------------------------------------------ tables

namespace rc {

// Least-squares affine function of the node indices on a full grid: the normal
// equations decouple, slope_a = sum y (i_a - mean_a) / sum (i_a - mean_a)^2.
void affine_fit(const double* y, const int n[3], double co[4]) {
  double mean[3], var[3], cov[3] = {0, 0, 0}, ysum = 0.0;
  for (int a = 0; a < 3; ++a) {
    mean[a] = 0.5 * (n[a] - 1);
    // sum over the grid of (i - mean)^2 = (other sizes) * n (n^2 - 1) / 12
    var[a] = (double)n[a] * ((double)n[a] * n[a] - 1.0) / 12.0 * ((double)n[0] * n[1] * n[2] / n[a]);
  }
  int64_t idx = 0;
  for (int i0 = 0; i0 < n[0]; ++i0)
    for (int i1 = 0; i1 < n[1]; ++i1)
      for (int i2 = 0; i2 < n[2]; ++i2, ++idx) {
        const double v = y[idx];
        ysum += v;
        cov[0] += v * (i0 - mean[0]);
        cov[1] += v * (i1 - mean[1]);
        cov[2] += v * (i2 - mean[2]);
      }
  const double vol = (double)n[0] * n[1] * n[2];
  co[0] = ysum / vol;
  for (int a = 0; a < 3; ++a) {
    co[a + 1] = cov[a] / var[a];
    co[0] -= co[a + 1] * mean[a];
  }
}

// float -> bfloat16 bits, round to nearest, ties to even (finite values)
uint16_t bf16_bits(float v) {
  uint32_t b;
  std::memcpy(&b, &v, 4);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

float bf16_round(float v) {
  const uint32_t b = (uint32_t)bf16_bits(v) << 16;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}

// the residuals as stored: rounded to bfloat16 for that storage form
void round_storage(rc_tables_s* t) {
  if (t->spec.value_dtype != RC_VALUE_BF16) return;
  for (float& v : t->resid) v = bf16_round(v);
}

std::vector<float> storage_values(const rc_table_spec& s, const float* resid) {
  const size_t n = (size_t)(3 * volume(s.cool) + volume(s.coul));
  std::vector<float> v(resid, resid + n);
  if (s.value_dtype == RC_VALUE_BF16)
    for (float& x : v) x = bf16_round(x);
  return v;
}

void fill_geom(rc_tables_s* t) {
  fill_axes(t->spec, t->geom.ax);
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) t->geom.coef[k][j] = t->coef[k][j];
  for (int j = 0; j < 4; ++j) t->geom.coef_se[j] = t->coef[1][j] + t->coef[2][j];
  const AxisP &a = t->geom.ax[1], &b = t->geom.ax[4];
  t->geom.same_te = a.lo == b.lo && a.inv_d == b.inv_d && a.n == b.n;
}

rc_status upload(rc_tables_s* t, void* stream) {
  const int64_t vc = volume(t->spec.cool), vk = volume(t->spec.coul);
  const bool bf = t->spec.value_dtype == RC_VALUE_BF16;
  const size_t cool_bytes = (bf ? 8 : 16) * (size_t)vc, coul_bytes = (bf ? 2 : 4) * (size_t)vk;
  std::vector<float> packed;
  std::vector<uint16_t> packed16;
  try {
    if (bf) packed16.resize(4 * (size_t)vc + (size_t)vk);
    else packed.resize(4 * (size_t)vc);
  } catch (...) {
    return fail(RC_ENOMEM, "host allocation of the packed tables failed");
  }
  for (int64_t i = 0; i < vc; ++i) {
    const float v[4] = {t->resid[i], t->resid[vc + i], t->resid[2 * vc + i], 0.0f};
    for (int k = 0; k < 4; ++k) {
      if (bf) packed16[4 * i + k] = bf16_bits(v[k]);
      else packed[4 * i + k] = v[k];
    }
  }
  if (bf)
    for (int64_t i = 0; i < vk; ++i) packed16[4 * vc + i] = bf16_bits(t->resid[3 * vc + i]);
  fill_geom(t);
  hipError_t e = hipSuccess;
  hipStream_t s = (hipStream_t)stream;
  if (t->external) {
    // the caller's storage: parts at the offsets of storage_layout
    char* base = (char*)t->spec.external_storage;
    const StorageLayout L = storage_layout(t->spec);
    t->d_geom = (TableGeom*)(base + L.geom);
    t->d_cool = base + L.cool;
    t->d_coul = base + L.coul;
  } else {
    e = hipMalloc(&t->d_geom, sizeof(TableGeom));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(table geometry)");
    e = hipMalloc(&t->d_cool, cool_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(cooling tables)");
    e = hipMalloc(&t->d_coul, coul_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(Coulomb table)");
  }
  e = hipMemcpy(t->d_geom, &t->geom, sizeof(TableGeom), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "table geometry upload");
  const void* hc = bf ? (const void*)packed16.data() : (const void*)packed.data();
  const void* hk = bf ? (const void*)(packed16.data() + 4 * vc) : (const void*)(t->resid.data() + 3 * vc);
  e = hipMemcpyAsync(t->d_cool, hc, cool_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(t->d_coul, hk, coul_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  // external storage of FP32 tables holds the cell-blocked copy too: built
  // now, so that no later call allocates it
  if (t->external && t->spec.value_dtype == RC_VALUE_F32) return ensure_cells(t, s);
  return RC_OK;
}

// cell-blocked copies: corner (a, b, c) of cell (i0, i1, i2) at
// ((i0 (n1 - 1) + i1) (n2 - 1) + i2) 8 + a 4 + b 2 + c; the cooling copy holds
// the solver's {brem, se} pair of each corner
__global__ __launch_bounds__(256) void k_cells_cool(const float4* nodes, float2* cells, int n0, int n1, int n2) {
  const int64_t total = (int64_t)(n0 - 1) * (n1 - 1) * (n2 - 1) * 8;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(j & 7);
    int64_t c = j >> 3;
    const int i2 = (int)(c % (n2 - 1));
    c /= (n2 - 1);
    const int i1 = (int)(c % (n1 - 1));
    const int i0 = (int)(c / (n1 - 1));
    cells[j] = brem_se(nodes[((int64_t)(i0 + (k >> 2)) * n1 + i1 + ((k >> 1) & 1)) * n2 + i2 + (k & 1)]);
  }
}

__global__ __launch_bounds__(256) void k_cells_coul(const float* nodes, float* cells, int n0, int n1, int n2) {
  const int64_t total = (int64_t)(n0 - 1) * (n1 - 1) * (n2 - 1) * 8;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(j & 7);
    int64_t c = j >> 3;
    const int i2 = (int)(c % (n2 - 1));
    c /= (n2 - 1);
    const int i1 = (int)(c % (n1 - 1));
    const int i0 = (int)(c / (n1 - 1));
    cells[j] = nodes[((int64_t)(i0 + (k >> 2)) * n1 + i1 + ((k >> 1) & 1)) * n2 + i2 + (k & 1)];
  }
}

rc_status ensure_cells(rc_tables_s* t, hipStream_t s) {
  if (t->spec.value_dtype != RC_VALUE_F32)
    return set_error(RC_EUNSUPPORTED, "the cell-blocked table layout holds FP32 tables only");
  std::lock_guard<std::mutex> lock(t->cells_lock);
  if (t->d_cool_cells && t->d_coul_cells) return RC_OK;
  const rc_axes &a = t->spec.cool, &k = t->spec.coul;
  const int64_t nc = (int64_t)(a.n[0] - 1) * (a.n[1] - 1) * (a.n[2] - 1) * 8;
  const int64_t nk = (int64_t)(k.n[0] - 1) * (k.n[1] - 1) * (k.n[2] - 1) * 8;
  void *dc = nullptr, *dk = nullptr;
  hipError_t e = hipSuccess;
  if (t->external) {
    const StorageLayout L = storage_layout(t->spec);
    dc = (char*)t->spec.external_storage + L.cool_cells;
    dk = (char*)t->spec.external_storage + L.coul_cells;
  } else {
    e = hipMalloc(&dc, sizeof(float2) * nc);
    if (e == hipSuccess) e = hipMalloc(&dk, sizeof(float) * nk);
  }
  if (e == hipSuccess) {
    const auto grid = [](int64_t m) { return (unsigned)std::min<int64_t>((m + 255) / 256, 1 << 16); };
    hipLaunchKernelGGL(k_cells_cool, dim3(grid(nc)), dim3(256), 0, s, (const float4*)t->d_cool, (float2*)dc, a.n[0],
                       a.n[1], a.n[2]);
    hipLaunchKernelGGL(k_cells_coul, dim3(grid(nk)), dim3(256), 0, s, (const float*)t->d_coul, (float*)dk, k.n[0],
                       k.n[1], k.n[2]);
    e = hipGetLastError();
    // complete before the pointers become visible to calls on other streams
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) {
    if (dc && !t->external) (void)hipFree(dc);
    if (dk && !t->external) (void)hipFree(dk);
    return hip_fail(e, "building the cell-blocked tables");
  }
  t->d_cool_cells = dc;
  t->d_coul_cells = dk;
  return RC_OK;
}

void destroy_tables(rc_tables_s* t) {
  if (!t) return;
  if (!t->external) {
    if (t->d_geom) (void)hipFree(t->d_geom);
    if (t->d_cool) (void)hipFree(t->d_cool);
    if (t->d_coul) (void)hipFree(t->d_coul);
    if (t->d_cool_cells) (void)hipFree(t->d_cool_cells);
    if (t->d_coul_cells) (void)hipFree(t->d_coul_cells);
  }
  if (t->d_counter) (void)hipFree(t->d_counter);
  if (t->d_gscratch) (void)hipFree(t->d_gscratch);
  if (t->d_step_scratch) (void)hipFree(t->d_step_scratch);
  t->magic = 0;
  delete t;
}

rc_status new_tables(const rc_table_spec* spec, rc_tables_s** out) {
  rc_tables_s* t = new (std::nothrow) rc_tables_s();
  if (!t) return fail(RC_ENOMEM, "host allocation of the table handle failed");
  t->spec = *spec;
  t->magic = kTablesMagic;
  if (hipGetDevice(&t->device) != hipSuccess) t->device = -1;
  if (spec->external_storage) {
    // caller-owned device memory on this device, aligned and large enough
    const StorageLayout L = storage_layout(*spec);
    hipPointerAttribute_t pa{};
    const bool on_device = hipPointerGetAttributes(&pa, spec->external_storage) == hipSuccess &&
                           pa.type == hipMemoryTypeDevice && pa.device == t->device;
    (void)hipGetLastError();   // a host pointer leaves an error behind; the message below reports it
    const char* bad = !on_device ? "external_storage is not device memory of the current device"
                    : ((uintptr_t)spec->external_storage & 255) ? "external_storage is not 256-byte aligned"
                    : spec->external_bytes < L.total ? "external_bytes is below rc_tables_storage_bytes(spec)"
                    : nullptr;
    if (bad) {
      delete t;
      return fail(RC_EINVAL, bad);
    }
    t->external = true;
  }
  const int64_t vc = volume(spec->cool), vk = volume(spec->coul);
  try {
    t->resid.assign((size_t)(3 * vc + vk), 0.0f);
  } catch (...) {
    delete t;
    return fail(RC_ENOMEM, "host allocation of table residuals failed");
  }
  *out = t;
  return RC_OK;
}

bool handle_ok(rc_tables t) { return t && t->magic == kTablesMagic; }

}  // namespace rc

// node evaluation: one thread per node
__global__ void k_nodes_cool(rc_axes ax, int compton_literal, double* yb, double* ys, double* ye) {
  const int64_t n = (int64_t)ax.n[0] * ax.n[1] * ax.n[2];
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i2 = (int)(idx % ax.n[2]);
    const int i1 = (int)((idx / ax.n[2]) % ax.n[1]);
    const int i0 = (int)(idx / ((int64_t)ax.n[1] * ax.n[2]));
    const double N = exp10(ax.lo[0] + i0 * (ax.hi[0] - ax.lo[0]) / (ax.n[0] - 1));
    const double T = exp10(ax.lo[1] + i1 * (ax.hi[1] - ax.lo[1]) / (ax.n[1] - 1));
    const double B = exp10(ax.lo[2] + i2 * (ax.hi[2] - ax.lo[2]) / (ax.n[2] - 1));
    yb[idx] = node_brem(N, T);
    node_synch_eta(N, T, B, compton_literal != 0, &ys[idx], &ye[idx]);
  }
}

__global__ void k_nodes_coul(rc_axes ax, double ln_lambda, int theta_i_me, double* yc) {
  const int64_t n = (int64_t)ax.n[0] * ax.n[1] * ax.n[2];
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i2 = (int)(idx % ax.n[2]);
    const int i1 = (int)((idx / ax.n[2]) % ax.n[1]);
    const int i0 = (int)(idx / ((int64_t)ax.n[1] * ax.n[2]));
    const double ne = exp10(ax.lo[0] + i0 * (ax.hi[0] - ax.lo[0]) / (ax.n[0] - 1));
    const double Te = exp10(ax.lo[1] + i1 * (ax.hi[1] - ax.lo[1]) / (ax.n[1] - 1));
    const double Ti = exp10(ax.lo[2] + i2 * (ax.hi[2] - ax.lo[2]) / (ax.n[2] - 1));
    yc[idx] = node_coul(ne, Te, Ti, ln_lambda, theta_i_me != 0);
  }
}

namespace {

rc_status finish_from_values(rc_tables_s* t, const std::vector<double>& y, void* stream) {
  const int64_t vc = volume(t->spec.cool), vk = volume(t->spec.coul);
  for (int k = 0; k < 4; ++k) {
    const rc_axes& a = (k < 3) ? t->spec.cool : t->spec.coul;
    const double* src = y.data() + (k < 3 ? k * vc : 3 * vc);
    const int64_t v = (k < 3) ? vc : vk;
    bool holes = false;
    for (int64_t i = 0; i < v; ++i) {
      if (std::isfinite(src[i])) continue;
      // the literal Compton reading leaves eta nodes without a value (NaN)
      if (!(k == RC_TAB_ETA && t->spec.compton_exponent == RC_COMPTON_LITERAL && std::isnan(src[i])))
        return fail(RC_EDEVICE, "table build produced a non-finite node value");
      holes = true;
    }
    // a table with nodes without a value keeps a zero affine part: the
    // residual is the log2 value itself (NaN stays NaN)
    if (holes) for (int j = 0; j < 4; ++j) t->coef[k][j] = 0.0;
    else affine_fit(src, a.n, t->coef[k]);
    float* dst = t->resid.data() + (k < 3 ? k * vc : 3 * vc);
    int64_t idx = 0;
    for (int i0 = 0; i0 < a.n[0]; ++i0)
      for (int i1 = 0; i1 < a.n[1]; ++i1)
        for (int i2 = 0; i2 < a.n[2]; ++i2, ++idx) {
          const double base = t->coef[k][0] + t->coef[k][1] * i0 + t->coef[k][2] * i1 + t->coef[k][3] * i2;
          dst[idx] = (float)(src[idx] - base);
        }
  }
  round_storage(t);
  return upload(t, stream);
}

}  // namespace

extern "C" rc_status rc_build_tables(const rc_table_spec* spec, void* stream, rc_tables* out) {
  if (!out) return fail(RC_EINVAL, "rc_build_tables: out is NULL");
  *out = nullptr;
  if (!spec_ok(spec)) return fail(RC_EINVAL, "rc_build_tables: invalid table spec");
  rc_tables_s* t = nullptr;
  rc_status st = new_tables(spec, &t);
  if (st != RC_OK) return st;
  const int64_t vc = volume(spec->cool), vk = volume(spec->coul);
  double* d_y = nullptr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMalloc(&d_y, sizeof(double) * (3 * vc + vk));
  if (e != hipSuccess) { destroy_tables(t); return hip_fail(e, "hipMalloc(node values)"); }
  const int blk = 128;
  const int gc = (int)std::min<int64_t>((vc + blk - 1) / blk, 65535);
  const int gk = (int)std::min<int64_t>((vk + blk - 1) / blk, 65535);
  hipLaunchKernelGGL(k_nodes_cool, dim3(gc), dim3(blk), 0, s, spec->cool,
                     spec->compton_exponent == RC_COMPTON_LITERAL ? 1 : 0, d_y, d_y + vc, d_y + 2 * vc);
  hipLaunchKernelGGL(k_nodes_coul, dim3(gk), dim3(blk), 0, s, spec->coul, spec->ln_lambda,
                     spec->theta_i_mass == RC_THETA_I_ME ? 1 : 0, d_y + 3 * vc);
  e = hipGetLastError();
  std::vector<double> y;
  if (e == hipSuccess) {
    try {
      y.resize((size_t)(3 * vc + vk));
    } catch (...) {
      (void)hipFree(d_y);
      destroy_tables(t);
      return fail(RC_ENOMEM, "host allocation of node values failed");
    }
    e = hipMemcpyAsync(y.data(), d_y, sizeof(double) * y.size(), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_y);
  if (e != hipSuccess) { destroy_tables(t); return hip_fail(e, "table node evaluation"); }
  st = finish_from_values(t, y, stream);
  if (st != RC_OK) { destroy_tables(t); return st; }
  *out = t;
  return RC_OK;
}

extern "C" rc_status rc_tables_import(const rc_table_spec* spec, const float* resid, const double* coeffs,
                                      void* stream, rc_tables* out) {
  if (!out) return fail(RC_EINVAL, "rc_tables_import: out is NULL");
  *out = nullptr;
  if (!spec_ok(spec)) return fail(RC_EINVAL, "rc_tables_import: invalid table spec");
  if (!resid || !coeffs) return fail(RC_EINVAL, "rc_tables_import: resid or coeffs is NULL");
  rc_tables_s* t = nullptr;
  rc_status st = new_tables(spec, &t);
  if (st != RC_OK) return st;
  const int64_t vc_i = volume(spec->cool);
  for (size_t i = 0; i < t->resid.size(); ++i) {
    // nodes without a value (NaN) only in the eta table of the literal Compton reading
    const bool hole_ok = spec->compton_exponent == RC_COMPTON_LITERAL && (int64_t)i >= 2 * vc_i &&
                         (int64_t)i < 3 * vc_i && std::isnan(resid[i]);
    if (!std::isfinite(resid[i]) && !hole_ok) {
      destroy_tables(t);
      return fail(RC_EINVAL, "rc_tables_import: non-finite residual");
    }
    t->resid[i] = resid[i];
  }
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) {
      if (!std::isfinite(coeffs[4 * k + j])) { destroy_tables(t); return fail(RC_EINVAL, "rc_tables_import: non-finite coefficient"); }
      t->coef[k][j] = coeffs[4 * k + j];
    }
  round_storage(t);
  st = upload(t, stream);
  if (st != RC_OK) { destroy_tables(t); return st; }
  *out = t;
  return RC_OK;
}

extern "C" rc_status rc_tables_export(rc_tables t, float* resid, double* coeffs) {
  if (!handle_ok(t)) return fail(RC_ESTATE, "rc_tables_export: invalid table handle");
  if (resid) std::memcpy(resid, t->resid.data(), sizeof(float) * t->resid.size());
  if (coeffs)
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) coeffs[4 * k + j] = t->coef[k][j];
  return RC_OK;
}

extern "C" rc_status rc_tables_info(rc_tables t, rc_table_spec* spec, int64_t* n_values) {
  if (!handle_ok(t)) return fail(RC_ESTATE, "rc_tables_info: invalid table handle");
  if (spec) *spec = t->spec;
  if (n_values) *n_values = (int64_t)t->resid.size();
  return RC_OK;
}

extern "C" rc_status rc_tables_destroy(rc_tables t) {
  if (!t) return RC_OK;
  if (!handle_ok(t)) return fail(RC_ESTATE, "rc_tables_destroy: invalid table handle");
  destroy_tables(t);
  return RC_OK;
}

// ------------------------------------------------------------------ file I/O

namespace {

constexpr char kFileMagic[8] = {'R', 'C', 'T', 'A', 'B', 'L', 'E', '4'};

// FNV-1a, 64 bit, over the payload bytes
uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

}  // namespace

extern "C" rc_status rc_tables_save(rc_tables t, const char* path) {
  if (!handle_ok(t)) return fail(RC_ESTATE, "rc_tables_save: invalid table handle");
  if (!path) return fail(RC_EINVAL, "rc_tables_save: path is NULL");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(RC_EIO, std::string("rc_tables_save: cannot open ") + path);
  const uint64_t n = t->resid.size();
  // the file holds the tables, not where they lived
  rc_table_spec spec = t->spec;
  spec.external_storage = nullptr;
  spec.external_bytes = 0;
  uint64_t h = 1469598103934665603ULL;
  h = fnv1a(&spec, sizeof(spec), h);
  h = fnv1a(t->coef, sizeof(t->coef), h);
  h = fnv1a(t->resid.data(), sizeof(float) * n, h);
  bool ok = std::fwrite(kFileMagic, 1, 8, f) == 8 && std::fwrite(&spec, sizeof(spec), 1, f) == 1 &&
            std::fwrite(&n, sizeof(n), 1, f) == 1 && std::fwrite(t->coef, sizeof(t->coef), 1, f) == 1 &&
            std::fwrite(t->resid.data(), sizeof(float), n, f) == n && std::fwrite(&h, sizeof(h), 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? RC_OK : fail(RC_EIO, std::string("rc_tables_save: write failed for ") + path);
}

extern "C" rc_status rc_tables_load(const char* path, void* stream, rc_tables* out) {
  if (!out) return fail(RC_EINVAL, "rc_tables_load: out is NULL");
  *out = nullptr;
  if (!path) return fail(RC_EINVAL, "rc_tables_load: path is NULL");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(RC_EIO, std::string("rc_tables_load: cannot open ") + path);
  char magic[8];
  rc_table_spec spec;
  uint64_t n = 0, h = 0;
  double coef[4][4];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kFileMagic, 8) == 0 &&
            std::fread(&spec, sizeof(spec), 1, f) == 1 && std::fread(&n, sizeof(n), 1, f) == 1 &&
            std::fread(coef, sizeof(coef), 1, f) == 1;
  if (!ok || !spec_ok(&spec) || n != (uint64_t)(3 * volume(spec.cool) + volume(spec.coul))) {
    std::fclose(f);
    return fail(RC_EIO, std::string("rc_tables_load: malformed header in ") + path);
  }
  std::vector<float> resid;
  try {
    resid.resize(n);
  } catch (...) {
    std::fclose(f);
    return fail(RC_ENOMEM, "rc_tables_load: host allocation failed");
  }
  ok = std::fread(resid.data(), sizeof(float), n, f) == n && std::fread(&h, sizeof(h), 1, f) == 1;
  std::fclose(f);
  if (!ok) return fail(RC_EIO, std::string("rc_tables_load: truncated file ") + path);
  uint64_t hc = 1469598103934665603ULL;
  hc = fnv1a(&spec, sizeof(spec), hc);
  hc = fnv1a(coef, sizeof(coef), hc);
  hc = fnv1a(resid.data(), sizeof(float) * n, hc);
  if (hc != h) return fail(RC_EIO, std::string("rc_tables_load: checksum mismatch in ") + path);
  return rc_tables_import(&spec, resid.data(), &coef[0][0], stream, out);
}

// ------------------------------------------------------------------ host self-tests

extern "C" rc_status rc_selftest_node_host(const rc_table_spec* spec, int32_t table, int32_t i0, int32_t i1,
                                           int32_t i2, double* value) {
  if (!spec_ok(spec) || !value || table < 0 || table > 3) return fail(RC_EINVAL, "rc_selftest_node_host: bad argument");
  const rc_axes& a = (table < 3) ? spec->cool : spec->coul;
  if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= a.n[0] || i1 >= a.n[1] || i2 >= a.n[2])
    return fail(RC_EINVAL, "rc_selftest_node_host: node index out of range");
  const double u0 = exp10(node_u(a, 0, i0)), u1 = exp10(node_u(a, 1, i1)), u2 = exp10(node_u(a, 2, i2));
  if (table == RC_TAB_BREM) {
    *value = node_brem(u0, u1);
  } else if (table == RC_TAB_COUL) {
    *value = node_coul(u0, u1, u2, spec->ln_lambda, spec->theta_i_mass == RC_THETA_I_ME);
  } else {
    double ys, ye;
    node_synch_eta(u0, u1, u2, spec->compton_exponent == RC_COMPTON_LITERAL, &ys, &ye);
    *value = (table == RC_TAB_SYNCH) ? ys : ye;
  }
  return RC_OK;
}

extern "C" rc_status rc_selftest_special_host(int32_t which, const double* x, double* y, int64_t n) {
  if (!x || !y || n < 0 || which < 0 || which > 9) return fail(RC_EINVAL, "rc_selftest_special_host: bad argument");
  for (int64_t i = 0; i < n; ++i) {
    double k0, k1, k2;
    switch (which) {
      case 0: case 1: case 2:
        kve012(x[i], &k0, &k1, &k2);
        y[i] = which == 0 ? k0 : (which == 1 ? k1 : k2);
        break;
      case 3: y[i] = exp(ln_tail(x[i])); break;
      case 4: y[i] = solve_xc(x[i]); break;
      case 5: y[i] = flog(x[i]); break;
      case 6: y[i] = flog10(x[i]); break;
      case 7: y[i] = flog1p(x[i]); break;
      case 8: y[i] = fexp(x[i]); break;
      default: y[i] = fexp2(x[i]); break;
    }
  }
  return RC_OK;
}

extern "C" rc_status rc_selftest_step_host(const rc_table_spec* spec, const float* resid, const double* coeffs,
                                           const double* n_e, const double* T_e, const double* T_i,
                                           const double* B, const double* H, const double* T_floor_gas, int64_t n,
                                           double dt,
                                           const rc_step_opts* opts, double* T_e_new, double* T_i_new,
                                           double* Q_rad, double* Q_cc, uint8_t* status) {
  if (!spec_ok(spec) || !resid || !coeffs) return fail(RC_EINVAL, "rc_selftest_step_host: bad table arguments");
  if (!n_e || !T_e || !T_i || !B || !H || !opts || n < 0 || !(dt > 0.0) || !std::isfinite(dt))
    return fail(RC_EINVAL, "rc_selftest_step_host: bad argument");
  rc_tables_s host;                       // host-only handle: no device memory
  host.spec = *spec;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) host.coef[k][j] = coeffs[4 * k + j];
  StepParams P;
  rc_status st = make_params(&host, dt, opts, &P, true);
  if (st != RC_OK) return st;
  const int64_t vc = volume(spec->cool);
  const std::vector<float> stored = storage_values(*spec, resid);
  std::vector<float4> cool((size_t)vc);
  for (int64_t i = 0; i < vc; ++i) cool[i] = make_float4(stored[i], stored[vc + i], stored[2 * vc + i], 0.0f);
  GlobalTab tab{cool.data(), stored.data() + 3 * vc, spec->cool.n[1], spec->cool.n[2], spec->coul.n[1],
                spec->coul.n[2]};
  for (int64_t i = 0; i < n; ++i) {
    CellOut o;
    if (opts->variant == RC_VARIANT_DIRECT) {
      direct_rates(P, n_e[i], T_e[i], T_i[i], B[i], H[i], T_floor_gas ? T_floor_gas[i] : 0.0, &o);
    } else if (opts->scheme == RC_SCHEME_NEWTON && opts->passes == 2 && !bad_input(n_e[i]) && !bad_input(T_e[i]) &&
               !bad_input(T_i[i]) && !bad_input(B[i]) && !bad_input(H[i])) {
      // the two-pass step's per-cell path: the first round, the resume
      // record, then a fresh solver resuming from it (the device passes)
      CellSolver<GlobalTab> first(tab, P);
      const double s0 = first.setup(n_e[i], T_e[i], T_i[i], B[i], H[i], dt, T_floor_gas ? T_floor_gas[i] : 0.0);
      o.status = first.clamp;
      NewtonState ns;
      first.newton_begin(s0, ns);
      if (!first.newton_round(ns, &o)) {
        NewtonResume rec;
        CellSolver<GlobalTab>::save_resume(ns, &rec);
        CellSolver<GlobalTab> second(tab, P);
        const double s1 = second.setup(n_e[i], T_e[i], T_i[i], B[i], H[i], dt, T_floor_gas ? T_floor_gas[i] : 0.0);
        NewtonState ns2;
        second.load_resume(s1, rec, ns2);
        while (!second.newton_round(ns2, &o)) {
        }
      }
    } else {
      cool_cell_any(tab, P, n_e[i], T_e[i], T_i[i], B[i], H[i], T_floor_gas ? T_floor_gas[i] : 0.0, false, &o);
    }
    if (T_e_new) T_e_new[i] = o.T_e_new;
    if (T_i_new) T_i_new[i] = o.T_i_new;
    if (Q_rad) Q_rad[i] = o.q_rad;
    if (Q_cc) Q_cc[i] = o.q_cc;
    if (status) status[i] = o.status;
  }
  return RC_OK;
}
