// Upstream per-cell inputs (thermal scale height, gas-temperature floor), the
// radiation-pressure temperature correction and the downstream coupling of
// the cooling to the gas energy-momentum: elementwise, HBM-bound kernels (one
// read of the inputs, one write of the outputs per cell).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "radcool.h"
#include "rc_disk.hpp"
#include "rc_internal.hpp"

namespace rc {
namespace {

struct DiskArgs {
  const double *rho, *P, *u, *r;
  double *H, *Tf;
  double gamma, a, h_floor, r_g;
};

struct RadpArgs {
  const double *n_e, *T_e, *H;
  double* T_out;
  uint8_t* thick;
  double tau_crit;
};

struct CouplingArgs {
  const double *n_e, *T_e, *T_i, *T_e_new, *T_i_new;
  const double* u[4];
  const double* sqrt_g;
  double* U[4];
  double* lambda;
  double dt;
};

RC_HD bool ok_pos(double v) { return v > 0.0 && std::isfinite(v); }
RC_HD bool ok_nonneg(double v) { return v >= 0.0 && std::isfinite(v); }

// one cell of rc_disk_inputs; invalid inputs give NaN outputs
RC_HD void disk_cell(const DiskArgs& d, int64_t i) {
  const double rho = d.rho[i], P = d.P[i], u = d.u[i], r = d.r[i];
  const bool ok = ok_nonneg(rho) && ok_pos(P) && ok_nonneg(u) && ok_pos(r);
  const double nan = __builtin_nan("");
  if (d.H) d.H[i] = ok ? disk_scale_height(rho, P, u, r, d.a, d.gamma, d.r_g) : nan;
  if (d.Tf) d.Tf[i] = ok ? floor_gas_temperature(r, d.a, d.h_floor) : nan;
}

// one cell of rc_rad_pressure_correction; invalid inputs give NaN, not thick
RC_HD void radp_cell(const RadpArgs& a, int64_t i) {
  const double n_e = a.n_e[i], T_e = a.T_e[i], H = a.H[i];
  const bool ok = ok_pos(n_e) && ok_pos(T_e) && ok_pos(H);
  const bool thick = ok && n_e * kSigmaT * H > a.tau_crit;
  a.T_out[i] = !ok ? __builtin_nan("") : (thick ? rad_pressure_temperature(n_e, T_e) : T_e);
  if (a.thick) a.thick[i] = thick ? 1 : 0;
}

// one cell of rc_apply_cooling: U_mu += dt sqrt(-g) (-lambda u_mu); a cell
// whose lambda is not finite keeps U
RC_HD void coupling_cell(const CouplingArgs& a, int64_t i) {
  const double lam = cooling_lambda(a.n_e[i], a.T_e[i], a.T_i[i], a.T_e_new[i], a.T_i_new[i], a.dt);
  if (a.lambda) a.lambda[i] = std::isfinite(lam) ? lam : __builtin_nan("");
  if (!std::isfinite(lam)) return;
  const double f = -a.dt * (a.sqrt_g ? a.sqrt_g[i] : 1.0) * lam;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
    if (a.U[mu]) a.U[mu][i] += f * a.u[mu][i];
}

__global__ __launch_bounds__(256) void k_coupling(CouplingArgs a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    coupling_cell(a, i);
}

__global__ __launch_bounds__(256) void k_disk_inputs(DiskArgs d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    disk_cell(d, i);
}

__global__ __launch_bounds__(256) void k_rad_pressure(RadpArgs a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    radp_cell(a, i);
}

rc_status disk_args(const double* rho, const double* P, const double* u, const double* r, int64_t n,
                    const rc_disk_params* p, double* H, double* Tf, const char* who, DiskArgs* d) {
  if (n < 0) return set_error(RC_EINVAL, (std::string(who) + ": n < 0").c_str());
  if (!p || !(p->gamma > 1.0) || !std::isfinite(p->gamma) || !(std::fabs(p->spin) <= 1.0) ||
      !(p->h_floor >= 0.0) || !std::isfinite(p->h_floor) || !(p->r_g > 0.0) || !std::isfinite(p->r_g))
    return set_error(RC_EINVAL, (std::string(who) + ": parameters need gamma > 1, |spin| <= 1, h_floor >= 0, r_g > 0").c_str());
  if (n > 0 && (!rho || !P || !u || !r)) return set_error(RC_EINVAL, (std::string(who) + ": an input pointer is NULL").c_str());
  *d = DiskArgs{rho, P, u, r, H, Tf, p->gamma, p->spin, p->h_floor, p->r_g};
  return RC_OK;
}

rc_status radp_args(const double* n_e, const double* T_e, const double* H, int64_t n, double tau_crit,
                    double* T_out, uint8_t* thick, const char* who, RadpArgs* a) {
  if (n < 0) return set_error(RC_EINVAL, (std::string(who) + ": n < 0").c_str());
  if (!(tau_crit >= 0.0) || !std::isfinite(tau_crit)) return set_error(RC_EINVAL, (std::string(who) + ": tau_crit must be finite and >= 0").c_str());
  if (n > 0 && (!n_e || !T_e || !H || !T_out)) return set_error(RC_EINVAL, (std::string(who) + ": a pointer is NULL").c_str());
  *a = RadpArgs{n_e, T_e, H, T_out, thick, tau_crit};
  return RC_OK;
}

rc_status coupling_args(const double* n_e, const double* T_e, const double* T_i, const double* T_e_new,
                        const double* T_i_new, int64_t n, double dt, const rc_coupling* c, double* lambda,
                        const char* who, CouplingArgs* a) {
  if (n < 0) return set_error(RC_EINVAL, (std::string(who) + ": n < 0").c_str());
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(RC_EINVAL, (std::string(who) + ": dt must be finite and > 0").c_str());
  if (!c) return set_error(RC_EINVAL, (std::string(who) + ": coupling is NULL").c_str());
  if (n > 0 && (!n_e || !T_e || !T_i || !T_e_new || !T_i_new || !c->u_cov[0] || !c->u_cov[1] || !c->u_cov[2] ||
                !c->u_cov[3]))
    return set_error(RC_EINVAL, (std::string(who) + ": a state, temperature or velocity pointer is NULL").c_str());
  *a = CouplingArgs{n_e, T_e, T_i, T_e_new, T_i_new, {c->u_cov[0], c->u_cov[1], c->u_cov[2], c->u_cov[3]},
                    c->sqrt_g, {c->U[0], c->U[1], c->U[2], c->U[3]}, lambda, dt};
  return RC_OK;
}

unsigned stream_grid(int64_t n) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t want = (n + 255) / 256, cap = (int64_t)(cus > 0 ? cus : 256) * 16;
  return (unsigned)(want < cap ? want : cap);
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_disk_inputs(const double* rho, const double* P, const double* u, const double* r, int64_t n,
                                    const rc_disk_params* params, double* H_th, double* T_floor_gas, void* stream) {
  DiskArgs d;
  const rc_status st = disk_args(rho, P, u, r, n, params, H_th, T_floor_gas, "rc_disk_inputs", &d);
  if (st != RC_OK || n == 0) return st;
  hipLaunchKernelGGL(k_disk_inputs, dim3(stream_grid(n)), dim3(256), 0, (hipStream_t)stream, d, n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RC_OK : hip_fail(e, "rc_disk_inputs launch");
}

extern "C" rc_status rc_rad_pressure_correction(const double* n_e, const double* T_e, const double* H, int64_t n,
                                                double tau_crit, double* T_e_out, uint8_t* thick, void* stream) {
  RadpArgs a;
  const rc_status st = radp_args(n_e, T_e, H, n, tau_crit, T_e_out, thick, "rc_rad_pressure_correction", &a);
  if (st != RC_OK || n == 0) return st;
  hipLaunchKernelGGL(k_rad_pressure, dim3(stream_grid(n)), dim3(256), 0, (hipStream_t)stream, a, n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RC_OK : hip_fail(e, "rc_rad_pressure_correction launch");
}

extern "C" rc_status rc_selftest_disk_host(const double* rho, const double* P, const double* u, const double* r,
                                           int64_t n, const rc_disk_params* params, double* H_th,
                                           double* T_floor_gas) {
  DiskArgs d;
  const rc_status st = disk_args(rho, P, u, r, n, params, H_th, T_floor_gas, "rc_selftest_disk_host", &d);
  if (st != RC_OK) return st;
  for (int64_t i = 0; i < n; ++i) disk_cell(d, i);
  return RC_OK;
}

extern "C" rc_status rc_selftest_radp_host(const double* n_e, const double* T_e, const double* H, int64_t n,
                                           double tau_crit, double* T_e_out, uint8_t* thick) {
  RadpArgs a;
  const rc_status st = radp_args(n_e, T_e, H, n, tau_crit, T_e_out, thick, "rc_selftest_radp_host", &a);
  if (st != RC_OK) return st;
  for (int64_t i = 0; i < n; ++i) radp_cell(a, i);
  return RC_OK;
}

extern "C" rc_status rc_apply_cooling(const double* n_e, const double* T_e, const double* T_i, const double* T_e_new,
                                      const double* T_i_new, int64_t n, double dt, const rc_coupling* coupling,
                                      double* lambda, void* stream) {
  CouplingArgs a;
  const rc_status st = coupling_args(n_e, T_e, T_i, T_e_new, T_i_new, n, dt, coupling, lambda, "rc_apply_cooling", &a);
  if (st != RC_OK || n == 0) return st;
  hipLaunchKernelGGL(k_coupling, dim3(stream_grid(n)), dim3(256), 0, (hipStream_t)stream, a, n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RC_OK : hip_fail(e, "rc_apply_cooling launch");
}

extern "C" rc_status rc_selftest_coupling_host(const double* n_e, const double* T_e, const double* T_i,
                                               const double* T_e_new, const double* T_i_new, int64_t n, double dt,
                                               const rc_coupling* coupling, double* lambda) {
  CouplingArgs a;
  const rc_status st =
      coupling_args(n_e, T_e, T_i, T_e_new, T_i_new, n, dt, coupling, lambda, "rc_selftest_coupling_host", &a);
  if (st != RC_OK) return st;
  for (int64_t i = 0; i < n; ++i) coupling_cell(a, i);
  return RC_OK;
}
