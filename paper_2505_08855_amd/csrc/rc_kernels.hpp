// Argument blocks and the output store shared by the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "radcool.h"
#include "rc_step.hpp"

namespace rc {

struct StateArgs {
  const double* n_e;
  const double* T_e;
  const double* T_i;
  const double* B;
  const double* H;
  const double* T_floor_gas;   // optional per-cell gas-temperature floor (NULL = none)
};

__device__ inline double floor_gas_at(const StateArgs& s, int64_t i) { return s.T_floor_gas ? s.T_floor_gas[i] : 0.0; }

struct OutArgs {
  double* T_e_new;
  double* T_i_new;
  void* Q_rad;          // double, or float when rates_f32
  void* Q_cc;
  double* Q_brem;
  double* Q_syn;
  double* eta;
  uint8_t* status;
  int rates_f32;        // element type of Q_rad and Q_cc (RC_RATE_F32)
};

inline OutArgs out_args(const rc_out* out, const rc_step_opts* opts) {
  return OutArgs{out->T_e_new, out->T_i_new, out->Q_rad, out->Q_cc, out->Q_brem, out->Q_syn, out->eta, out->status,
                 opts->rate_dtype == RC_RATE_F32 ? 1 : 0};
}

// one rate output element (Q_rad or Q_cc) in the caller's element type
__device__ inline void put_rate(void* p, int f32, int64_t i, double v) {
  if (f32) ((float*)p)[i] = (float)v;
  else ((double*)p)[i] = v;
}

__device__ inline void store(const OutArgs& o, int64_t i, const CellOut& r) {
  if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
  if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
  if (o.Q_rad) put_rate(o.Q_rad, o.rates_f32, i, r.q_rad);
  if (o.Q_cc) put_rate(o.Q_cc, o.rates_f32, i, r.q_cc);
  if (o.Q_brem) o.Q_brem[i] = r.q_brem;
  if (o.Q_syn) o.Q_syn[i] = r.q_syn;
  if (o.eta) o.eta[i] = r.eta;
  if (o.status) o.status[i] = r.status;
}

}  // namespace rc
