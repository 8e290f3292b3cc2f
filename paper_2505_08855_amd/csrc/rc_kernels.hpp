// Argument blocks and the output store shared by the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
  double* Q_rad;
  double* Q_cc;
  double* Q_brem;
  double* Q_syn;
  double* eta;
  uint8_t* status;
};

__device__ inline void store(const OutArgs& o, int64_t i, const CellOut& r) {
  if (o.T_e_new) o.T_e_new[i] = r.T_e_new;
  if (o.T_i_new) o.T_i_new[i] = r.T_i_new;
  if (o.Q_rad) o.Q_rad[i] = r.q_rad;
  if (o.Q_cc) o.Q_cc[i] = r.q_cc;
  if (o.Q_brem) o.Q_brem[i] = r.q_brem;
  if (o.Q_syn) o.Q_syn[i] = r.q_syn;
  if (o.eta) o.eta[i] = r.eta;
  if (o.status) o.status[i] = r.status;
}

}  // namespace rc
