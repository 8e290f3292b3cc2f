// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "radcool.h"
#include "rc_step.hpp"

namespace rc {

constexpr uint32_t kTablesMagic = 0x52435442u;  // "RCTB"

}  // namespace rc

struct rc_tables_s {
  uint32_t magic = 0;
  int device = -1;
  rc_table_spec spec{};
  double coef[4][4] = {};
  std::vector<float> resid;         // host copy of the storage form, [brem][synch][eta][coul]
  float4* d_cool = nullptr;         // interleaved {brem, synch, eta, 0} per cooling node
  float* d_coul = nullptr;          // planar Coulomb residuals
  // texture objects for the sampling variant (created on first use)
  hipArray_t tex_arr[4] = {nullptr, nullptr, nullptr, nullptr};
  hipTextureObject_t tex[4] = {0, 0, 0, 0};
  bool tex_ready = false;
  void* d_counter = nullptr;        // work-queue counter of the batched kernel (allocated on first use)
  void* d_gscratch = nullptr;       // backward: synch * eta table-gradient accumulator (first use)
};

namespace rc {

rc_status set_error(rc_status s, const char* msg);
rc_status hip_fail(hipError_t e, const char* what);
bool handle_ok(rc_tables t);
bool spec_ok(const rc_table_spec* s);
int64_t volume(const rc_axes& a);
void fill_axes(const rc_table_spec& s, AxisP ax[6]);
rc_status make_params(rc_tables t, double dt, const rc_step_opts* o, StepParams* P);
void release_textures(rc_tables_s* t);

}  // namespace rc
