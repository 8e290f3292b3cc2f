// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
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
  // device storage: FP32 form float4 {brem, synch, eta, 0} per cooling node and
  // float per Coulomb node; bfloat16 form uint2 (4 x bf16) and uint16
  void* d_cool = nullptr;
  void* d_coul = nullptr;
  rc::TableGeom geom{};             // axes and affine coefficients (host copy)
  rc::TableGeom* d_geom = nullptr;  // the same in device memory, read by the kernels
  void* d_counter = nullptr;        // work-queue counter of the batched kernel (allocated on first use)
  int batched_grid = 0;             // workgroups of the last rc_cool_step_batched launch (0 = none)
  void* d_gscratch = nullptr;       // backward: table-gradient records and accumulators (first use)
  size_t gscratch_bytes = 0;        // its size (grows with the cell count)
  void* d_step_scratch = nullptr;   // two-pass Newton step: resume records, classes, tile lists (first use)
  size_t step_scratch_bytes = 0;    // its size (grows with the cell count)
  // cell-blocked copies of the FP32 tables (RC_VARIANT_CELL; built on first use)
  void* d_cool_cells = nullptr;
  void* d_coul_cells = nullptr;
  std::mutex cells_lock;
  // geometry, node tables and cell-blocked copy live in the caller's
  // spec.external_storage (not freed by the library)
  bool external = false;
};

namespace rc {

rc_status set_error(rc_status s, const char* msg);
rc_status hip_fail(hipError_t e, const char* what);
bool handle_ok(rc_tables t);
bool spec_ok(const rc_table_spec* s);

// Offsets (bytes, each 256-aligned) of the parts of a table set's device
// memory in external storage, and the total.
struct StorageLayout {
  size_t geom, cool, coul, cool_cells, coul_cells, total;
  bool cells;           // FP32 tables: the cell-blocked copy is part of the storage
};
StorageLayout storage_layout(const rc_table_spec& s);
int64_t volume(const rc_axes& a);
void fill_axes(const rc_table_spec& s, AxisP ax[6]);
// fill t->geom from t->spec and t->coef
void fill_geom(rc_tables_s* t);
// Validate the options and fill P; P->g points to the device copy of the table
// geometry, or with host = true (host self-tests) to the host copy.
rc_status make_params(rc_tables t, double dt, const rc_step_opts* o, StepParams* P, bool host = false);
// host copy of residuals in their storage form (bfloat16-rounded for that form)
std::vector<float> storage_values(const rc_table_spec& s, const float* resid);

// Build the cell-blocked copies of t's FP32 tables on stream s if they do not
// exist yet (allocates; ordered before later work on s).
rc_status ensure_cells(rc_tables_s* t, hipStream_t s);

// Call f with the table accessor of t's storage form (GlobalTab or GlobalTabBF16).
template <class F>
auto with_tab(const rc_tables_s* t, F&& f) {
  const rc_table_spec& s = t->spec;
  if (s.value_dtype == RC_VALUE_BF16)
    return f(GlobalTabBF16{(const uint2*)t->d_cool, (const unsigned short*)t->d_coul, s.cool.n[1], s.cool.n[2],
                           s.coul.n[1], s.coul.n[2]});
  return f(GlobalTab{(const float4*)t->d_cool, (const float*)t->d_coul, s.cool.n[1], s.cool.n[2], s.coul.n[1],
                     s.coul.n[2]});
}

// The accessor of t's cell-blocked copy (ensure_cells has built it).
inline CellTab cell_tab(const rc_tables_s* t) {
  const rc_table_spec& s = t->spec;
  return CellTab{(const float4*)t->d_cool, (const float*)t->d_coul, (const float2*)t->d_cool_cells,
                 (const float*)t->d_coul_cells, s.cool.n[1], s.cool.n[2], s.coul.n[1], s.coul.n[2]};
}

}  // namespace rc
