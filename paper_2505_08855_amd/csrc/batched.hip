// Batched form: a persistent kernel over (mesh block, accretion state) work
// items taken from an atomic queue, the entry point rc_cool_step_batched, and
// captured launch plans (hipGraph) with a small autotuner over the launch
// shape.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "radcool.h"
#include "rc_internal.hpp"
#include "rc_kernels.hpp"

namespace rc {

struct BatchArgs {
  const rc_block* blocks;
  int n_blocks;
  int n_states;
  int64_t n_total;
  unsigned* counter;      // work-queue counter
  const double* dt;       // per-state dt, device memory
  unsigned* wg_items;     // per workgroup: work items taken from the queue
};

// device scratch of a batched launch: the counter in the first 256 bytes, the
// per-state dt after it, then one item count per workgroup
constexpr size_t kBatchDtOffset = 256;
constexpr size_t kBatchItemsOffset = kBatchDtOffset + sizeof(double) * RC_MAX_STATES;
constexpr size_t kBatchScratch = kBatchItemsOffset + sizeof(unsigned) * RC_MAX_GRID;

__global__ void k_reset_counter(unsigned* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0u;
}

// Each workgroup repeatedly takes the next block index from the queue and
// advances all of that block's cells; it exits when the index passes the last
// block, which every workgroup reaches because the counter only grows.  On
// exit it records how many items it took.
template <int SCHEME, class Tab>
__global__ __launch_bounds__(256) void k_batched(Tab tab, StepParams P, StateArgs s, OutArgs o, BatchArgs b) {
  __shared__ int item;
  const bool diag = o.Q_brem || o.Q_syn || o.eta;
  unsigned taken = 0;
  for (;;) {
    if (threadIdx.x == 0) item = (int)atomicAdd(b.counter, 1u);
    __syncthreads();
    const int w = item;
    __syncthreads();
    if (w >= b.n_blocks) break;
    ++taken;
    const rc_block blk = b.blocks[w];
    if (blk.first_cell < 0 || blk.n_cells <= 0 || blk.first_cell > b.n_total - blk.n_cells || blk.state_id < 0 ||
        blk.state_id >= b.n_states)
      continue;
    const double dt = b.dt[blk.state_id];
    for (int k = threadIdx.x; k < blk.n_cells; k += blockDim.x) {
      const int64_t i = blk.first_cell + k;
      CellOut r;
      cool_cell<SCHEME>(tab, P, dt, s.n_e[i], s.T_e[i], s.T_i[i], s.B[i], s.H[i], floor_gas_at(s, i), diag, &r);
      store(o, i, r);
    }
  }
  if (threadIdx.x == 0) b.wg_items[blockIdx.x] = taken;
}

namespace {

rc_status check_batch_args(rc_tables t, const rc_state* state, int64_t n_total, const rc_block* blocks,
                           int32_t n_blocks, const double* dts, int32_t n_states, const rc_step_opts* opts,
                           const rc_out* out, StepParams* P, BatchArgs* b) {
  if (!handle_ok(t)) return set_error(RC_ESTATE, "batched: invalid table handle");
  if (!state || !out || !opts) return set_error(RC_EINVAL, "batched: state, out or opts is NULL");
  if (n_total < 0 || n_blocks < 0) return set_error(RC_EINVAL, "batched: negative size");
  if (n_states < 1 || n_states > RC_MAX_STATES || !dts)
    return set_error(RC_EINVAL, "batched: n_states must lie in [1, RC_MAX_STATES] with dt_per_state given");
  for (int k = 0; k < n_states; ++k)
    if (!(dts[k] > 0.0) || !std::isfinite(dts[k])) return set_error(RC_EINVAL, "batched: dt_per_state must be finite and > 0");
  rc_status st = make_params(t, dts[0], opts, P);
  if (st != RC_OK) return st;
  if (opts->variant != RC_VARIANT_AUTO && opts->variant != RC_VARIANT_GLOBAL && opts->variant != RC_VARIANT_CELL)
    return set_error(RC_EUNSUPPORTED, "batched: only the global-table and cell-blocked variants are batched");
  if (n_blocks > 0 && !blocks) return set_error(RC_EINVAL, "batched: blocks is NULL");
  if (n_total > 0 && (!state->n_e || !state->T_e || !state->T_i || !state->B || !state->H))
    return set_error(RC_EINVAL, "batched: a state pointer is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return set_error(RC_ESTATE, "batched: tables live on another device than the current one");
  b->blocks = blocks;
  b->n_blocks = n_blocks;
  b->n_states = n_states;
  b->n_total = n_total;
  return RC_OK;
}

// counter + per-state dt in device scratch; dt copied in on the stream
rc_status fill_scratch(void* scratch, const double* dts, int n_states, hipStream_t hs, BatchArgs* b) {
  b->counter = (unsigned*)scratch;
  b->dt = (const double*)((char*)scratch + kBatchDtOffset);
  b->wg_items = (unsigned*)((char*)scratch + kBatchItemsOffset);
  const hipError_t e = hipMemcpyAsync((char*)scratch + kBatchDtOffset, dts, sizeof(double) * n_states,
                                      hipMemcpyHostToDevice, hs);
  return e == hipSuccess ? RC_OK : hip_fail(e, "batched: copying dt_per_state");
}

// the cell-blocked copy serves AUTO (FP32 tables) and CELL
bool batched_cells(const rc_tables_s* t, const rc_step_opts* opts) {
  return opts->variant == RC_VARIANT_CELL ||
         (opts->variant == RC_VARIANT_AUTO && t->spec.value_dtype == RC_VALUE_F32);
}

hipError_t launch_batched(int scheme, const rc_tables_s* t, bool cells, const StepParams& P, const StateArgs& s,
                          const OutArgs& o, const BatchArgs& b, int block, int grid, hipStream_t hs) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, hs, b.counter);
  const auto launch = [&](auto tab) {
    using Tab = decltype(tab);
    if (scheme == RC_SCHEME_NEWTON)
      hipLaunchKernelGGL((k_batched<SCHEME_NEWTON, Tab>), dim3(grid), dim3(block), 0, hs, tab, P, s, o, b);
    else if (scheme == RC_SCHEME_EXPLICIT16)
      hipLaunchKernelGGL((k_batched<SCHEME_EXPLICIT16, Tab>), dim3(grid), dim3(block), 0, hs, tab, P, s, o, b);
    else
      hipLaunchKernelGGL((k_batched<SCHEME_RATES, Tab>), dim3(grid), dim3(block), 0, hs, tab, P, s, o, b);
    return 0;
  };
  if (cells) {
    launch(cell_tab(t));
  } else {
    with_tab(t, launch);
  }
  return hipGetLastError();
}

int compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

}  // namespace
}  // namespace rc

using namespace rc;

struct rc_plan_s {
  uint32_t magic = 0;
  rc_tables t = nullptr;
  StepParams P;
  StateArgs s;
  OutArgs o;
  BatchArgs b;
  int scheme = 0;
  bool cells = false;   // the step reads the cell-blocked table copy
  int block = 256, grid = 0;
  double tuned_ms = 0.0;
  int last_grid = 0;    // workgroups of the plan's most recent launch (0 = none yet)
  unsigned* counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static constexpr uint32_t kPlanMagic = 0x52435050u;  // "RCPP"

extern "C" rc_status rc_cool_step_batched(rc_tables t, const rc_state* state, int64_t n_total, const rc_block* blocks,
                                          int32_t n_blocks, const double* dt_per_state, int32_t n_states,
                                          const rc_step_opts* opts, const rc_out* out, void* stream) {
  StepParams P;
  BatchArgs b;
  rc_status st = check_batch_args(t, state, n_total, blocks, n_blocks, dt_per_state, n_states, opts, out, &P, &b);
  if (st != RC_OK) return st;
  if (n_blocks == 0 || n_total == 0) return RC_OK;
  const bool cells = batched_cells(t, opts);
  if (cells && (st = ensure_cells(t, (hipStream_t)stream)) != RC_OK) return st;
  if (!t->d_counter) {
    const hipError_t ae = hipMalloc(&t->d_counter, kBatchScratch);
    if (ae != hipSuccess) return hip_fail(ae, "hipMalloc(batched scratch)");
  }
  st = fill_scratch(t->d_counter, dt_per_state, n_states, (hipStream_t)stream, &b);
  if (st != RC_OK) return st;
  StateArgs s{state->n_e, state->T_e, state->T_i, state->B, state->H, state->T_floor_gas};
  const OutArgs o = out_args(out, opts);
  const int block = opts->block ? opts->block : 256;
  const int grid = opts->grid ? opts->grid : compute_units() * 4;
  const hipError_t e = launch_batched(opts->scheme, t, cells, P, s, o, b, block, grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rc_cool_step_batched launch");
  t->batched_grid = grid;
  return RC_OK;
}

namespace {
rc_status copy_items(const void* scratch, int grid, uint32_t* items, int32_t capacity, int32_t* grid_out,
                     const char* who) {
  if (grid <= 0 || !scratch) return set_error(RC_ESTATE, who);
  if (capacity < 0) return set_error(RC_EINVAL, "workgroup items: negative capacity");
  hipError_t e = hipDeviceSynchronize();
  const int m = grid < capacity ? grid : capacity;
  if (e == hipSuccess && items && m > 0)
    e = hipMemcpy(items, (const char*)scratch + kBatchItemsOffset, sizeof(unsigned) * (size_t)m,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "workgroup items: reading the counts");
  if (grid_out) *grid_out = grid;
  return RC_OK;
}
}  // namespace

extern "C" rc_status rc_batched_workgroup_items(rc_tables t, uint32_t* items, int32_t capacity, int32_t* grid) {
  if (!handle_ok(t)) return set_error(RC_ESTATE, "rc_batched_workgroup_items: invalid table handle");
  return copy_items(t->d_counter, t->batched_grid, items, capacity, grid,
                    "rc_batched_workgroup_items: no batched launch on this table handle yet");
}

extern "C" rc_status rc_plan_create(rc_tables t, const rc_state* state, int64_t n_total, const rc_block* blocks,
                                    int32_t n_blocks, const double* dt_per_state, int32_t n_states,
                                    const rc_step_opts* opts, const rc_out* out, int32_t autotune, void* stream,
                                    rc_plan* plan) {
  if (!plan) return set_error(RC_EINVAL, "rc_plan_create: plan is NULL");
  *plan = nullptr;
  StepParams P;
  BatchArgs b;
  rc_status st = check_batch_args(t, state, n_total, blocks, n_blocks, dt_per_state, n_states, opts, out, &P, &b);
  if (st != RC_OK) return st;
  if (n_blocks < 1) return set_error(RC_EINVAL, "rc_plan_create: a plan needs at least one block");
  hipStream_t hs = (hipStream_t)stream;
  // validate every block on the host once
  std::vector<rc_block> hb(n_blocks);
  hipError_t e = hipMemcpyAsync(hb.data(), blocks, sizeof(rc_block) * n_blocks, hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return hip_fail(e, "rc_plan_create: reading blocks");
  for (const rc_block& k : hb)
    if (k.first_cell < 0 || k.n_cells <= 0 || k.first_cell > n_total - k.n_cells || k.state_id < 0 || k.state_id >= n_states)
      return set_error(RC_EINVAL, "rc_plan_create: a block lies outside the state arrays or names an unknown state");
  rc_plan_s* p = new (std::nothrow) rc_plan_s();
  if (!p) return set_error(RC_ENOMEM, "rc_plan_create: host allocation failed");
  p->t = t;
  p->P = P;
  p->s = StateArgs{state->n_e, state->T_e, state->T_i, state->B, state->H, state->T_floor_gas};
  p->o = out_args(out, opts);
  p->b = b;
  p->scheme = opts->scheme;
  p->cells = batched_cells(t, opts);
  if (p->cells && (st = ensure_cells(t, hs)) != RC_OK) {   // before any capture
    delete p;
    return st;
  }
  e = hipMalloc(&p->counter, kBatchScratch);
  if (e != hipSuccess) { delete p; return hip_fail(e, "rc_plan_create: hipMalloc(counter)"); }
  st = fill_scratch(p->counter, dt_per_state, n_states, hs, &p->b);
  if (st == RC_OK && hipStreamSynchronize(hs) != hipSuccess) st = set_error(RC_EDEVICE, "rc_plan_create: copying dt");
  if (st != RC_OK) { (void)hipFree(p->counter); delete p; return st; }
  const int cus = compute_units();
  p->block = opts->block ? opts->block : 256;
  p->grid = opts->grid ? opts->grid : cus * 4;
  if (autotune) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int blocks_c[3] = {64, 128, 256};
    const int per_cu[4] = {1, 2, 4, 8};
    float best = 1e30f;
    for (int bi = 0; bi < 3; ++bi) {
      for (int gi = 0; gi < (opts->grid ? 1 : 4); ++gi) {
        const int blk = blocks_c[bi], grid = opts->grid ? opts->grid : cus * per_cu[gi];
        p->last_grid = grid;
        e = launch_batched(p->scheme, t, p->cells, p->P, p->s, p->o, p->b, blk, grid, hs);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, hs);
        if (e == hipSuccess) e = launch_batched(p->scheme, t, p->cells, p->P, p->s, p->o, p->b, blk, grid, hs);
        if (e == hipSuccess) e = hipEventRecord(e1, hs);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          (void)hipFree(p->counter);
          delete p;
          return hip_fail(e, "rc_plan_create: autotune launch");
        }
        if (ms < best) { best = ms; p->block = blk; p->grid = grid; }
      }
    }
    p->tuned_ms = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  // capture counter reset + persistent kernel on a private stream
  hipStream_t cap;
  e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = launch_batched(p->scheme, t, p->cells, p->P, p->s, p->o, p->b, p->block, p->grid, cap);
    e = hipStreamEndCapture(cap, &p->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->counter);
    delete p;
    return hip_fail(e, "rc_plan_create: graph capture");
  }
  p->magic = kPlanMagic;
  *plan = p;
  return RC_OK;
}

extern "C" rc_status rc_plan_launch(rc_plan plan, void* stream) {
  if (!plan || plan->magic != kPlanMagic) return set_error(RC_ESTATE, "rc_plan_launch: invalid plan");
  if (!handle_ok(plan->t)) return set_error(RC_ESTATE, "rc_plan_launch: the plan's tables were destroyed");
  const hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rc_plan_launch");
  plan->last_grid = plan->grid;
  return RC_OK;
}

extern "C" rc_status rc_plan_workgroup_items(rc_plan plan, uint32_t* items, int32_t capacity, int32_t* grid) {
  if (!plan || plan->magic != kPlanMagic) return set_error(RC_ESTATE, "rc_plan_workgroup_items: invalid plan");
  return copy_items(plan->counter, plan->last_grid, items, capacity, grid,
                    "rc_plan_workgroup_items: the plan has not been launched yet");
}

extern "C" rc_status rc_plan_info(rc_plan plan, int32_t* block, int32_t* grid, double* tuned_ms) {
  if (!plan || plan->magic != kPlanMagic) return set_error(RC_ESTATE, "rc_plan_info: invalid plan");
  if (block) *block = plan->block;
  if (grid) *grid = plan->grid;
  if (tuned_ms) *tuned_ms = plan->tuned_ms;
  return RC_OK;
}

extern "C" rc_status rc_plan_destroy(rc_plan plan) {
  if (!plan) return RC_OK;
  if (plan->magic != kPlanMagic) return set_error(RC_ESTATE, "rc_plan_destroy: invalid plan");
  plan->magic = 0;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->counter) (void)hipFree(plan->counter);
  delete plan;
  return RC_OK;
}
