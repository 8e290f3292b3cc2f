/*
 * radcool.h - C ABI of the MI355X (gfx950) two-temperature radiative cooling
 * source step.
 *
 * The operation (paper "Black hole spectral states revealed in GRMHD
 * simulations with texture memory accelerated cooling", arXiv:2505.08855):
 * for every cell of a GRMHD grid, given the electron density n_e [cm^-3], the
 * electron and ion temperatures T_e, T_i [K], the field strength |B| [G] and
 * the thermal scale height H [cm] (Sections II.F and II.G list the cell
 * parameters), read the cooling and Coulomb rates from log-spaced tables by
 * multilinear interpolation (Section III.A), bridge the optically thin cooling
 * to the thick limit (Section II.D, eq. total_cooling) and update the electron
 * and ion internal energies over dt (Section III.B.1), implicitly (backward
 * Euler, solved by Newton) or explicitly (16 substeps, 30 % limiter), with the
 * temperature floor of Section III.B.2.
 *
 * Conventions shared by every entry point:
 *   - All functions return rc_status: RC_OK (0) or a negative error code; they
 *     never abort.  On error, rc_last_error() returns a message (thread-local,
 *     valid until the next call on the same thread).
 *   - Arguments that can be checked on the host are checked before anything is
 *     launched: NULL required pointers, negative sizes, dt <= 0 or not finite,
 *     malformed table specs give RC_EINVAL and nothing runs.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Step and backward calls are asynchronous on that stream and never
 *     synchronise it; table build, import, export and file I/O are synchronous.
 *   - Per-cell arrays are device pointers to contiguous FP64 arrays of length
 *     n (8-byte aligned; 256-byte alignment gives full-speed loads), owned by
 *     the caller.  Output arrays may not alias inputs.
 *   - Per-cell problems are not errors: they set bits in the status byte and
 *     leave the outputs defined (see RC_ST_*).
 *   - Units are cgs throughout.
 */
#ifndef RADCOOL_H
#define RADCOOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RC_OK = 0,
  RC_EINVAL = -1,        /* bad argument (host-detectable) */
  RC_ENOMEM = -2,        /* device or host allocation failed */
  RC_EDEVICE = -3,       /* a HIP call failed; message has hipGetErrorString */
  RC_EUNSUPPORTED = -4,  /* valid request this build or device cannot serve */
  RC_ESTATE = -5,        /* object in the wrong state (e.g. destroyed handle) */
  RC_EIO = -6            /* file read/write failed or file malformed */
} rc_status;

/* Table identifiers and their content (values stored as log2):
 *   RC_TAB_BREM  log2(N^2 f_brem(theta_e)),     N = n_e H  (Sec. II.A)
 *   RC_TAB_SYNCH log2 Q_syn(N, T_e, B, H = 1cm)            (Sec. II.B, eq. synchrotron)
 *   RC_TAB_ETA   log2 eta_comp(nu_c) at H = 1cm            (Sec. II.C)
 *   RC_TAB_COUL  log2(Q_cc / (T_i - T_e))                  (Sec. II.G, eq. coulomb_collisions)
 * The three cooling tables share the axes (log10 N, log10 T_e, log10 B); the
 * Coulomb table has the axes (log10 n_e, log10 T_e, log10 T_i).  The paper's
 * 4-D cooling table over (H, B, n_e, T_e) reduces exactly to these 3-D tables:
 * every rate depends on n_e and H only through N = n_e H apart from explicit
 * powers of H (Q_brem = v_brem / H^2, Q_syn = v_synch / H, eta = v_eta). */
enum { RC_TAB_BREM = 0, RC_TAB_SYNCH = 1, RC_TAB_ETA = 2, RC_TAB_COUL = 3, RC_NUM_TABLES = 4 };

/* Per-cell status bits (uint8). */
enum {
  RC_ST_INVALID = 1,     /* an input was not finite or <= 0: T' = NaN, rates = NaN */
  RC_ST_CLAMP_COOL = 2,  /* a cooling-table coordinate of the input state was out of range (clamped) */
  RC_ST_CLAMP_COUL = 4,  /* a Coulomb-table coordinate of the input state was out of range (clamped) */
  RC_ST_FLOOR = 8,       /* the implicit update ended on the temperature floor */
  RC_ST_MAXITER = 16,    /* the solver hit max_iter; outputs are the best bracketed iterate */
  RC_ST_GAS_FLOOR = 32,  /* radiative cooling off for the step: input T_e + T_i below T_floor_gas */
  RC_ST_NO_RATE = 64     /* literal Compton reading only (RC_COMPTON_LITERAL): the cooling at the
                            input state has no value, Q_rad = NaN.  Tables: a cooling-table corner
                            of the cell's table cell holds no value (eta <= 0 at that node);
                            DIRECT: eta <= 0 (or not finite) at the cell.  Not set when the
                            cooling is off (T_e < T_floor, or the gas-temperature floor). */
};

/* One table's three axes, log10-spaced: node k of axis a is
 * lo[a] + k (hi[a] - lo[a]) / (n[a] - 1), k = 0 .. n[a]-1.  n[a] >= 2, lo < hi. */
typedef struct {
  int32_t n[3];
  double lo[3];
  double hi[3];
} rc_axes;

/* Storage precision of the table residuals (the values minus their
 * least-squares affine part in node-index space, which is kept in FP64). */
enum { RC_VALUE_F32 = 0, RC_VALUE_BF16 = 1 };

/* Readings of two printed formulas (Sec. II.C and II.G), selectable so that
 * the printed forms stay on record and testable.
 *   compton_exponent: RC_COMPTON_DERIVED (default) takes the Compton
 *     enhancement with the exponent -1 - ln P / ln A, which makes it the
 *     geometric series 1 + P (A-1) sum_{j<k} (PA)^j over k = ln(3 theta/E)/ln A
 *     scatterings; RC_COMPTON_LITERAL takes the exponent 1 - ln P / ln A exactly
 *     as printed, eta = 1 + P (A-1)/(1 - PA) [1 - (E/3 theta)^(1 - ln P/ln A)]
 *     (eta = 1 for E >= 3 theta in both), which is negative wherever P A > 1.
 *     Table nodes where that eta is not positive hold no value (NaN), so the
 *     log2 table cannot be interpolated there: such cells get RC_ST_NO_RATE.
 *     Tables built with RC_COMPTON_LITERAL serve the rates scheme only (rates
 *     at the input state); the Newton and explicit schemes, the batched form
 *     and the backward pass return RC_EUNSUPPORTED for them.
 *   theta_i_mass: RC_THETA_I_MP (default) takes theta_i = k T_i / m_p c^2;
 *     RC_THETA_I_ME takes the printed theta_i = k T_i / m_e c^2.  Only theta_i
 *     changes (the prefactor keeps m_e / m_p).  Both readings give a complete
 *     Coulomb table and every scheme accepts it. */
enum { RC_COMPTON_DERIVED = 0, RC_COMPTON_LITERAL = 1 };
enum { RC_THETA_I_MP = 0, RC_THETA_I_ME = 1 };

typedef struct {
  rc_axes cool;          /* log10 N [cm^-2], log10 T_e [K], log10 B [G] */
  rc_axes coul;          /* log10 n_e [cm^-3], log10 T_e [K], log10 T_i [K] */
  double ln_lambda;      /* Coulomb logarithm, Sec. II.G (default 20) */
  int32_t value_dtype;   /* RC_VALUE_F32 (default) or RC_VALUE_BF16: the residual
                            rounded once more, to nearest-even bfloat16 (storage
                            experiment: half the table bytes, 2^-9 relative
                            rounding of the residual) */
  int32_t compton_exponent;  /* RC_COMPTON_DERIVED (default) or RC_COMPTON_LITERAL */
  int32_t theta_i_mass;      /* RC_THETA_I_MP (default) or RC_THETA_I_ME */
  int32_t reserved;          /* must be 0 */
  void* external_storage;    /* NULL (default): the library allocates and owns the
                                device memory of the tables.  Otherwise caller-owned
                                device memory on the current device, 256-byte aligned,
                                of at least rc_tables_storage_bytes(spec) bytes, that
                                rc_build_tables / rc_tables_import put the tables into
                                (geometry, node tables and, for FP32 tables, the
                                cell-blocked copy, built at once instead of on first
                                use); rc_tables_destroy does not free it, and the
                                caller keeps it alive and unmodified until then.
                                Saved table files never hold it. */
  uint64_t external_bytes;   /* size of external_storage in bytes (0 when it is NULL) */
} rc_table_spec;

typedef struct rc_tables_s* rc_tables;   /* opaque, library-owned device tables */

/* Per-cell input state: device pointers, FP64, length n.  T_floor_gas is
 * optional (NULL = none): a per-cell floor on the gas temperature T_e + T_i
 * [K] (Sec. III.B.2, e.g. from rc_disk_inputs); a cell whose input gas
 * temperature lies below it has zero radiative cooling for the step (Coulomb
 * exchange still acts) and status bit RC_ST_GAS_FLOOR. */
typedef struct {
  const double* n_e;
  const double* T_e;
  const double* T_i;
  const double* B;
  const double* H;
  const double* T_floor_gas;
} rc_state;

/* Per-cell outputs: device pointers, length n; NULL = not written.
 * Rates are reported at the INPUT state (the paper's cooling function);
 * Q_rad is zero when T_e < T_floor.  The effective applied cooling is
 * (u - u') / dt. */
typedef struct {
  double* T_e_new;
  double* T_i_new;
  void* Q_rad;           /* bridged radiative cooling, erg cm^-3 s^-1; double, or float
                            with opts.rate_dtype = RC_RATE_F32 */
  void* Q_cc;            /* Coulomb exchange, > 0 when ions heat electrons; as Q_rad */
  uint8_t* status;       /* RC_ST_* bits */
  double* Q_brem;        /* optional diagnostics */
  double* Q_syn;
  double* eta;
} rc_out;

enum { RC_SCHEME_NEWTON = 0, RC_SCHEME_EXPLICIT16 = 1, RC_SCHEME_RATES = 2 };

/* How the tables are read.  AUTO selects CELL for FP32 tables and GLOBAL for
 * bfloat16 tables.  GLOBAL gathers the corners with plain global loads,
 * through the vector L1 and L2 caches.  LDS stages,
 * per workgroup, the box of table nodes its cells can reach (their N and B
 * cells of the cooling tables over the whole T_e axis, their n_e cells of the
 * Coulomb table over the whole T_e x T_i plane) in 256 bytes of LDS per
 * workgroup thread (64 KiB at 256) when it fits,
 * and reads the tables from there; a box that does not fit is read from global
 * memory.  Results equal GLOBAL's.  Its workgroup is opts.block threads (0 =
 * 256).  It pays only for spatially coherent cell order.  TEX names the texture-memory path
 * of the paper's GPU (Sec. III.A); gfx950 exposes no texture sampling to HIP,
 * so it returns RC_EUNSUPPORTED.  DIRECT evaluates the closed forms of
 * Sec. II per cell instead of tables (rates scheme only).  Every variant
 * reads the synchrotron and Compton tables as their sum se = log2(eta Q_syn)
 * (they enter the rates only as that product): se's residual at a node is
 * the single-precision sum of the two stored residuals (one IEEE addition,
 * rounded to nearest) and its affine part the sum of theirs.  CELL reads a
 * cell-blocked copy of the FP32 tables, the 8 corners of every table cell
 * stored together (a cooling cell's 8 {brem, se} pairs in one aligned
 * 64-byte block, a Coulomb cell's 8 values in 32 bytes), so that a corner
 * gather touches one block instead of four node pairs, for 4 times the
 * cooling and 8 times the Coulomb table memory (about 200 MiB at 128^3
 * nodes).  The copy is
 * built on the first CELL (or AUTO) call for an FP32 table set: that call
 * allocates device memory and synchronizes its stream; later calls do
 * neither (make one call before capturing a graph).  Results equal GLOBAL's.
 * RC_EUNSUPPORTED for bfloat16 tables. */
enum { RC_VARIANT_AUTO = 0, RC_VARIANT_GLOBAL = 1, RC_VARIANT_LDS = 2, RC_VARIANT_TEX = 3, RC_VARIANT_DIRECT = 4,
       RC_VARIANT_CELL = 5 };

typedef struct {
  int32_t scheme;        /* RC_SCHEME_*: backward Euler (Newton), 16-substep explicit, or rates only */
  int32_t variant;       /* RC_VARIANT_*: how tables are read; DIRECT evaluates closed forms (no tables) */
  int32_t max_iter;      /* Newton iteration cap (default 60) */
  int32_t block;         /* threads per workgroup (one cell per thread): 64, 128, 192
                            or 256; 0 = library choice (64 for the Newton scheme,
                            256 otherwise) */
  double T_floor;        /* K, cooling is zero below it (Sec. III.B.2; default 1e6) */
  double tol;            /* target relative accuracy of T_e' (default 1e-12): a Newton step
                            below sqrt(tol) in ln T_e' ends the solve */
  int32_t passes;        /* Newton scheme, variants AUTO, CELL and GLOBAL: 0 = library
                            choice (1), 1 = one kernel, every cell solved by its own
                            thread in cell order; 2 = two passes: every cell's first
                            Newton round in cell order, then the unfinished cells,
                            grouped per tile of 4096 cells by the length of their
                            first proposed step, resumed so that the cells of a
                            wavefront need similar numbers of rounds.  Identical
                            results; two passes keep device scratch in the table
                            handle (59 bytes per cell, allocated (hipMalloc) on the
                            first call and whenever n grows past what it holds), so
                            two-pass calls that overlap on one table handle must use
                            the same stream.  Ignored by other schemes and variants. */
  int32_t grid;          /* batched form only: workgroups of the persistent launch,
                            0 = library choice (4 per compute unit for
                            rc_cool_step_batched; the tuned or the same default for a
                            plan); otherwise 1 .. RC_MAX_GRID.  Ignored by the other
                            entry points. */
  int32_t rate_dtype;    /* element type of out->Q_rad and out->Q_cc: RC_RATE_F64
                            (default, double) or RC_RATE_F32 (float, the FP64 value
                            rounded to nearest: 8 instead of 16 bytes per cell) */
  int32_t reserved;      /* must be 0 */
} rc_step_opts;

enum { RC_RATE_F64 = 0, RC_RATE_F32 = 1 };

#define RC_MAX_GRID 65536

/* Fill *spec with the default axes (n points per axis):
 *   cooling: log10 N in [15, 29], log10 T_e in [5.95, 12.05], log10 B in [-0.5, 10.5]
 *   Coulomb: log10 n_e in [9.5, 20.5], log10 T_e in [5.95, 12.05], log10 T_i in [5.95, 14.05]
 * and ln_lambda = 20, FP32 storage, the derived Compton exponent and theta_i with
 * m_p.  Returns RC_EINVAL for spec == NULL or n < 2. */
rc_status rc_default_spec(rc_table_spec* spec, int32_t n);

/* Device bytes the tables of *spec occupy, for spec->external_storage: the
 * geometry record, the node tables (16 bytes per cooling node and 4 per
 * Coulomb node for FP32 residuals; 8 and 2 for bfloat16) and, for FP32
 * tables, the cell-blocked copy (64 bytes per cooling cell, 32 per Coulomb
 * cell), each part 256-byte aligned.  Host only (no device call); the
 * external_storage fields of *spec are ignored.  RC_EINVAL for an invalid
 * spec or bytes == NULL. */
rc_status rc_tables_storage_bytes(const rc_table_spec* spec, uint64_t* bytes);

/* Fill *opts with: Newton scheme, AUTO variant, max_iter 60, block 0,
 * T_floor 1e6 K, tol 1e-12, passes 0, grid 0, FP64 rates. */
rc_status rc_default_opts(rc_step_opts* opts);

/* Build the four tables on the current device from the closed forms of Sec. II
 * (node values in FP64 on the GPU; a least-squares affine function of the node
 * indices is removed from each log2 table on the host and the residual is
 * stored in FP32, or in bfloat16 when spec->value_dtype says so).
 * Synchronous.  *out receives a new handle owned by the caller (release with
 * rc_tables_destroy).  With spec->external_storage the tables are put there;
 * the node evaluation still takes temporary device memory (8 bytes per node,
 * freed before the call returns).  RC_EINVAL for external storage that is
 * too small, not 256-byte aligned or not device memory of the current device. */
rc_status rc_build_tables(const rc_table_spec* spec, void* stream, rc_tables* out);

/* Create tables from host data in the storage form: resid holds the FP32
 * residuals of the four tables back to back, each C-ordered [i0][i1][i2] over
 * its axes (three cooling tables of n0*n1*n2 values, then the Coulomb table),
 * and coeffs holds 4 x 4 FP64 affine coefficients (c0, c1, c2, c3 per table,
 * value = c0 + c1 i0 + c2 i1 + c3 i2 + resid).  For RC_VALUE_BF16 the
 * residuals are rounded to bfloat16 (nearest, ties to even) on import, and
 * export returns the rounded values.  Synchronous; host buffers are only read
 * during the call.  With spec->external_storage (checked as for
 * rc_build_tables) the call allocates no device memory. */
rc_status rc_tables_import(const rc_table_spec* spec, const float* resid, const double* coeffs,
                           void* stream, rc_tables* out);

/* Copy the storage form out to host buffers laid out as in rc_tables_import
 * (either pointer may be NULL).  Synchronous. */
rc_status rc_tables_export(rc_tables t, float* resid, double* coeffs);

/* Spec of a table set and the number of residual values (sum over the four tables). */
rc_status rc_tables_info(rc_tables t, rc_table_spec* spec, int64_t* n_values);

/* Save to / load from a binary file: header (magic, version, spec without its
 * external_storage fields), the coefficients, the residuals and a 64-bit
 * checksum of the payload.  Load verifies the checksum (RC_EIO on mismatch)
 * and returns library-owned tables. */
rc_status rc_tables_save(rc_tables t, const char* path);
rc_status rc_tables_load(const char* path, void* stream, rc_tables* out);

rc_status rc_tables_destroy(rc_tables t);

/* One cooling source step over n cells (Sec. III.B): rates at the input state
 * and, unless scheme == RC_SCHEME_RATES, the updated temperatures.  n == 0 is
 * a no-op.  Asynchronous on stream. */
rc_status rc_cool_step(rc_tables t, const rc_state* state, int64_t n, double dt,
                       const rc_step_opts* opts, const rc_out* out, void* stream);

/* Allocation-free variant of rc_cool_step, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation.  Same arguments, semantics and results as
 * rc_cool_step (the same kernels), but it calls no hipMalloc, no hipFree and
 * no allocating library routine (rc_cool_step allocates the two-pass step's
 * scratch and the cell-blocked table copy on first use):
 *  - the two-pass Newton step's scratch (resume records, classes, tile lists
 *    and counts, about 59 bytes per cell) lives in a static device array
 *    sized for RC_NOALLOC_MAX_CELLS cells (about 59 MiB), which every device
 *    the library runs on holds until the process ends;
 *  - n > RC_NOALLOC_MAX_CELLS returns RC_EINVAL before any launch;
 *  - the cell-blocked table copy is read only if an earlier rc_cool_step or
 *    rc_cool_step_batched on these tables built it: AUTO otherwise reads the
 *    node layout (identical results), RC_VARIANT_CELL returns RC_ESTATE.
 * The static scratch is shared by every call on a device and keeps the last
 * call's contents; each call writes every scratch entry before reading it,
 * so nothing has to start at zero.  Calls that overlap on one device (on
 * different streams, or from threads without ordering) race on it and must
 * be serialised by the caller. */
#define RC_NOALLOC_MAX_CELLS (1 << 20)
rc_status rc_cool_step_noalloc(rc_tables t, const rc_state* state, int64_t n, double dt,
                               const rc_step_opts* opts, const rc_out* out, void* stream);

/* One adaptive-mesh block of one accretion-rate state: cells first_cell ..
 * first_cell + n_cells - 1 of the state and output arrays, advanced with
 * dt_per_state[state_id]. */
typedef struct {
  int64_t first_cell;
  int32_t n_cells;
  int32_t state_id;
} rc_block;

#define RC_MAX_STATES 64

/* Batched form: many uneven blocks and several states in one launch of a
 * persistent kernel whose workgroups take blocks from an atomic work queue
 * (every workgroup exits once the queue is drained).  blocks is a device array
 * of n_blocks entries; blocks whose range lies outside [0, n_total) or whose
 * state_id is outside [0, n_states) are skipped.  dt_per_state is a host array
 * of n_states (1 .. RC_MAX_STATES) positive finite values.  Same per-cell
 * semantics as rc_cool_step; variants AUTO, GLOBAL and CELL (AUTO reads the
 * cell-blocked copy of FP32 tables, built on first use as described for
 * RC_VARIANT_CELL), others RC_EUNSUPPORTED.  opts->grid sets the number of
 * workgroups (0 = 4 per compute unit).  Uses internal device scratch (the
 * queue counter, the per-state dt and the per-workgroup item counts, 257 KiB)
 * allocated on first use per table handle; calls that overlap on one table
 * handle must use the same stream.  Asynchronous on stream. */
rc_status rc_cool_step_batched(rc_tables t, const rc_state* state, int64_t n_total, const rc_block* blocks,
                               int32_t n_blocks, const double* dt_per_state, int32_t n_states,
                               const rc_step_opts* opts, const rc_out* out, void* stream);

/* A captured launch plan for a fixed batched problem (the same buffers every
 * replay): the counter reset (a one-thread kernel) and the persistent kernel,
 * captured into a hipGraph and instantiated once.  With autotune != 0 the
 * workgroup size (64, 128, 256) and the persistent grid (1, 2, 4 or 8
 * workgroups per compute unit; only opts->grid when that is set) are chosen
 * by timing each candidate with HIP events on the given stream (the outputs
 * are written during tuning).  Without autotuning the plan takes opts->block
 * (0 = 256) and opts->grid (0 = 4 per compute unit).
 * blocks is copied to the host once to validate every range (RC_EINVAL).
 * The plan keeps pointers, not copies, of state, out and blocks; the
 * cell-blocked table copy, when the variant reads it, is built before the
 * capture. */
typedef struct rc_plan_s* rc_plan;
rc_status rc_plan_create(rc_tables t, const rc_state* state, int64_t n_total, const rc_block* blocks,
                         int32_t n_blocks, const double* dt_per_state, int32_t n_states,
                         const rc_step_opts* opts, const rc_out* out, int32_t autotune, void* stream,
                         rc_plan* plan);
/* Replay the plan's graph on stream (asynchronous). */
rc_status rc_plan_launch(rc_plan plan, void* stream);

/* Work-queue diagnostics: how many work items (blocks) each workgroup of the
 * most recent batched launch took from the queue, skipped blocks included (the
 * counts sum to n_blocks).  rc_batched_workgroup_items reads the last
 * rc_cool_step_batched launch on the table handle, rc_plan_workgroup_items the
 * last launch of the plan (including its tuning launches).  Waits for the
 * device (hipDeviceSynchronize), then copies min(grid, capacity) counts to the
 * host array items (may be NULL); *grid (may be NULL) receives the number of
 * workgroups of that launch.  RC_ESTATE when no launch has been made. */
rc_status rc_batched_workgroup_items(rc_tables t, uint32_t* items, int32_t capacity, int32_t* grid);
rc_status rc_plan_workgroup_items(rc_plan plan, uint32_t* items, int32_t capacity, int32_t* grid);
/* Chosen launch shape and the tuned time of one launch (ms, 0 if not tuned). */
rc_status rc_plan_info(rc_plan plan, int32_t* block, int32_t* grid, double* tuned_ms);
rc_status rc_plan_destroy(rc_plan plan);

/* Forward outputs the backward pass reads (device pointers, length n). */
typedef struct {
  const double* T_e_new;
  const double* T_i_new;
  const uint8_t* status;
} rc_fwd;

/* Upstream cotangents of the forward outputs (device pointers, length n);
 * NULL = zero. */
typedef struct {
  const double* T_e_new;
  const double* T_i_new;
  const double* Q_rad;
  const double* Q_cc;
} rc_cotangent;

/* Gradients written by the backward pass (device pointers).  The five
 * per-cell arrays (length n) are overwritten; NULL = not written.  tables
 * (n_values doubles, laid out as the residuals of rc_tables_import: gradient
 * with respect to each table's log2 node values) is accumulated (+=); the
 * per-cell contributions are grouped by buckets of table cells and summed
 * with atomic adds in local memory (and, for table cells crowded with more
 * contributions than one workgroup takes, in device memory), so their
 * summation order, and the last bits of the values, vary from run to run;
 * NULL = not computed. */
typedef struct {
  double* n_e;
  double* T_e;
  double* T_i;
  double* B;
  double* H;
  double* tables;
} rc_grad;

/* Vector-Jacobian product of rc_cool_step (differentiation form).  For the
 * Newton scheme the forward outputs define (T_e', T_i') implicitly through the
 * backward-Euler equations of Sec. III.B.1; the adjoint solves the transposed
 * 2x2 Jacobian per cell (implicit function theorem) at the converged solution
 * (on a floor-projected cell T_e' is constant).  The input-state rates Q_rad,
 * Q_cc add their direct derivatives.  RC_SCHEME_RATES is supported (T' = T);
 * RC_SCHEME_EXPLICIT16, the DIRECT variant and tables of the literal Compton
 * exponent give RC_EUNSUPPORTED.  fwd must hold the outputs of a
 * forward call with the same tables, state, dt and options.  Table reads
 * follow opts->variant as in rc_cool_step: AUTO and CELL read FP32 tables
 * through the cell-blocked copy (a call that finds it missing builds it:
 * allocates and synchronizes its stream), GLOBAL and LDS the node layout;
 * every variant gives the same gradients.  With table
 * gradients the call keeps device scratch in the table handle: per-point
 * records, their keys and their bucket placement (about 200 bytes per cell)
 * plus 24 doubles per table cell, allocated
 * (hipMalloc) on the first call and whenever n grows past what it holds
 * (n up to 2^31 - 1 with table gradients: record positions are 32-bit);
 * backward calls with table gradients that overlap on one table handle must
 * therefore use the same stream.  Asynchronous on stream. */
rc_status rc_cool_step_backward(rc_tables t, const rc_state* state, int64_t n, double dt,
                                const rc_step_opts* opts, const rc_fwd* fwd, const rc_cotangent* cot,
                                const rc_grad* grad, void* stream);

/* Disk parameters of the upstream inputs (Sec. II.F, III.B.2). */
typedef struct {
  double gamma;          /* adiabatic index (the paper's runs: 5/3) */
  double spin;           /* dimensionless black-hole spin a, |a| <= 1 (the paper: 0.9375) */
  double h_floor;        /* target thickness (H/R)_floor of the temperature floor (the paper: 0.1) */
  double r_g;            /* gravitational radius G M / c^2 [cm] */
} rc_disk_params;

/* Per-cell inputs upstream of the step, from GRMHD primitives (device
 * pointers, FP64, length n): rest-mass density rho [g cm^-3], gas pressure P
 * and internal energy density u = rho eps [erg cm^-3], radius r [r_g].
 * Writes (either may be NULL):
 *   H_th        = c_s / Omega_K [cm], c_s^2 = gamma P / (rho c^2 + u + P),
 *                 Omega_K = 1 / (r^(3/2) + a) in c / r_g   (Sec. II.F, eq. H_thermal);
 *   T_floor_gas = (pi/2) (h_floor Omega_K r)^2 m_p c^2 / k_B [K], the floor on the
 *                 gas temperature T_e + T_i (Sec. III.B.2; P / rho = k (T_e + T_i) / m_p),
 *                 ready for rc_state.T_floor_gas.
 * Cells with a non-finite input, rho < 0, u < 0, P <= 0 or r <= 0 get NaN.
 * RC_EINVAL for NULL inputs, n < 0, gamma <= 1, |spin| > 1, h_floor < 0 or
 * r_g <= 0.  Asynchronous on stream. */
rc_status rc_disk_inputs(const double* rho, const double* P, const double* u, const double* r, int64_t n,
                         const rc_disk_params* params, double* H_th, double* T_floor_gas, void* stream);

/* Radiation-pressure temperature correction (Sec. IV, eq. total_pressure),
 * a post-processing step: where tau_sca = n_e sigma_T H > tau_crit (the paper:
 * 4.6, fewer than 1 % of photons escaping unscattered) the pressure
 * n_e k (T_e + T_i) is shared between radiation and gas with T_i held, and
 * T_e_out solves a T^4 + n_e k T = n_e k T_e (a = 4 sigma_SB / c; unique root,
 * T_e_out < T_e); elsewhere T_e_out = T_e.  Device pointers, FP64, length n;
 * thick (uint8, may be NULL) flags the corrected cells.  Cells with a
 * non-finite or non-positive input get NaN and thick = 0.  Asynchronous on
 * stream. */
rc_status rc_rad_pressure_correction(const double* n_e, const double* T_e, const double* H, int64_t n,
                                     double tau_crit, double* T_e_out, uint8_t* thick, void* stream);

/* Downstream coupling of the cooling to the gas (Sec. II.E, eqs.
 * energy-momentum_eq and 4-force_calc): the 4-force density
 * G_mu = -lambda u_mu applied over dt to the conserved energy-momentum
 * densities U_mu = sqrt(-g) T^t_mu,
 *   U_mu += dt sqrt(-g) G_mu = -dt sqrt(-g) lambda u_mu,
 * with lambda the energy per unit volume and time the step removed from the
 * gas [erg cm^-3 s^-1],
 *   lambda = 1.5 n_e k_B [(T_e - T_e') + (T_i - T_i')] / dt,
 * which for the backward-Euler step equals Q_rad at the new temperatures.  In
 * the fluid frame (u_mu = (-1, 0, 0, 0)) U_0 = -e sqrt(-g) rises by
 * dt sqrt(-g) lambda: the gas energy falls by the radiated energy.
 *   u_cov:  covariant 4-velocity u_0..u_3 (dimensionless, c = 1), required;
 *   sqrt_g: sqrt(-g) per cell, NULL for 1;
 *   U:      the four conserved densities, updated in place (the caller's
 *           units, consistent with lambda dt); a NULL component is skipped.
 * Device pointers, FP64 SoA, length n; the library keeps none of them. */
typedef struct {
  const double* u_cov[4];
  const double* sqrt_g;
  double* U[4];
} rc_coupling;

/* Apply the cooling of a step (its input temperatures T_e, T_i and outputs
 * T_e_new, T_i_new) to the gas energy-momentum as above; lambda (may be NULL)
 * receives the per-cell lambda.  A cell whose lambda is not finite (an
 * invalid step) keeps U and gets lambda = NaN.  RC_EINVAL for n < 0, dt not
 * finite and positive, coupling NULL, or a NULL temperature, n_e or velocity
 * pointer with n > 0.  Asynchronous on stream. */
rc_status rc_apply_cooling(const double* n_e, const double* T_e, const double* T_i, const double* T_e_new,
                           const double* T_i_new, int64_t n, double dt, const rc_coupling* coupling, double* lambda,
                           void* stream);

/* The paper's own cooling-table layout (Sec. II.F, III.A), for comparison
 * with the exact 3-D column tables: log2 of the bridged Q_total on a 4-D grid
 * over log10 H [cm], log10 B [G], log10 n_e [cm^-3], log10 T_e [K] (node k of
 * axis d at lo[d] + k (hi[d] - lo[d]) / (n[d] - 1)), stored as plain FP32 log2
 * values C-ordered [H][B][n_e][T_e], read by 4-D multilinear interpolation
 * (clamped at the edges).  The paper's flattening of n_e and T_e into one
 * texture axis is a texture-memory constraint and changes no value. */
typedef struct {
  int32_t n[4];
  double lo[4];
  double hi[4];
} rc_axes4;
typedef struct rc_table4d_s* rc_table4d;

/* The paper's ranges with n points per axis: H in [1e3, 1e12], B in [1, 1e10],
 * n_e in [1e2, 1e25], T_e in [1e2, 1e15] (the paper: n = 100). */
rc_status rc_paper_axes4(rc_axes4* axes, int32_t n);
/* Evaluate every node from the closed forms on the current device
 * (synchronous; 100^4 nodes take 400 MB of device memory). */
rc_status rc_build_table4d(const rc_axes4* axes, void* stream, rc_table4d* out);
/* Create from host FP32 log2 values laid out as above (synchronous). */
rc_status rc_table4d_import(const rc_axes4* axes, const float* values, void* stream, rc_table4d* out);
/* Copy the axes and / or the values to host memory (either may be NULL; synchronous). */
rc_status rc_table4d_export(rc_table4d t, rc_axes4* axes, float* values);
rc_status rc_table4d_destroy(rc_table4d t);
/* Q_rad (bridged total cooling, erg cm^-3 s^-1; zero below T_floor) at every
 * cell from the 4-D table; status (may be NULL) gets RC_ST_INVALID or
 * RC_ST_CLAMP_COOL.  state->T_i and state->T_floor_gas are not read.
 * Asynchronous on stream. */
rc_status rc_rates4d(rc_table4d t, const rc_state* state, int64_t n, double T_floor, double* Q_rad,
                     uint8_t* status, void* stream);

/* The physical constants compiled into the library, in this order:
 * c, k_B, h, m_e, m_p, e, sigma_T, sigma_SB; returns how many were written
 * (at most n). */
int32_t rc_constants(double* out, int32_t n);

/* Host-side self-test of the node evaluator: evaluates table `table` at node
 * (i0, i1, i2) of spec on the host CPU with the same source the GPU kernels
 * are compiled from, writing the log2 value to *value.  For tests only; no
 * step entry point ever calls it. */
rc_status rc_selftest_node_host(const rc_table_spec* spec, int32_t table, int32_t i0, int32_t i1,
                                int32_t i2, double* value);

/* Host-side self-test of special functions (same source as the device code):
 * which = 0,1,2: exponentially scaled K_nu(x) for nu = which;
 * which = 3: the synchrotron tail integral J(x) = int_x^inf s I'(s) ds;
 * which = 4: x_c solving ln(I'(x)/x) = x (input is the log right side);
 * which = 5..9: the solver's own elementary functions ln x, log10 x,
 * ln(1 + x), e^x, 2^x (finite arguments; positive for the logarithms).
 * For tests only. */
rc_status rc_selftest_special_host(int32_t which, const double* x, double* y, int64_t n);

/* Host-side self-test of the per-cell step (same source as the GPU kernel)
 * on tables given in the storage form of rc_tables_import (host memory):
 * host arrays of length n.  For tests only. */
rc_status rc_selftest_step_host(const rc_table_spec* spec, const float* resid, const double* coeffs,
                                const double* n_e, const double* T_e, const double* T_i,
                                const double* B, const double* H, const double* T_floor_gas, int64_t n, double dt,
                                const rc_step_opts* opts, double* T_e_new, double* T_i_new,
                                double* Q_rad, double* Q_cc, uint8_t* status);

/* Host-side self-tests of rc_disk_inputs and rc_rad_pressure_correction: the
 * same per-cell source on host arrays.  For tests only. */
rc_status rc_selftest_disk_host(const double* rho, const double* P, const double* u, const double* r, int64_t n,
                                const rc_disk_params* params, double* H_th, double* T_floor_gas);
rc_status rc_selftest_radp_host(const double* n_e, const double* T_e, const double* H, int64_t n, double tau_crit,
                                double* T_e_out, uint8_t* thick);

/* Host-side self-test of rc_apply_cooling: the same per-cell source on host
 * arrays (rc_coupling pointing to host memory).  For tests only. */
rc_status rc_selftest_coupling_host(const double* n_e, const double* T_e, const double* T_i, const double* T_e_new,
                                    const double* T_i_new, int64_t n, double dt, const rc_coupling* coupling,
                                    double* lambda);

/* Host-side self-tests of the 4-D table: node values (log2 Q_total at the
 * given states) and the rates read from host FP32 values.  For tests only. */
rc_status rc_selftest_node4d_host(const double* H, const double* B, const double* n_e, const double* T, int64_t n,
                                  double* log2_q);
rc_status rc_selftest_rates4d_host(const rc_axes4* axes, const float* values, const double* n_e, const double* T_e,
                                   const double* B, const double* H, int64_t n, double T_floor, double* Q_rad,
                                   uint8_t* status);

/* Host-side self-test of the per-cell adjoint (same source as the GPU
 * kernel) on tables in storage form (host memory).  Arrays of length n; cot_*
 * may be NULL (zero); g_tables (n_values doubles) is accumulated.  For tests
 * only. */
rc_status rc_selftest_backward_host(const rc_table_spec* spec, const float* resid, const double* coeffs,
                                    const double* n_e, const double* T_e, const double* T_i, const double* B,
                                    const double* H, const double* T_e_new, const double* T_i_new,
                                    const uint8_t* status, const double* cot_T_e_new, const double* cot_T_i_new,
                                    const double* cot_Q_rad, const double* cot_Q_cc, int64_t n, double dt,
                                    const rc_step_opts* opts, double* g_n_e, double* g_T_e, double* g_T_i,
                                    double* g_B, double* g_H, double* g_tables);

/* Message of the last error on this thread ("" if none). */
const char* rc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RADCOOL_H */
