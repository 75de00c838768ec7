/*
 * mttkrp.h -- C ABI of an MI355X (gfx950) sparse MTTKRP / CP-ALS library.
 *
 * The operation (Sec. II-A, Eq. (1) and the elementwise update after it):
 * for an N-mode sparse tensor X with nonzeros (c_0..c_{N-1}, val) and dense
 * factor matrices A_m (I_m x R), the MTTKRP along mode n is
 *
 *     M_n[i, r] = sum over nonzeros with c_n == i of  val * prod_{m != n} A_m[c_m, r].
 *
 * CP-ALS (Sec. II-A, CPD paragraph) computes it along every mode in turn and
 * re-solves each factor from it.
 *
 * Following the paper's tensor format (Sec. III-C, "mode-specific copies"),
 * mttkrp_layout_build keeps one copy of the nonzeros per output mode, each
 * ordered by its output index and split into nonzero-balanced partitions
 * (Sec. III-B, load-balancing scheme 2), and the per-mode kernel accumulates
 * every output row on chip and writes it once (Sec. IV-B), with no global
 * atomics.
 *
 * Conventions for every call:
 *  - Indices are 0-based.  Matrices are row-major with R contiguous values per
 *    row.  "host" pointers are CPU memory, "device" pointers are memory of the
 *    current HIP device.
 *  - Every call returns a status and never aborts.  Arguments are validated
 *    on the host before anything is enqueued; mttkrp_last_error() then holds
 *    a message (per calling thread).  Errors raised by the HIP runtime are
 *    reported as MTTKRP_EHIP, at the latest by the next call.
 *  - Device work is enqueued on `stream` (0 = the null stream) and is
 *    asynchronous unless stated otherwise.  A handle owns scratch memory
 *    (carry rows, CP-ALS workspace), so one handle must be used by one stream
 *    at a time; different handles are independent.
 *  - Results are reproducible bit for bit for a fixed handle (including its
 *    parts_per_cu), R and dtype: no atomics, fixed summation order.  The one
 *    exception is mttkrp_run_scheme2, kept to compare with the paper's
 *    atomic-based scheme.
 */
#ifndef MTTKRP_H
#define MTTKRP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mttkrp_layout* mttkrp_handle; /* opaque; owns all device copies and workspace */

typedef enum {
    MTTKRP_OK = 0,
    MTTKRP_EINVAL = 1,        /* null pointer, bad N / mode / R / dims, or handle misuse */
    MTTKRP_ERANGE = 2,        /* a coordinate is >= the dimension of its mode */
    MTTKRP_ENOMEM = 3,        /* footprint over the budget (not a "small tensor"), or allocation failed */
    MTTKRP_EUNSUPPORTED = 4,  /* N or R outside the compiled set */
    MTTKRP_ENOTSPD = 5,       /* CP-ALS: a normal-equation matrix is not positive definite */
    MTTKRP_EHIP = 6           /* HIP runtime error */
} mttkrp_status;

/* Factor storage used for the row gathers. */
enum { MTTKRP_FP32 = 0, MTTKRP_BF16 = 1 };

/* Limits: 3 <= N <= MTTKRP_MAX_MODES, every dim in [1, 2^31 - 1], nnz < 2^32,
 * R in {16, 32, 64}. */
#define MTTKRP_MAX_MODES 8

typedef struct {
    int parts_per_cu;          /* workgroup partitions per compute unit for the MTTKRP launch; 0 = default (8) */
    int factor_dtype;          /* gather precision used inside cpd_als_iter: MTTKRP_FP32 or MTTKRP_BF16 */
    int max_R;                 /* largest R the handle will run with (16, 32 or 64); sizes the workspace; 0 = 64 */
    uint64_t hbm_budget_bytes; /* refuse to build (MTTKRP_ENOMEM) when the footprint exceeds this; 0 = no budget */
    int host_only;             /* 1: build the host arrays only (for inspection); no device memory, runs refused */
    int hot_rows;              /* rows of each input factor kept in LDS during a run: the most frequently
                                  gathered ones.  -1 = as many as fit, 0 = none (default), k > 0 = at most k */
    int build_on_host;         /* 1: sort the mode copies on the host.  0 (default): on the device when the
                                  packed coordinate key of all N indices fits 128 bits, 1 <= nnz < 2^31 and
                                  hot_rows is 0 (the copies are identical either way; the device build
                                  holds a transient scratch of about nnz * (4N + 48) bytes) */
    int partitioner;           /* how each mode copy is split into workgroup partitions (Sec. III-B):
                                  MTTKRP_PART_NNZ (default): equal nonzero ranges, rows cut by a range
                                  boundary combined by a deterministic fix-up (scheme 2 without atomics);
                                  MTTKRP_PART_ROWS_LPT: scheme 1, whole output rows dealt to lpt_parts
                                  partitions, longest first to the least-loaded partition (built on the
                                  host; no hot rows; not usable in batches or the gather probe) */
    int lpt_parts;             /* partitions (the paper's kappa) of MTTKRP_PART_ROWS_LPT; 0 = one per
                                  compute unit */
    int hot_steps;             /* 1: lay the copies out in wave steps for rank max_R and factor_dtype
                                  (3- and 4-mode tensors; built on the host): each input's most gathered
                                  rows are held in LDS, every output row's nonzeros are ordered by which
                                  of their input rows are held there, and rows are padded with zero
                                  entries to whole steps of one wave, so that steps whose rows are all held
                                  skip the global gathers.  Runs then need R = max_R (fp32, or bf16 when
                                  factor_dtype is MTTKRP_BF16); not usable in batches, the gather probe or
                                  mttkrp_run_scheme2; hot_rows and partitioner are ignored.  0 (default): off */
    int wide_indices;          /* 1: always store 32-bit input coordinates.  0 (default): a copy whose input
                                  dimensions are all <= 65536 stores them as uint16 (3- to 5-mode tensors,
                                  nonzero split, no hot rows or steps; the paper's memory model counts
                                  log2 of the dimension per index, Sec. III-C) */
    int part_threads;          /* partition-kernel workgroup size for fp32 runs of 3-mode tensors without hot
                                  rows or steps: 256, 512 or 1024 threads; 0 (default) = 512.  Ignored elsewhere */
    int part_gathers;          /* nonzeros whose row gathers each lane group keeps in flight in those runs: 2
                                  or 4; 0 (default) = 2 at R = 16, else 4.  Ignored elsewhere.  Both change
                                  the partitioning, so results change by rounding only */
    int relabel;               /* 1: renumber every mode's indices by decreasing nonzero count (ties: lower
                                  index first) before building, so the most gathered factor rows lie
                                  together (rows shorter than a cache line then share lines; the LDS hot
                                  rows of hot_rows are picked by the same count).  Every row index the
                                  handle then takes or produces is in the new numbering: factors passed to
                                  runs and CP-ALS, MTTKRP outputs, hot-row tables.  mttkrp_layout_perm
                                  gives the map.  0 (default): the caller's numbering */
    int als_solve;             /* CP-ALS normal equations A_n V = M (Sec. II-A): 0 (default) V^{-1} by the sweep
                                  operator (FP64, one workgroup) and M V^{-1} on the FP64 matrix cores;
                                  1: V = L L^T by Cholesky (FP64) and every row of M solved by forward and
                                  back substitution (FP64).  Both reject the same non-SPD V; 1 is slower */
} mttkrp_opts;

enum { MTTKRP_PART_NNZ = 0, MTTKRP_PART_ROWS_LPT = 1 };

/* Fill `o` with the defaults listed above. */
void mttkrp_opts_default(mttkrp_opts* o);

/* Device bytes a handle for this tensor would hold: N mode copies (Sec. III-C:
 * the paper's memory formula is N * nnz * bits-per-nonzero; here each copy
 * stores N-1 uint32 input indices, one fp32 value, 1 bit of row-start flag
 * and a 32-bit row index per 32 nonzeros, plus 4 bytes per output row) and
 * the workspace sized by opts->max_R and opts->factor_dtype.  Host only; opts
 * may be NULL.  Used for admission before anything is built. */
mttkrp_status mttkrp_footprint(const uint32_t* dims /* host, N */, int N, uint64_t nnz,
                               const mttkrp_opts* opts, uint64_t* bytes /* host, out */);

/* Build the N mode-specific copies (Sec. III-B/III-C) of a COO tensor.
 *   coo_idx: host, nnz x N uint32, row-major (nonzero k at coo_idx[k*N .. k*N+N-1])
 *   vals:    host, nnz float
 *   dims:    host, N
 * The inputs are borrowed for the call only (validated and copied).  Duplicate
 * coordinates are allowed and add up.  nnz == 0 is valid (all outputs zero).
 * Each copy is ordered by (output index, other indices in cyclic order,
 * input position).  The sort runs on the device, on `stream`, when the
 * packed key of all N indices fits 128 bits (see opts->build_on_host); the
 * COO tensor is then uploaded to a transient scratch allocation that is freed
 * before returning.  Otherwise it runs on the host and the copies are
 * uploaded on `stream`.  Either way the call returns once the copies are on
 * the device, and the copies are identical.
 * On success *out receives a handle to release with mttkrp_layout_free. */
mttkrp_status mttkrp_layout_build(const uint32_t* coo_idx, const float* vals, uint64_t nnz,
                                  const uint32_t* dims, int N, const mttkrp_opts* opts,
                                  hipStream_t stream, mttkrp_handle* out);

/* Device scratch bytes mttkrp_layout_build_in needs beside the handle's own
 * memory, for these dims, nnz and opts: the sort and decode buffers of the
 * device build (about nnz * (4N + 48) bytes), or 0 when the copies will be
 * built on the host (opts->build_on_host, hot rows, keys over 128 bits).
 * Host only; opts may be NULL. */
mttkrp_status mttkrp_build_scratch_bytes(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts* opts,
                                         uint64_t* bytes /* host, out */);

/* As mttkrp_layout_build, but in caller-owned device memory, for callers that
 * must not allocate or free device memory from the library (a serving loop
 * whose other streams must keep running: freeing device memory synchronises
 * the whole device).
 *   dev_mem:     device, 256-byte aligned, dev_bytes >= mttkrp_footprint(...);
 *                the handle borrows it: keep it until mttkrp_layout_free and
 *                until every enqueued call that uses the handle has completed
 *   dev_scratch: device, 256-byte aligned, scratch_bytes >=
 *                mttkrp_build_scratch_bytes(...), used only during this call;
 *                may be NULL (then the copies are built on the host)
 * The copies are identical to mttkrp_layout_build's.  The call synchronises
 * `stream` (only) before it returns.  mttkrp_layout_free of such a handle
 * releases host state only and never waits on the device.  Errors as
 * mttkrp_layout_build; MTTKRP_EINVAL when dev_bytes is too small. */
mttkrp_status mttkrp_layout_build_in(const uint32_t* coo_idx, const float* vals, uint64_t nnz,
                                     const uint32_t* dims, int N, const mttkrp_opts* opts, void* dev_mem,
                                     uint64_t dev_bytes, void* dev_scratch, uint64_t scratch_bytes,
                                     hipStream_t stream, mttkrp_handle* out);

/* Device bytes held by the handle (0 for a host-only handle). */
uint64_t mttkrp_layout_bytes(mttkrp_handle h);

/* MTTKRP along `mode` (Alg. 1's body for one mode; Alg. 2 per partition).
 *   factors: host array of N device pointers; factors[m] is A_m, I_m x R fp32.
 *            factors[mode] is not read and may be NULL.
 *   out:     device, I_mode x R fp32, overwritten (rows without nonzeros get 0).
 * R must be 16, 32 or 64 and <= the handle's max_R. */
mttkrp_status mttkrp_run(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                         hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): mttkrp_run
 * with its carry rows (partials of rows cut by partition boundaries) in a
 * fixed device array of mttkrp_noalloc_scratch_bytes() = 4 MiB that the
 * library holds on each device it runs on until the process ends, instead
 * of the handle's workspace.  The call allocates and frees nothing.  Same
 * arguments, result (bitwise mttkrp_run's), layout and errors as
 * mttkrp_run; in addition MTTKRP_EINVAL when the current device is not the
 * handle's, and MTTKRP_ENOMEM when the launch needs more carry rows than the
 * array holds (more than 8192 partitions at R = 64, 16384 at R = 32).  The
 * array needs no clearing: every carry row the fix-up reads is written by the
 * same call first.  All calls on one device share the array, so calls that
 * overlap on one device (different streams, or different host threads) race
 * and must be ordered by the caller. */
mttkrp_status mttkrp_run_noalloc(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                 hipStream_t stream);
uint64_t mttkrp_noalloc_scratch_bytes(void);

/* Same, with bfloat16 factor rows (uint16 bit patterns, I_m x R) gathered and
 * multiplied in FP32 with FP32 accumulation. */
mttkrp_status mttkrp_run_bf16(mttkrp_handle h, int mode, const uint16_t* const* factors, float* out, int R,
                              hipStream_t stream);

/* Prepare CP-ALS state for `factors` (host array of N device pointers to
 * I_m x R fp32): the FP64 Gram matrices A_m^T A_m, and the bf16 copies when
 * opts->factor_dtype is MTTKRP_BF16.  Call before the first cpd_als_iter and
 * again whenever the factors were changed by anything but cpd_als_iter. */
mttkrp_status cpd_als_init(mttkrp_handle h, const float* const* factors, int R, hipStream_t stream);

/* One CP-ALS sweep over all modes (textbook ALS, see Sec. II-A): for each
 * mode n, V = Hadamard product of the other Gram matrices (FP64), M = MTTKRP
 * along n, A_n = M V^{-1} with V^{-1} from symmetric pivoting (the sweep
 * operator; its pivots are V's Cholesky pivots; FP64 arithmetic, fp32 store), columns
 * normalised to unit 2-norm with the norms in lambda, Gram of A_n updated.
 *   factors: host array of N device pointers, updated in place
 *   lambda:  device, R doubles (out: the norms of the last mode)
 *   fit_out: device, 1 double (out: 1 - |X - Xhat| / |X|), may be NULL
 * Returns MTTKRP_ENOTSPD if a V is not positive definite (detected on the
 * device; reported by this call, which then synchronises the stream). */
mttkrp_status cpd_als_iter(mttkrp_handle h, float* const* factors, double* lambda, int R, double* fit_out,
                           hipStream_t stream);

/* For comparison only: the MTTKRP with the paper's load balancing scheme 2
 * (Sec. III-B: equal nonzero chunks per workgroup, partial results of rows
 * that span chunks added with global atomics) instead of mttkrp_run's
 * deterministic carry fix-up.  Same arguments, layout and errors as
 * mttkrp_run (fp32 factors); the output is zeroed by a kernel first.  The
 * order of the atomic additions varies, so results agree with mttkrp_run up
 * to rounding only and need not repeat bit for bit. */
mttkrp_status mttkrp_run_scheme2(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                 hipStream_t stream);

/* Measurement aid for the on-chip gather ceiling (not part of the method):
 * the index/value stream and factor-row gathers of the MTTKRP along `mode`,
 * with the same partitions, lane groups and loads as mttkrp_run (fp32) or
 * mttkrp_run_bf16, but the products, row sums, stores and fix-up replaced by
 * an XOR fold of the loaded bits.  what = 0 streams the mode copy only;
 * what = 1 also gathers every factor row the nonzeros name; what = 2 issues
 * the same gather instructions with one lane of each row's lane group
 * reading (1/L of the bytes); what = 3 gathers row (index & 63) in place of
 * row index, so every gather hits rows resident in L1.  Variants 2 and 3 are
 * compiled for 3- and 4-mode tensors; for more modes they fail with
 * MTTKRP_EHIP (invalid launch).
 *   factors:      host array of N device pointers (factors[mode] unused), rows
 *                 of R fp32 values (factor_dtype MTTKRP_FP32) or R bf16 bit
 *                 patterns (MTTKRP_BF16)
 * Writes nothing the caller owns; it may write the handle's carry workspace,
 * so it must not overlap an MTTKRP on the same handle.  Errors as mttkrp_run. */
mttkrp_status mttkrp_gather_probe(mttkrp_handle h, int mode, const void* const* factors, int factor_dtype, int R,
                                  int what, hipStream_t stream);

/* Launch facts of a handle, for tuning and reports. */
typedef struct {
    uint32_t cu_count;            /* compute units of the handle's device */
    uint32_t lds_per_workgroup;   /* LDS bytes a workgroup may allocate on that device */
    uint32_t hot_rows;            /* rows per input factor the MTTKRP kernel keeps in LDS */
    uint32_t wg_threads;          /* threads per MTTKRP workgroup */
    uint32_t parts_per_cu;        /* MTTKRP workgroups launched per compute unit */
    uint32_t lpt_parts;           /* scheme-1 partitions (MTTKRP_PART_ROWS_LPT), 0 for the nonzero split */
    uint32_t step_entries;        /* hot-steps copies: entries per wave step (0: nonzero-ordered copies) */
    uint32_t idx16_modes;         /* bit n set: the copy of output mode n stores 16-bit input coordinates */
    uint32_t gathers_in_flight;   /* nonzeros' row gathers in flight per lane group (fp32 runs at max_R;
                                     0 for hot-steps copies) */
} mttkrp_info;

mttkrp_status mttkrp_layout_info(mttkrp_handle h, mttkrp_info* info);

/* The renumbering of a layout built with opts.relabel = 1: new_of_old (host,
 * I_mode entries, written) receives the new index of each original index of
 * `mode`.  MTTKRP_EINVAL for a layout built without relabel. */
mttkrp_status mttkrp_layout_perm(mttkrp_handle h, int mode, uint32_t* new_of_old);

/* Launch plan of the per-mode MTTKRP for a tensor of nnz nonzeros and N modes
 * (host only, no device needed): the nonzero-balanced partitions of the
 * paper's load-balancing scheme 2 (Sec. III-B), one workgroup each.  Every
 * lane group adds at most 4096 consecutive nonzeros in one FP32 register
 * chain, for any nnz < 2^32, so rounding grows with at most 4096 terms per
 * chain; partials beyond that are combined in LDS and in FP64.
 *   parts_per_cu: the target number of partitions per compute unit (<= 0: 8)
 *   cu_count:     compute units of the device (0: 256, the MI355X) */
typedef struct {
    uint32_t wg_threads;          /* threads per partition workgroup */
    uint32_t lane_groups;         /* lane groups per workgroup (one 16-byte row slice per lane) */
    uint32_t lanes_per_group;     /* lanes that share one factor row */
    uint32_t nonzeros_per_group;  /* consecutive nonzeros one lane group adds in registers (<= 4096) */
    uint64_t nonzeros_per_part;   /* nonzeros per workgroup partition */
    uint32_t nparts;              /* workgroups of the launch */
    uint64_t carry_bytes;         /* carry rows the handle reserves for rows cut by partitions (at max_R = R) */
} mttkrp_plan;

mttkrp_status mttkrp_launch_plan(uint64_t nnz, int N, int R, int factor_dtype, int parts_per_cu, uint32_t cu_count,
                                 mttkrp_plan* out);

/* ---- Batching: many small tensors per launch ----
 * A batch groups handles of tensors with the same N.  mttkrp_batch_run runs
 * the MTTKRP along one mode for every tensor of the batch with one
 * partition-kernel launch and one fix-up launch: a static list of (tensor,
 * partition) work items, walked by a grid of resident workgroups.  Every
 * tensor keeps the partitioning mttkrp_run gives it, so each tensor's result
 * is bitwise the same as mttkrp_run on its handle, whatever else is in the
 * batch. */
typedef struct mttkrp_batch* mttkrp_batch_handle;

/* layouts: host array of `count` device handles (same N, each with max_R >= R).
 * The handles must outlive the batch.  Each tensor is partitioned with its own
 * handle's parts_per_cu.  opts (may be NULL) sets the batch's gather precision
 * with factor_dtype: MTTKRP_FP32 (default; mttkrp_batch_run) or MTTKRP_BF16
 * (mttkrp_batch_run_bf16, and cpd_als_batch_iter_async on layouts built with
 * factor_dtype MTTKRP_BF16); its other fields are validated only.  Allocates
 * the batch's descriptor tables and carry rows. */
mttkrp_status mttkrp_batch_create(const mttkrp_handle* layouts, int count, int R, const mttkrp_opts* opts,
                                  mttkrp_batch_handle* out);

/* factors: host array of count * N device pointers, tensor t's A_m at
 *          [t * N + m] (I_m x R fp32; the mode's own entry is not read);
 * outs:    host array of count device pointers, tensor t's I_mode x R fp32
 *          output (overwritten).
 * When the pointers differ from the previous call's, the descriptor tables
 * are re-uploaded on `stream`, which is then synchronised (only it). */
mttkrp_status mttkrp_batch_run(mttkrp_batch_handle b, int mode, const float* const* factors, float* const* outs,
                               hipStream_t stream);

/* Same for a batch created with factor_dtype MTTKRP_BF16: factors are bf16 bit
 * patterns (uint16, I_m x R), gathered and multiplied in FP32 with FP32
 * accumulation; each tensor's result is bitwise mttkrp_run_bf16 on its handle.
 * MTTKRP_EINVAL on an fp32 batch (and mttkrp_batch_run on a bf16 one). */
mttkrp_status mttkrp_batch_run_bf16(mttkrp_batch_handle b, int mode, const uint16_t* const* factors,
                                    float* const* outs, hipStream_t stream);

/* One CP-ALS sweep for every tensor of the batch, enqueued only (capturable):
 * per mode, each tensor's FP64 normal-equation kernels around one batched
 * MTTKRP launch pair.  Every tensor must have been prepared with
 * cpd_als_init(h, ..., R), and every layout's factor_dtype must be the
 * batch's: with MTTKRP_BF16 the MTTKRPs gather the layouts' bf16 factor copies,
 * refreshed after each mode update by one batched cast.  Each tensor's results
 * are bitwise those of cpd_als_iter_async on its own handle.
 *   factors: host array of count * N device pointers (updated in place)
 *   lambdas: host array of count device pointers (R doubles each)
 *   fits:    host array of count device pointers (1 double each) or NULL */
mttkrp_status cpd_als_batch_iter_async(mttkrp_batch_handle b, float* const* factors, double* const* lambdas,
                                       double* const* fits, hipStream_t stream);

/* Autotuner for the partition size of batched tensors (the paper sizes its
 * partitions per SM, Sec. III-B; here the size is measured, not modelled):
 * for each candidate parts_per_cu, set it on every layout, build the batch and
 * time `reps` batched all-mode MTTKRP passes after one warm-up pass, with HIP
 * events on `stream`.  With more than 4 candidates the 4 fastest are timed
 * again over 4 x reps passes.  The fastest candidate stays set on the layouts
 * (so mttkrp_run, cpd_als_iter and later batches use it; results change by
 * rounding only) and is returned.  Synchronises the stream.
 *   candidates: n_candidates values in [1, 64]; NULL = {1, 2, 4, 8, 16}
 *   factors:    host array of count * N device pointers, as mttkrp_batch_run
 *   outs:       host array of count * N device pointers, tensor t's mode-n
 *               output (I_n x R fp32, overwritten) at [t * N + n]
 *   times_ms:   NULL or one float per candidate: time of one all-mode pass
 *               (for the 4 finalists, from the second timing)
 *   best_ppc:   out: the chosen parts_per_cu */
mttkrp_status mttkrp_batch_autotune(const mttkrp_handle* layouts, int count, int R, const int* candidates,
                                    int n_candidates, const float* const* factors, float* const* outs, int reps,
                                    hipStream_t stream, int* best_ppc, float* times_ms);

/* A launch shape of the partition kernel, as the shape autotuner sets it. */
typedef struct {
    int parts_per_cu;   /* partitions per compute unit, [1, 64] */
    int threads;        /* opts.part_threads: 0, 256, 512 or 1024 */
    int gathers;        /* opts.part_gathers: 0, 2 or 4 */
} mttkrp_part_shape;

/* As mttkrp_batch_autotune over launch shapes: each candidate sets
 * parts_per_cu, part_threads and part_gathers on every layout (the shape
 * fields apply to fp32 runs of 3-mode tensors without hot rows, and are
 * ignored elsewhere).  The fastest stays set and is returned in *best.
 *   candidates: n_candidates shapes, or NULL for the defaults listed by
 *               mttkrp_batch_autotune_default_shapes(layouts[0]'s N)
 *   times_ms:   NULL or one float per candidate */
mttkrp_status mttkrp_batch_autotune_shape(const mttkrp_handle* layouts, int count, int R,
                                          const mttkrp_part_shape* candidates, int n_candidates,
                                          const float* const* factors, float* const* outs, int reps,
                                          hipStream_t stream, mttkrp_part_shape* best, float* times_ms);

/* The same for one layout: each candidate is timed as `reps` passes of
 * mttkrp_run along every mode (fp32 factors) after a warm-up pass, and the
 * fastest stays set on h (mttkrp_run and cpd_als_iter then use it).
 * Synchronises the stream.  MTTKRP_EUNSUPPORTED on hot-steps copies.
 *   factors: host array of N device pointers (I_m x R fp32)
 *   outs:    host array of N device pointers, the mode-n output (I_n x R fp32,
 *            overwritten) at [n] */
mttkrp_status mttkrp_autotune_shape(mttkrp_handle h, int R, const mttkrp_part_shape* candidates, int n_candidates,
                                    const float* const* factors, float* const* outs, int reps, hipStream_t stream,
                                    mttkrp_part_shape* best, float* times_ms);

/* The default candidates of mttkrp_batch_autotune_shape and
 * mttkrp_autotune_shape for N-mode tensors (parts_per_cu 1, 2, 4, 8, 16, 32;
 * for N = 3 each with threads 256, 512, 1024 and gathers 2, 4): written to out
 * when it is not NULL (room for 36); returns their number. */
int mttkrp_batch_autotune_default_shapes(int N, mttkrp_part_shape* out);

/* Release a batch (not its layouts).  A batch that allocated its own device
 * memory synchronises the device first; one from mttkrp_batch_create_in
 * releases host state only.  NULL is ignored. */
void mttkrp_batch_free(mttkrp_batch_handle b);

/* Device bytes mttkrp_batch_create_in needs for these layouts and R (host
 * only; the same checks as mttkrp_batch_create). */
mttkrp_status mttkrp_batch_bytes(const mttkrp_handle* layouts, int count, int R, uint64_t* bytes /* host, out */);

/* As mttkrp_batch_create, in caller-owned device memory (dev_mem: 256-byte
 * aligned, dev_bytes >= mttkrp_batch_bytes), for callers that must not make
 * the library allocate or free device memory.  The tables are uploaded on
 * `stream`, which is synchronised (only it) before the call returns.  Keep
 * dev_mem until mttkrp_batch_free and until every enqueued call using the
 * batch has completed. */
mttkrp_status mttkrp_batch_create_in(const mttkrp_handle* layouts, int count, int R, const mttkrp_opts* opts,
                                     void* dev_mem, uint64_t dev_bytes, hipStream_t stream,
                                     mttkrp_batch_handle* out);

/* As cpd_als_iter, but only enqueued: nothing is read back and the stream is
 * not synchronised, so sweeps can be captured into a HIP graph and replayed.
 * A V that is not positive definite sets a sticky device flag (and makes the
 * factors NaN); cpd_als_status reports it. */
mttkrp_status cpd_als_iter_async(mttkrp_handle h, float* const* factors, double* lambda, int R, double* fit_out,
                                 hipStream_t stream);

/* MTTKRP_ENOTSPD if any sweep since the last check met a V that is not
 * positive definite (then clears the flag), else MTTKRP_OK.  Synchronises the
 * stream. */
mttkrp_status cpd_als_status(mttkrp_handle h, hipStream_t stream);

/* Release a handle.  A handle from mttkrp_layout_build frees its device
 * memory and synchronises the device first; one from mttkrp_layout_build_in
 * releases host state only (the caller owns the memory).  NULL is ignored. */
void mttkrp_layout_free(mttkrp_handle h);

/* Message of the last failed call on this thread ("" if none). */
const char* mttkrp_last_error(void);

/* The scheme-1 partitioner alone (host only): rows of the given nonzero
 * counts dealt to kappa partitions by longest processing time first (Sec.
 * III-B, scheme 1; Graham's rule, whose makespan is at most (4/3 - 1/(3
 * kappa)) times the optimum, the bound the paper quotes): rows by decreasing
 * count, ties to the lower row, each to the least-loaded partition, ties to
 * the lower partition.
 *   loads:     host, nrows counts
 *   part:      host out, nrows partition indices
 *   part_load: host out (may be NULL), kappa sums */
mttkrp_status mttkrp_lpt_partition(const uint64_t* loads, uint64_t nrows, uint32_t kappa, uint32_t* part,
                                   uint64_t* part_load);

/* Host view of one mode copy of a host-only handle (for inspection and tests).
 * All pointers stay valid until mttkrp_layout_free. */
typedef struct {
    uint64_t nnz;                 /* nonzeros */
    uint64_t nnz_pad;             /* array length: nnz rounded up to a multiple of 32 */
    uint64_t nrows_nz;            /* output rows with at least one nonzero */
    uint64_t nempty;              /* output rows without nonzeros */
    int n_in;                     /* N - 1 */
    int in_modes[MTTKRP_MAX_MODES - 1];      /* the input modes, increasing */
    const uint32_t* idx[MTTKRP_MAX_MODES - 1]; /* idx[j][k]: coordinate in mode in_modes[j] of nonzero k,
                                                   or 0x80000000 | s for the row in hot slot s */
    const float* val;             /* value of nonzero k */
    const uint32_t* winfo;        /* 2 words per 32 nonzeros: row-start bits, row ordinal of the first */
    const uint32_t* row_id;       /* output row of each nonempty row, increasing (nrows_nz) */
    const uint32_t* empty_rows;   /* rows without nonzeros, increasing (nempty) */
    const uint64_t* src_pos;      /* position in the caller's COO input of nonzero k (nnz entries; for
                                     scheme-1 copies nnz_pad entries, all ones at gap entries) */
    uint64_t nhot;                /* rows per input mode served from LDS */
    const uint32_t* hot_rows[MTTKRP_MAX_MODES - 1]; /* hot_rows[j][s]: row of mode in_modes[j] in slot s */
    uint64_t step_entries;        /* hot-steps copies: entries per step; the arrays then hold nsteps steps
                                     (nnz_pad = steps padded to 32, times step_entries), entry e of step s
                                     at (s / 32) * 32 * step_entries + e * 32 + s % 32, winfo per 32 steps;
                                     padding entries have value 0 and coordinate 0x80000000 | nhot */
    uint64_t nsteps;
    uint64_t nparts;              /* scheme-1 partitions (0 for the nonzero split) */
    const uint64_t* part_range;   /* 2 * nparts: first position and nonzeros of each partition; the rows of
                                     partition p, in increasing order, fill [first, first + nonzeros) and
                                     every first is a multiple of 32 (entries between partitions are
                                     zero and belong to none) */
} mttkrp_mode_view;

mttkrp_status mttkrp_layout_view(mttkrp_handle h, int mode, mttkrp_mode_view* v);

#ifdef __cplusplus
}
#endif

#endif /* MTTKRP_H */
