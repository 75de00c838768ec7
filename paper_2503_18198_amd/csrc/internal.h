// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <stdint.h>

#include <vector>
#include <hip/hip_runtime.h>

#include "mttkrp.h"

namespace mk {

constexpr int kWG = 256;                       // threads per workgroup in every kernel here
constexpr int kMaxIn = MTTKRP_MAX_MODES - 1;   // input modes per nonzero, at most
constexpr int kMaxIn16 = 4;                    // input modes up to which 16-bit coordinate kernels exist

// One mode-specific copy of the tensor in device memory (Sec. III-C).
// Nonzeros are ordered by output row; arrays are padded to nnz_pad (a
// multiple of 32) with zero entries that the kernels never use.
struct DevMode {
    uint64_t nnz = 0, nnz_pad = 0, nrows_nz = 0, nempty = 0;
    int n_in = 0;
    int in_modes[kMaxIn] = {};
    uint32_t in_dims[kMaxIn] = {};     // I_m of each input mode
    const uint32_t* idx[kMaxIn] = {};  // SoA input-mode coordinates
    const float* val = nullptr;
    const uint2* winfo = nullptr;      // per 32 nonzeros: {row-start bits, ordinal of the row holding the first}
    const uint32_t* row_id = nullptr;  // ordinal -> output row
    const uint32_t* empty_rows = nullptr;
    // Scheme 1 (whole rows per partition): {first position, nonzeros} of each
    // of nprange partitions; null for the nonzero-balanced split.
    const uint64_t* prange = nullptr;
    uint32_t nprange = 0;
    // Hot-steps copy (step_P > 0): the arrays hold nsteps steps of step_P
    // entries, transposed per 32 steps, and winfo describes steps.
    uint32_t step_P = 0;
    uint64_t nsteps = 0;
    // idx16: the input coordinate arrays hold uint16 (every input dimension
    // <= 65536, 3- to 5-mode tensors, nonzero-ordered copies without hot rows).
    bool idx16 = false;
};

// Launch geometry of one MTTKRP call.
struct Geometry {
    int lanes;          // lanes per group: 16 bytes of a factor row per lane
    int groups;         // lane groups per workgroup
    uint32_t gsz;       // nonzeros per lane group (multiple of 32)
    uint64_t wgc;       // nonzeros per workgroup partition = groups * gsz
    uint32_t nparts;    // workgroups (partitions)
    uint32_t grid = 0;  // hot-steps copies: resident workgroups that walk the partitions
    // A tuned partition-kernel shape (3-mode tensors, fp32 factors, no hot
    // rows): threads per workgroup and gathers in flight; 0 = the default.
    int threads = 0, gathers = 0;
};

// Partitions of about nnz / target_parts nonzeros, with at most max_parts
// partitions and, unless max_parts forbids it, at most max_gsz nonzeros per
// lane group (the length of its FP32 accumulation chain); workgroups of
// `threads` threads (0: the default for n_in).  The caller sets the tuned
// shape fields.
Geometry plan_geometry(uint64_t nnz, int n_in, int R, int dtype, int target_parts, uint32_t max_parts,
                       uint32_t max_gsz, int threads = 0);

// The partition kernel's default shape for n_in inputs, rank R and dtype.
void default_part_shape(int n_in, int R, int dtype, int* threads, int* gathers);

// Whether a tuned shape (threads per workgroup, gathers in flight) is compiled.
bool tuned_shape_supported(int threads, int gathers);

// Launch plan of a hot-steps copy of nsteps steps: gsz = steps per wave run
// (a multiple of 32, at most max_chain / passes), groups = waves per
// workgroup, wgc = steps per partition, nparts partitions (at most max_parts).
Geometry plan_step_geometry(uint64_t nsteps, int R, int dtype, uint32_t P, int target_parts, uint32_t max_parts,
                            uint32_t max_chain, uint32_t cu_count);

// Entries per step of a hot-steps copy laid out for rank R and factor dtype:
// the lane groups one wave runs at that rank and dtype.
uint32_t step_entries(int R, int dtype);

// LDS bytes of the step kernel for n_in inputs, rank R, element bytes es, nhot hot rows each.
uint32_t step_kernel_lds_bytes(int n_in, int R, int es, uint32_t nhot);

// Threads per partition workgroup for n_in input modes.
int partition_wg_threads(int n_in);

// Threads per workgroup of the step kernel (hot-steps copies).
int step_wg_threads();

// Dynamic LDS of the partition kernel for n_in input modes and nhot cached rows per mode.
uint32_t partition_lds_bytes(int n_in, int R, int dtype, uint32_t nhot);

// Enqueue the per-mode MTTKRP: partition kernel then fix-up kernel.  With
// atomic_cut (the paper's scheme 2, for comparison) the output (out_rows x R)
// is zeroed first and rows cut by partition boundaries are added with global
// atomics instead of the deterministic carry fix-up.
// `fac` and `hot_rows` hold the N-1 input factors and their hot-row tables in
// the order of m.in_modes; nhot rows of each are cached in LDS.
hipError_t launch_mttkrp(const DevMode& m, int R, int dtype, const void* const* fac,
                         const uint32_t* const* hot_rows, uint32_t nhot, float* out, float* carry,
                         const Geometry& g, hipStream_t s, bool atomic_cut = false, uint32_t out_rows = 0);

// Gather-ceiling probe of one mode (stream and row gathers, no arithmetic);
// what = 0: stream only, 1: stream and gathers.  Writes only (rarely) carry.
hipError_t launch_gather_probe(const DevMode& m, int R, int dtype, const void* const* fac, float* carry,
                               const Geometry& g, int what, hipStream_t s);

// Batched launches: device descriptor arrays plus (tensor, item) work lists.
size_t part_desc_bytes(int n_in);
void fill_part_desc(void* dst, const DevMode& m, int R, int dtype, const void* const* fac, float* out, float* carry,
                    uint32_t gsz);
size_t fix_desc_bytes();
// Returns the number of fix-up blocks of this copy.
uint32_t fill_fix_desc(void* dst, const DevMode& m, const Geometry& g, float* carry, float* out, int R);
// threads, gathers: the batch's tuned shape (0, 0: the default kernels).
hipError_t launch_batch_part(int n_in, int R, int dtype, int threads, int gathers, const void* descs,
                             const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s);
hipError_t launch_batch_fixup(const void* descs, const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s);

// CP-ALS helpers (als_kernels.hip).  All FP64 unless noted.
// One normal-equation inverse per job: V = Hadamard product of the Gram
// matrices of every mode but `skip`, W = V^{-1}; *flag = 1 if V is not SPD
// (cleared first when reset_flag).  jobs: device array of `count` entries.
struct InvJob {
    const double* grams;   // N x R x R
    double* V;             // R x R
    double* W;             // R x R
    double* flag;          // 1 double
};

struct AlsWork {
    double* grams = nullptr;     // N x R x R
    double* V = nullptr;         // R x R
    double* W = nullptr;         // R x R (V^{-1})
    double* part = nullptr;      // per-block partial sums: max_blocks x (R x R)
    double* colsq = nullptr;     // R
    double* lam = nullptr;       // R
    double* scal = nullptr;      // small scalars: [0] fit, [1] not-positive-definite flag
    float* M = nullptr;          // max_I x R fp32 (MTTKRP output)
    uint16_t* bf16[MTTKRP_MAX_MODES] = {};  // bf16 copies of the factors (optional)
    InvJob* job = nullptr;       // device copy of {grams, V, W, scal + 1} for the inverse kernel
    int max_blocks = 0;
};

hipError_t als_gram(const float* A, uint32_t I, int R, double* G_out, AlsWork& w, hipStream_t s);
hipError_t als_hadamard(const double* grams, int N, int skip, int R, double* V, double* flag, int reset_flag,
                        hipStream_t s);
// solve 0: W = V^{-1} (sweep operator); 1: W = V's Cholesky factor L.
hipError_t als_normal_eq_inverse(const InvJob* jobs, int count, int N, int skip, int R, int reset_flag, int solve,
                                 hipStream_t s);

// The row passes of one mode update of one tensor (a "job"): A = M W with
// column norms into lam and A normalised; the Gram matrix of A; the fit.
// A job's rows are split into nb blocks of rpb rows (plan_dense_blocks); the
// *_jobs entry points run one job passed by value (jobs == NULL, grid = its
// blocks) or a device job table with a device (job, block) work list of
// nwork items, in one launch per kernel for every job.  Each job's arithmetic
// and reduction order are the same either way.
struct DenseJob {
    const float* M;        // I x R MTTKRP output
    const double* W;       // R x R inverse of V
    float* A;              // I x R factor being updated (fp32)
    double* lam;           // R column norms
    double* part;          // per-block partial sums (>= nb x R x R)
    double* colsq;         // R (fit: column dot products)
    double* G_out;         // R x R Gram matrix of A
    const double* grams;   // N x R x R (fit)
    double* fit_out;       // 1 double (fit)
    double* lam_out;       // R (fit: the caller's lambda)
    double normX2;         // |X|^2 (fit)
    uint16_t* A16;         // bf16 copy of A (batched casts), or null
    uint32_t I, rpb, nb;
    int N;
};
void plan_dense_blocks(uint32_t I, int max_blocks, DenseJob& j);
// solve: as als_normal_eq_inverse, for the W the jobs hold (0: M W; 1: substitution with L).
hipError_t als_solve_normalize_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork,
                                    int count, int R, int solve, hipStream_t s);
hipError_t als_gram_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork, int count,
                         int R, hipStream_t s);
// als_solve_normalize_jobs followed by als_gram_jobs; for R = 16 and 32 with
// the V^{-1} solve the Gram partials come from the store pass itself.
hipError_t als_solve_normalize_gram_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work,
                                         uint32_t nwork, int count, int R, int solve, hipStream_t s);
hipError_t als_fit_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork, int count,
                        int R, hipStream_t s);
hipError_t cast_bf16(const float* A, uint64_t n, uint16_t* out, hipStream_t s);
// bf16 copies of every job's A into its A16 over a (job, row block) work list.
hipError_t cast_bf16_jobs(const DenseJob* jobs, const uint2* work, uint32_t nwork, int R, hipStream_t s);

// Device memory of one mode copy, sized for nnz_pad nonzeros and I_n rows:
// N-1 index arrays, values, per-word row info, and the row lists (nonempty
// rows first, then the empty rows, I_n entries in all).
struct DeviceModeSlots {
    uint32_t* idx[kMaxIn] = {};   // uint16 arrays when idx16
    bool idx16 = false;
    float* val = nullptr;
    uint2* winfo = nullptr;
    uint32_t* rows = nullptr;
};

// Whether the copies of this tensor can be built on the device: 1 <= nnz < 2^31
// and the packed coordinate key (all N indices) fits 128 bits.
bool device_build_applies(const uint32_t* dims, int N, uint64_t nnz);

// Device scratch bytes of build_device_modes (0 when the device build does not apply).
uint64_t device_build_scratch_bytes(const uint32_t* dims, int N, uint64_t nnz);

// Build all N mode copies on the device into `slots` (same arrays and order as
// the host build) and the duplicate-merged |X|^2; uploads the COO tensor to a
// scratch region: ext_scratch (256-byte aligned, at least
// device_build_scratch_bytes) or, when that is NULL, an allocation freed
// before returning.  Synchronises `s`.
hipError_t build_device_modes(const uint32_t* coo_host, const float* vals_host, uint64_t nnz, const uint32_t* dims,
                              int N, const std::vector<DeviceModeSlots>& slots, std::vector<DevMode>& modes,
                              double* normX2, void* ext_scratch, uint64_t ext_scratch_bytes, hipStream_t s);

// Record `msg` as this thread's last error and return `s`.
mttkrp_status set_error(mttkrp_status s, const char* msg);

// mttkrp_run (fp32 factors) with the carry rows of partition-cut rows in
// `carry` (device memory of `device`, carry_bytes long) instead of the
// handle's workspace.  MTTKRP_EINVAL when `device` is not the handle's,
// MTTKRP_ENOMEM when the launch needs more than carry_bytes.
mttkrp_status run_fp32_with_carry(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                  int device, float* carry, uint64_t carry_bytes, hipStream_t stream);

}  // namespace mk
