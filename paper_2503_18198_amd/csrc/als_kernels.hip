// CP-ALS update kernels (FP64 arithmetic).
//
// The paper computes CPD by alternating least squares around the MTTKRP and
// normalises the factors (Sec. II-A).  The least-squares step is the
// textbook one: A_n = M V^{-1} with V the Hadamard product of the other
// factors' Gram matrices.  R <= 64 here, so V is tiny: by default its inverse
// comes from one workgroup (sweep operator, whose pivots are those of V's
// Cholesky factorisation, so non-SPD V is caught) and the I_n x R products
// M V^{-1} are row passes on the FP64 matrix cores; opt-in, V is factored by
// Cholesky and every row of M is solved by substitution.  Every reduction writes per-block partials that a
// second kernel adds in block order, so results repeat bit for bit.

#include <math.h>

#include "internal.h"

namespace mk {
namespace {

constexpr int kRowsTile = 16;   // rows staged in LDS per step of the row passes

// Block b of a job covers rows [b * rpb, min((b+1) * rpb, I)).
__device__ __forceinline__ void block_rows(uint32_t I, uint32_t rpb, uint32_t b, uint32_t& r0, uint32_t& r1)
{
    r0 = min((uint64_t)b * rpb, (uint64_t)I);
    r1 = min((uint64_t)r0 + rpb, (uint64_t)I);
}

// The (job, block) a workgroup of a row pass works on: with a job table,
// work[blockIdx.x] names both; without one, the single job passed by value
// and block blockIdx.x.
__device__ __forceinline__ const DenseJob& pick_job(const DenseJob& single, const DenseJob* jobs, const uint2* work,
                                                    uint32_t& blk)
{
    if (!jobs) {
        blk = blockIdx.x;
        return single;
    }
    const uint2 w = work[blockIdx.x];
    blk = w.y;
    return jobs[w.x];
}

// part[b][r*R + c] = sum over the block's rows i of A[i][r] * A[i][c].
// Thread (bi, bj) of a 16 x 16 grid owns the B x B entry block (B = R/16)
// with rows bi*B.. and columns bj*B..; rows are staged 16 at a time in LDS.
template <int R>
__global__ __launch_bounds__(kWG) void gram_partial_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                           const uint2* __restrict__ work)
{
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const float* __restrict__ A = jb.A;
    const uint32_t I = jb.I;
    double* __restrict__ part = jb.part;
    constexpr int B = R / 16;
    __shared__ double tile[kRowsTile * R];
    const int tid = threadIdx.x;
    const int bi = tid / 16, bj = tid % 16;
    double acc[B][B];
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) acc[i][j] = 0.0;
    uint32_t r0, r1;
    block_rows(I, jb.rpb, blk, r0, r1);
    for (uint32_t i0 = r0; i0 < r1; i0 += kRowsTile) {
        const uint32_t nrow = min((uint32_t)kRowsTile, r1 - i0);
        __syncthreads();
        for (int e = tid; e < kRowsTile * R; e += kWG)
            tile[e] = e < (int)(nrow * R) ? (double)A[(uint64_t)i0 * R + e] : 0.0;
        __syncthreads();
#pragma unroll 4
        for (int t = 0; t < kRowsTile; ++t) {
            double x[B], y[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                x[i] = tile[t * R + bi * B + i];
                y[i] = tile[t * R + bj * B + i];
            }
#pragma unroll
            for (int i = 0; i < B; ++i)
#pragma unroll
                for (int j = 0; j < B; ++j) acc[i][j] += x[i] * y[j];
        }
    }
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) part[(uint64_t)blk * R * R + (bi * B + i) * R + bj * B + j] = acc[i][j];
}

// out[e] = sum over blocks b of part[b * K + e], one wave per entry: lane j
// adds blocks j, j+64, ... in order, then a fixed butterfly adds the 64 lane
// sums.  Workgroup g serves job g / per_job (per_job = ceil(K / 4)); `which`
// picks the job's output: 0 lam (op: sqrt, 1 in place of 0 -> column norms),
// 1 the Gram matrix G_out, 2 colsq.
__global__ __launch_bounds__(kWG) void reduce_partials_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                              int K, int which)
{
    const int per_job = (K + kWG / 64 - 1) / (kWG / 64);
    const DenseJob& jb = jobs ? jobs[blockIdx.x / per_job] : single;
    const int e = (blockIdx.x % per_job) * (kWG / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (e >= K) return;
    const double* __restrict__ part = jb.part;
    const int nblk = (int)jb.nb;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(uint64_t)b * K + e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        if (which == 0) jb.lam[e] = s > 0.0 ? sqrt(s) : 1.0;
        else if (which == 1) jb.G_out[e] = s;
        else jb.colsq[e] = s;
    }
}

// V = Hadamard product of all Gram matrices except `skip` (skip = -1: all).
// reset_flag: clear the not-positive-definite flag at the start of a sweep.
__global__ __launch_bounds__(kWG) void hadamard_kernel(const double* __restrict__ grams, int N, int skip, int R,
                                                       double* __restrict__ V, double* flag, int reset_flag)
{
    const int RR = R * R;
    for (int e = threadIdx.x; e < RR; e += kWG) {
        double v = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != skip) v *= grams[(uint64_t)m * RR + e];
        V[e] = v;
    }
    if (reset_flag && threadIdx.x == 0) *flag = 0.0;
}

// V^{-1} of the symmetric positive definite R x R matrix V by R sweeps of the
// sweep operator (Goodnight, 1979), all in LDS: sweeping pivot k maps A to
//   A[i][j] - A[i][k] A[k][j] / d,  A[i][k] / d,  A[k][j] / d,  -1 / d
// (d = A[k][k]; the four cases are i,j != k, j == k, i == k, and both), and
// after every pivot has been swept A = -V^{-1}.  For SPD V the pivots are the
// squared diagonal of V's Cholesky factor, so a pivot that is not positive
// beyond rounding (relative to V_kk) means V is not SPD to working precision:
// then *flag = 1 and W is filled with NaN.  Each sweep updates all R^2
// entries in parallel from one LDS copy of A into the other, so one barrier
// per sweep separates it from the next.
//
// One workgroup per job: job b first forms its V = Hadamard product of the
// Gram matrices of every mode but `skip` (kept in LDS and stored to V), then
// inverts it into W.  One launch serves one tensor or every tensor of a batch.
template <int R>
__global__ __launch_bounds__(kWG) void normal_eq_inverse_kernel(const InvJob* __restrict__ jobs, int N, int skip,
                                                                int reset_flag)
{
    constexpr int RR = R * R;
    constexpr int kPer = (RR + kWG - 1) / kWG;   // entries per thread
    __shared__ double Abuf[2][RR];
    __shared__ double diag0[R];
    const InvJob jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    for (int e = tid; e < RR; e += kWG) {
        double v = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != skip) v *= jb.grams[(uint64_t)m * RR + e];
        Abuf[0][e] = v;
        jb.V[e] = v;
    }
    __syncthreads();
    if (tid < R) diag0[tid] = Abuf[0][tid * R + tid];
    __syncthreads();
    bool bad = false;   // every thread tests the same pivots, so this is uniform
    for (int k = 0; k < R; ++k) {
        const double* A = Abuf[k & 1];
        double* An = Abuf[(k + 1) & 1];
        double d = A[k * R + k];
        if (!(d > 64.0 * 2.220446049250313e-16 * fabs(diag0[k])) || !isfinite(d)) {
            bad = true;
            d = 1.0;
        }
        const double inv = 1.0 / d;
        double nv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = tid + q * kWG;
            const int i = e / R;
            const int j = e % R;
            nv[q] = 0.0;
            if (e < RR) {
                const double aik = A[i * R + k];
                const double akj = A[k * R + j];
                if (i == k && j == k) nv[q] = -inv;
                else if (i == k) nv[q] = akj * inv;
                else if (j == k) nv[q] = aik * inv;
                else nv[q] = A[e] - aik * akj * inv;
            }
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = tid + q * kWG;
            if (e < RR) An[e] = nv[q];
        }
        __syncthreads();
    }
    const double* A = Abuf[R & 1];
    for (int e = tid; e < RR; e += kWG) jb.W[e] = bad ? __longlong_as_double(0x7ff8000000000000ll) : -A[e];
    if (tid == 0) {
        if (reset_flag) *jb.flag = 0.0;
        if (bad) *jb.flag = 1.0;
    }
}

// ---- The Cholesky solve (opt-in, mttkrp_opts.als_solve = 1) ----
//
// Cholesky factor of the symmetric positive definite R x R normal-equation
// matrix V (the textbook CP-ALS solve): one workgroup per job forms V = the
// Hadamard product of the Gram matrices of every mode but `skip` (kept in LDS
// and stored to V), then factors V = L L^T in place, right-looking: at step k
// the pivot d is the Schur complement's diagonal entry, L_kk = sqrt(d), the
// column below is divided by L_kk and the trailing lower triangle loses
// L_ik L_jk (all entries of a step in parallel, barriers between steps).  The
// pivot test is the sweep operator's, on the same pivots: a failure sets
// *flag = 1 and fills W with NaN.  Otherwise W holds L (lower triangle; zeros
// above).  One launch serves one tensor or every tensor of a batch.
template <int R>
__global__ __launch_bounds__(kWG) void normal_eq_cholesky_kernel(const InvJob* __restrict__ jobs, int N, int skip,
                                                                 int reset_flag)
{
    constexpr int RR = R * R;
    __shared__ double A[RR];
    __shared__ double diag0[R];
    const InvJob jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    for (int e = tid; e < RR; e += kWG) {
        double v = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != skip) v *= jb.grams[(uint64_t)m * RR + e];
        A[e] = v;
        jb.V[e] = v;
    }
    __syncthreads();
    if (tid < R) diag0[tid] = A[tid * R + tid];
    __syncthreads();
    bool bad = false;   // every thread tests the same pivots, so this is uniform
    for (int k = 0; k < R; ++k) {
        double d = A[k * R + k];
        if (!(d > 64.0 * 2.220446049250313e-16 * fabs(diag0[k])) || !isfinite(d)) {
            bad = true;
            d = 1.0;
        }
        const double lkk = sqrt(d);
        const double inv = 1.0 / lkk;
        __syncthreads();                              // every thread has read the pivot
        for (int i = k + 1 + tid; i < R; i += kWG) A[i * R + k] *= inv;
        if (tid == 0) A[k * R + k] = lkk;
        __syncthreads();
        // Trailing lower triangle: entries (i, j) with k < j <= i < R.
        for (int e = tid; e < RR; e += kWG) {
            const int i = e / R, j = e % R;
            if (j > k && j <= i) A[e] -= A[i * R + k] * A[j * R + k];
        }
        __syncthreads();
    }
    for (int e = tid; e < RR; e += kWG) {
        const int i = e / R, j = e % R;
        jb.W[e] = bad ? __longlong_as_double(0x7ff8000000000000ll) : (j <= i ? A[e] : 0.0);
    }
    if (tid == 0) {
        if (reset_flag) *jb.flag = 0.0;
        if (bad) *jb.flag = 1.0;
    }
}

// Rows of M V^{-1} (FP64) by substitution with the Cholesky factor L of V
// (in W): forward L y = m, then backward L^T x = y, one row per thread,
// both in column order (after x_k is final, the rows it enters are updated),
// so the R - k updates of a step are independent.  L and 1/L_kk sit in LDS
// and are read by every lane at the same address, one column of L per step
// (compiler barriers keep the scheduler from holding all of L in registers).
// op 0: per-block column sums of squares -> part[b][c]: for R <= 32 each
// thread adds its rows in registers and the 64 lanes of a wave are then added
// by a fixed butterfly; for R = 64 every row's squares go through the
// butterfly at once into a per-wave LDS sum; the waves are added in order.
// op 1: A[i][c] = x[c] / lam[c], stored as fp32.
template <int R>
__global__ __launch_bounds__(kWG) void chol_solve_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                         const uint2* __restrict__ work, int op)
{
    constexpr int kWaves = kWG / 64;
    constexpr bool kRegSums = R <= 32;
    __shared__ double sL[R * R];
    __shared__ double sdinv[R];
    __shared__ double sscale[R];
    __shared__ double swave[kWaves][R];
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < R * R; e += kWG) sL[e] = jb.W[e];
    for (int e = tid; e < kWaves * R; e += kWG) swave[e / R][e % R] = 0.0;
    __syncthreads();
    if (tid < R) {
        sdinv[tid] = 1.0 / sL[tid * R + tid];
        sscale[tid] = op == 1 ? 1.0 / jb.lam[tid] : 0.0;
    }
    __syncthreads();
    uint32_t r0, r1;
    block_rows(jb.I, jb.rpb, blk, r0, r1);
    double colsq[kRegSums ? R : 1];
#pragma unroll
    for (int c = 0; c < (kRegSums ? R : 1); ++c) colsq[c] = 0.0;
    // Every wave runs the same number of row steps, so the butterflies below
    // always have all 64 lanes (rows past the block's end contribute zero).
    const uint32_t nsteps = (r1 - r0 + kWG - 1) / kWG;
    for (uint32_t it = 0; it < nsteps; ++it) {
        const uint32_t i = r0 + it * kWG + tid;
        const bool live = i < r1;
        double x[R];
        if (live) {
            const float4* mrow = reinterpret_cast<const float4*>(jb.M + (uint64_t)i * R);
#pragma unroll
            for (int q = 0; q < R / 4; ++q) {
                const float4 v = mrow[q];
                x[4 * q] = v.x;
                x[4 * q + 1] = v.y;
                x[4 * q + 2] = v.z;
                x[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) x[c] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            asm volatile("" ::: "memory");   // one column of L in registers at a time
            x[k] *= sdinv[k];
#pragma unroll
            for (int j = k + 1; j < R; ++j) x[j] -= sL[j * R + k] * x[k];
        }
#pragma unroll
        for (int k = R - 1; k >= 0; --k) {
            asm volatile("" ::: "memory");
            x[k] *= sdinv[k];
#pragma unroll
            for (int j = 0; j < k; ++j) x[j] -= sL[k * R + j] * x[k];
        }
        if (op == 0) {
            if constexpr (kRegSums) {
#pragma unroll
                for (int c = 0; c < R; ++c) colsq[c] += x[c] * x[c];
            } else {
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    double t = x[c] * x[c];
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
                    if (lane == 0) swave[wave][c] += t;
                }
            }
        } else if (live) {
            float4* arow = reinterpret_cast<float4*>(jb.A + (uint64_t)i * R);
#pragma unroll
            for (int q = 0; q < R / 4; ++q)
                arow[q] = make_float4((float)(x[4 * q] * sscale[4 * q]), (float)(x[4 * q + 1] * sscale[4 * q + 1]),
                                      (float)(x[4 * q + 2] * sscale[4 * q + 2]),
                                      (float)(x[4 * q + 3] * sscale[4 * q + 3]));
        }
    }
    if (op == 0) {
        if constexpr (kRegSums) {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                double t = colsq[c];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
                if (lane == 0) swave[wave][c] = t;
            }
        }
        __syncthreads();
        if (tid < R) {
            double t = 0.0;
            for (int w = 0; w < kWaves; ++w) t += swave[w][tid];
            jb.part[(uint64_t)blk * R + tid] = t;
        }
    }
}

// Rows of M W (FP64).  Thread (ri of 32, column group cg of 8) computes the
// B = R/8 columns cg*B.. of rows ri, ri+32, ... (RB rows: register blocking,
// so each W value read from LDS feeds RB products).  The M tile is staged in
// LDS with a padded row stride so the 8 rows a wave reads at once fall in
// different banks.  op 0: per-block column sums of squares -> part[b][c].
// op 1: A[i][c] = (M W)[i][c] / lam[c], stored as fp32.
template <int R>
__global__ __launch_bounds__(kWG) void mw_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                 const uint2* __restrict__ work, int op)
{
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const float* __restrict__ M = jb.M;
    const double* __restrict__ W = jb.W;
    const uint32_t I = jb.I;
    const double* __restrict__ lam = jb.lam;
    float* __restrict__ A = jb.A;
    double* __restrict__ part = jb.part;
    constexpr int B = R / 8;
    constexpr int RB = R == 64 ? 1 : 4;        // rows per thread (LDS: 64 KB static limit)
    constexpr int kRows = (kWG / 8) * RB;
    constexpr int SP = R + 1;                  // padded stride of the staged M rows
    static_assert(kRows * SP >= kWG * B, "column partials reuse the M tile");
    __shared__ double sW[R * R];
    __shared__ double sM[kRows * SP];
    const int tid = threadIdx.x;
    for (int e = tid; e < R * R; e += kWG) sW[e] = W[e];
    const int ri = tid / 8;
    const int cg = tid % 8;
    double inv[B];
    double colsq[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
        inv[j] = op == 1 ? 1.0 / lam[cg * B + j] : 0.0;
        colsq[j] = 0.0;
    }
    uint32_t r0, r1;
    block_rows(I, jb.rpb, blk, r0, r1);
    for (uint32_t i0 = r0; i0 < r1; i0 += kRows) {
        const uint32_t nrow = min((uint32_t)kRows, r1 - i0);
        __syncthreads();
        for (int e = tid; e < kRows * R; e += kWG) {
            const int rr = e / R, cc = e % R;
            sM[rr * SP + cc] = (uint32_t)rr < nrow ? (double)M[((uint64_t)i0 + rr) * R + cc] : 0.0;
        }
        __syncthreads();
        double acc[RB][B];
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int j = 0; j < B; ++j) acc[q][j] = 0.0;
#pragma unroll 4
        for (int k = 0; k < R; ++k) {
            double w[B];
#pragma unroll
            for (int j = 0; j < B; ++j) w[j] = sW[k * R + cg * B + j];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const double m = sM[(ri + 32 * q) * SP + k];
#pragma unroll
                for (int j = 0; j < B; ++j) acc[q][j] += m * w[j];
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const uint32_t rr = ri + 32 * q;
            if (rr < nrow) {
                const uint64_t row = i0 + rr;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    if (op == 0) colsq[j] += acc[q][j] * acc[q][j];
                    else A[row * R + cg * B + j] = (float)(acc[q][j] * inv[j]);
                }
            }
        }
    }
    if (op == 0) {
        __syncthreads();
        double* sred = sM;
#pragma unroll
        for (int j = 0; j < B; ++j) sred[(cg * B + j) * 32 + ri] = colsq[j];
        __syncthreads();
        if (tid < R) {
            double t = 0.0;
            for (int r = 0; r < 32; ++r) t += sred[tid * 32 + r];
            part[(uint64_t)blk * R + tid] = t;
        }
    }
}

// ---- FP64 matrix-core versions of the two row passes (R = 16, 32) ----
//
// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; item q of its result is
// D[l / 16 + 4 q][l % 16].
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Rows of M W on matrix cores; same job, blocks and outputs as mw_kernel.
// Each wave takes 16-row tiles.  Lane (lr = l % 16, lq = l / 16) loads
// M[row lr][16h + 4lq .. +3] as one 16-byte load; its j-th value is the
// A operand of k-step 4h + j, whose k index lq stands for k = 16h + 4lq + j,
// so the B operand of that step is W[16h + 4lq + j][16t + lr].
// GRAM (with op 1): the store pass also adds the Gram partials of the
// stored rows.  Item q of a column tile's result is row tile + lq + 4q,
// column 16t + lr of A: for each q that is exactly the operand a Gram
// matrix-core step over those 4 rows takes (as in gram_mfma_kernel), so
// A^T A needs no second pass over A.
template <int R, bool GRAM = false>
__global__ __launch_bounds__(kWG) void mw_mfma_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                      const uint2* __restrict__ work, int op)
{
    static_assert(R == 16 || R == 32, "matrix-core row pass for R = 16 or 32");
    constexpr int CT = R / 16;   // column tiles
    constexpr int H = R / 16;    // 16-wide k chunks
    __shared__ double sred[GRAM ? 4 * R * R : R * 16];
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const float* __restrict__ M = jb.M;
    const double* __restrict__ W = jb.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    double wf[H][4][CT];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < CT; ++t) wf[h][j][t] = W[(16 * h + 4 * lq + j) * R + 16 * t + lr];
    double inv[CT];
    double colsq[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        inv[t] = op == 1 ? 1.0 / jb.lam[16 * t + lr] : 0.0;
        colsq[t] = 0.0;
    }
    f64x4 gacc[CT][CT];
    if constexpr (GRAM) {
#pragma unroll
        for (int a = 0; a < CT; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b) gacc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    uint32_t r0, r1;
    block_rows(jb.I, jb.rpb, blk, r0, r1);
    for (uint32_t tile = r0 + 16u * wave; tile < r1; tile += 64u) {
        const uint32_t row = tile + lr;
        f64x4 acc[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float4 m = {0.f, 0.f, 0.f, 0.f};
            if (row < r1) m = *reinterpret_cast<const float4*>(M + (uint64_t)row * R + 16 * h + 4 * lq);
            const double a[4] = {(double)m.x, (double)m.y, (double)m.z, (double)m.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int t = 0; t < CT; ++t) acc[t] = mfma_f64(a[j], wf[h][j][t], acc[t]);
        }
        if constexpr (GRAM) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t rr = tile + lq + 4 * q;
                double x[CT];
#pragma unroll
                for (int t = 0; t < CT; ++t) {
                    x[t] = 0.0;
                    if (rr < r1) {
                        const float v = (float)(acc[t][q] * inv[t]);
                        jb.A[(uint64_t)rr * R + 16 * t + lr] = v;
                        x[t] = (double)v;
                    }
                }
#pragma unroll
                for (int a = 0; a < CT; ++a)
#pragma unroll
                    for (int b = 0; b < CT; ++b) gacc[a][b] = mfma_f64(x[a], x[b], gacc[a][b]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < CT; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t rr = tile + lq + 4 * q;
                    if (rr < r1) {
                        if (op == 0) colsq[t] += acc[t][q] * acc[t][q];
                        else jb.A[(uint64_t)rr * R + 16 * t + lr] = (float)(acc[t][q] * inv[t]);
                    }
                }
        }
    }
    if constexpr (GRAM) {
        // The four waves' tiles, added in a fixed order.
#pragma unroll
        for (int a = 0; a < CT; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    sred[wave * R * R + (16 * a + lq + 4 * q) * R + 16 * b + lr] = gacc[a][b][q];
        __syncthreads();
        for (int e = threadIdx.x; e < R * R; e += kWG)
            jb.part[(uint64_t)blk * R * R + e] =
                ((sred[e] + sred[R * R + e]) + sred[2 * R * R + e]) + sred[3 * R * R + e];
        return;
    }
    if (op == 0) {
        // Column c = 16t + lr: 16 partials (4 waves x 4 lane quarters), added in a fixed order.
#pragma unroll
        for (int t = 0; t < CT; ++t) sred[(16 * t + lr) * 16 + wave * 4 + lq] = colsq[t];
        __syncthreads();
        if (threadIdx.x < R) {
            double v = 0.0;
            for (int k = 0; k < 16; ++k) v += sred[threadIdx.x * 16 + k];
            jb.part[(uint64_t)blk * R + threadIdx.x] = v;
        }
    }
}

// Gram partials of the block's rows on matrix cores: D = sum_i A[i]^T A[i]
// over 4-row steps; the A operand is A^T (lane: row i0 + lq, column 16rt + lr),
// the B operand A itself (row i0 + lq, column 16ct + lr).  Each wave takes
// every fourth 4-row step; the four waves' tiles are added in a fixed order.
template <int R>
__global__ __launch_bounds__(kWG) void gram_mfma_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                        const uint2* __restrict__ work)
{
    static_assert(R == 16 || R == 32, "matrix-core Gram for R = 16 or 32");
    constexpr int T = R / 16;
    __shared__ double sacc[4 * R * R];
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const float* __restrict__ A = jb.A;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    f64x4 acc[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    uint32_t r0, r1;
    block_rows(jb.I, jb.rpb, blk, r0, r1);
    for (uint32_t i0 = r0 + 4u * wave; i0 < r1; i0 += 16u) {
        const uint32_t row = i0 + lq;
        double x[T];
#pragma unroll
        for (int h = 0; h < T; ++h) x[h] = row < r1 ? (double)A[(uint64_t)row * R + 16 * h + lr] : 0.0;
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) acc[a][b] = mfma_f64(x[a], x[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                sacc[wave * R * R + (16 * a + lq + 4 * q) * R + 16 * b + lr] = acc[a][b][q];
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += kWG)
        jb.part[(uint64_t)blk * R * R + e] =
            ((sacc[e] + sacc[R * R + e]) + sacc[2 * R * R + e]) + sacc[3 * R * R + e];
}

// part[b][c] = sum over the block's rows of M[i][c] * A[i][c].
__global__ __launch_bounds__(kWG) void coldot_kernel(DenseJob single, const DenseJob* __restrict__ jobs,
                                                     const uint2* __restrict__ work, int R)
{
    uint32_t blk;
    const DenseJob& jb = pick_job(single, jobs, work, blk);
    const float* __restrict__ M = jb.M;
    const float* __restrict__ A = jb.A;
    const uint32_t I = jb.I;
    double* __restrict__ part = jb.part;
    __shared__ double sred[kWG];
    const int tid = threadIdx.x;
    const int rows_per_pass = kWG / R;
    const int c = tid % R;
    const int ri = tid / R;
    double s = 0.0;
    uint32_t r0, r1;
    block_rows(I, jb.rpb, blk, r0, r1);
    for (uint32_t i = r0 + ri; i < r1; i += rows_per_pass)
        s += (double)M[(uint64_t)i * R + c] * (double)A[(uint64_t)i * R + c];
    sred[tid] = s;
    __syncthreads();
    if (tid < R) {
        double t = 0.0;
        for (int j = 0; j < rows_per_pass; ++j) t += sred[j * R + tid];
        part[(uint64_t)blk * R + tid] = t;
    }
}

// fit = 1 - sqrt(max(0, |X|^2 + lam^T (*G) lam - 2 sum_r lam_r dot_r)) / |X|.
__global__ __launch_bounds__(kWG) void fit_kernel(DenseJob single, const DenseJob* __restrict__ jobs, int R)
{
    const DenseJob& jb = jobs ? jobs[blockIdx.x] : single;
    const double* __restrict__ dot = jb.colsq;
    const double* __restrict__ lam = jb.lam;
    const double* __restrict__ grams = jb.grams;
    const int N = jb.N;
    const double normX2 = jb.normX2;
    double* fit_out = jb.fit_out;
    double* lam_out = jb.lam_out;
    __shared__ double sx[kWG];
    __shared__ double sd[kWG];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double x = 0.0;
    for (int e = tid; e < RR; e += kWG) {
        double v = 1.0;
        for (int m = 0; m < N; ++m) v *= grams[(uint64_t)m * RR + e];
        x += lam[e / R] * v * lam[e % R];
    }
    sx[tid] = x;
    sd[tid] = tid < R ? lam[tid] * dot[tid] : 0.0;
    if (lam_out && tid < R) lam_out[tid] = lam[tid];
    __syncthreads();
    if (tid == 0) {
        double xh = 0.0, inner = 0.0;
        for (int j = 0; j < kWG; ++j) xh += sx[j];
        for (int j = 0; j < R; ++j) inner += sd[j];
        const double res = normX2 + xh - 2.0 * inner;
        if (fit_out) *fit_out = 1.0 - sqrt(res > 0.0 ? res : 0.0) / sqrt(normX2);
    }
}

// Round fp32 to bfloat16, nearest-even on the bit pattern; NaN stays NaN.
__global__ __launch_bounds__(kWG) void cast_bf16_kernel(const float* __restrict__ A, uint64_t n,
                                                        uint16_t* __restrict__ out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kWG) {
        const uint32_t b = __float_as_uint(A[i]);
        uint16_t h;
        if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) h = (uint16_t)((b >> 16) | 0x0040u);
        else h = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
        out[i] = h;
    }
}

uint32_t nblocks_for(uint32_t I, int max_blocks, uint32_t& rpb)
{
    uint32_t nb = (I + 63) / 64;
    if (nb > (uint32_t)max_blocks) nb = (uint32_t)max_blocks;
    if (nb < 1) nb = 1;
    rpb = (I + nb - 1) / nb;
    return nb;
}

}  // namespace

hipError_t als_hadamard(const double* grams, int N, int skip, int R, double* V, double* flag, int reset_flag,
                        hipStream_t s)
{
    hipLaunchKernelGGL(hadamard_kernel, dim3(1), dim3(kWG), 0, s, grams, N, skip, R, V, flag, reset_flag);
    return hipGetLastError();
}

hipError_t als_normal_eq_inverse(const InvJob* jobs, int count, int N, int skip, int R, int reset_flag, int solve,
                                 hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (solve == 1) {
        switch (R) {
            case 16: hipLaunchKernelGGL(normal_eq_cholesky_kernel<16>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
            case 32: hipLaunchKernelGGL(normal_eq_cholesky_kernel<32>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
            case 64: hipLaunchKernelGGL(normal_eq_cholesky_kernel<64>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (R) {
        case 16: hipLaunchKernelGGL(normal_eq_inverse_kernel<16>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
        case 32: hipLaunchKernelGGL(normal_eq_inverse_kernel<32>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
        case 64: hipLaunchKernelGGL(normal_eq_inverse_kernel<64>, dim3(count), dim3(kWG), 0, s, jobs, N, skip, reset_flag); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void plan_dense_blocks(uint32_t I, int max_blocks, DenseJob& j)
{
    j.I = I;
    j.nb = nblocks_for(I, max_blocks, j.rpb);
}

// Each entry point runs either one job (passed by value, grid = its blocks)
// or a job table with a (job, block) work list of `nwork` items.
namespace {
struct Launch {
    const DenseJob& single;
    const DenseJob* jobs;
    const uint2* work;
    uint32_t nwork;   // row-pass workgroups
    int count;        // jobs
    uint32_t grid() const { return jobs ? nwork : single.nb; }
};

// R = 16 and 32 run on the FP64 matrix cores; R = 64 on the vector units.
template <int R>
void launch_solve(const Launch& L, int op, hipStream_t s)
{
    hipLaunchKernelGGL(chol_solve_kernel<R>, dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work, op);
}

template <int R>
void launch_mw(const Launch& L, int op, hipStream_t s)
{
    if constexpr (R <= 32)
        hipLaunchKernelGGL(mw_mfma_kernel<R>, dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work, op);
    else
        hipLaunchKernelGGL(mw_kernel<R>, dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work, op);
}

template <int R>
void launch_gram(const Launch& L, hipStream_t s)
{
    if constexpr (R <= 32)
        hipLaunchKernelGGL(gram_mfma_kernel<R>, dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work);
    else
        hipLaunchKernelGGL(gram_partial_kernel<R>, dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work);
}

void launch_reduce(const Launch& L, int K, int which, hipStream_t s)
{
    const int per_job = (K + kWG / 64 - 1) / (kWG / 64);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((uint32_t)(per_job * (L.jobs ? L.count : 1))), dim3(kWG), 0, s,
                       L.single, L.jobs, K, which);
}
}  // namespace

hipError_t als_solve_normalize_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork,
                                    int count, int R, int solve, hipStream_t s)
{
    const Launch L{single, jobs, work, nwork, count};
    if (L.grid() == 0) return hipSuccess;
    for (int op = 0; op < 2; ++op) {
        switch (R * 2 + (solve == 1 ? 1 : 0)) {
            case 32: launch_mw<16>(L, op, s); break;
            case 64: launch_mw<32>(L, op, s); break;
            case 128: launch_mw<64>(L, op, s); break;
            case 33: launch_solve<16>(L, op, s); break;
            case 65: launch_solve<32>(L, op, s); break;
            case 129: launch_solve<64>(L, op, s); break;
            default: return hipErrorInvalidValue;
        }
        if (op == 0) launch_reduce(L, R, 0, s);
    }
    return hipGetLastError();
}

hipError_t als_solve_normalize_gram_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work,
                                         uint32_t nwork, int count, int R, int solve, hipStream_t s)
{
    if (solve == 1 || R > 32) {
        const hipError_t e = als_solve_normalize_jobs(single, jobs, work, nwork, count, R, solve, s);
        return e != hipSuccess ? e : als_gram_jobs(single, jobs, work, nwork, count, R, s);
    }
    const Launch L{single, jobs, work, nwork, count};
    if (L.grid() == 0) return hipSuccess;
    if (R == 16) {
        launch_mw<16>(L, 0, s);
        launch_reduce(L, R, 0, s);
        hipLaunchKernelGGL((mw_mfma_kernel<16, true>), dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work, 1);
    } else if (R == 32) {
        launch_mw<32>(L, 0, s);
        launch_reduce(L, R, 0, s);
        hipLaunchKernelGGL((mw_mfma_kernel<32, true>), dim3(L.grid()), dim3(kWG), 0, s, L.single, L.jobs, L.work, 1);
    } else {
        return hipErrorInvalidValue;
    }
    launch_reduce(L, R * R, 1, s);
    return hipGetLastError();
}

hipError_t als_gram_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork, int count,
                         int R, hipStream_t s)
{
    const Launch L{single, jobs, work, nwork, count};
    if (L.grid() == 0) return hipSuccess;
    switch (R) {
        case 16: launch_gram<16>(L, s); break;
        case 32: launch_gram<32>(L, s); break;
        case 64: launch_gram<64>(L, s); break;
        default: return hipErrorInvalidValue;
    }
    launch_reduce(L, R * R, 1, s);
    return hipGetLastError();
}

hipError_t als_fit_jobs(const DenseJob& single, const DenseJob* jobs, const uint2* work, uint32_t nwork, int count,
                        int R, hipStream_t s)
{
    const Launch L{single, jobs, work, nwork, count};
    if (L.grid() == 0) return hipSuccess;
    hipLaunchKernelGGL(coldot_kernel, dim3(L.grid()), dim3(kWG), 0, s, single, jobs, work, R);
    launch_reduce(L, R, 2, s);
    hipLaunchKernelGGL(fit_kernel, dim3((uint32_t)(jobs ? count : 1)), dim3(kWG), 0, s, single, jobs, R);
    return hipGetLastError();
}

hipError_t als_gram(const float* A, uint32_t I, int R, double* G_out, AlsWork& w, hipStream_t s)
{
    DenseJob j{};
    j.A = const_cast<float*>(A);
    j.part = w.part;
    j.G_out = G_out;
    plan_dense_blocks(I, w.max_blocks, j);
    return als_gram_jobs(j, nullptr, nullptr, 0, 1, R, s);
}

// Round-to-nearest-even bf16 copies of many tensors' factors: work item
// (job, block) casts rows [block * rpb, min((block + 1) * rpb, I)) of job's A
// into its A16, with the same rounding as cast_bf16_kernel.
__global__ __launch_bounds__(kWG) void cast_bf16_jobs_kernel(const DenseJob* __restrict__ jobs,
                                                             const uint2* __restrict__ work, uint32_t nwork, int R)
{
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint2 wk = work[w];
        const DenseJob& j = jobs[wk.x];
        const uint64_t r0 = (uint64_t)wk.y * j.rpb;
        const uint64_t r1 = min(r0 + j.rpb, (uint64_t)j.I);
        if (r0 >= r1) continue;
        const uint64_t n = (r1 - r0) * (uint64_t)R;
        const float* A = j.A + r0 * R;
        uint16_t* out = j.A16 + r0 * R;
        for (uint64_t i = threadIdx.x; i < n; i += kWG) {
            const uint32_t b = __float_as_uint(A[i]);
            uint16_t h;
            if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) h = (uint16_t)((b >> 16) | 0x0040u);
            else h = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
            out[i] = h;
        }
    }
}

hipError_t cast_bf16_jobs(const DenseJob* jobs, const uint2* work, uint32_t nwork, int R, hipStream_t s)
{
    if (nwork == 0) return hipSuccess;
    const uint32_t grid = nwork < 4096u ? nwork : 4096u;
    hipLaunchKernelGGL(cast_bf16_jobs_kernel, dim3(grid), dim3(kWG), 0, s, jobs, work, nwork, R);
    return hipGetLastError();
}

hipError_t cast_bf16(const float* A, uint64_t n, uint16_t* out, hipStream_t s)
{
    uint64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(cast_bf16_kernel, dim3((uint32_t)blocks), dim3(kWG), 0, s, A, n, out);
    return hipGetLastError();
}

}  // namespace mk
