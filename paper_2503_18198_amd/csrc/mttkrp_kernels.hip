// Per-mode sparse MTTKRP for gfx950 (CDNA4, wave64).
//
// The paper's per-partition thread block (Alg. 2) gives each nonzero a
// column of R threads: load the nonzero, gather the N-1 input factor rows,
// multiply them element by element with the value, add the product into the
// output row (Sec. IV-B).  Here the same per-nonzero work is mapped onto
// CDNA4 as follows.
//
//  * A lane group of L = R*sizeof(T)/16 lanes owns one factor row per
//    gather: each lane loads one 16-byte slice, so a row is one coalesced
//    128-byte (fp32, R=32) access.  A wave runs 64/L groups side by side.
//  * Every lane group walks its own contiguous run of `gsz` nonzeros of the
//    mode copy (nonzero-balanced partitions, Sec. III-B scheme 2).  It
//    streams indices and values 32 nonzeros at a time with full-line loads,
//    shares them inside the group with ds_swizzle, keeps up to U nonzeros'
//    row gathers in flight, and accumulates the current output row in
//    registers.  A row that ends inside the group's run is stored once with
//    a plain store.
//  * A workgroup is G consecutive lane groups (one partition).  The partial
//    first/last rows of every group are combined in LDS in group order; rows
//    complete inside the workgroup are stored once.  A row cut by a
//    workgroup boundary leaves one partial per workgroup in `carry`, and the
//    fix-up kernel adds those in workgroup order.  No global atomics, a fixed
//    summation order, so results repeat bit for bit.
//  * Row boundaries come from one bit per nonzero ("starts a new output
//    row") plus, per 32 nonzeros, the ordinal of the row holding the first
//    one; ordinals map to output rows through the list of nonempty rows.
#include "internal.h"
#include "part_kernel.h"
#include "step_kernel.h"

namespace mk {

// Instantiated in part_n3.hip .. part_n8.hip.
extern template size_t part_desc_bytes_nin<2>();
extern template void fill_part_desc_nin<2>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<2>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template size_t part_desc_bytes_nin<3>();
extern template void fill_part_desc_nin<3>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<3>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template size_t part_desc_bytes_nin<4>();
extern template void fill_part_desc_nin<4>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<4>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template size_t part_desc_bytes_nin<5>();
extern template void fill_part_desc_nin<5>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<5>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template size_t part_desc_bytes_nin<6>();
extern template void fill_part_desc_nin<6>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<6>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template size_t part_desc_bytes_nin<7>();
extern template void fill_part_desc_nin<7>(void*, const DevMode&, int, int, const void* const*, float*, float*, uint32_t);
extern template hipError_t launch_batch_part_nin<7>(int, int, const void*, const uint2*, uint32_t, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<2>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<3>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<4>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<5>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<6>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_nin<7>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                                uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);

extern template hipError_t launch_part_tuned_wg<256>(const DevMode&, int, int, const void* const*, float*, float*,
                                                    const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_tuned_wg<512>(const DevMode&, int, int, const void* const*, float*, float*,
                                                    const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_part_tuned_wg<1024>(const DevMode&, int, int, const void* const*, float*, float*,
                                                     const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_batch_part_tuned_wg<256>(int, int, const void*, const uint2*, uint32_t, uint32_t,
                                                          hipStream_t);
extern template hipError_t launch_batch_part_tuned_wg<512>(int, int, const void*, const uint2*, uint32_t, uint32_t,
                                                          hipStream_t);
extern template hipError_t launch_batch_part_tuned_wg<1024>(int, int, const void*, const uint2*, uint32_t, uint32_t,
                                                           hipStream_t);
extern template hipError_t launch_step_nin<2>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                             uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);
extern template hipError_t launch_step_nin<3>(const DevMode&, int, int, const void* const*, const uint32_t* const*,
                                             uint32_t, float*, float*, const Geometry&, uint32_t, hipStream_t);

namespace {

struct FixArgs {
    const uint2* winfo;
    const uint32_t* row_id;
    const uint32_t* empty_rows;
    float* carry;
    float* out;
    uint64_t wgc;          // nonzeros per workgroup partition
    uint32_t nparts;
    uint32_t nbound;       // partition boundaries (nparts - 1, or 0 when no row is cut)
    uint64_t nempty;
    int R;
    int phase;             // 0: one pass; 1 then 2: chunk sums, then rows (see fixup_body)
};

constexpr int kEmptyPerBlock = 64;
constexpr int kBoundsPerBlock = kWG / 64;   // one wave per partition boundary
constexpr uint32_t kChunk = 64;              // partitions per chunk sum of a long cut row

// Fix-up blocks of a copy with nbound partition boundaries.
__host__ __device__ inline uint32_t fixup_bound_blocks(uint32_t nbound)
{
    return (nbound + kBoundsPerBlock - 1) / kBoundsPerBlock;
}

// Adds, in FP64, the R-float partials carry[slot(j) of partition part(j)] for
// j = 0 .. n-1, over 256 / R interleaved streams of 4 columns per lane, then
// the streams in stream order; lanes of stream 0 return the 4 sums of their
// columns (col = (lane % (R / 4)) * 4), the other lanes return garbage.
template <typename PartOf>
__device__ __forceinline__ double4 sum_partials(const FixArgs& a, uint32_t n, int lane, PartOf part_of)
{
    const int R = a.R;
    const int C4 = R / 4;                         // lanes per partial
    const int S = 64 / C4;                        // partial streams
    const int col = (lane % C4) * 4;
    const int st = lane / C4;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll 4
    for (uint32_t j = (uint32_t)st; j < n; j += (uint32_t)S) {
        const uint64_t slot_row = part_of(j);     // partition * 2 + slot
        const float4 c = *reinterpret_cast<const float4*>(a.carry + slot_row * R + col);
        t0 += (double)c.x;
        t1 += (double)c.y;
        t2 += (double)c.z;
        t3 += (double)c.w;
    }
    double4 sum = make_double4(t0, t1, t2, t3);
    for (int k = 1; k < S; ++k) {
        const int src = (lane % C4) + k * C4;
        sum.x += __shfl(t0, src, 64);
        sum.y += __shfl(t1, src, 64);
        sum.z += __shfl(t2, src, 64);
        sum.w += __shfl(t3, src, 64);
    }
    return sum;
}

// Block `blk` of the fix-up of one mode copy.  A row r cut by partition
// boundaries has one partial in `carry` for each partition holding part of
// it: partition pa, where it starts (slot 0 if pa itself starts inside r,
// else slot 1), and partitions qf .. pb, which start inside it (slot 0).
// The first fixup_bound_blocks(nbound) blocks take the boundaries, one wave
// each (boundary q = blk * kBoundsPerBlock + wave + 1, where partition q
// starts); the other blocks zero rows without nonzeros, kEmptyPerBlock each.
//  phase 0: the wave at the first boundary qf of each cut row adds all of its
//           partials in partition order and stores the row;
//  phase 1: every partition p of qf+1 .. pb with p % kChunk == 0 (a chunk
//           leader) replaces its slot 0 with the sum of slot 0 over
//           p .. min(p + kChunk - 1, pb);
//  phase 2: the wave at qf adds pa's partial, slot 0 of qf up to the first
//           chunk leader, and every chunk leader's sum, in partition order.
// Every sum is formed in FP64 in a fixed order, so results repeat bit for bit.
__device__ __forceinline__ void fixup_body(const FixArgs& a, uint32_t blk)
{
    const int tid = threadIdx.x;
    const int R = a.R;
    const uint32_t nbb = fixup_bound_blocks(a.nbound);
    if (blk < nbb) {
        const int lane = tid & 63;
        const uint32_t bidx = blk * kBoundsPerBlock + (uint32_t)(tid >> 6);
        if (bidx >= a.nbound) return;
        const uint32_t q = bidx + 1;                  // partition q begins at q * wgc
        const auto winfo_of = [&](uint32_t p) { return a.winfo[((uint64_t)p * a.wgc) >> 5]; };
        const uint2 wq = winfo_of(q);
        if (wq.x & 1u) return;                        // a row starts at the boundary: nothing is cut
        const uint32_t r = wq.y;                      // ordinal of the cut row
        const uint2 wp = winfo_of(q - 1);
        const bool interior = !(wp.x & 1u) && wp.y == r;   // the row was already cut at boundary q-1
        const int C4 = R / 4;
        const int col = (lane % C4) * 4;
        const bool stream0 = lane < C4;
        if (a.phase == 1) {
            if (!interior || q % kChunk != 0) return;
            // The chunk's partitions that start inside r form a prefix.
            const uint32_t p = q + (uint32_t)lane;
            const uint64_t out_m = __ballot(p >= a.nparts || winfo_of(p).y != r);
            const uint32_t cnt = out_m ? (uint32_t)__ffsll((long long)out_m) - 1 : 64u;
            const double4 sum = sum_partials(a, cnt, lane, [&](uint32_t j) { return ((uint64_t)q + j) * 2; });
            if (stream0)
                *reinterpret_cast<float4*>(a.carry + (uint64_t)q * 2 * R + col) =
                    make_float4((float)sum.x, (float)sum.y, (float)sum.z, (float)sum.w);
            return;
        }
        if (interior) return;
        const uint32_t pa = q - 1;
        const uint64_t slot_a = (wp.y == r) ? 0 : 1;  // pa starts inside r (slot 0) or r starts inside pa
        // Partitions q, q+1, ..., pb start inside the row; they form a prefix
        // of those after q (the row ordinal of a partition's first nonzero
        // never decreases).  The 64 partitions after q are tested at once; a
        // row reaching past them is ended by a 64-way search: with p = lo
        // inside the row and p = hi past it (hi = nparts counts as past),
        // lane l tests lo + (l+1) * step.
        const auto past = [&](uint32_t p) { return p >= a.nparts || winfo_of(p).y != r; };
        uint32_t pb;
        {
            const uint64_t m = __ballot(past(q + 1 + (uint32_t)lane));
            if (m != 0) {
                pb = q + (uint32_t)__ffsll((long long)m) - 1;
            } else {
                uint32_t lo = q + 64, hi = a.nparts;
                while (hi - lo > 1) {
                    const uint32_t step = (hi - lo + 63) / 64;
                    const uint32_t pl = lo + ((uint32_t)lane + 1) * step;
                    const uint64_t mm = __ballot(pl >= hi || past(pl));
                    const uint32_t f = (uint32_t)__ffsll((long long)mm) - 1;   // lane 63 always tests >= hi
                    hi = min(hi, lo + (f + 1) * step);
                    lo = lo + f * step;
                }
                pb = lo;
            }
        }
        // Contributions: j = 0 is pa; j = 1 .. n1 are partitions q .. q + n1 - 1;
        // then (phase 2) the chunk leaders l0, l0 + kChunk, ... <= pb.
        uint32_t n1 = pb - q + 1, n2 = 0, l0 = 0;
        if (a.phase == 2) {
            l0 = (q / kChunk + 1) * kChunk;
            if (l0 <= pb) {
                n1 = l0 - q;
                n2 = (pb - l0) / kChunk + 1;
            }
        }
        const double4 sum = sum_partials(a, 1 + n1 + n2, lane, [&](uint32_t j) -> uint64_t {
            if (j == 0) return (uint64_t)pa * 2 + slot_a;
            if (j <= n1) return ((uint64_t)q + j - 1) * 2;
            return ((uint64_t)l0 + (uint64_t)(j - 1 - n1) * kChunk) * 2;
        });
        if (stream0)
            *reinterpret_cast<float4*>(a.out + (uint64_t)a.row_id[r] * R + col) =
                make_float4((float)sum.x, (float)sum.y, (float)sum.z, (float)sum.w);
    } else {
        if (a.phase == 1) return;
        const uint64_t e0 = (uint64_t)(blk - nbb) * kEmptyPerBlock;
        const uint64_t e1 = min(e0 + kEmptyPerBlock, a.nempty);
        const uint64_t n = (e1 - e0) * (uint64_t)R;
        for (uint64_t t = tid; t < n; t += kWG) {
            const uint64_t e = e0 + t / R;
            a.out[(uint64_t)a.empty_rows[e] * R + (t % R)] = 0.0f;
        }
    }
}

__global__ __launch_bounds__(kWG) void mttkrp_fixup_kernel(FixArgs a) { fixup_body(a, blockIdx.x); }

// The fix-ups of many tensors' copies of one mode in one launch.
__global__ __launch_bounds__(kWG) void mttkrp_batch_fixup_kernel(const FixArgs* __restrict__ descs,
                                                                 const uint2* __restrict__ work, uint32_t nwork)
{
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint2 wk = work[w];
        const FixArgs a = descs[wk.x];
        fixup_body(a, wk.y);
        __syncthreads();
    }
}

}  // namespace

Geometry plan_geometry(uint64_t nnz, int n_in, int R, int dtype, int target_parts, uint32_t max_parts, uint32_t max_gsz,
                       int threads)
{
    Geometry g;
    g.lanes = lanes_per_row(R, dtype);
    g.groups = (threads > 0 ? threads : part_wg(n_in)) / g.lanes;
    if (target_parts < 1) target_parts = 1;
    max_gsz = max_gsz < 32 ? 32 : max_gsz / 32 * 32;
    uint64_t per_group = (nnz + (uint64_t)target_parts * g.groups - 1) / ((uint64_t)target_parts * g.groups);
    uint64_t gsz = (per_group + 31) / 32 * 32;
    if (gsz < 32) gsz = 32;
    if (gsz > max_gsz) gsz = max_gsz;   // bound every lane group's FP32 accumulation chain
    uint64_t wgc = gsz * g.groups;
    uint64_t parts = (nnz + wgc - 1) / wgc;
    if (parts > max_parts) {
        const uint64_t pg = (nnz + (uint64_t)max_parts * g.groups - 1) / ((uint64_t)max_parts * g.groups);
        gsz = (pg + 31) / 32 * 32;
        wgc = gsz * g.groups;
        parts = (nnz + wgc - 1) / wgc;
    }
    g.gsz = (uint32_t)gsz;
    g.wgc = wgc;
    g.nparts = (uint32_t)parts;
    return g;
}

uint32_t partition_lds_bytes(int n_in, int R, int dtype, uint32_t nhot) { return part_lds_bytes(n_in, R, dtype, nhot); }

uint32_t step_entries(int R, int dtype) { return 64u / (uint32_t)lanes_per_row(R, dtype); }

uint32_t step_kernel_lds_bytes(int n_in, int R, int es, uint32_t nhot) { return step_lds_bytes(n_in, R, es, nhot); }

Geometry plan_step_geometry(uint64_t nsteps, int R, int dtype, uint32_t P, int target_parts, uint32_t max_parts,
                            uint32_t max_chain, uint32_t cu_count)
{
    Geometry g;
    g.lanes = lanes_per_row(R, dtype);
    g.groups = kStepWaves;
    const uint32_t passes = P / step_entries(R, dtype);   // entries one lane group adds per step
    if (target_parts < 1) target_parts = 1;
    uint64_t max_w = max_chain / (passes ? passes : 1);
    max_w = max_w < 32 ? 32 : max_w / 32 * 32;
    uint64_t per = (nsteps + (uint64_t)target_parts * kStepWaves - 1) / ((uint64_t)target_parts * kStepWaves);
    uint64_t w = (per + 31) / 32 * 32;
    if (w < 32) w = 32;
    if (w > max_w) w = max_w;
    uint64_t parts = (nsteps + w * kStepWaves - 1) / (w * kStepWaves);
    if (parts > max_parts) {
        const uint64_t pw = (nsteps + (uint64_t)max_parts * kStepWaves - 1) / ((uint64_t)max_parts * kStepWaves);
        w = (pw + 31) / 32 * 32;
        parts = (nsteps + w * kStepWaves - 1) / (w * kStepWaves);
    }
    g.gsz = (uint32_t)w;
    g.wgc = w * kStepWaves;
    g.nparts = (uint32_t)parts;
    g.grid = g.nparts < cu_count ? g.nparts : (cu_count ? cu_count : 1u);
    return g;
}

int partition_wg_threads(int n_in) { return part_wg(n_in); }

void default_part_shape(int n_in, int R, int dtype, int* threads, int* gathers)
{
    *threads = part_wg(n_in);
    *gathers = part::gathers_in_flight(n_in, R, dtype);
}

bool tuned_shape_supported(int threads, int gathers)
{
    return (threads == 256 || threads == 512 || threads == 1024) && (gathers == 2 || gathers == 4);
}

static hipError_t launch_part_tuned(const DevMode& m, int R, const void* const* fac, float* out, float* carry,
                                    const Geometry& g, uint32_t atomic_cut, hipStream_t s)
{
    switch (g.threads) {
        case 256: return launch_part_tuned_wg<256>(m, R, g.gathers, fac, out, carry, g, atomic_cut, s);
        case 512: return launch_part_tuned_wg<512>(m, R, g.gathers, fac, out, carry, g, atomic_cut, s);
        case 1024: return launch_part_tuned_wg<1024>(m, R, g.gathers, fac, out, carry, g, atomic_cut, s);
        default: return hipErrorInvalidValue;
    }
}

int step_wg_threads() { return kStepWG; }

// out[0..n) = 0 (a kernel, not a memset, so that it can sit in a captured graph).
__global__ __launch_bounds__(kWG) void zero_fill_kernel(float* __restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kWG) p[i] = 0.0f;
}

hipError_t launch_mttkrp(const DevMode& m, int R, int dtype, const void* const* fac,
                         const uint32_t* const* hot_rows, uint32_t nhot, float* out, float* carry,
                         const Geometry& g, hipStream_t s, bool atomic_cut, uint32_t out_rows)
{
    hipError_t e = hipSuccess;
    if (atomic_cut) {
        // The paper's scheme 2: zero the output, add rows cut by partition
        // boundaries with global atomics, no fix-up.
        const uint64_t n = (uint64_t)out_rows * R;
        uint64_t blocks = (n + kWG - 1) / kWG;
        if (blocks > 4096) blocks = 4096;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(zero_fill_kernel, dim3((uint32_t)blocks), dim3(kWG), 0, s, out, n);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint32_t ac = atomic_cut ? 1u : 0u;
    if (m.nnz > 0 && m.step_P) {
        // Hot-steps copy: one resident workgroup per compute unit walks the partitions.
        const uint32_t grid = g.grid ? g.grid : 1u;
        switch (m.n_in) {
            case 2: e = launch_step_nin<2>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, grid, s); break;
            case 3: e = launch_step_nin<3>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, grid, s); break;
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    } else if (m.nnz > 0 && g.threads) {
        // A tuned launch shape (3-mode tensors, fp32 factors, no hot rows).
        if (dtype != MTTKRP_FP32 || nhot) return hipErrorInvalidValue;
        e = launch_part_tuned(m, R, fac, out, carry, g, ac, s);
        if (e != hipSuccess) return e;
    } else if (m.nnz > 0) {
        switch (m.n_in) {
            case 2: e = launch_part_nin<2>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            case 3: e = launch_part_nin<3>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            case 4: e = launch_part_nin<4>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            case 5: e = launch_part_nin<5>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            case 6: e = launch_part_nin<6>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            case 7: e = launch_part_nin<7>(m, R, dtype, fac, hot_rows, nhot, out, carry, g, ac, s); break;
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    if (atomic_cut) return hipSuccess;
    FixArgs f;
    f.winfo = m.winfo;
    f.row_id = m.row_id;
    f.empty_rows = m.empty_rows;
    f.carry = carry;
    f.out = out;
    f.wgc = g.wgc;
    f.nparts = m.nnz > 0 ? g.nparts : 0;
    f.nbound = f.nparts > 1 && !m.prange ? f.nparts - 1 : 0;   // scheme-1 partitions cut no rows
    f.nempty = m.nempty;
    f.R = R;
    f.phase = 0;
    const uint64_t eblocks = (m.nempty + kEmptyPerBlock - 1) / kEmptyPerBlock;
    const uint32_t nbb = fixup_bound_blocks(f.nbound);
    if (f.nbound > kChunk) {
        // A row may span more than kChunk partitions: chunk sums first.
        f.phase = 1;
        hipLaunchKernelGGL(mttkrp_fixup_kernel, dim3(nbb), dim3(kWG), 0, s, f);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        f.phase = 2;
    }
    const uint64_t blocks = nbb + eblocks;
    if (blocks > 0) {
        hipLaunchKernelGGL(mttkrp_fixup_kernel, dim3((uint32_t)blocks), dim3(kWG), 0, s, f);
        e = hipGetLastError();
    }
    return e;
}

size_t fix_desc_bytes() { return sizeof(FixArgs); }

uint32_t fill_fix_desc(void* dst, const DevMode& m, const Geometry& g, float* carry, float* out, int R)
{
    FixArgs& f = *static_cast<FixArgs*>(dst);
    f.winfo = m.winfo;
    f.row_id = m.row_id;
    f.empty_rows = m.empty_rows;
    f.carry = carry;
    f.out = out;
    f.wgc = g.wgc;
    f.nparts = m.nnz > 0 ? g.nparts : 0;
    f.nbound = f.nparts > 1 ? f.nparts - 1 : 0;
    f.nempty = m.nempty;
    f.R = R;
    f.phase = 0;   // batches add each cut row in one pass
    return fixup_bound_blocks(f.nbound) + (uint32_t)((m.nempty + kEmptyPerBlock - 1) / kEmptyPerBlock);
}

hipError_t launch_batch_fixup(const void* descs, const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s)
{
    if (nwork == 0) return hipSuccess;
    hipLaunchKernelGGL(mttkrp_batch_fixup_kernel, dim3(grid), dim3(kWG), 0, s, static_cast<const FixArgs*>(descs), work,
                       nwork);
    return hipGetLastError();
}

hipError_t launch_batch_part(int n_in, int R, int dtype, int threads, int gathers, const void* descs,
                             const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s)
{
    if (nwork == 0) return hipSuccess;
    if (threads) {
        if (n_in != 2 || dtype != MTTKRP_FP32) return hipErrorInvalidValue;
        switch (threads) {
            case 256: return launch_batch_part_tuned_wg<256>(R, gathers, descs, work, nwork, grid, s);
            case 512: return launch_batch_part_tuned_wg<512>(R, gathers, descs, work, nwork, grid, s);
            case 1024: return launch_batch_part_tuned_wg<1024>(R, gathers, descs, work, nwork, grid, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (n_in) {
        case 2: return launch_batch_part_nin<2>(R, dtype, descs, work, nwork, grid, s);
        case 3: return launch_batch_part_nin<3>(R, dtype, descs, work, nwork, grid, s);
        case 4: return launch_batch_part_nin<4>(R, dtype, descs, work, nwork, grid, s);
        case 5: return launch_batch_part_nin<5>(R, dtype, descs, work, nwork, grid, s);
        case 6: return launch_batch_part_nin<6>(R, dtype, descs, work, nwork, grid, s);
        case 7: return launch_batch_part_nin<7>(R, dtype, descs, work, nwork, grid, s);
        default: return hipErrorInvalidValue;
    }
}

size_t part_desc_bytes(int n_in)
{
    switch (n_in) {
        case 2: return part_desc_bytes_nin<2>();
        case 3: return part_desc_bytes_nin<3>();
        case 4: return part_desc_bytes_nin<4>();
        case 5: return part_desc_bytes_nin<5>();
        case 6: return part_desc_bytes_nin<6>();
        case 7: return part_desc_bytes_nin<7>();
        default: return 0;
    }
}

void fill_part_desc(void* dst, const DevMode& m, int R, int dtype, const void* const* fac, float* out, float* carry,
                    uint32_t gsz)
{
    switch (m.n_in) {
        case 2: fill_part_desc_nin<2>(dst, m, R, dtype, fac, out, carry, gsz); break;
        case 3: fill_part_desc_nin<3>(dst, m, R, dtype, fac, out, carry, gsz); break;
        case 4: fill_part_desc_nin<4>(dst, m, R, dtype, fac, out, carry, gsz); break;
        case 5: fill_part_desc_nin<5>(dst, m, R, dtype, fac, out, carry, gsz); break;
        case 6: fill_part_desc_nin<6>(dst, m, R, dtype, fac, out, carry, gsz); break;
        case 7: fill_part_desc_nin<7>(dst, m, R, dtype, fac, out, carry, gsz); break;
        default: break;
    }
}

}  // namespace mk
