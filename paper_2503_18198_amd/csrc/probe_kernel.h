// Gather-ceiling probe kernels, instantiated per mode count in probe_n*.hip:
// the memory traffic of one mode's MTTKRP without its arithmetic.  Same
// partitions, lane groups (16 bytes of a factor row per lane, 8 for bf16 rows
// of R = 16), batch stream loads and row gathers as the partition kernel; the
// products, row sums, stores and fix-up are replaced by an XOR fold of the
// loaded bits.  Timing it beside the MTTKRP gives the on-chip ceiling of a
// tensor's own index pattern (what = 1) and of the stream alone (what = 0).
// Two variants split the gather cost (3- and 4-mode tensors): what = 2 issues
// the same gather instructions with only the first lane of each lane group
// reading (the others take the out-of-range offset, which reads zero), so it
// moves 1/L of the bytes; what = 3 gathers row (index & 63) instead of row
// index, which stays in L1 (index & 63 <= index, so every row read exists).
#pragma once

#include "part_kernel.h"

namespace mk {
namespace part {

template <int NIN, int R, int DT, int WHAT, bool IDX16>
__global__ __launch_bounds__(part_wg(NIN)) void gather_probe_kernel(PartArgs<NIN> a)
{
    constexpr int kWGT = part_wg(NIN);
    constexpr int E = vals_per_lane(R, DT);
    constexpr int L = R / E;
    constexpr int V = 32 / L;
    constexpr int G = kWGT / L;
    constexpr int U = gathers_in_flight(NIN, R, DT);
    using ST = typename Slice<R, DT>::T;

    const int tid = threadIdx.x;
    const int g = tid / L;
    const int gl = tid % L;
    const uint64_t g_beg = ((uint64_t)blockIdx.x * G + g) * a.gsz;
    uint32_t x = 0;
    if (g_beg < a.nnz) {
        const uint64_t g_end = min(g_beg + (uint64_t)a.gsz, a.nnz);
        __amdgpu_buffer_rsrc_t rsrc[NIN];
#pragma unroll
        for (int m = 0; m < NIN; ++m) rsrc[m] = make_rsrc(a.fac[m], a.fac_bytes[m]);
        for (uint64_t b = g_beg; b < g_end; b += 32) {
            Batch<NIN, V> bt;
            load_batch<NIN, V, IDX16>(a, b, gl, bt);
            const int nvalid = (int)min((uint64_t)32, g_end - b);
            x ^= bt.w.x ^ bt.w.y;
            if constexpr (WHAT == 0) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    x ^= bt.val[j];
#pragma unroll
                    for (int m = 0; m < NIN; ++m) x ^= bt.idx[m][j];
                }
            } else {
                static_for<0, 32 / U>([&](auto SB) {
                    constexpr int sb = decltype(SB)::value * U;
                    ST r[U][NIN];
                    static_for<0, U>([&](auto UU) {
                        constexpr int u = decltype(UU)::value;
                        constexpr int k = sb + u;
                        const bool valid = k < nvalid;
                        x ^= group_bcast<L, k / V>(bt.val[k % V]);
                        static_for<0, NIN>([&](auto M) {
                            constexpr int m = decltype(M)::value;
                            uint32_t v = group_bcast<L, k / V>(bt.idx[m][k % V]);
                            if constexpr (WHAT == 3) v &= 63u;
                            const bool use = valid && (WHAT != 2 || gl == 0);
                            const uint32_t off =
                                use ? (v * (uint32_t)R + (uint32_t)(gl * E)) * Slice<R, DT>::kElem : kSkipOffset;
                            r[u][m] = load_buffer<R, DT>(rsrc[m], off);
                        });
                    });
                    static_for<0, U>([&](auto UU) {
                        constexpr int u = decltype(UU)::value;
                        static_for<0, NIN>([&](auto M) {
                            constexpr int m = decltype(M)::value;
                            if constexpr (Slice<R, DT>::kBytes == 16) x ^= r[u][m].x ^ r[u][m].y ^ r[u][m].z ^ r[u][m].w;
                            else x ^= r[u][m].x ^ r[u][m].y;
                        });
                    });
                });
            }
        }
    }
    // Practically never taken; keeps every load live.  The carry workspace is
    // scratch that the next MTTKRP rewrites.
    if (x == 0x9E3779B9u) a.carry[blockIdx.x] = 1.0f;
}

template <int NIN, int R, int DT>
hipError_t launch_probe_r(const PartArgs<NIN>& a, uint32_t grid, int what, hipStream_t s)
{
    auto go = [&](auto what_c, auto idx16_c) {
        hipLaunchKernelGGL((gather_probe_kernel<NIN, R, DT, decltype(what_c)::value, decltype(idx16_c)::value>),
                           dim3(grid), dim3(part_wg(NIN)), 0, s, a);
        return hipGetLastError();
    };
    auto by_what = [&](auto idx16_c) {
        switch (what) {
            case 0: return go(std::integral_constant<int, 0>{}, idx16_c);
            case 1: return go(std::integral_constant<int, 1>{}, idx16_c);
            case 2:
            case 3:
                // The split variants are compiled for 3- and 4-mode tensors only.
                if constexpr (NIN <= 3) {
                    if (what == 2) return go(std::integral_constant<int, 2>{}, idx16_c);
                    return go(std::integral_constant<int, 3>{}, idx16_c);
                } else {
                    return hipErrorInvalidValue;
                }
            default: return hipErrorInvalidValue;
        }
    };
    if constexpr (NIN <= kMaxIn16) {
        if (a.idx16) return by_what(std::true_type{});
    }
    return by_what(std::false_type{});
}

template <int NIN>
hipError_t launch_probe_nin(const DevMode& m, int R, int dtype, const void* const* fac, float* carry,
                            const Geometry& g, int what, hipStream_t s)
{
    PartArgs<NIN> a;
    fill_part_args<NIN>(a, m, R, dtype, fac, nullptr, 0, nullptr, carry, g.gsz);
    if (dtype == MTTKRP_FP32) {
        switch (R) {
            case 16: return launch_probe_r<NIN, 16, MTTKRP_FP32>(a, g.nparts, what, s);
            case 32: return launch_probe_r<NIN, 32, MTTKRP_FP32>(a, g.nparts, what, s);
            case 64: return launch_probe_r<NIN, 64, MTTKRP_FP32>(a, g.nparts, what, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (R) {
        case 16: return launch_probe_r<NIN, 16, MTTKRP_BF16>(a, g.nparts, what, s);
        case 32: return launch_probe_r<NIN, 32, MTTKRP_BF16>(a, g.nparts, what, s);
        case 64: return launch_probe_r<NIN, 64, MTTKRP_BF16>(a, g.nparts, what, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace part
}  // namespace mk
