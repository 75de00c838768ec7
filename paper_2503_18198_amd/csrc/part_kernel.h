// Partition kernel of the per-mode MTTKRP; the design is described at the top
// of mttkrp_kernels.hip.  Included by one translation unit per mode count
// (part_n3.hip .. part_n8.hip) so the instantiations build in parallel.
#pragma once

#include <type_traits>

#include "internal.h"

namespace mk {
namespace part {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}

// Value of lane SRC of each aligned group of L lanes, for every lane of the
// group (ds_swizzle in bit mode: and-mask keeps the group, or-mask picks SRC).
template <int L, int SRC>
__device__ __forceinline__ uint32_t group_bcast(uint32_t x)
{
    static_assert(L >= 1 && L <= 32 && (L & (L - 1)) == 0 && SRC >= 0 && SRC < L, "bad group broadcast");
    if constexpr (L == 1) {
        return x;
    } else {
        constexpr int pattern = (0x1F & ~(L - 1)) | (SRC << 5);
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, pattern);
    }
}

// V consecutive 32-bit words of the streamed mode copy (read once: non-temporal).
template <int V>
__device__ __forceinline__ void load_words(const uint32_t* p, uint32_t (&w)[V])
{
    if constexpr (V >= 4) {
        static_for<0, V / 4>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p) + j);
            w[4 * j + 0] = v.x;
            w[4 * j + 1] = v.y;
            w[4 * j + 2] = v.z;
            w[4 * j + 3] = v.w;
        });
    } else if constexpr (V == 2) {
        const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
        w[0] = v.x;
        w[1] = v.y;
    } else {
        w[0] = __builtin_nontemporal_load(p);
    }
}

// Elements per 16-byte slice.
template <int DT>
constexpr int vec_of() { return DT == MTTKRP_FP32 ? 4 : 8; }

// The 16-byte slice `gl` of row `row` of an I x R factor.
template <int R, int DT>
__device__ __forceinline__ u32x4 load_slice(const void* fac, uint32_t row, int gl)
{
    if constexpr (DT == MTTKRP_FP32) {
        const float* p = static_cast<const float*>(fac) + (uint64_t)row * R + gl * 4;
        return *reinterpret_cast<const u32x4*>(p);
    } else {
        const uint16_t* p = static_cast<const uint16_t*>(fac) + (uint64_t)row * R + gl * 8;
        return *reinterpret_cast<const u32x4*>(p);
    }
}

// Unpack a slice into VEC floats (bf16 -> fp32 is exact: the bf16 bits are the
// high half of the fp32 pattern).
template <int DT>
__device__ __forceinline__ void unpack(const u32x4 v, float* f)
{
    if constexpr (DT == MTTKRP_FP32) {
        f[0] = __uint_as_float(v.x);
        f[1] = __uint_as_float(v.y);
        f[2] = __uint_as_float(v.z);
        f[3] = __uint_as_float(v.w);
    } else {
        f[0] = __uint_as_float(v.x << 16);
        f[1] = __uint_as_float(v.x & 0xffff0000u);
        f[2] = __uint_as_float(v.y << 16);
        f[3] = __uint_as_float(v.y & 0xffff0000u);
        f[4] = __uint_as_float(v.z << 16);
        f[5] = __uint_as_float(v.z & 0xffff0000u);
        f[6] = __uint_as_float(v.w << 16);
        f[7] = __uint_as_float(v.w & 0xffff0000u);
    }
}

template <int VEC>
__device__ __forceinline__ void store_vec(float* dst, const float* v)
{
    static_for<0, VEC / 4>([&](auto J) {
        constexpr int j = decltype(J)::value;
        f32x4 t = {v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        *reinterpret_cast<f32x4*>(dst + 4 * j) = t;
    });
}

template <int NIN>
struct PartArgs {
    const uint32_t* idx[NIN];
    const void* fac[NIN];
    const float* val;
    const uint2* winfo;
    const uint32_t* row_id;
    float* out;
    float* carry;
    uint64_t nnz;
    uint32_t nrows_nz;
    uint32_t gsz;
};

// One workgroup = one partition of G * gsz consecutive nonzeros.
template <int NIN, int R, int DT>
__global__ __launch_bounds__(kWG) void mttkrp_part_kernel(PartArgs<NIN> a)
{
    constexpr int VEC = vec_of<DT>();
    constexpr int L = R / VEC;          // lanes per group
    constexpr int G = kWG / L;          // groups per workgroup
    constexpr int V = 32 / L;           // streamed words per lane per 32 nonzeros
    constexpr int U = NIN <= 2 ? 8 : (NIN <= 4 ? 4 : 2);  // nonzeros with gathers in flight
    static_assert(R % VEC == 0 && L >= 2 && L <= 16 && 32 % U == 0, "unsupported shape");

    __shared__ float s_head[G * R];     // partial sum of each group's first row
    __shared__ float s_tail[G * R];     // partial sum of each group's last row (if different)
    __shared__ int s_trow[G];           // ordinal of the last row, -1 if the group has one row
    __shared__ int s_hstart[G];         // 1: group's first nonzero starts a row; 0: continues one; -1: empty

    const int tid = threadIdx.x;
    const int g = tid / L;
    const int gl = tid % L;
    const int wave_grp0 = (tid & 63) & ~(L - 1);   // wave lane of this group's lane 0
    const uint64_t wg_beg = (uint64_t)blockIdx.x * G * a.gsz;
    const uint64_t g_beg = wg_beg + (uint64_t)g * a.gsz;

    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.0f;
    int first_row = -1;
    int cur = -1;
    int hstart = -1;

    if (g_beg < a.nnz) {
        const uint64_t g_end = min(g_beg + (uint64_t)a.gsz, a.nnz);
        const uint2 w0 = a.winfo[g_beg >> 5];
        first_row = cur = (int)w0.y;
        hstart = (int)(w0.x & 1u);
        for (uint64_t b = g_beg; b < g_end; b += 32) {
            const uint2 w = a.winfo[b >> 5];
            const int nvalid = (int)min((uint64_t)32, g_end - b);
            uint32_t flags = w.x;
            if (b == g_beg) flags &= ~1u;
            if (nvalid < 32) flags &= (1u << nvalid) - 1u;

            uint32_t sidx[NIN][V];
            uint32_t sval[V];
            static_for<0, NIN>([&](auto M) {
                constexpr int m = decltype(M)::value;
                load_words<V>(a.idx[m] + b + gl * V, sidx[m]);
            });
            load_words<V>(reinterpret_cast<const uint32_t*>(a.val) + b + gl * V, sval);
            // Output rows of the next L row ordinals, for the stores of this batch.
            const int rbase = cur;
            const uint32_t rid_pf = a.row_id[min((uint32_t)(rbase + gl), a.nrows_nz - 1u)];

            static_for<0, 32 / U>([&](auto SB) {
                constexpr int sb = decltype(SB)::value * U;
                if (sb < nvalid) {
                    u32x4 gv[U][NIN];
                    float vv[U];
                    static_for<0, U>([&](auto UU) {
                        constexpr int u = decltype(UU)::value;
                        constexpr int k = sb + u;
                        constexpr int src = k / V;
                        constexpr int reg = k % V;
                        vv[u] = __uint_as_float(group_bcast<L, src>(sval[reg]));
                        static_for<0, NIN>([&](auto M) {
                            constexpr int m = decltype(M)::value;
                            const uint32_t row = group_bcast<L, src>(sidx[m][reg]);
                            if (k < nvalid) gv[u][m] = load_slice<R, DT>(a.fac[m], row, gl);
                            else gv[u][m] = u32x4{0u, 0u, 0u, 0u};
                        });
                    });
                    static_for<0, U>([&](auto UU) {
                        constexpr int u = decltype(UU)::value;
                        constexpr int k = sb + u;
                        if (k < nvalid) {
                            float p[VEC];
                            unpack<DT>(gv[u][0], p);
#pragma unroll
                            for (int e = 0; e < VEC; ++e) p[e] *= vv[u];
                            static_for<1, NIN>([&](auto M) {
                                constexpr int m = decltype(M)::value;
                                float q[VEC];
                                unpack<DT>(gv[u][m], q);
#pragma unroll
                                for (int e = 0; e < VEC; ++e) p[e] *= q[e];
                            });
                            if ((flags >> k) & 1u) {
                                // Row `cur` ends before nonzero k.
                                if (cur == first_row) {
#pragma unroll
                                    for (int e = 0; e < VEC; ++e) s_head[g * R + gl * VEC + e] = acc[e];
                                } else {
                                    const int o = cur - rbase;
                                    uint32_t rid;
                                    if (o < L)
                                        rid = (uint32_t)__builtin_amdgcn_ds_bpermute((wave_grp0 + o) << 2,
                                                                                    (int)rid_pf);
                                    else
                                        rid = a.row_id[cur];
                                    store_vec<VEC>(a.out + (uint64_t)rid * R + gl * VEC, acc);
                                }
                                ++cur;
#pragma unroll
                                for (int e = 0; e < VEC; ++e) acc[e] = p[e];
                            } else {
#pragma unroll
                                for (int e = 0; e < VEC; ++e) acc[e] += p[e];
                            }
                        }
                    });
                }
            });
        }
        if (cur == first_row) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) s_head[g * R + gl * VEC + e] = acc[e];
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) s_tail[g * R + gl * VEC + e] = acc[e];
        }
    }
    if (gl == 0) {
        s_trow[g] = (first_row >= 0 && cur != first_row) ? cur : -1;
        s_hstart[g] = hstart;
    }
    __syncthreads();

    // ---- combine the groups' first/last rows in group order ----
    const uint64_t next_beg = wg_beg + (uint64_t)G * a.gsz;
    const bool row_continues = next_beg < a.nnz && !(a.winfo[next_beg >> 5].x & 1u);
    const int hs = s_hstart[g];
    if (hs < 0) return;
    const int trow = s_trow[g];

    // A run starts at this group's first row (if g == 0 or a row starts with the
    // group) and/or at its last row; its owner adds the following groups' first
    // rows while they continue it.
    auto emit = [&](const float* src, int row, bool from_first_of_wg, bool extend) {
        float sum[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) sum[e] = src[g * R + gl * VEC + e];
        bool reaches_end = extend;
        if (extend) {
            for (int j = g + 1; j < G; ++j) {
                if (s_hstart[j] != 0) {
                    reaches_end = false;
                    break;
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e) sum[e] += s_head[j * R + gl * VEC + e];
                if (s_trow[j] >= 0) {
                    reaches_end = false;
                    break;
                }
            }
        }
        const bool head_split = from_first_of_wg && s_hstart[0] == 0;
        const bool tail_split = reaches_end && row_continues;
        if (head_split || tail_split) {
            float* dst = a.carry + ((uint64_t)blockIdx.x * 2 + (from_first_of_wg ? 0 : 1)) * R + gl * VEC;
            store_vec<VEC>(dst, sum);
        } else {
            const uint32_t rid = a.row_id[row];
            store_vec<VEC>(a.out + (uint64_t)rid * R + gl * VEC, sum);
        }
    };
    if (g == 0 || hs == 1) emit(s_head, first_row, g == 0, trow < 0);
    if (trow >= 0) emit(s_tail, trow, false, true);
}

template <int NIN, int R, int DT>
hipError_t launch_part(const DevMode& m, const void* const* fac, float* out, float* carry, const Geometry& g,
                       hipStream_t s)
{
    PartArgs<NIN> a;
    for (int j = 0; j < NIN; ++j) {
        a.idx[j] = m.idx[j];
        a.fac[j] = fac[j];
    }
    a.val = m.val;
    a.winfo = m.winfo;
    a.row_id = m.row_id;
    a.out = out;
    a.carry = carry;
    a.nnz = m.nnz;
    a.nrows_nz = (uint32_t)m.nrows_nz;
    a.gsz = g.gsz;
    hipLaunchKernelGGL((mttkrp_part_kernel<NIN, R, DT>), dim3(g.nparts), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

template <int NIN, int DT>
hipError_t dispatch_r(const DevMode& m, int R, const void* const* fac, float* out, float* carry, const Geometry& g,
                      hipStream_t s)
{
    switch (R) {
        case 16: return launch_part<NIN, 16, DT>(m, fac, out, carry, g, s);
        case 32: return launch_part<NIN, 32, DT>(m, fac, out, carry, g, s);
        case 64: return launch_part<NIN, 64, DT>(m, fac, out, carry, g, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace part

template <int NIN>
hipError_t launch_part_nin(const DevMode& m, int R, int dtype, const void* const* fac, float* out, float* carry,
                           const Geometry& g, hipStream_t s)
{
    return dtype == MTTKRP_FP32 ? part::dispatch_r<NIN, MTTKRP_FP32>(m, R, fac, out, carry, g, s)
                                : part::dispatch_r<NIN, MTTKRP_BF16>(m, R, fac, out, carry, g, s);
}

}  // namespace mk
