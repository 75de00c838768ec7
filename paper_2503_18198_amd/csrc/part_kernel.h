// Partition kernel of the per-mode MTTKRP; the overall design is described at
// the top of mttkrp_kernels.hip.  Included by one translation unit per mode
// count (part_n3.hip .. part_n8.hip) so the instantiations build in parallel.
//
// Per workgroup (part_wg threads, one partition of G * gsz nonzeros):
//  1. When the layout has hot rows (the most frequently gathered rows of each
//     input factor, coordinates stored as kHotBit | slot), they are copied
//     into LDS.
//  2. Each lane group of L lanes (16 bytes of a factor row per lane: 4 fp32 or
//     8 bf16 values; bf16 rows of R = 16 use 8 bytes) walks gsz consecutive
//     nonzeros, 32 at a time: indices and values are streamed with full-line
//     non-temporal loads and shared in the group with ds_swizzle; U nonzeros'
//     row gathers are issued before any is used; hot rows come from LDS, the
//     rest from global memory.  The running row sum stays in registers and a
//     row that ends inside the run is stored once.
//  3. The first and last row partials of every group go to LDS (reusing the
//     hot-row area) and are added in group order; rows cut by the
//     workgroup's ends go to the carry buffer for the fix-up kernel.
#pragma once

#include <type_traits>

#include "internal.h"

namespace mk {

constexpr uint32_t kHotBitDev = 0x80000000u;

// Threads per partition workgroup: 512 for 3-mode tensors (lane state fits in
// 128 registers, so four workgroups of 8 waves fill a CU); with 4 or more
// modes the per-nonzero state is larger, so 256-thread workgroups.  Measured
// on the 20M-nonzero Zipf(1.2) R=32 tensor: 512 threads with 8 partitions per
// CU beat 1024 threads with 2 by 9%.
#ifndef MK_WG_3MODE
#define MK_WG_3MODE 512
#endif
#ifndef MK_U_3MODE
#define MK_U_3MODE 4
#endif
constexpr int part_wg(int n_in) { return n_in <= 2 ? MK_WG_3MODE : 256; }

// Factor values each lane gathers and accumulates: 16 bytes of a row, i.e. 4
// fp32 or 8 bf16 values (bf16 rows of R = 16 keep 4 per lane, so a row still
// spans more than one lane), and the lanes that share one row.
constexpr int vals_per_lane(int R, int dtype) { return (dtype == MTTKRP_BF16 && R >= 32) ? 8 : 4; }
constexpr int lanes_per_row(int R, int dtype) { return R / vals_per_lane(R, dtype); }

// Dynamic LDS bytes of a partition workgroup.
inline uint32_t part_lds_bytes(int n_in, int R, int dtype, uint32_t nhot, int threads = 0)
{
    const uint32_t groups = (threads ? threads : part_wg(n_in)) / lanes_per_row(R, dtype);
    const uint32_t es = dtype == MTTKRP_FP32 ? 4 : 2;
    const uint32_t hot = (uint32_t)n_in * nhot * (uint32_t)R * es;
    const uint32_t slots = 2u * groups * (uint32_t)R * 4u;
    return (hot > slots ? hot : slots) + 2u * groups * 4u;
}

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
// group (ds_swizzle in bit mode: the and-mask keeps the group, the or-mask
// selects SRC).
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

// One lane's consecutive factor values of a row: kVals values of kElem bytes.
template <int R, int DT>
struct Slice {
    static constexpr int kVals = vals_per_lane(R, DT);
    static constexpr int kElem = DT == MTTKRP_FP32 ? 4 : 2;
    static constexpr int kBytes = kVals * kElem;
    using T = typename std::conditional<kBytes == 16, u32x4, u32x2>::type;
};

// Buffer-resource loads: 32-bit offsets, and an offset past the end returns
// zero without touching memory, which turns a skipped gather into a no-op
// lane instead of a branch.
constexpr uint32_t kRsrcWord3 = 0x00020000u;   // raw buffer, gfx9-family format bits
constexpr uint32_t kSkipOffset = 0xFFFFFFF0u;  // beyond every factor (factors are < 4 GiB - 16)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, (int)kRsrcWord3);
}

template <int R, int DT>
__device__ __forceinline__ typename Slice<R, DT>::T load_buffer(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (Slice<R, DT>::kBytes == 16) return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    else return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}

typedef __attribute__((address_space(3))) const char lds_char;

template <int R, int DT>
__device__ __forceinline__ typename Slice<R, DT>::T load_lds(lds_char* base, uint32_t slot, int gl)
{
    lds_char* p = base + (slot * R + gl * Slice<R, DT>::kVals) * Slice<R, DT>::kElem;
    return *reinterpret_cast<__attribute__((address_space(3))) const typename Slice<R, DT>::T*>(p);
}

// bf16 -> fp32 is exact: the bf16 bits are the high half of the fp32 pattern.
template <int R, int DT>
__device__ __forceinline__ void unpack(const typename Slice<R, DT>::T v, float (&f)[Slice<R, DT>::kVals])
{
    if constexpr (DT == MTTKRP_FP32) {
        f[0] = __uint_as_float(v.x);
        f[1] = __uint_as_float(v.y);
        f[2] = __uint_as_float(v.z);
        f[3] = __uint_as_float(v.w);
    } else {
        constexpr int W = Slice<R, DT>::kVals / 2;   // 32-bit words, two bf16 each
#pragma unroll
        for (int i = 0; i < W; ++i) {
            f[2 * i] = __uint_as_float(v[i] << 16);
            f[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
        }
    }
}

// E consecutive fp32 values (E = 4 or 8) with 16-byte stores.
template <int E>
__device__ __forceinline__ void store_vals(float* dst, const float (&v)[E])
{
#pragma unroll
    for (int j = 0; j < E / 4; ++j) {
        const f32x4 t = {v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        *reinterpret_cast<f32x4*>(dst + 4 * j) = t;
    }
}

template <int NIN>
struct PartArgs {
    const uint32_t* idx[NIN];
    const void* fac[NIN];
    const uint32_t* hot_rows[NIN];
    uint32_t fac_bytes[NIN];   // bytes of each input factor (< 4 GiB - 16)
    const float* val;
    const uint2* winfo;
    const uint32_t* row_id;
    float* out;
    float* carry;
    uint64_t nnz;
    uint32_t nrows_nz;
    uint32_t gsz;
    uint32_t nhot;       // hot slots per input mode held in LDS
    uint32_t atomic_cut; // rows cut by a partition boundary: 0 partial to carry, 1 global atomic add to out
    const uint64_t* prange; // scheme 1: {first position, nonzeros} per partition (whole rows); null: part * G * gsz
    uint32_t idx16;         // 1: the input coordinates are uint16 (every input dimension <= 65536)
};

// Nonzeros whose row gathers are issued before the first is used, chosen so
// that a 1024-thread workgroup (128 registers per lane) does not spill.
#ifndef MK_U_BF16_WIDE
#define MK_U_BF16_WIDE 4
#endif
constexpr int gathers_in_flight(int n_in, int R, int dtype)
{
    if (vals_per_lane(R, dtype) == 8) return MK_U_BF16_WIDE;
    if (n_in <= 2) return (dtype == MTTKRP_FP32 && R == 16) ? 2 : MK_U_3MODE;
    if (n_in <= 3) return (dtype == MTTKRP_FP32 && R == 16) ? 2 : 4;
    return 2;
}

// State of one lane group while it walks its run of nonzeros (E values per lane).
template <int E>
struct GroupState {
    float acc[E];
    float head[E];
    int first_row;
    int cur;
};

// The streamed part of one batch of 32 nonzeros: each lane of a group holds
// V consecutive words of every input-coordinate array and of the values.
template <int NIN, int V>
struct Batch {
    uint32_t idx[NIN][V];
    uint32_t val[V];
    uint2 w;   // {row-start bits, ordinal of the row holding the first nonzero}
};

template <int NIN, int V, bool IDX16 = false>
__device__ __forceinline__ void load_batch(const PartArgs<NIN>& a, uint64_t b, int gl, Batch<NIN, V>& bt)
{
    static_for<0, NIN>([&](auto M) {
        constexpr int m = decltype(M)::value;
        if constexpr (IDX16) {
            // V uint16 coordinates = V / 2 words, widened in registers
            static_assert(V % 2 == 0, "16-bit coordinates need an even count per lane");
            uint32_t w[V / 2];
            load_words<V / 2>(reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint16_t*>(a.idx[m]) + b +
                                                                gl * V),
                              w);
#pragma unroll
            for (int i = 0; i < V / 2; ++i) {
                bt.idx[m][2 * i] = w[i] & 0xFFFFu;
                bt.idx[m][2 * i + 1] = w[i] >> 16;
            }
        } else {
            load_words<V>(a.idx[m] + b + gl * V, bt.idx[m]);
        }
    });
    load_words<V>(reinterpret_cast<const uint32_t*>(a.val) + b + gl * V, bt.val);
    bt.w = a.winfo[b >> 5];
}

// Store the finished row `cur` (ordinal) of a group, or keep it as the
// group's head partial if it is the group's first row.
template <int R, int DT, int NIN>
__device__ __forceinline__ void flush_row(const PartArgs<NIN>& a, GroupState<vals_per_lane(R, DT)>& st, int rbase,
                                          uint32_t rid_pf, int gl, int wave_grp0)
{
    constexpr int E = vals_per_lane(R, DT);
    constexpr int L = R / E;
    if (st.cur == st.first_row) {
#pragma unroll
        for (int e = 0; e < E; ++e) st.head[e] = st.acc[e];
    } else {
        const int o = st.cur - rbase;
        uint32_t rid;
        if (o < L) rid = (uint32_t)__builtin_amdgcn_ds_bpermute((wave_grp0 + o) << 2, (int)rid_pf);
        else rid = a.row_id[st.cur];
        store_vals<E>(a.out + (uint64_t)rid * R + gl * E, st.acc);
    }
}

// One batch of 32 consecutive nonzeros starting at b (b is a multiple of 32).
// FULL: all 32 are valid (no per-nonzero bounds tests).  HOT: coordinates
// may name LDS hot-row slots.
template <int NIN, int R, int DT, bool HOT, bool FULL, int U>
__device__ __forceinline__ void process_batch(const PartArgs<NIN>& a, const __amdgpu_buffer_rsrc_t (&rsrc)[NIN],
                                              lds_char* hot_lds, GroupState<vals_per_lane(R, DT)>& st,
                                              const Batch<NIN, 32 / lanes_per_row(R, DT)>& bt,
                                              int nvalid, bool first_batch, int gl, int wave_grp0)
{
    constexpr int E = vals_per_lane(R, DT);
    constexpr int L = R / E;
    constexpr int V = 32 / L;
    using ST = typename Slice<R, DT>::T;

    uint32_t flags = bt.w.x;
    if (first_batch) flags &= ~1u;
    if (!FULL && nvalid < 32) flags &= (1u << nvalid) - 1u;
    // Output rows of the next L row ordinals, for the stores of this batch.
    const int rbase = st.cur;
    const uint32_t rid_pf = a.row_id[min((uint32_t)(rbase + gl), a.nrows_nz - 1u)];

    static_for<0, 32 / U>([&](auto SB) {
        constexpr int sb = decltype(SB)::value * U;
        if (FULL || sb < nvalid) {
            // (a) Coordinates and values of the sub-batch, shared in the group.
            uint32_t vidx[U][NIN];
            float vv[U];
            static_for<0, U>([&](auto UU) {
                constexpr int u = decltype(UU)::value;
                constexpr int k = sb + u;
                vv[u] = __uint_as_float(group_bcast<L, k / V>(bt.val[k % V]));
                static_for<0, NIN>([&](auto M) {
                    constexpr int m = decltype(M)::value;
                    vidx[u][m] = group_bcast<L, k / V>(bt.idx[m][k % V]);
                });
            });
            // (b) Every gather of the sub-batch is issued before any is used.
            // Buffer loads: a lane with nothing to gather (past the end, or a
            // hot row) gets an out-of-range offset and reads zero.
            ST gg[U][NIN];
            ST hh[U][NIN];
            static_for<0, U>([&](auto UU) {
                constexpr int u = decltype(UU)::value;
                constexpr int k = sb + u;
                static_for<0, NIN>([&](auto M) {
                    constexpr int m = decltype(M)::value;
                    const uint32_t v = vidx[u][m];
                    const bool valid = FULL || k < nvalid;
                    if constexpr (HOT) {
                        const bool hot = (v & kHotBitDev) != 0;
                        const uint32_t off = (valid && !hot) ? (v * (uint32_t)R + (uint32_t)(gl * E)) * Slice<R, DT>::kElem
                                                             : kSkipOffset;
                        gg[u][m] = load_buffer<R, DT>(rsrc[m], off);
                        hh[u][m] = ST{};
                        if (valid && hot)
                            hh[u][m] = load_lds<R, DT>(hot_lds + (size_t)m * a.nhot * R * Slice<R, DT>::kElem,
                                                       v & ~kHotBitDev, gl);
                    } else {
                        const uint32_t off = valid ? (v * (uint32_t)R + (uint32_t)(gl * E)) * Slice<R, DT>::kElem
                                                   : kSkipOffset;
                        gg[u][m] = load_buffer<R, DT>(rsrc[m], off);
                    }
                });
            });
            // (c) Products; the last factor is fused into the row sum.
            const uint32_t sub = (flags >> sb) & ((1u << U) - 1u);
            float p[U][E];
            float ql[U][E];
            static_for<0, U>([&](auto UU) {
                constexpr int u = decltype(UU)::value;
                static_for<0, NIN>([&](auto M) {
                    constexpr int m = decltype(M)::value;
                    ST sl = gg[u][m];
                    if constexpr (HOT) sl = sl | hh[u][m];
                    float q[E];
                    unpack<R, DT>(sl, q);
                    if constexpr (m == 0) {
#pragma unroll
                        for (int e = 0; e < E; ++e) p[u][e] = q[e] * vv[u];
                    } else if constexpr (m < NIN - 1) {
#pragma unroll
                        for (int e = 0; e < E; ++e) p[u][e] *= q[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < E; ++e) ql[u][e] = q[e];
                    }
                });
                if constexpr (NIN == 1) {
#pragma unroll
                    for (int e = 0; e < E; ++e) ql[u][e] = 1.0f;
                }
            });
            if (sub == 0) {
                // No row ends inside this sub-batch (the common case).
                static_for<0, U>([&](auto UU) {
                    constexpr int u = decltype(UU)::value;
                    if (FULL || sb + u < nvalid) {
#pragma unroll
                        for (int e = 0; e < E; ++e) st.acc[e] = fmaf(p[u][e], ql[u][e], st.acc[e]);
                    }
                });
            } else {
                static_for<0, U>([&](auto UU) {
                    constexpr int u = decltype(UU)::value;
                    if (FULL || sb + u < nvalid) {
                        if ((sub >> u) & 1u) {
                            flush_row<R, DT, NIN>(a, st, rbase, rid_pf, gl, wave_grp0);
                            ++st.cur;
#pragma unroll
                            for (int e = 0; e < E; ++e) st.acc[e] = p[u][e] * ql[u][e];
                        } else {
#pragma unroll
                            for (int e = 0; e < E; ++e) st.acc[e] = fmaf(p[u][e], ql[u][e], st.acc[e]);
                        }
                    }
                });
            }
        }
    });
}

// The work of one partition `part` (a workgroup's share) of one mode copy.
// WGT threads per workgroup and UU nonzeros' gathers in flight per lane
// group: the library defaults (part_wg, gathers_in_flight) or a tuned shape.
template <int NIN, int R, int DT, bool HOT, bool IDX16 = false, int WGT = part_wg(NIN),
          int UU = gathers_in_flight(NIN, R, DT)>
__device__ __forceinline__ void partition_body(const PartArgs<NIN>& a, uint32_t part, char* smem)
{
    constexpr int kPartWG = WGT;
    constexpr int E = vals_per_lane(R, DT);
    constexpr int L = R / E;            // lanes per group
    constexpr int V = 32 / L;
    constexpr int G = kPartWG / L;      // groups per workgroup
    static_assert(R % E == 0 && L >= 2 && L <= 16, "unsupported rank");

    const int tid = threadIdx.x;
    const int g = tid / L;
    const int gl = tid % L;
    const int wave_grp0 = (tid & 63) & ~(L - 1);

    // 1. Hot rows of every input factor into LDS: 16-byte chunks, eight per
    //    thread in flight (row numbers first, then the data, then the stores).
    const uint32_t row_bytes = R * Slice<R, DT>::kElem;
    if (HOT && a.nhot) {
        constexpr int F = 8;
        const uint32_t cpr = row_bytes / 16;
        const uint32_t chunks = a.nhot * cpr;
        static_for<0, NIN>([&](auto M) {
            constexpr int m = decltype(M)::value;
            char* dst = smem + (size_t)m * a.nhot * row_bytes;
            const char* fac = static_cast<const char*>(a.fac[m]);
            for (uint32_t c0 = tid; c0 < chunks; c0 += F * kPartWG) {
                uint32_t row[F];
                u32x4 d[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t c = c0 + f * kPartWG;
                    row[f] = c < chunks ? a.hot_rows[m][c / cpr] : 0u;
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t c = c0 + f * kPartWG;
                    if (c < chunks)
                        d[f] = *reinterpret_cast<const u32x4*>(fac + (uint64_t)row[f] * row_bytes + (c % cpr) * 16);
                }
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t c = c0 + f * kPartWG;
                    if (c < chunks)
                        *reinterpret_cast<u32x4*>(dst + (size_t)(c / cpr) * row_bytes + (c % cpr) * 16) = d[f];
                }
            }
        });
        __syncthreads();
    }

    // 2. Walk this group's run of nonzeros, streaming one batch ahead.  A
    //    nonzero-balanced partition is G runs of gsz; a scheme-1 partition
    //    (whole rows, its own length) is split into G runs of a multiple of 32.
    uint64_t wg_beg, wg_end;
    uint32_t gsz;
    if (a.prange) {
        wg_beg = a.prange[2 * part];
        wg_end = wg_beg + a.prange[2 * part + 1];
        const uint64_t per = (wg_end - wg_beg + G - 1) / G;
        gsz = (uint32_t)(per < 32 ? 32 : (per + 31) / 32 * 32);
    } else {
        wg_beg = (uint64_t)part * G * a.gsz;
        wg_end = a.nnz;
        gsz = a.gsz;
    }
    const uint64_t g_beg = wg_beg + (uint64_t)g * gsz;
    GroupState<E> st;
#pragma unroll
    for (int e = 0; e < E; ++e) st.acc[e] = st.head[e] = 0.0f;
    st.first_row = -1;
    st.cur = -1;
    int hstart = -1;
    if (g_beg < wg_end) {
        const uint64_t g_end = min(g_beg + (uint64_t)gsz, wg_end);
        lds_char* hot_lds = (lds_char*)smem;
        __amdgpu_buffer_rsrc_t rsrc[NIN];
#pragma unroll
        for (int m = 0; m < NIN; ++m) rsrc[m] = make_rsrc(a.fac[m], a.fac_bytes[m]);
        Batch<NIN, V> cur_b, next_b;
        load_batch<NIN, V, IDX16>(a, g_beg, gl, cur_b);
        st.first_row = st.cur = (int)cur_b.w.y;
        hstart = (int)(cur_b.w.x & 1u);
        uint64_t b = g_beg;
        for (; b + 32 <= g_end; b += 32) {
            if (b + 32 < g_end) load_batch<NIN, V, IDX16>(a, b + 32, gl, next_b);
            process_batch<NIN, R, DT, HOT, true, UU>(a, rsrc, hot_lds, st, cur_b, 32, b == g_beg, gl, wave_grp0);
            cur_b = next_b;
        }
        if (b < g_end)
            process_batch<NIN, R, DT, HOT, false, UU>(a, rsrc, hot_lds, st, cur_b, (int)(g_end - b), b == g_beg, gl,
                                                  wave_grp0);
    }
    __syncthreads();   // every group is done with the hot rows

    // 3. Group partials into LDS, then combine them in group order.
    float* s_head = reinterpret_cast<float*>(smem);
    float* s_tail = s_head + G * R;
    int* s_trow = reinterpret_cast<int*>(smem + (a.nhot * NIN * row_bytes > 2u * G * R * 4u
                                                     ? a.nhot * NIN * row_bytes
                                                     : 2u * G * R * 4u));
    int* s_hstart = s_trow + G;
    const bool multi = st.first_row >= 0 && st.cur != st.first_row;
    if (st.first_row >= 0) {
        store_vals<E>(s_head + g * R + gl * E, multi ? st.head : st.acc);
        if (multi) store_vals<E>(s_tail + g * R + gl * E, st.acc);
    }
    if (gl == 0) {
        s_trow[g] = multi ? st.cur : -1;
        s_hstart[g] = hstart;
    }
    __syncthreads();

    // Scheme-1 partitions hold whole rows: nothing continues past their end.
    const uint64_t next_beg = wg_beg + (uint64_t)G * gsz;
    const bool row_continues = !a.prange && next_beg < a.nnz && !(a.winfo[next_beg >> 5].x & 1u);
    const int hs = s_hstart[g];
    const int trow = s_trow[g];

    // A run starts at this group's first row (if g == 0 or a row starts with
    // the group) and/or at its last row; its owner adds the following groups'
    // first rows while they continue it.
    auto emit = [&](const float* src, int row, bool from_first_of_wg, bool extend) {
        float sum[E];
#pragma unroll
        for (int e = 0; e < E; ++e) sum[e] = src[g * R + gl * E + e];
        bool reaches_end = extend;
        if (extend) {
            for (int j = g + 1; j < G; ++j) {
                if (s_hstart[j] != 0) {
                    reaches_end = false;
                    break;
                }
#pragma unroll
                for (int e = 0; e < E; ++e) sum[e] += s_head[j * R + gl * E + e];
                if (s_trow[j] >= 0) {
                    reaches_end = false;
                    break;
                }
            }
        }
        const bool head_split = from_first_of_wg && s_hstart[0] == 0;
        const bool tail_split = reaches_end && row_continues;
        if ((head_split || tail_split) && a.atomic_cut) {
            float* dst = a.out + (uint64_t)a.row_id[row] * R + gl * E;
#pragma unroll
            for (int e = 0; e < E; ++e) atomicAdd(dst + e, sum[e]);
        } else if (head_split || tail_split)
            store_vals<E>(a.carry + ((uint64_t)part * 2 + (from_first_of_wg ? 0 : 1)) * R + gl * E, sum);
        else
            store_vals<E>(a.out + (uint64_t)a.row_id[row] * R + gl * E, sum);
    };
    if (hs >= 0) {
        if (g == 0 || hs == 1) emit(s_head, st.first_row, g == 0, trow < 0);
        if (trow >= 0) emit(s_tail, trow, false, true);
    }
}

template <int NIN, int R, int DT, bool HOT, bool IDX16 = false, int WGT = part_wg(NIN),
          int UU = gathers_in_flight(NIN, R, DT)>
__global__ __launch_bounds__(WGT) void mttkrp_part_kernel(PartArgs<NIN> a)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    partition_body<NIN, R, DT, HOT, IDX16, WGT, UU>(a, blockIdx.x, smem);
}

// Many tensors' copies of the same mode in one launch: a static list of
// (tensor, partition) work items, walked by a grid of resident workgroups.
template <int NIN, int R, int DT, int WGT = part_wg(NIN), int UU = gathers_in_flight(NIN, R, DT)>
__global__ __launch_bounds__(WGT) void mttkrp_batch_part_kernel(const PartArgs<NIN>* __restrict__ descs,
                                                                const uint2* __restrict__ work, uint32_t nwork)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint2 wk = work[w];
        const PartArgs<NIN> a = descs[wk.x];
        if constexpr (NIN <= kMaxIn16) {
            if (a.idx16) partition_body<NIN, R, DT, false, true, WGT, UU>(a, wk.y, smem);
            else partition_body<NIN, R, DT, false, false, WGT, UU>(a, wk.y, smem);
        } else {
            partition_body<NIN, R, DT, false, false, WGT, UU>(a, wk.y, smem);
        }
        __syncthreads();   // the next item reuses the LDS
    }
}

template <int NIN>
void fill_part_args(PartArgs<NIN>& a, const DevMode& m, int R, int dtype, const void* const* fac,
                    const uint32_t* const* hot_rows, uint32_t nhot, float* out, float* carry, uint32_t gsz)
{
    const uint32_t es = dtype == MTTKRP_FP32 ? 4u : 2u;
    for (int j = 0; j < NIN; ++j) {
        a.idx[j] = m.idx[j];
        a.fac[j] = fac[j];
        a.hot_rows[j] = hot_rows ? hot_rows[j] : nullptr;
        a.fac_bytes[j] = (uint32_t)((uint64_t)m.in_dims[j] * R * es);
    }
    a.val = m.val;
    a.winfo = m.winfo;
    a.row_id = m.row_id;
    a.out = out;
    a.carry = carry;
    a.nnz = m.nnz;
    a.nrows_nz = (uint32_t)m.nrows_nz;
    a.gsz = gsz;
    a.nhot = nhot;
    a.atomic_cut = 0;
    a.prange = m.prange;
    a.idx16 = m.idx16 ? 1u : 0u;
}

template <int NIN, int R, int DT, bool HOT, bool IDX16 = false, int WGT = part_wg(NIN),
          int UU = gathers_in_flight(NIN, R, DT)>
hipError_t launch_part(const DevMode& m, const void* const* fac, const uint32_t* const* hot_rows, uint32_t nhot,
                       float* out, float* carry, const Geometry& g, uint32_t atomic_cut, hipStream_t s)
{
    PartArgs<NIN> a;
    fill_part_args<NIN>(a, m, R, DT, fac, hot_rows, nhot, out, carry, g.gsz);
    a.atomic_cut = atomic_cut;
    const uint32_t lds = part_lds_bytes(NIN, R, DT, nhot, WGT);
    static uint32_t lds_set = 0;   // largest dynamic LDS size already allowed for this instantiation
    if (lds > lds_set) {
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&mttkrp_part_kernel<NIN, R, DT, HOT, IDX16, WGT, UU>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL((mttkrp_part_kernel<NIN, R, DT, HOT, IDX16, WGT, UU>), dim3(m.prange ? m.nprange : g.nparts),
                       dim3(WGT), lds, s, a);
    return hipGetLastError();
}

template <int NIN, int DT>
hipError_t dispatch_r(const DevMode& m, int R, const void* const* fac, const uint32_t* const* hot_rows, uint32_t nhot,
                      float* out, float* carry, const Geometry& g, uint32_t atomic_cut, hipStream_t s)
{
    if (nhot) {
        switch (R) {
            case 16: return launch_part<NIN, 16, DT, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
            case 32: return launch_part<NIN, 32, DT, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
            case 64: return launch_part<NIN, 64, DT, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
            default: return hipErrorInvalidValue;
        }
    }
    if constexpr (NIN <= kMaxIn16) {
        if (m.idx16) {
            switch (R) {
                case 16: return launch_part<NIN, 16, DT, false, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
                case 32: return launch_part<NIN, 32, DT, false, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
                case 64: return launch_part<NIN, 64, DT, false, true>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
                default: return hipErrorInvalidValue;
            }
        }
    }
    switch (R) {
        case 16: return launch_part<NIN, 16, DT, false>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
        case 32: return launch_part<NIN, 32, DT, false>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
        case 64: return launch_part<NIN, 64, DT, false>(m, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NIN, int R, int DT, int WGT = part_wg(NIN), int UU = gathers_in_flight(NIN, R, DT)>
hipError_t launch_batch_part(const void* descs, const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s)
{
    const uint32_t lds = part_lds_bytes(NIN, R, DT, 0, WGT);
    static uint32_t lds_set = 0;
    if (lds > lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mttkrp_batch_part_kernel<NIN, R, DT, WGT, UU>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL((mttkrp_batch_part_kernel<NIN, R, DT, WGT, UU>), dim3(grid), dim3(WGT), lds, s,
                       static_cast<const PartArgs<NIN>*>(descs), work, nwork);
    return hipGetLastError();
}

}  // namespace part

// Launch shapes the autotuner may pick for fp32 factors of 3-mode tensors
// without hot rows: workgroups of WGT = 256, 512 or 1024 threads and 2 or 4
// nonzeros' gathers in flight per lane group.  Each workgroup size is
// instantiated in a file of its own (part_tuned_<WGT>.hip); a shape equal to
// the default of its rank runs through the default kernels instead.
template <int R, int WGT, int UU>
hipError_t launch_tuned_r(const DevMode& m, const void* const* fac, float* out, float* carry, const Geometry& g,
                          uint32_t atomic_cut, hipStream_t s)
{
    if constexpr (WGT == part_wg(2) && UU == part::gathers_in_flight(2, R, MTTKRP_FP32)) {
        return hipErrorInvalidValue;
    } else {
        if (m.idx16)
            return part::launch_part<2, R, MTTKRP_FP32, false, true, WGT, UU>(m, fac, nullptr, 0, out, carry, g,
                                                                             atomic_cut, s);
        return part::launch_part<2, R, MTTKRP_FP32, false, false, WGT, UU>(m, fac, nullptr, 0, out, carry, g,
                                                                          atomic_cut, s);
    }
}

template <int R, int WGT, int UU>
hipError_t launch_batch_tuned_r(const void* descs, const uint2* work, uint32_t nwork, uint32_t grid, hipStream_t s)
{
    if constexpr (WGT == part_wg(2) && UU == part::gathers_in_flight(2, R, MTTKRP_FP32))
        return hipErrorInvalidValue;
    else
        return part::launch_batch_part<2, R, MTTKRP_FP32, WGT, UU>(descs, work, nwork, grid, s);
}

template <int WGT>
hipError_t launch_part_tuned_wg(const DevMode& m, int R, int gathers, const void* const* fac, float* out, float* carry,
                                const Geometry& g, uint32_t atomic_cut, hipStream_t s)
{
    if (m.n_in != 2) return hipErrorInvalidValue;
#define MK_TUNED(RR, UU) \
    if (R == RR && gathers == UU) return launch_tuned_r<RR, WGT, UU>(m, fac, out, carry, g, atomic_cut, s);
    MK_TUNED(16, 2) MK_TUNED(16, 4) MK_TUNED(32, 2) MK_TUNED(32, 4) MK_TUNED(64, 2) MK_TUNED(64, 4)
#undef MK_TUNED
    return hipErrorInvalidValue;
}

template <int WGT>
hipError_t launch_batch_part_tuned_wg(int R, int gathers, const void* descs, const uint2* work, uint32_t nwork,
                                      uint32_t grid, hipStream_t s)
{
#define MK_TUNED(RR, UU) \
    if (R == RR && gathers == UU) return launch_batch_tuned_r<RR, WGT, UU>(descs, work, nwork, grid, s);
    MK_TUNED(16, 2) MK_TUNED(16, 4) MK_TUNED(32, 2) MK_TUNED(32, 4) MK_TUNED(64, 2) MK_TUNED(64, 4)
#undef MK_TUNED
    return hipErrorInvalidValue;
}

// Descriptor of one tensor's mode copy for the batched partition kernel.
template <int NIN>
size_t part_desc_bytes_nin() { return sizeof(part::PartArgs<NIN>); }

template <int NIN>
void fill_part_desc_nin(void* dst, const DevMode& m, int R, int dtype, const void* const* fac, float* out,
                        float* carry, uint32_t gsz)
{
    part::fill_part_args<NIN>(*static_cast<part::PartArgs<NIN>*>(dst), m, R, dtype, fac, nullptr, 0, out, carry, gsz);
}

template <int NIN>
hipError_t launch_batch_part_nin(int R, int dtype, const void* descs, const uint2* work, uint32_t nwork, uint32_t grid,
                                 hipStream_t s)
{
    if (dtype == MTTKRP_FP32) {
        switch (R) {
            case 16: return part::launch_batch_part<NIN, 16, MTTKRP_FP32>(descs, work, nwork, grid, s);
            case 32: return part::launch_batch_part<NIN, 32, MTTKRP_FP32>(descs, work, nwork, grid, s);
            case 64: return part::launch_batch_part<NIN, 64, MTTKRP_FP32>(descs, work, nwork, grid, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (R) {
        case 16: return part::launch_batch_part<NIN, 16, MTTKRP_BF16>(descs, work, nwork, grid, s);
        case 32: return part::launch_batch_part<NIN, 32, MTTKRP_BF16>(descs, work, nwork, grid, s);
        case 64: return part::launch_batch_part<NIN, 64, MTTKRP_BF16>(descs, work, nwork, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NIN>
hipError_t launch_part_nin(const DevMode& m, int R, int dtype, const void* const* fac,
                           const uint32_t* const* hot_rows, uint32_t nhot, float* out, float* carry,
                           const Geometry& g, uint32_t atomic_cut, hipStream_t s)
{
    return dtype == MTTKRP_FP32
               ? part::dispatch_r<NIN, MTTKRP_FP32>(m, R, fac, hot_rows, nhot, out, carry, g, atomic_cut, s)
               : part::dispatch_r<NIN, MTTKRP_BF16>(m, R, fac, hot_rows, nhot, out, carry, g, atomic_cut, s);
}

}  // namespace mk
