// Step kernel of the per-mode MTTKRP on hot-steps copies (see build_step_copy):
// every output row's nonzeros are ordered by which of their input rows are
// hot, and rows are padded to whole steps of P entries.
//
// A wave walks a contiguous run of steps.  In one step its G lane groups (L
// lanes each, a 16-byte slice of a factor row per lane) take G entries of the
// same output row, so a row's partial sums sit in G groups' registers and are
// added across groups (a fixed butterfly) when the row ends.  For each input
// the wave asks whether any of its entries names a cold row and whether any
// names a hot one: a step whose rows are all hot for an input reads them from
// LDS and issues no global gather for it; an all-cold one issues no LDS read;
// only the steps where a row's hot/cold class changes issue both.  Since rows
// are sorted by class, most steps are one or the other.
//
// One workgroup of 1024 threads per compute unit holds the hot rows of every
// input (and one zero row each, named by padding entries) in LDS for its
// whole life and walks partitions blockIdx.x, blockIdx.x + gridDim.x, ...
// A partition is 16 consecutive wave runs; the first/last row partials of
// the waves are combined in LDS in wave order and rows cut by the partition's
// ends go to the carry buffer, which the fix-up kernel adds in partition
// order, exactly as for the nonzero-ordered copies.  No atomics: results
// repeat bit for bit.
#pragma once

#include "part_kernel.h"

namespace mk {

constexpr int kStepWG = 1024;
constexpr int kStepWaves = kStepWG / 64;

template <int NIN>
struct StepArgs {
    const uint32_t* idx[NIN];   // step copy, transposed per 32 steps
    const void* fac[NIN];
    const uint32_t* hot_rows[NIN];
    uint32_t fac_bytes[NIN];
    const float* val;
    const uint2* winfo;         // per 32 steps: {row-start bits, ordinal of the row holding the first step}
    const uint32_t* row_id;
    uint32_t nrows_nz;          // entries of row_id
    float* out;
    float* carry;
    uint64_t nsteps;
    uint32_t wsz;               // steps per wave run (multiple of 32)
    uint32_t nparts;
    uint32_t nhot;              // hot rows per input; slot nhot is the zero row
    uint32_t P;                 // entries per step (a multiple of the groups per wave)
};

// LDS bytes of a step workgroup: hot rows (+ the zero row) of every input at R
// values of `es` bytes, then the wave partials.
inline uint32_t step_lds_bytes(int n_in, int R, int es, uint32_t nhot)
{
    return (uint32_t)n_in * (nhot + 1u) * (uint32_t)R * (uint32_t)es + 2u * kStepWaves * (uint32_t)R * 4u +
           2u * kStepWaves * 4u;
}

namespace step {

using part::f32x4;
using part::group_bcast;
using part::load_buffer;
using part::load_lds;
using part::load_words;
using part::lds_char;
using part::make_rsrc;
using part::Slice;
using part::static_for;
using part::store_vals;
using part::unpack;
using part::kSkipOffset;

// The value x of lane ^ d (d a power of two below 64): DPP for d = 8 (a
// rotation by half of each 16-lane row), ds_swizzle for the other d < 32,
// ds_bpermute for d = 32.
template <int d>
__device__ __forceinline__ float lane_xor(float x, int lane)
{
    if constexpr (d == 8) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
    } else if constexpr (d < 32) {
        constexpr int pattern = 0x1F | (d << 10);   // ds_swizzle bit mode: xor d
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), pattern));
    } else {
        return __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, __float_as_int(x)));
    }
}

// Sum over the G = 64 / L lane groups of v[0..E) (lane gl of group g holds
// elements gl * E .. gl * E + E - 1 of group g's partial row), scattered:
// each stage pairs lanes lane ^ (L << k) and halves the values a lane keeps
// (the lane whose bit is set keeps the upper half) until one is left; the
// remaining stages add the pair's copies.  Returns the sum of element
// gl * E + er, er = this lane's index; lanes of groups g < min(E, G) hold
// distinct elements.  A fixed pairing tree: the same bits every time, and
// both lanes of a pair compute the same sum.
template <int L, int E>
__device__ __forceinline__ float sum_groups_scatter(const float (&v)[E], int lane, int& er)
{
    float cur[E];
#pragma unroll
    for (int e = 0; e < E; ++e) cur[e] = v[e];
    er = 0;
    static_for<0, 6>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int d = L << k;
        constexpr int n = E >> k;          // values a lane holds before this stage
        if constexpr (d < 64 && n >= 2) {
            constexpr int h = n / 2;
            const bool up = (lane & d) != 0;
            float keep[h], snd[h];
#pragma unroll
            for (int i = 0; i < h; ++i) {
                keep[i] = up ? cur[i + h] : cur[i];
                snd[i] = up ? cur[i] : cur[i + h];
            }
#pragma unroll
            for (int i = 0; i < h; ++i) cur[i] = keep[i] + lane_xor<d>(snd[i], lane);
            if (up) er += h;
        } else if constexpr (d < 64) {
            cur[0] = cur[0] + lane_xor<d>(cur[0], lane);
        }
    });
    return cur[0];
}

template <int NIN, int R, int DT, int SUB>
__device__ __forceinline__ void step_body(const StepArgs<NIN>& a, char* smem)
{
    constexpr int E = vals_per_lane(R, DT);
    constexpr int L = R / E;        // lanes per group
    constexpr int G = 64 / L;       // groups per wave
    constexpr int V = 32 / L;       // words per lane of a 32-step column
    constexpr int W = kStepWaves;
    constexpr int kOwn = E < G ? E : G;   // groups whose lanes hold distinct elements of a summed row
    constexpr int kEs = Slice<R, DT>::kElem;
    constexpr int U = (NIN <= 2 && SUB == 1 && E == 4) ? 8 : (NIN <= 2 ? 4 : 2);   // entries per chunk, whose loads are issued before the first is used
    using ST = typename Slice<R, DT>::T;
    static_assert(R % E == 0 && L >= 2 && L <= 16 && NIN >= 2, "unsupported rank or mode count");
    static_assert(SUB >= 1 && (32 * SUB) % U == 0, "bad pass count");

    const int tid = threadIdx.x;
    // The wave index, and everything derived from it (the wave's run, its
    // batches, row bits and ordinals), is the same in every lane: kept in
    // scalar registers, so the per-step tests are scalar branches.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane / L;
    const int gl = lane % L;
    const uint32_t row_bytes = R * kEs;
    const uint32_t hot_stride = (a.nhot + 1u) * row_bytes;   // bytes of one input's hot rows

    // 1. Hot rows of every input, then its zero row, into LDS.
    {
        const uint32_t cpr = row_bytes / 16;
        const uint32_t chunks = (a.nhot + 1u) * cpr;
        static_for<0, NIN>([&](auto M) {
            constexpr int m = decltype(M)::value;
            char* dst = smem + (size_t)m * hot_stride;
            const char* fac = static_cast<const char*>(a.fac[m]);
            for (uint32_t c = tid; c < chunks; c += kStepWG) {
                const uint32_t r = c / cpr;
                part::u32x4 d = {0u, 0u, 0u, 0u};
                if (r < a.nhot) d = *reinterpret_cast<const part::u32x4*>(fac + (uint64_t)a.hot_rows[m][r] * row_bytes +
                                                                         (c % cpr) * 16);
                *reinterpret_cast<part::u32x4*>(dst + (size_t)r * row_bytes + (c % cpr) * 16) = d;
            }
        });
    }
    __syncthreads();

    char* pbase = smem + (size_t)NIN * hot_stride;
    float* s_head = reinterpret_cast<float*>(pbase);
    float* s_tail = s_head + W * R;
    int* s_trow = reinterpret_cast<int*>(s_tail + W * R);
    int* s_hstart = s_trow + W;
    __amdgpu_buffer_rsrc_t rsrc[NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) rsrc[m] = make_rsrc(a.fac[m], a.fac_bytes[m]);
    lds_char* hot_lds = (lds_char*)smem;

    for (uint32_t part_i = blockIdx.x; part_i < a.nparts; part_i += gridDim.x) {
        const uint64_t wg_beg = (uint64_t)part_i * W * a.wsz;
        const uint64_t w_beg = wg_beg + (uint64_t)wave * a.wsz;
        float acc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = 0.0f;
        // Row sums over the groups are held scattered: this lane's element of
        // a summed row is gl * E + er (lanes of groups g >= kOwn repeat those
        // of lower groups).
        float head_v = 0.0f, tail_v = 0.0f;
        int er = 0;
        int first_row = -1, cur = -1, hstart = -1;
        // Output rows of the ordinals rid_base, rid_base + 1, ... (one per
        // lane), loaded once per 32-step batch: a row that ends inside the
        // batch finds its row there instead of waiting on a load.
        int rid_base = 0;
        uint32_t rid_pf = 0;

        // The row `cur` ended: its sum over the groups is stored, or kept as
        // the wave's head partial if it is the wave's first row.
        auto row_end = [&]() {
            const float tot = sum_groups_scatter<L, E>(acc, lane, er);
            if (cur == first_row) {
                head_v = tot;
            } else {
                const uint32_t rid = (uint32_t)__builtin_amdgcn_readlane((int)rid_pf, cur - rid_base);
                if (g < kOwn) a.out[(uint64_t)rid * R + gl * E + er] = tot;
            }
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0.0f;
        };

        if (w_beg < a.nsteps) {
            const uint64_t w_end = min(w_beg + (uint64_t)a.wsz, a.nsteps);
            for (uint64_t b = w_beg; b < w_end; b += 32) {
                const int nvalid = (int)min((uint64_t)32, w_end - b);
                const uint2 wi = a.winfo[b >> 5];
                uint32_t flags = wi.x;
                if (b == w_beg) {
                    first_row = cur = (int)wi.y;
                    hstart = (int)(flags & 1u);
                    flags &= ~1u;
                }
                rid_base = cur;
                rid_pf = a.row_id[min((uint32_t)(cur + lane), a.nrows_nz - 1u)];
                // The batch's columns: pass t of step s takes entry t * G + g.
                const uint64_t col0 = (b >> 5) * 32ull * a.P;
                uint32_t cw[SUB][NIN][V], cv[SUB][V];
                static_for<0, SUB>([&](auto T) {
                    constexpr int t = decltype(T)::value;
                    const uint64_t col = col0 + (uint64_t)(t * G + g) * 32ull + (uint64_t)gl * V;
                    static_for<0, NIN>([&](auto M) {
                        constexpr int m = decltype(M)::value;
                        load_words<V>(a.idx[m] + col, cw[t][m]);
                    });
                    load_words<V>(reinterpret_cast<const uint32_t*>(a.val) + col, cv[t]);
                });
                // Entries q = s * SUB + t in order, U at a time ("chunks").
                static_for<0, 32 * SUB / U>([&](auto QB) {
                    constexpr int q0 = decltype(QB)::value * U;
                    if (q0 / SUB < nvalid) {
                        uint32_t vidx[U][NIN];
                        float vv[U];
                        static_for<0, U>([&](auto UU) {
                            constexpr int u = decltype(UU)::value;
                            constexpr int s = (q0 + u) / SUB, t = (q0 + u) % SUB;
                            vv[u] = __uint_as_float(group_bcast<L, s / V>(cv[t][s % V]));
                            static_for<0, NIN>([&](auto M) {
                                constexpr int m = decltype(M)::value;
                                vidx[u][m] = group_bcast<L, s / V>(cw[t][m][s % V]);
                            });
                        });
                        ST x[U][NIN];
                        constexpr int s_last = (q0 + U - 1) / SUB;
                        if (s_last < nvalid) {
                            // Whole chunk.  Per input, the wave learns whether any
                            // of the chunk's rows is cold and whether any is hot
                            // (one wave-wide vote each): all cold, the rows come
                            // by global gathers; all hot, from LDS; both (a class
                            // boundary), cold lanes gather (hot ones get an
                            // out-of-range offset and read 0) and hot lanes add
                            // their LDS row (cold ones the zero row).
                            static_for<0, NIN>([&](auto M) {
                                constexpr int m = decltype(M)::value;
                                lds_char* base = hot_lds + (size_t)m * hot_stride;
                                uint32_t hot_or = 0u, hot_and = kHotBitDev;
                                static_for<0, U>([&](auto UU) {
                                    hot_or |= vidx[decltype(UU)::value][m];
                                    hot_and &= vidx[decltype(UU)::value][m];
                                });
                                const bool some_cold = __builtin_amdgcn_ballot_w64((hot_and & kHotBitDev) == 0u) != 0ull;
                                const bool some_hot = __builtin_amdgcn_ballot_w64((hot_or & kHotBitDev) != 0u) != 0ull;
                                if (!some_hot) {
                                    static_for<0, U>([&](auto UU) {
                                        constexpr int u = decltype(UU)::value;
                                        x[u][m] = load_buffer<R, DT>(
                                            rsrc[m], (vidx[u][m] * (uint32_t)R + (uint32_t)(gl * E)) * kEs);
                                    });
                                } else if (!some_cold) {
                                    static_for<0, U>([&](auto UU) {
                                        constexpr int u = decltype(UU)::value;
                                        x[u][m] = load_lds<R, DT>(base, vidx[u][m] & ~kHotBitDev, gl);
                                    });
                                } else {
                                    static_for<0, U>([&](auto UU) {
                                        constexpr int u = decltype(UU)::value;
                                        const uint32_t v = vidx[u][m];
                                        x[u][m] = load_buffer<R, DT>(
                                            rsrc[m], (v & kHotBitDev) ? kSkipOffset
                                                                      : (v * (uint32_t)R + (uint32_t)(gl * E)) * kEs);
                                    });
                                    static_for<0, U>([&](auto UU) {
                                        constexpr int u = decltype(UU)::value;
                                        const uint32_t v = vidx[u][m];
                                        x[u][m] = x[u][m] | load_lds<R, DT>(base, (v & kHotBitDev) ? (v & ~kHotBitDev)
                                                                                                   : a.nhot, gl);
                                    });
                                }
                            });
                        } else {
                            // The run's ragged end: entries past it read nothing.
                            static_for<0, U>([&](auto UU) {
                                constexpr int u = decltype(UU)::value;
                                constexpr int s = (q0 + u) / SUB;
                                static_for<0, NIN>([&](auto M) {
                                    constexpr int m = decltype(M)::value;
                                    x[u][m] = ST{};
                                    if (s < nvalid) {
                                        const uint32_t v = vidx[u][m];
                                        const bool hot = (v & kHotBitDev) != 0;
                                        x[u][m] = load_buffer<R, DT>(
                                            rsrc[m], hot ? kSkipOffset : (v * (uint32_t)R + (uint32_t)(gl * E)) * kEs);
                                        x[u][m] = x[u][m] | load_lds<R, DT>(hot_lds + (size_t)m * hot_stride,
                                                                            hot ? (v & ~kHotBitDev) : a.nhot, gl);
                                    }
                                });
                            });
                        }
                        // Products and row sums; row ends are tested only in
                        // chunks where a row starts.
                        auto use = [&](auto UU, bool test_rows) {
                            constexpr int u = decltype(UU)::value;
                            constexpr int s = (q0 + u) / SUB, t = (q0 + u) % SUB;
                            if (s < nvalid) {
                                if (t == 0 && test_rows && ((flags >> s) & 1u)) {
                                    row_end();
                                    ++cur;
                                }
                                float p[E];
                                static_for<0, NIN>([&](auto M) {
                                    constexpr int m = decltype(M)::value;
                                    float q[E];
                                    unpack<R, DT>(x[u][m], q);
                                    if constexpr (m == 0) {
#pragma unroll
                                        for (int e = 0; e < E; ++e) p[e] = q[e] * vv[u];
                                    } else if constexpr (m < NIN - 1) {
#pragma unroll
                                        for (int e = 0; e < E; ++e) p[e] *= q[e];
                                    } else {
#pragma unroll
                                        for (int e = 0; e < E; ++e) acc[e] = fmaf(p[e], q[e], acc[e]);
                                    }
                                });
                            }
                        };
                        constexpr uint32_t chunk_bits = ((1u << (s_last - q0 / SUB + 1)) - 1u) << (q0 / SUB);
                        if (flags & chunk_bits) {
                            static_for<0, U>([&](auto UU) { use(UU, true); });
                        } else {
                            static_for<0, U>([&](auto UU) { use(UU, false); });
                        }
                    }
                });
            }
            // The run's last row: its sum over the groups.
            const float tot = sum_groups_scatter<L, E>(acc, lane, er);
            if (cur == first_row) head_v = tot;
            else tail_v = tot;
        }

        // 3. Wave partials into LDS, then combined in wave order.
        const bool multi = first_row >= 0 && cur != first_row;
        if (first_row >= 0 && g < kOwn) {
            s_head[wave * R + gl * E + er] = head_v;
            if (multi) s_tail[wave * R + gl * E + er] = tail_v;
        }
        if (lane == 0) {
            s_trow[wave] = multi ? cur : -1;
            s_hstart[wave] = hstart;
        }
        __syncthreads();

        const uint64_t next_beg = wg_beg + (uint64_t)W * a.wsz;
        const bool row_continues = next_beg < a.nsteps && !(a.winfo[next_beg >> 5].x & 1u);
        const int hs = s_hstart[wave];
        const int trow = s_trow[wave];
        auto emit = [&](const float* src, int row, bool from_first_of_wg, bool extend) {
            float sum[E];
#pragma unroll
            for (int e = 0; e < E; ++e) sum[e] = src[wave * R + gl * E + e];
            bool reaches_end = extend;
            if (extend) {
                for (int j = wave + 1; j < W; ++j) {
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
            if (head_split || tail_split)
                store_vals<E>(a.carry + ((uint64_t)part_i * 2 + (from_first_of_wg ? 0 : 1)) * R + gl * E, sum);
            else
                store_vals<E>(a.out + (uint64_t)a.row_id[row] * R + gl * E, sum);
        };
        if (g == 0 && hs >= 0) {
            if (wave == 0 || hs == 1) emit(s_head, first_row, wave == 0, trow < 0);
            if (trow >= 0) emit(s_tail, trow, false, true);
        }
        __syncthreads();   // the next partition reuses the partial slots
    }
}

}  // namespace step

template <int NIN, int R, int DT, int SUB>
__global__ __launch_bounds__(kStepWG) void mttkrp_step_kernel(StepArgs<NIN> a)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    step::step_body<NIN, R, DT, SUB>(a, smem);
}

template <int NIN, int R, int DT, int SUB>
hipError_t launch_step_sub(const StepArgs<NIN>& a, uint32_t grid, hipStream_t s)
{
    const uint32_t lds = step_lds_bytes(NIN, R, DT == MTTKRP_FP32 ? 4 : 2, a.nhot);
    static uint32_t lds_set = 0;
    if (lds > lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mttkrp_step_kernel<NIN, R, DT, SUB>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL((mttkrp_step_kernel<NIN, R, DT, SUB>), dim3(grid), dim3(kStepWG), lds, s, a);
    return hipGetLastError();
}

// Passes per step: the copy's entries per step over this launch's lane groups per wave (1 or 2).
template <int NIN, int R, int DT>
hipError_t launch_step_kernel(const StepArgs<NIN>& a, uint32_t grid, hipStream_t s)
{
    constexpr uint32_t G = 64 / (R / vals_per_lane(R, DT));
    if (a.P == G) return launch_step_sub<NIN, R, DT, 1>(a, grid, s);
    if (a.P == 2 * G) return launch_step_sub<NIN, R, DT, 2>(a, grid, s);
    return hipErrorInvalidValue;
}

// Fill the arguments of one step-copy launch and start it; `fac` and
// `hot_rows` in the order of m.in_modes.
template <int NIN>
hipError_t launch_step_nin(const DevMode& m, int R, int dtype, const void* const* fac,
                           const uint32_t* const* hot_rows, uint32_t nhot, float* out, float* carry,
                           const Geometry& g, uint32_t grid, hipStream_t s)
{
    StepArgs<NIN> a;
    const uint32_t es = dtype == MTTKRP_FP32 ? 4u : 2u;
    for (int j = 0; j < NIN; ++j) {
        a.idx[j] = m.idx[j];
        a.fac[j] = fac[j];
        a.hot_rows[j] = hot_rows[j];
        a.fac_bytes[j] = (uint32_t)((uint64_t)m.in_dims[j] * R * es);
    }
    a.val = m.val;
    a.winfo = m.winfo;
    a.row_id = m.row_id;
    a.nrows_nz = (uint32_t)m.nrows_nz;
    a.out = out;
    a.carry = carry;
    a.nsteps = m.nsteps;
    a.wsz = g.gsz;
    a.nparts = g.nparts;
    a.nhot = nhot;
    a.P = m.step_P;
    if (dtype == MTTKRP_FP32) {
        switch (R) {
            case 16: return launch_step_kernel<NIN, 16, MTTKRP_FP32>(a, grid, s);
            case 32: return launch_step_kernel<NIN, 32, MTTKRP_FP32>(a, grid, s);
            case 64: return launch_step_kernel<NIN, 64, MTTKRP_FP32>(a, grid, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (R) {
        case 16: return launch_step_kernel<NIN, 16, MTTKRP_BF16>(a, grid, s);
        case 32: return launch_step_kernel<NIN, 32, MTTKRP_BF16>(a, grid, s);
        case 64: return launch_step_kernel<NIN, 64, MTTKRP_BF16>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mk
