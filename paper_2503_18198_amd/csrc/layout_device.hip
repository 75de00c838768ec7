// Device construction of the mode-specific copies (Sec. III-B scheme 2 order,
// Sec. III-C COO copies): the same arrays, in the same order, as the host
// build, for tensors whose packed coordinate keys fit 128 bits.
//
// Per mode: a packed key per nonzero (output index in the top bits, then the
// other indices in cyclic order), a stable radix sort of (key, position)
// pairs (keys over 64 bits: by the low word, then stably by the high word),
// so equal coordinates keep their input order, then the
// structure-of-arrays copy decoded from the sorted keys, the row-start bits
// with the per-word row ordinals, and the lists of nonempty and empty rows.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace mk {

namespace {

struct KeyFields {
    int nf;                 // input modes, in cyclic order after the output mode
    int mode[kMaxIn];       // their mode numbers
    int bits[kMaxIn];       // bits of each field (0 for a dimension of 1)
    int shift[kMaxIn];      // position of each field in the key
    int slot[kMaxIn];       // position among the increasing input modes (the SoA array)
    int row_mode, row_bits, row_shift;
};

struct DecodeOut {
    void* idx[kMaxIn];   // uint32 arrays, or uint16 where bit j of narrow is set
    uint32_t narrow;
    float* val;
};

__device__ __forceinline__ void put_idx(const DecodeOut& out, int j, uint64_t k, uint32_t v)
{
    if ((out.narrow >> j) & 1u) static_cast<uint16_t*>(out.idx[j])[k] = (uint16_t)v;
    else static_cast<uint32_t*>(out.idx[j])[k] = v;
}

using u128 = unsigned __int128;

// Key k from its low and high words (no high words: keys of at most 64 bits).
__device__ __forceinline__ u128 key_at(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi, uint64_t k)
{
    u128 v = lo[k];
    if (hi) v |= (u128)hi[k] << 64;
    return v;
}

__device__ __forceinline__ uint64_t row_of(u128 key, const KeyFields& kf)
{
    return kf.row_bits ? (uint64_t)(key >> kf.row_shift) : 0;
}

__global__ void pack_keys_kernel(const uint32_t* __restrict__ coo, uint64_t nnz, int N, KeyFields kf,
                                 uint64_t* __restrict__ lo, uint64_t* __restrict__ hi, uint32_t* __restrict__ pos)
{
    const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const uint32_t* p = coo + k * (uint64_t)N;
    u128 v = p[kf.row_mode];
    for (int f = 0; f < kf.nf; ++f)
        if (kf.bits[f]) v = (v << kf.bits[f]) | p[kf.mode[f]];
    lo[k] = (uint64_t)v;
    if (hi) hi[k] = (uint64_t)(v >> 64);
    pos[k] = (uint32_t)k;
}

// dst[k] = src[pos[k]]
__global__ void gather_u64_kernel(const uint64_t* __restrict__ src, const uint32_t* __restrict__ pos, uint64_t n,
                                  uint64_t* __restrict__ dst)
{
    const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[pos[k]];
}

// Input-mode coordinates from the sorted keys, values gathered by position;
// the padding up to a multiple of 32 is zero.
__global__ void decode_kernel(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi,
                              const uint32_t* __restrict__ pos,
                              const float* __restrict__ val_in, uint64_t nnz, uint64_t nnz_pad, KeyFields kf,
                              DecodeOut out)
{
    const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (k >= nnz_pad) return;
    if (k >= nnz) {
        for (int f = 0; f < kf.nf; ++f) put_idx(out, kf.slot[f], k, 0u);
        out.val[k] = 0.0f;
        return;
    }
    const u128 x = key_at(lo, hi, k);
    for (int f = 0; f < kf.nf; ++f) {
        const uint32_t mask = kf.bits[f] ? (uint32_t)((1ull << kf.bits[f]) - 1ull) : 0u;
        put_idx(out, kf.slot[f], k, (uint32_t)(x >> kf.shift[f]) & mask);
    }
    out.val[k] = val_in[pos[k]];
}

// Per 32 nonzeros: a bit per nonzero that starts an output row, and the count.
__global__ void row_bits_kernel(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi, uint64_t nnz,
                                uint64_t nwords, KeyFields kf,
                                uint32_t* __restrict__ bits_out, uint32_t* __restrict__ count_out)
{
    const uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t bits = 0;
    const uint64_t k0 = w * 32;
    uint64_t prev = k0 ? row_of(key_at(lo, hi, k0 - 1), kf) : ~0ull;
    for (int b = 0; b < 32 && k0 + b < nnz; ++b) {
        const uint64_t r = row_of(key_at(lo, hi, k0 + b), kf);
        if (r != prev) bits |= 1u << b;
        prev = r;
    }
    bits_out[w] = bits;
    count_out[w] = (uint32_t)__popc(bits);
}

// winfo = {row-start bits, ordinal of the row holding the word's first
// nonzero}; row_id[ordinal] = output row; marks the rows that are present.
__global__ void row_lists_kernel(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi,
                                 const uint32_t* __restrict__ bits_in,
                                 const uint32_t* __restrict__ before, uint64_t nwords, KeyFields kf,
                                 uint2* __restrict__ winfo, uint32_t* __restrict__ row_id,
                                 uint8_t* __restrict__ empty_flag)
{
    const uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const uint32_t bits = bits_in[w];
    const uint32_t b0 = before[w];
    winfo[w] = make_uint2(bits, b0 + (bits & 1u) - 1u);
    uint32_t m = bits;
    while (m) {
        const int b = __ffs(m) - 1;
        m &= m - 1;
        const uint32_t row = (uint32_t)row_of(key_at(lo, hi, w * 32 + b), kf);
        row_id[b0 + (uint32_t)__popc(bits & ((1u << b) - 1u))] = row;
        empty_flag[row] = 0;
    }
}

__global__ void fill_u8_kernel(uint8_t* p, uint64_t n, uint8_t v)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Squared value of every run of equal coordinates (duplicates summed first),
// at the run's first nonzero; zero elsewhere.
__global__ void run_squares_kernel(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi,
                                   const float* __restrict__ val, uint64_t nnz, double* __restrict__ sq)
{
    const uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const u128 key = key_at(lo, hi, k);
    if (k > 0 && key_at(lo, hi, k - 1) == key) {
        sq[k] = 0.0;
        return;
    }
    double v = val[k];
    for (uint64_t j = k + 1; j < nnz && key_at(lo, hi, j) == key; ++j) v += val[j];
    sq[k] = v * v;
}

int bits_for(uint32_t d)
{
    int b = 0;
    while ((1ull << b) < (uint64_t)d) ++b;
    return b;
}

uint32_t blocks_for(uint64_t n, int threads) { return (uint32_t)((n + threads - 1) / threads); }

}  // namespace

bool device_build_applies(const uint32_t* dims, int N, uint64_t nnz)
{
    if (nnz == 0 || nnz >= (1ull << 31)) return false;
    int bits = 0;
    for (int m = 0; m < N; ++m) bits += bits_for(dims[m]);
    return bits <= 128;   // the key of every mode holds all N fields
}

namespace {

// Byte offsets of the device build's scratch arrays in one allocation.
struct ScratchPlan {
    uint64_t o_coo, o_val, o_key, o_tkey, o_hi, o_pos, o_tpos, o_sq, o_bits, o_cnt, o_before, o_flag, o_small, o_cub;
    uint64_t cub_b, total;
};

hipError_t plan_scratch(const uint32_t* dims, int N, uint64_t nnz, ScratchPlan& p)
{
    const uint64_t nnz_pad = (nnz + 31) / 32 * 32;
    const uint64_t nwords = nnz_pad / 32;
    uint32_t max_dim = 0;
    for (int m = 0; m < N; ++m) max_dim = std::max(max_dim, dims[m]);
    // hipCUB scratch sizes (size queries only: nothing is enqueued)
    hipStream_t s = nullptr;
    size_t sort_b = 0, scan_b = 0, sel_b = 0, red_b = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                                      (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)nnz, 0, 64, s);
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (int)nwords, s);
    if (e == hipSuccess)
        e = hipcub::DeviceSelect::Flagged(nullptr, sel_b, hipcub::CountingInputIterator<uint32_t>(0),
                                          (const uint8_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                          (int)max_dim, s);
    if (e == hipSuccess)
        e = hipcub::DeviceReduce::Sum(nullptr, red_b, (const double*)nullptr, (double*)nullptr, (int)nnz, s);
    if (e != hipSuccess) return e;
    p.cub_b = std::max(std::max(sort_b, scan_b), std::max(sel_b, red_b));
    auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
    p.o_coo = 0;
    p.o_val = p.o_coo + al(nnz * N * 4);
    p.o_key = p.o_val + al(nnz * 4);
    p.o_tkey = p.o_key + al(nnz * 8);
    p.o_hi = p.o_tkey + al(nnz * 8);
    p.o_pos = p.o_hi + al(nnz * 8);
    p.o_tpos = p.o_pos + al(nnz * 4);
    p.o_sq = p.o_tpos + al(nnz * 4);
    p.o_bits = p.o_sq + al(nnz * 8);
    p.o_cnt = p.o_bits + al(nwords * 4);
    p.o_before = p.o_cnt + al(nwords * 4);
    p.o_flag = p.o_before + al(nwords * 4);
    p.o_small = p.o_flag + al(max_dim);
    p.o_cub = p.o_small + 256;
    p.total = p.o_cub + al(p.cub_b);
    return hipSuccess;
}

}  // namespace

uint64_t device_build_scratch_bytes(const uint32_t* dims, int N, uint64_t nnz)
{
    if (!device_build_applies(dims, N, nnz)) return 0;
    ScratchPlan p;
    if (plan_scratch(dims, N, nnz, p) != hipSuccess) return 0;
    return p.total;
}

hipError_t build_device_modes(const uint32_t* coo_host, const float* vals_host, uint64_t nnz, const uint32_t* dims,
                              int N, const std::vector<DeviceModeSlots>& slots, std::vector<DevMode>& modes,
                              double* normX2, void* ext_scratch, uint64_t ext_scratch_bytes, hipStream_t s)
{
    const uint64_t nnz_pad = (nnz + 31) / 32 * 32;
    const uint64_t nwords = nnz_pad / 32;
    uint32_t max_dim = 0;
    for (int m = 0; m < N; ++m) max_dim = std::max(max_dim, dims[m]);
    ScratchPlan sp;
    hipError_t e = plan_scratch(dims, N, nnz, sp);
    if (e != hipSuccess) return e;
    const size_t cub_b = sp.cub_b;
    const uint64_t o_coo = sp.o_coo, o_val = sp.o_val, o_key = sp.o_key, o_tkey = sp.o_tkey, o_hi = sp.o_hi,
                   o_pos = sp.o_pos, o_tpos = sp.o_tpos, o_sq = sp.o_sq, o_bits = sp.o_bits, o_cnt = sp.o_cnt,
                   o_before = sp.o_before, o_flag = sp.o_flag, o_small = sp.o_small, o_cub = sp.o_cub;
    // One scratch region: the caller's, or an allocation freed before returning.
    char* base = nullptr;
    const bool own = ext_scratch == nullptr;
    if (own) {
        e = hipMalloc(&base, sp.total);
        if (e != hipSuccess) return e;
    } else {
        if (ext_scratch_bytes < sp.total || reinterpret_cast<uintptr_t>(ext_scratch) % 256) return hipErrorInvalidValue;
        base = static_cast<char*>(ext_scratch);
    }
    uint32_t* d_coo = (uint32_t*)(base + o_coo);
    float* d_val = (float*)(base + o_val);
    uint64_t* d_key = (uint64_t*)(base + o_key);
    uint64_t* d_tkey = (uint64_t*)(base + o_tkey);
    uint64_t* d_hi = (uint64_t*)(base + o_hi);
    uint32_t* d_pos = (uint32_t*)(base + o_pos);
    uint32_t* d_tpos = (uint32_t*)(base + o_tpos);
    double* d_sq = (double*)(base + o_sq);
    uint32_t* d_bits = (uint32_t*)(base + o_bits);
    uint32_t* d_cnt = (uint32_t*)(base + o_cnt);
    uint32_t* d_before = (uint32_t*)(base + o_before);
    uint8_t* d_flag = (uint8_t*)(base + o_flag);
    uint32_t* d_small = (uint32_t*)(base + o_small);    // [0] empty-row count; as double: |X|^2
    void* d_cub = base + o_cub;

    e = hipMemcpyAsync(d_coo, coo_host, nnz * N * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_val, vals_host, nnz * 4, hipMemcpyHostToDevice, s);

    constexpr int T = 256;
    modes.assign(N, DevMode{});
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        const DeviceModeSlots& sl = slots[n];
        DevMode& d = modes[n];
        KeyFields kf{};
        kf.nf = N - 1;
        int below = 0;
        for (int f = N - 2; f >= 0; --f) {
            const int m = (n + 1 + f) % N;
            kf.mode[f] = m;
            kf.bits[f] = bits_for(dims[m]);
            kf.shift[f] = below;
            kf.slot[f] = m < n ? m : m - 1;
            below += kf.bits[f];
        }
        kf.row_mode = n;
        kf.row_bits = bits_for(dims[n]);
        kf.row_shift = below;
        const int key_bits = below + kf.row_bits;

        // Sorted keys end in (lo, hi) with positions in pos.
        const bool wide = key_bits > 64;
        const uint64_t* lo = d_tkey;
        const uint64_t* hi = nullptr;
        const uint32_t* pos = d_tpos;
        pack_keys_kernel<<<blocks_for(nnz, T), T, 0, s>>>(d_coo, nnz, N, kf, d_key, wide ? d_hi : nullptr, d_pos);
        size_t b = cub_b;
        e = hipcub::DeviceRadixSort::SortPairs(d_cub, b, d_key, d_tkey, d_pos, d_tpos, (int)nnz, 0,
                                               wide ? 64 : std::max(key_bits, 1), s);
        if (e != hipSuccess) break;
        if (wide) {
            // then stably by the high word: the high words in low-word order go
            // to d_tkey, are sorted into d_hi with positions into d_pos, and the
            // low words are gathered by the final positions into d_tkey
            gather_u64_kernel<<<blocks_for(nnz, T), T, 0, s>>>(d_hi, d_tpos, nnz, d_tkey);
            b = cub_b;
            e = hipcub::DeviceRadixSort::SortPairs(d_cub, b, d_tkey, d_hi, d_tpos, d_pos, (int)nnz, 0,
                                                   key_bits - 64, s);
            if (e != hipSuccess) break;
            gather_u64_kernel<<<blocks_for(nnz, T), T, 0, s>>>(d_key, d_pos, nnz, d_tkey);
            hi = d_hi;
            pos = d_pos;
        }
        DecodeOut out{};
        for (int j = 0; j < N - 1; ++j) out.idx[j] = sl.idx[j];
        out.narrow = sl.idx16 ? (1u << (N - 1)) - 1u : 0u;
        out.val = sl.val;
        decode_kernel<<<blocks_for(nnz_pad, T), T, 0, s>>>(lo, hi, pos, d_val, nnz, nnz_pad, kf, out);
        row_bits_kernel<<<blocks_for(nwords, T), T, 0, s>>>(lo, hi, nnz, nwords, kf, d_bits, d_cnt);
        b = cub_b;
        e = hipcub::DeviceScan::ExclusiveSum(d_cub, b, d_cnt, d_before, (int)nwords, s);
        if (e != hipSuccess) break;
        fill_u8_kernel<<<blocks_for(dims[n], T), T, 0, s>>>(d_flag, dims[n], 1);
        row_lists_kernel<<<blocks_for(nwords, T), T, 0, s>>>(lo, hi, d_bits, d_before, nwords, kf, sl.winfo,
                                                            sl.rows, d_flag);
        // row counts: the scan's last entry plus the last word's count
        uint32_t tail[2] = {0, 0};
        e = hipMemcpyAsync(&tail[0], d_before + (nwords - 1), 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&tail[1], d_cnt + (nwords - 1), 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        const uint64_t nrows_nz = (uint64_t)tail[0] + tail[1];
        // empty rows, increasing, right after the nonempty ones
        b = cub_b;
        e = hipcub::DeviceSelect::Flagged(d_cub, b, hipcub::CountingInputIterator<uint32_t>(0), d_flag,
                                          sl.rows + nrows_nz, d_small, (int)dims[n], s);
        if (e != hipSuccess) break;
        uint32_t nempty = 0;
        e = hipMemcpyAsync(&nempty, d_small, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        if (nrows_nz + nempty != dims[n]) {   // cannot happen: a row is either present or not
            e = hipErrorUnknown;
            break;
        }

        d.nnz = nnz;
        d.nnz_pad = nnz_pad;
        d.nrows_nz = nrows_nz;
        d.nempty = nempty;
        d.n_in = N - 1;
        for (int j = 0; j < N - 1; ++j) {
            const int m = j < n ? j : j + 1;
            d.in_modes[j] = m;
            d.in_dims[j] = dims[m];
            d.idx[j] = sl.idx[j];
        }
        d.idx16 = sl.idx16;
        d.val = sl.val;
        d.winfo = sl.winfo;
        d.row_id = sl.rows;
        d.empty_rows = sl.rows + nrows_nz;

        if (n == 0) {
            // |X|^2 with duplicate coordinates merged (equal keys are adjacent)
            run_squares_kernel<<<blocks_for(nnz, T), T, 0, s>>>(lo, hi, sl.val, nnz, d_sq);
            b = cub_b;
            e = hipcub::DeviceReduce::Sum(d_cub, b, d_sq, (double*)d_small, (int)nnz, s);
            if (e == hipSuccess) e = hipMemcpyAsync(normX2, d_small, 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    }
    if (e == hipSuccess) e = hipGetLastError();
    // The scratch is released (or handed back) only once every kernel above is done.
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (!own) return e;
    const hipError_t ef = hipFree(base);
    return e != hipSuccess ? e : ef;
}

}  // namespace mk
