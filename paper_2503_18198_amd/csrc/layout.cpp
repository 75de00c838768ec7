// Host construction of the mode-specific copies (Sec. III-B scheme 2 order,
// Sec. III-C COO copies).  Runs once per tensor; O(nnz log(row length)) per mode.
#include "layout.h"

#include <algorithm>
#include <functional>
#include <numeric>
#include <thread>
#include <utility>

#include "mttkrp.h"

namespace mk {

namespace {

void parallel_for(uint64_t n, int threads, const std::function<void(uint64_t, uint64_t)>& f)
{
    if (threads <= 1 || n < (1u << 16)) {
        f(0, n);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(threads);
    for (int t = 0; t < threads; ++t) {
        const uint64_t lo = n * (uint64_t)t / (uint64_t)threads;
        const uint64_t hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
        ts.emplace_back(f, lo, hi);
    }
    for (auto& t : ts) t.join();
}

// Split rows [0, I) into `threads` ranges of about equal nonzero count.
void parallel_rows(const std::vector<uint64_t>& start, int threads,
                   const std::function<void(uint64_t, uint64_t)>& f)
{
    const uint64_t I = start.size() - 1;
    const uint64_t nnz = start[I];
    if (threads <= 1 || nnz < (1u << 16)) {
        f(0, I);
        return;
    }
    std::vector<uint64_t> cut(threads + 1, I);
    cut[0] = 0;
    for (int t = 1; t < threads; ++t) {
        const uint64_t target = nnz * (uint64_t)t / (uint64_t)threads;
        cut[t] = (uint64_t)(std::upper_bound(start.begin(), start.end(), target) - start.begin()) - 1;
        cut[t] = std::max(cut[t], cut[t - 1]);
    }
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
        if (cut[t + 1] > cut[t]) ts.emplace_back(f, cut[t], cut[t + 1]);
    for (auto& t : ts) t.join();
}

int bits_for(uint32_t d)
{
    int b = 0;
    while ((1ull << b) < (uint64_t)d) ++b;
    return b;
}

}  // namespace

std::string validate_coo(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N, bool* range_error)
{
    *range_error = false;
    if (N < 3 || N > MTTKRP_MAX_MODES) return "N must be between 3 and " + std::to_string(MTTKRP_MAX_MODES);
    if (!dims) return "dims is NULL";
    for (int m = 0; m < N; ++m)
        if (dims[m] == 0 || dims[m] > 0x7fffffffu)
            return "dims[" + std::to_string(m) + "] must be in [1, 2^31-1]";
    if (nnz >= (1ull << 32)) return "nnz must be below 2^32";
    if (nnz && !coo) return "coo_idx is NULL";
    for (uint64_t k = 0; k < nnz; ++k)
        for (int m = 0; m < N; ++m)
            if (coo[k * (uint64_t)N + m] >= dims[m]) {
                *range_error = true;
                return "nonzero " + std::to_string(k) + ": coordinate " + std::to_string(coo[k * (uint64_t)N + m]) +
                       " >= dims[" + std::to_string(m) + "] = " + std::to_string(dims[m]);
            }
    return "";
}

uint64_t mode_device_bytes(uint64_t nnz, int N, uint64_t I_mode)
{
    const uint64_t pad = (nnz + 31) / 32 * 32;
    return pad * (4ull * (N - 1) + 4ull) + (pad / 32) * 8ull + 4ull * I_mode;
}

std::vector<HotSet> select_hot_rows(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N, uint32_t k)
{
    std::vector<HotSet> hs(N);
    for (int m = 0; m < N; ++m) {
        std::vector<uint64_t> deg(dims[m], 0);
        for (uint64_t e = 0; e < nnz; ++e) deg[coo[e * N + m]]++;
        std::vector<uint32_t> cand;
        for (uint32_t i = 0; i < dims[m]; ++i)
            if (deg[i] >= 2) cand.push_back(i);
        const size_t take = std::min<size_t>(k, cand.size());
        std::partial_sort(cand.begin(), cand.begin() + take, cand.end(), [&](uint32_t a, uint32_t b) {
            return deg[a] != deg[b] ? deg[a] > deg[b] : a < b;
        });
        hs[m].rows.assign(cand.begin(), cand.begin() + take);
        hs[m].slot.assign(dims[m], -1);
        for (size_t j = 0; j < take; ++j) hs[m].slot[hs[m].rows[j]] = (int32_t)j;
    }
    return hs;
}

void build_host_mode(const uint32_t* coo, const float* vals, uint64_t nnz, const uint32_t* dims, int N, int mode,
                     bool keep_src_pos, int threads, const std::vector<HotSet>* hot, HostMode& out)
{
    const int n = mode;
    const uint64_t I = dims[n];
    out = HostMode{};
    out.mode = n;
    for (int m = 0; m < N; ++m)
        if (m != n) out.in_modes.push_back(m);
    const int n_in = N - 1;
    out.nnz = nnz;
    out.nnz_pad = (nnz + 31) / 32 * 32;

    // 1. Stable counting sort by output index: rows in increasing order,
    //    caller's order inside each row.
    std::vector<uint64_t> start(I + 1, 0);
    for (uint64_t k = 0; k < nnz; ++k) start[coo[k * N + n] + 1]++;
    for (uint64_t i = 0; i < I; ++i) start[i + 1] += start[i];
    std::vector<uint32_t> perm(nnz);
    {
        std::vector<uint64_t> fill(start.begin(), start.end() - 1);
        for (uint64_t k = 0; k < nnz; ++k) perm[fill[coo[k * N + n]]++] = (uint32_t)k;
    }

    // 2. Inside each row: by the other indices in cyclic order, then by input position.
    std::vector<int> cyc;
    for (int j = 1; j < N; ++j) cyc.push_back((n + j) % N);
    int total_bits = 0;
    for (int m : cyc) total_bits += bits_for(dims[m]);
    if (total_bits <= 64) {
        std::vector<std::pair<uint64_t, uint32_t>> rec(nnz);
        std::vector<int> sh;
        for (int m : cyc) sh.push_back(bits_for(dims[m]));
        parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t k = lo; k < hi; ++k) {
                const uint32_t* p = coo + (uint64_t)perm[k] * N;
                uint64_t key = 0;
                for (size_t j = 0; j < cyc.size(); ++j) key = (sh[j] ? (key << sh[j]) : key) | p[cyc[j]];
                rec[k] = {key, perm[k]};
            }
        });
        parallel_rows(start, threads, [&](uint64_t r0, uint64_t r1) {
            for (uint64_t i = r0; i < r1; ++i)
                if (start[i + 1] - start[i] > 1) std::sort(rec.begin() + start[i], rec.begin() + start[i + 1]);
        });
        parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t k = lo; k < hi; ++k) perm[k] = rec[k].second;
        });
    } else {
        parallel_rows(start, threads, [&](uint64_t r0, uint64_t r1) {
            for (uint64_t i = r0; i < r1; ++i) {
                if (start[i + 1] - start[i] < 2) continue;
                std::sort(perm.begin() + start[i], perm.begin() + start[i + 1], [&](uint32_t a, uint32_t b) {
                    const uint32_t* pa = coo + (uint64_t)a * N;
                    const uint32_t* pb = coo + (uint64_t)b * N;
                    for (int m : cyc)
                        if (pa[m] != pb[m]) return pa[m] < pb[m];
                    return a < b;
                });
            }
        });
    }

    // 3. Structure-of-arrays copy, zero padded to a multiple of 32.
    out.idx.assign(n_in, std::vector<uint32_t>(out.nnz_pad, 0u));
    out.val.assign(out.nnz_pad, 0.0f);
    if (keep_src_pos) out.src_pos.resize(nnz);
    parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t k = lo; k < hi; ++k) {
            const uint64_t p = perm[k];
            for (int j = 0; j < n_in; ++j) {
                const int m = out.in_modes[j];
                const uint32_t v = coo[p * N + m];
                const int32_t sl = hot ? (*hot)[m].slot[v] : -1;
                out.idx[j][k] = sl >= 0 ? (kHotBit | (uint32_t)sl) : v;
            }
            out.val[k] = vals[p];
            if (keep_src_pos) out.src_pos[k] = p;
        }
    });

    // 4. Nonempty rows (row ordinal -> output row) and empty rows.
    for (uint64_t i = 0; i < I; ++i) {
        if (start[i + 1] > start[i]) out.row_id.push_back((uint32_t)i);
        else out.empty_rows.push_back((uint32_t)i);
    }
    out.nrows_nz = out.row_id.size();
    out.nempty = out.empty_rows.size();

    // 5. Per 32 nonzeros: a bit per nonzero that starts a row, and the
    //    ordinal of the row holding the word's first nonzero.
    const uint64_t nwords = out.nnz_pad / 32;
    out.winfo.assign(2 * nwords, 0u);
    for (uint64_t i = 0; i < I; ++i)
        if (start[i + 1] > start[i]) out.winfo[2 * (start[i] / 32)] |= 1u << (start[i] % 32);
    uint64_t before = 0;
    for (uint64_t w = 0; w < nwords; ++w) {
        const uint32_t bits = out.winfo[2 * w];
        out.winfo[2 * w + 1] = (uint32_t)(before + (bits & 1u) - 1u);
        before += (uint64_t)__builtin_popcount(bits);
    }
}

}  // namespace mk
