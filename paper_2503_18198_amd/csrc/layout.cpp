// Host construction of the mode-specific copies (Sec. III-B scheme 2 order,
// Sec. III-C COO copies).  Runs once per tensor: per mode, a stable radix sort
// of packed coordinate keys, one pass per 11 key bits.
#include "layout.h"

#include <sched.h>

#include <algorithm>
#include <queue>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <utility>

#include "mttkrp.h"

namespace mk {

int host_threads()
{
    int n = 0;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
    if (n <= 0) n = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 32));
}

namespace {

// Host worker threads shared by every layout build in the process.  A caller
// queues its tasks, runs the first itself and then runs queued tasks (its own
// or a concurrent caller's) until all of its own have finished, so builds on
// several caller threads share the workers and none waits idle on another's.
class TaskPool {
public:
    static TaskPool& instance()
    {
        static TaskPool* pool = new TaskPool(host_threads() - 1);   // lives until the process ends
        return *pool;
    }

    void run(int ntasks, const std::function<void(int)>& f)
    {
        if (ntasks <= 1 || workers_.empty()) {
            for (int i = 0; i < ntasks; ++i) f(i);
            return;
        }
        std::atomic<int> left(ntasks);
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (int i = 1; i < ntasks; ++i) queue_.push_back(Task{&f, i, &left});
        }
        work_cv_.notify_all();
        f(0);
        finish(left);
        while (left.load(std::memory_order_acquire) > 0) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (queue_.empty()) {
                    done_cv_.wait(lk, [&] { return left.load(std::memory_order_acquire) == 0 || !queue_.empty(); });
                    continue;
                }
                t = queue_.front();
                queue_.pop_front();
            }
            (*t.f)(t.i);
            finish(*t.left);
        }
    }

private:
    struct Task {
        const std::function<void(int)>* f = nullptr;
        int i = 0;
        std::atomic<int>* left = nullptr;
    };

    explicit TaskPool(int nworkers)
    {
        for (int w = 0; w < nworkers; ++w) workers_.emplace_back([this] { work(); });
        for (auto& t : workers_) t.detach();
    }

    void finish(std::atomic<int>& left)
    {
        if (left.fetch_sub(1, std::memory_order_acq_rel) == 1) {
            std::lock_guard<std::mutex> lk(mu_);   // the waiting caller checks `left` under this lock
            done_cv_.notify_all();
        }
    }

    void work()
    {
        for (;;) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu_);
                work_cv_.wait(lk, [&] { return !queue_.empty(); });
                t = queue_.front();
                queue_.pop_front();
            }
            (*t.f)(t.i);
            finish(*t.left);
        }
    }

    std::mutex mu_;
    std::condition_variable work_cv_, done_cv_;
    std::deque<Task> queue_;
    std::vector<std::thread> workers_;
};

// Chunks of at least 32K items, at most one per thread.
int chunks_for(uint64_t n, int threads)
{
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)std::max(threads, 1), n >> 15));
}

// Chunk t of `chunks` equal ranges of [0, n); the same split in every call.
void parallel_chunks(uint64_t n, int chunks, const std::function<void(int, uint64_t, uint64_t)>& f)
{
    TaskPool::instance().run(chunks, [&](int t) {
        f(t, n * (uint64_t)t / (uint64_t)chunks, n * (uint64_t)(t + 1) / (uint64_t)chunks);
    });
}

void parallel_for(uint64_t n, int threads, const std::function<void(uint64_t, uint64_t)>& f)
{
    parallel_chunks(n, chunks_for(n, threads), [&](int, uint64_t lo, uint64_t hi) { f(lo, hi); });
}

// Split rows [0, I) into `threads` ranges of about equal nonzero count.
void parallel_rows(const std::vector<uint64_t>& start, int threads,
                   const std::function<void(uint64_t, uint64_t)>& f)
{
    const uint64_t I = start.size() - 1;
    const uint64_t nnz = start[I];
    const int T = chunks_for(nnz, threads);
    std::vector<uint64_t> cut(T + 1, I);
    cut[0] = 0;
    for (int t = 1; t < T; ++t) {
        const uint64_t target = nnz * (uint64_t)t / (uint64_t)T;
        cut[t] = (uint64_t)(std::upper_bound(start.begin(), start.end(), target) - start.begin()) - 1;
        cut[t] = std::max(cut[t], cut[t - 1]);
    }
    TaskPool::instance().run(T, [&](int t) {
        if (cut[t + 1] > cut[t]) f(cut[t], cut[t + 1]);
    });
}

int bits_for(uint32_t d)
{
    int b = 0;
    while ((1ull << b) < (uint64_t)d) ++b;
    return b;
}

// Stable least-significant-digit radix sort of (key, pos) pairs on the low
// `bits` bits of the keys, 11 bits per pass, ping-ponging between the two
// buffer pairs.  A pass whose digit is the same for every key is skipped.
// Stability keeps equal keys in input order.  Returns true when the sorted
// pairs end in (tkey, tpos).
template <class K>
bool radix_sort_pairs(K* key, uint32_t* pos, K* tkey, uint32_t* tpos, uint64_t n, int bits, int threads)
{
    constexpr int kDigit = 11;   // 2048 buckets: fewer passes than bytes, histograms still in L1
    constexpr uint32_t kBuckets = 1u << kDigit;
    const int T = chunks_for(n, threads);
    std::vector<uint64_t> hist((size_t)T * kBuckets);
    bool swapped = false;
    for (int shift = 0; shift < bits; shift += kDigit) {
        parallel_chunks(n, T, [&](int t, uint64_t lo, uint64_t hi) {
            uint64_t* h = &hist[(size_t)t * kBuckets];
            std::fill(h, h + kBuckets, 0);
            for (uint64_t k = lo; k < hi; ++k) h[(uint32_t)(key[k] >> shift) & (kBuckets - 1)]++;
        });
        bool constant = false;
        uint64_t run = 0;
        for (uint32_t d = 0; d < kBuckets; ++d) {
            uint64_t tot = 0;
            for (int t = 0; t < T; ++t) {
                const uint64_t c = hist[(size_t)t * kBuckets + d];
                hist[(size_t)t * kBuckets + d] = run + tot;
                tot += c;
            }
            if (tot == n) constant = true;
            run += tot;
        }
        if (constant) continue;
        parallel_chunks(n, T, [&](int t, uint64_t lo, uint64_t hi) {
            uint64_t* o = &hist[(size_t)t * kBuckets];
            for (uint64_t k = lo; k < hi; ++k) {
                const uint64_t dst = o[(uint32_t)(key[k] >> shift) & (kBuckets - 1)]++;
                tkey[dst] = key[k];
                tpos[dst] = pos[k];
            }
        });
        std::swap(key, tkey);
        std::swap(pos, tpos);
        swapped = !swapped;
    }
    return swapped;
}

// Order of one mode copy by a packed integer key: the output index in the
// top bits, then the other indices in cyclic order.  Sorted stably from the
// input order, equal coordinates keep their input order.  Fills start (row
// starts), out.idx (decoded from the keys), out.val and out.src_pos.
template <class K>
void sort_by_packed_key(const uint32_t* coo, const float* vals, uint64_t nnz, const uint32_t* dims, int N, int n,
                        const std::vector<int>& cyc, int threads, const std::vector<HotSet>* hot, bool keep_src_pos,
                        BuildScratch& sc, std::vector<uint64_t>& start, HostMode& out)
{
    const uint64_t I = dims[n];
    const int nf = (int)cyc.size();
    std::vector<int> fbits(nf), fshift(nf), fslot(nf);
    int below = 0;
    for (int f = nf - 1; f >= 0; --f) {
        fbits[f] = bits_for(dims[cyc[f]]);
        fshift[f] = below;
        below += fbits[f];
        fslot[f] = cyc[f] < n ? cyc[f] : cyc[f] - 1;   // position among the increasing input modes
    }
    const int row_bits = bits_for(dims[n]);
    const int row_shift = below;
    if (sc.key.size() < nnz) {
        sc.key.resize(nnz);
        sc.tkey.resize(nnz);
        sc.pos.resize(nnz);
        sc.tpos.resize(nnz);
    }
    K* key = reinterpret_cast<K*>(sc.key.data());
    K* tkey = reinterpret_cast<K*>(sc.tkey.data());
    uint32_t* pos = sc.pos.data();
    uint32_t* tpos = sc.tpos.data();
    parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t k = lo; k < hi; ++k) {
            const uint32_t* p = coo + k * N;
            K v = (K)p[n];
            for (int f = 0; f < nf; ++f) v = fbits[f] ? ((v << fbits[f]) | (K)p[cyc[f]]) : v;
            key[k] = v;
            pos[k] = (uint32_t)k;
        }
    });
    if (radix_sort_pairs(key, pos, tkey, tpos, nnz, row_shift + row_bits, threads)) {
        std::swap(key, tkey);
        std::swap(pos, tpos);
    }

    auto row_of = [&](uint64_t k) -> uint64_t { return row_bits ? (uint64_t)(key[k] >> row_shift) : 0; };
    start.assign(I + 1, nnz);
    const bool use_hot = hot && !hot->empty() && !(*hot)[0].slot.empty();
    parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t k = lo; k < hi; ++k) {
            // rows from just after the previous nonzero's row up to this one start here
            const uint64_t r = row_of(k);
            for (uint64_t i = k ? row_of(k - 1) + 1 : 0; i <= r; ++i) start[i] = k;
            for (int f = 0; f < nf; ++f) {
                const uint32_t mask = fbits[f] ? (uint32_t)((1ull << fbits[f]) - 1) : 0u;
                const uint32_t v = (uint32_t)(key[k] >> fshift[f]) & mask;
                const int32_t sl = use_hot ? (*hot)[cyc[f]].slot[v] : -1;
                out.idx[fslot[f]][k] = sl >= 0 ? (kHotBit | (uint32_t)sl) : v;
            }
            out.val[k] = vals[pos[k]];
            if (keep_src_pos) out.src_pos[k] = pos[k];
        }
    });
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
    // the first offending nonzero, found by chunks in parallel
    const int T = chunks_for(nnz, host_threads());
    std::vector<uint64_t> bad(T, nnz);
    parallel_chunks(nnz, T, [&](int t, uint64_t lo, uint64_t hi) {
        for (uint64_t k = lo; k < hi && bad[t] == nnz; ++k)
            for (int m = 0; m < N; ++m)
                if (coo[k * (uint64_t)N + m] >= dims[m]) {
                    bad[t] = k;
                    break;
                }
    });
    const uint64_t k = *std::min_element(bad.begin(), bad.end());
    if (k == nnz) return "";
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
    if (k == 0) return hs;   // empty slot tables: no row is hot
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
                     bool keep_src_pos, int threads, const std::vector<HotSet>* hot, HostMode& out,
                     BuildScratch* scratch)
{
    const int n = mode;
    const uint64_t I = dims[n];
    out.mode = n;
    out.in_modes.clear();
    for (int m = 0; m < N; ++m)
        if (m != n) out.in_modes.push_back(m);
    const int n_in = N - 1;
    out.nnz = nnz;
    out.nnz_pad = (nnz + 31) / 32 * 32;
    // Buffers keep their capacity from an earlier mode; only the padding is cleared.
    out.idx.resize(n_in);
    for (auto& v : out.idx) {
        v.resize(out.nnz_pad);
        std::fill(v.begin() + nnz, v.end(), 0u);
    }
    out.val.resize(out.nnz_pad);
    std::fill(out.val.begin() + nnz, out.val.end(), 0.0f);
    out.src_pos.resize(keep_src_pos ? nnz : 0);
    out.row_id.clear();
    out.empty_rows.clear();
    out.part_range.clear();
    out.step_P = 0;
    out.nsteps = 0;

    std::vector<int> cyc;
    for (int j = 1; j < N; ++j) cyc.push_back((n + j) % N);
    int key_bits = bits_for(dims[n]);
    for (int m : cyc) key_bits += bits_for(dims[m]);
    std::vector<uint64_t> start;
    if (key_bits <= 128) {
        // 1-3. Radix sort of packed (row, cyclic others) keys; indices decoded from the keys.
        BuildScratch local;
        BuildScratch& sc = scratch ? *scratch : local;
        if (key_bits <= 64)
            sort_by_packed_key<uint64_t>(coo, vals, nnz, dims, N, n, cyc, threads, hot, keep_src_pos, sc, start, out);
        else
            sort_by_packed_key<unsigned __int128>(coo, vals, nnz, dims, N, n, cyc, threads, hot, keep_src_pos, sc,
                                                  start, out);
    } else {
        // 1. Stable counting sort by output index: rows in increasing order,
        //    caller's order inside each row.
        start.assign(I + 1, 0);
        for (uint64_t k = 0; k < nnz; ++k) start[coo[k * N + n] + 1]++;
        for (uint64_t i = 0; i < I; ++i) start[i + 1] += start[i];
        std::vector<uint32_t> perm(nnz);
        {
            std::vector<uint64_t> fill(start.begin(), start.end() - 1);
            for (uint64_t k = 0; k < nnz; ++k) perm[fill[coo[k * N + n]]++] = (uint32_t)k;
        }
        // 2. Inside each row: by the other indices in cyclic order, then by input position.
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
        // 3. Structure-of-arrays copy gathered from the caller's coordinates.
        const bool use_hot = hot && !hot->empty() && !(*hot)[0].slot.empty();
        parallel_for(nnz, threads, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t k = lo; k < hi; ++k) {
                const uint64_t p = perm[k];
                for (int j = 0; j < n_in; ++j) {
                    const int m = out.in_modes[j];
                    const uint32_t v = coo[p * N + m];
                    const int32_t sl = use_hot ? (*hot)[m].slot[v] : -1;
                    out.idx[j][k] = sl >= 0 ? (kHotBit | (uint32_t)sl) : v;
                }
                out.val[k] = vals[p];
                if (keep_src_pos) out.src_pos[k] = p;
            }
        });
    }

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

std::vector<uint32_t> lpt_assign(const uint64_t* load, uint64_t nrows, uint32_t kappa, std::vector<uint64_t>* part_load)
{
    std::vector<uint32_t> order(nrows);
    for (uint64_t i = 0; i < nrows; ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return load[a] > load[b]; });
    // Min-heap of (load, partition): the least-loaded partition, lowest index on ties.
    using Slot = std::pair<uint64_t, uint32_t>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (uint32_t p = 0; p < kappa; ++p) heap.push({0, p});
    std::vector<uint32_t> part(nrows, 0);
    std::vector<uint64_t> pl(kappa, 0);
    for (uint32_t r : order) {
        Slot s = heap.top();
        heap.pop();
        part[r] = s.second;
        s.first += load[r];
        pl[s.second] = s.first;
        heap.push(s);
    }
    if (part_load) *part_load = std::move(pl);
    return part;
}

uint64_t lpt_extra_bytes(int N, uint32_t kappa)
{
    // up to 31 gap entries per partition (N-1 indices and a value each), their
    // row-start words, and the partition table
    return (uint64_t)kappa * (31ull * 4ull * (uint64_t)N + 8ull) + 16ull * kappa + 256ull;
}

void lpt_regroup(HostMode& hm, uint32_t kappa)
{
    std::vector<uint64_t>& part_range = hm.part_range;
    const uint64_t nrows = hm.nrows_nz;
    const int n_in = (int)hm.idx.size();
    // Row extents in the sorted copy (ordinal order = increasing row).
    std::vector<uint64_t> beg(nrows + 1, hm.nnz);
    {
        uint64_t o = 0;
        for (uint64_t k = 0; k < hm.nnz; ++k)
            if ((hm.winfo[2 * (k / 32)] >> (k % 32)) & 1u) beg[o++] = k;
    }
    std::vector<uint64_t> len(nrows);
    for (uint64_t o = 0; o < nrows; ++o) len[o] = beg[o + 1] - beg[o];
    std::vector<uint64_t> pl;
    const std::vector<uint32_t> part = lpt_assign(len.data(), nrows, kappa, &pl);
    // Partition starts, each at a multiple of 32.
    part_range.assign(2 * (uint64_t)kappa, 0);
    uint64_t pos = 0;
    for (uint32_t p = 0; p < kappa; ++p) {
        part_range[2 * p] = pos;
        part_range[2 * p + 1] = pl[p];
        pos = (pos + pl[p] + 31) / 32 * 32;
    }
    const uint64_t total = pos < 32 ? 32 : pos;
    // Rows of each partition in increasing row order.
    std::vector<std::vector<uint32_t>> rows_of(kappa);
    for (uint64_t o = 0; o < nrows; ++o) rows_of[part[o]].push_back((uint32_t)o);
    std::vector<buf<uint32_t>> idx(n_in);
    for (auto& v : idx) v.assign(total, 0u);
    buf<float> val;
    val.assign(total, 0.0f);
    const bool keep_src = !hm.src_pos.empty();
    buf<uint64_t> src;
    if (keep_src) src.assign(total, ~0ull);
    std::vector<uint32_t> row_id;
    row_id.reserve(nrows);
    std::vector<uint32_t> winfo(2 * (total / 32), 0u);
    for (uint32_t p = 0; p < kappa; ++p) {
        uint64_t w = part_range[2 * p];
        for (uint32_t o : rows_of[p]) {
            winfo[2 * (w / 32)] |= 1u << (w % 32);
            row_id.push_back(hm.row_id[o]);
            for (int j = 0; j < n_in; ++j)
                std::copy(hm.idx[j].begin() + beg[o], hm.idx[j].begin() + beg[o + 1], idx[j].begin() + w);
            std::copy(hm.val.begin() + beg[o], hm.val.begin() + beg[o + 1], val.begin() + w);
            if (keep_src) std::copy(hm.src_pos.begin() + beg[o], hm.src_pos.begin() + beg[o + 1], src.begin() + w);
            w += len[o];
        }
    }
    // Ordinal of the row holding each word's first entry (gap entries count
    // with the row before them; no partition covers them).
    uint64_t before = 0;
    for (uint64_t wd = 0; wd < total / 32; ++wd) {
        const uint32_t bits = winfo[2 * wd];
        winfo[2 * wd + 1] = (uint32_t)(before + (bits & 1u) - 1u);
        before += (uint64_t)__builtin_popcount(bits);
    }
    for (int j = 0; j < n_in; ++j) hm.idx[j] = std::move(idx[j]);
    hm.val = std::move(val);
    hm.winfo = std::move(winfo);
    hm.row_id = std::move(row_id);
    hm.nnz_pad = total;
    hm.src_pos = std::move(src);   // per position (gap entries: all ones)
}

uint32_t class_rank(uint32_t cls)
{
    // position of cls in the reflected Gray sequence: inverse Gray code
    uint32_t r = cls;
    for (uint32_t sh = 1; sh < 32; sh <<= 1) r ^= r >> sh;
    return r;
}

uint64_t step_copy_steps_bound(uint64_t nnz, uint64_t rows, uint32_t P)
{
    const uint64_t steps = (nnz + (uint64_t)(P - 1) * rows + P - 1) / P;
    return (steps + 31) / 32 * 32;
}

void build_step_copy(const HostMode& hm, uint32_t P, uint32_t nhot, int threads, StepCopy& out)
{
    const int n_in = (int)hm.idx.size();
    const uint64_t nrows = hm.nrows_nz;
    // Row extents of the sorted copy.
    std::vector<uint64_t> beg(nrows + 1, hm.nnz);
    {
        uint64_t o = 0;
        for (uint64_t w = 0; w < hm.nnz_pad / 32; ++w) {
            uint32_t bits = hm.winfo[2 * w];
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1;
                beg[o++] = w * 32 + (uint64_t)b;
            }
        }
    }
    // First step of every row.
    std::vector<uint64_t> sbeg(nrows + 1, 0);
    for (uint64_t o = 0; o < nrows; ++o) sbeg[o + 1] = sbeg[o] + (beg[o + 1] - beg[o] + P - 1) / P;
    out.P = P;
    out.nsteps = sbeg[nrows];
    out.nsteps_pad = (out.nsteps + 31) / 32 * 32;
    if (out.nsteps_pad == 0) out.nsteps_pad = 32;
    const uint64_t len = out.nsteps_pad * P;
    out.idx.resize(n_in);
    const uint32_t pad_coord = kHotBit | nhot;   // the zero row after the hot rows
    for (auto& v : out.idx) v.assign(len, pad_coord);
    out.val.assign(len, 0.0f);
    auto at = [&](uint64_t s, uint32_t e) { return (s / 32) * 32 * P + (uint64_t)e * 32 + s % 32; };
    parallel_for(nrows, threads, [&](uint64_t o0, uint64_t o1) {
        std::vector<std::pair<uint32_t, uint32_t>> key;   // (class rank, offset in the row)
        for (uint64_t o = o0; o < o1; ++o) {
            const uint64_t b = beg[o], n = beg[o + 1] - beg[o];
            key.resize(n);
            for (uint64_t k = 0; k < n; ++k) {
                uint32_t cls = 0;
                for (int j = 0; j < n_in; ++j)
                    if (!(hm.idx[j][b + k] & kHotBit)) cls |= 1u << j;
                key[k] = {class_rank(cls), (uint32_t)k};
            }
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<uint32_t, uint32_t>& x, const std::pair<uint32_t, uint32_t>& y) {
                                 return x.first < y.first;
                             });
            for (uint64_t k = 0; k < n; ++k) {
                const uint64_t src = b + key[k].second;
                const uint64_t dst = at(sbeg[o] + k / P, (uint32_t)(k % P));
                for (int j = 0; j < n_in; ++j) out.idx[j][dst] = hm.idx[j][src];
                out.val[dst] = hm.val[src];
            }
        }
    });
    // Per 32 steps: row-start bits and the ordinal of the row holding the first step.
    const uint64_t nw = out.nsteps_pad / 32;
    out.winfo.assign(2 * nw, 0u);
    for (uint64_t o = 0; o < nrows; ++o) out.winfo[2 * (sbeg[o] / 32)] |= 1u << (sbeg[o] % 32);
    uint64_t before = 0;
    for (uint64_t w = 0; w < nw; ++w) {
        const uint32_t bits = out.winfo[2 * w];
        out.winfo[2 * w + 1] = (uint32_t)(before + (bits & 1u) - 1u);
        before += (uint64_t)__builtin_popcount(bits);
    }
}

}  // namespace mk
