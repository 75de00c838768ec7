// Host-side construction of the mode-specific tensor copies (Sec. III).
#pragma once

#include <stdint.h>

#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

namespace mk {

// An allocator that leaves trivially constructible elements uninitialised on
// resize, so large buffers are first touched by the threads that fill them
// instead of being zeroed by one thread.
template <class T>
struct UninitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <class U>
    UninitAlloc(const UninitAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept
    {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a)
    {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using buf = std::vector<T, UninitAlloc<T>>;

// One mode copy in host memory.  Nonzeros are ordered by (output index, then
// the other indices in cyclic order n+1, ..., N-1, 0, ..., n-1, then position
// in the caller's input), i.e. the hyperedges of the paper's hypergraph
// sorted by their output vertex (Sec. III-B, scheme 2), with a deterministic
// order inside each row.
struct HostMode {
    int mode = 0;
    std::vector<int> in_modes;                 // the N-1 input modes, increasing
    uint64_t nnz = 0, nnz_pad = 0, nrows_nz = 0, nempty = 0;
    std::vector<buf<uint32_t>> idx;            // [n_in][nnz_pad]
    buf<float> val;                            // [nnz_pad]
    std::vector<uint32_t> winfo;               // [2 * nnz_pad / 32]
    std::vector<uint32_t> row_id;              // [nrows_nz]
    std::vector<uint32_t> empty_rows;          // [nempty]
    buf<uint64_t> src_pos;                     // [nnz] (kept only on request)
    std::vector<uint64_t> part_range;          // scheme 1 only: {first position, nonzeros} per partition
    uint32_t step_P = 0;                       // hot-steps copy: entries per step (arrays hold steps, transposed)
    uint64_t nsteps = 0;
};

// Sort buffers of a build, kept across its modes so their pages are mapped once.
struct BuildScratch {
    buf<unsigned __int128> key, tkey;   // packed coordinate keys (64-bit keys use the first half)
    buf<uint32_t> pos, tpos;            // input positions carried with the keys
};

// Coordinates of rows served from the on-chip cache are stored as
// kHotBit | slot; slot indexes the hot-row table of that input mode.
constexpr uint32_t kHotBit = 0x80000000u;

// Per mode: the rows gathered most often (highest degree, at least 2, ties by
// row index), at most k of them, and for every row its slot or -1.
struct HotSet {
    std::vector<uint32_t> rows;   // slot -> row
    std::vector<int32_t> slot;    // row -> slot or -1
};

std::vector<HotSet> select_hot_rows(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N, uint32_t k);

// Host threads for layout builds: the CPUs this process may run on, at most 32.
int host_threads();

// Validate a COO tensor.  Returns an empty string when valid, else a message;
// *range_error is set when the failure is a coordinate out of range.
std::string validate_coo(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N, bool* range_error);

// Build the copy for output mode `mode` into `out`, reusing its buffers.
// `threads` host threads are used; `scratch` (may be null) is reused across calls.
void build_host_mode(const uint32_t* coo, const float* vals, uint64_t nnz, const uint32_t* dims, int N, int mode,
                     bool keep_src_pos, int threads, const std::vector<HotSet>* hot, HostMode& out,
                     BuildScratch* scratch = nullptr);

// Load balancing scheme 1 (Sec. III-B): whole output rows are dealt to kappa
// partitions by longest processing time first (Graham's rule, which meets the
// 4/3 bound the paper quotes): rows by decreasing nonzero count (ties: lower
// row first), each to the partition with the fewest nonzeros so far (ties:
// lower partition).  Returns the partition of every row; part_load (may be
// null) receives each partition's nonzeros.
std::vector<uint32_t> lpt_assign(const uint64_t* load, uint64_t nrows, uint32_t kappa,
                                 std::vector<uint64_t>* part_load);

// Regroup a copy for scheme 1: the rows of partition 0 in increasing row
// order, then those of partition 1, ...; each partition starts at a multiple
// of 32 (zero entries fill the gaps, covered by no partition).
// hm.part_range receives {first position, nonzeros} per partition; nnz_pad
// grows to the regrouped length, nnz and the empty rows are unchanged.
void lpt_regroup(HostMode& hm, uint32_t kappa);

// Bytes one mode copy may grow by when regrouped for kappa partitions.
uint64_t lpt_extra_bytes(int N, uint32_t kappa);

// A mode copy laid out in wave steps (the hot-steps layout): inside every
// output row the nonzeros are ordered by which of their input rows are hot
// (held in LDS; coordinates kHotBit | slot), all-hot first, then in the same
// cyclic index order as before; every row is padded with entries of value 0
// whose coordinates name the zero row kHotBit | nhot to a whole number of
// steps of P entries, so a step lies in one row and a wave can tell, for each
// input, whether all its lanes' rows are hot.  Storage is transposed per 32
// steps: entry e of step s sits at (s / 32) * 32 * P + e * 32 + s % 32, so
// the entries one lane group takes from 32 consecutive steps are contiguous.
struct StepCopy {
    uint32_t P = 0;                            // entries per step
    uint64_t nsteps = 0, nsteps_pad = 0;       // steps, and padded to a multiple of 32
    std::vector<buf<uint32_t>> idx;            // [n_in][nsteps_pad * P]
    buf<float> val;                            // [nsteps_pad * P]
    std::vector<uint32_t> winfo;               // per 32 steps: {row-start bits, ordinal of the row of the first}
};

// Order of a hot/cold class (bit j set: input j cold): reflected Gray code, so
// consecutive classes differ in one input.
uint32_t class_rank(uint32_t cls);

// Lay out a copy (built with hot sets) in steps of P entries.  Rows and their
// ordinals, empty rows and |X|^2 are those of hm.
void build_step_copy(const HostMode& hm, uint32_t P, uint32_t nhot, int threads, StepCopy& out);

// Steps of a step copy of a tensor whose mode has the given nonempty-row count,
// at most (bound used for footprints): ceil((nnz + (P - 1) * rows) / P) rounded up to 32.
uint64_t step_copy_steps_bound(uint64_t nnz, uint64_t rows, uint32_t P);

// Bytes of one mode copy on the device (arrays only, without alignment padding).
uint64_t mode_device_bytes(uint64_t nnz, int N, uint64_t I_mode);

}  // namespace mk
