// Host-side construction of the mode-specific tensor copies (Sec. III).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace mk {

// One mode copy in host memory.  Nonzeros are ordered by (output index, then
// the other indices in cyclic order n+1, ..., N-1, 0, ..., n-1, then position
// in the caller's input), i.e. the hyperedges of the paper's hypergraph
// sorted by their output vertex (Sec. III-B, scheme 2), with a deterministic
// order inside each row.
struct HostMode {
    int mode = 0;
    std::vector<int> in_modes;                 // the N-1 input modes, increasing
    uint64_t nnz = 0, nnz_pad = 0, nrows_nz = 0, nempty = 0;
    std::vector<std::vector<uint32_t>> idx;    // [n_in][nnz_pad]
    std::vector<float> val;                    // [nnz_pad]
    std::vector<uint32_t> winfo;               // [2 * nnz_pad / 32]
    std::vector<uint32_t> row_id;              // [nrows_nz]
    std::vector<uint32_t> empty_rows;          // [nempty]
    std::vector<uint64_t> src_pos;             // [nnz] (kept only on request)
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

// Validate a COO tensor.  Returns an empty string when valid, else a message;
// *range_error is set when the failure is a coordinate out of range.
std::string validate_coo(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N, bool* range_error);

// Build the copy for output mode `mode`.  `threads` host threads are used.
void build_host_mode(const uint32_t* coo, const float* vals, uint64_t nnz, const uint32_t* dims, int N, int mode,
                     bool keep_src_pos, int threads, const std::vector<HotSet>* hot, HostMode& out);

// Bytes of one mode copy on the device (arrays only, without alignment padding).
uint64_t mode_device_bytes(uint64_t nnz, int N, uint64_t I_mode);

}  // namespace mk
