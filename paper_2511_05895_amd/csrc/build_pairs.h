// Host-side construction of the merged arc-pair layout (bi-directional CSR).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace mf {

struct HostPairs {
    int32_t n = 0;
    int64_t m = 0;
    int32_t A = 0;
    std::vector<int32_t> row_ptr;   // n+1
    std::vector<int32_t> col;       // A
    std::vector<int32_t> twin;      // A
    std::vector<int32_t> cap;       // A
    std::vector<int32_t> edge2arc;  // m, -1 for self-loops
    int32_t max_pair_mult = 1;      // most input edges sharing one arc pair
};

// Argument checks of one graph: n >= 2, s and t distinct and in range,
// row_ptr non-decreasing from 0 to m < 2^31-1, col in [0, n), cap >= 0.
// Returns 0, or -1 with *err set.
int check_graph(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *cap,
                int32_t s, int32_t t, std::string *err);

// Per-edge capacity limit of a layout whose busiest arc pair merges `mult`
// input edges: after the deltas of one batch land, an arc's residual is at
// most twice the pair's capacity sum, which must fit int32.
int64_t edge_cap_limit(int32_t mult);

// Inputs must already be validated (row_ptr monotone 0..m, col in range,
// cap >= 0).  Returns 0, or -1 with *err set.
int build_pairs(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *cap,
                HostPairs *out, std::string *err);

}  // namespace mf
