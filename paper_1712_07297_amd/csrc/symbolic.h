// Integer (symbolic) part of the hierarchical solver: cluster tree, block
// patterns, colouring, processing order and fill partners of every level.
// Everything here depends on the sparsity pattern and the grid only, never on
// the numerical values or on the ranks (fill is recorded structurally).
#pragma once

#include <cstdint>
#include <vector>

namespace hs {

struct LevelSymbolic {
    int ncl = 0;
    int ncolors = 0;
    std::vector<int> color;      // colour of every cluster
    std::vector<int> order;      // clusters by (colour, index)
    std::vector<int> pos;        // processing position of every cluster
    std::vector<int> color_ptr;  // order[color_ptr[c] .. color_ptr[c+1]) = colour c
    std::vector<int> adj_ptr, adj;    // neighbours n(s) at the level start (sorted)
    std::vector<int> fill_ptr, fill;  // fill partners w(s) when s is processed (by position)
    std::vector<int> pat_ptr, pat;    // block pattern after the level (incl. diagonal, sorted)

    // block id of (a, b) in the final pattern, -1 if absent
    int block_id(int a, int b) const;
};

struct Symbolic {
    int64_t n = 0;
    int depth = 0;
    int nlevels = 0;
    std::vector<int> leaf_ptr;      // leaf c holds leaf_dofs[leaf_ptr[c] .. leaf_ptr[c+1])
    std::vector<int64_t> leaf_dofs; // ascending global ids per leaf
    std::vector<int> cluster_of;    // leaf of every unknown
    std::vector<int> local_of;      // position of every unknown in its leaf
    std::vector<LevelSymbolic> levels;
};

// Build the whole symbolic analysis.  Returns 0 or a negative HS_ERR_* code.
int build_symbolic(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int nx, int ny, int nz,
                   int leaf, Symbolic& out);

}  // namespace hs
