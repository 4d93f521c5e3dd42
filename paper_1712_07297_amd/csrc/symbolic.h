// Integer (symbolic) part of the hierarchical solver: cluster tree, block
// patterns, colouring, processing order and fill partners of every level.
// Everything here depends on the sparsity pattern and the grid only, never on
// the numerical values or on the ranks (fill is recorded structurally).
#pragma once

#include <cstdint>
#include <memory>
#include <new>
#include <utility>
#include <vector>

namespace hs {

// Allocator whose value construction leaves scalars uninitialised: resize(n)
// on a vector of it allocates without zeroing, so arrays that are written in
// full afterwards (on several host threads) are touched once, by the writers.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <class U, class... Args>
    void construct(U* p, Args&&... args) {
        ::new ((void*)p) U(std::forward<Args>(args)...);
    }
};
using ivec = std::vector<int, NoInitAlloc<int>>;
using i64vec = std::vector<int64_t, NoInitAlloc<int64_t>>;

struct LevelSymbolic {
    int ncl = 0;
    int ncolors = 0;
    ivec color;      // colour of every cluster
    ivec order;      // clusters by (colour, index)
    ivec pos;        // processing position of every cluster
    ivec color_ptr;  // order[color_ptr[c] .. color_ptr[c+1]) = colour c
    ivec adj_ptr, adj;    // neighbours n(s) at the level start (sorted)
    ivec fill_ptr, fill;  // fill partners w(s) when s is processed (by position)
    ivec pat_ptr, pat;    // block pattern after the level (incl. diagonal, sorted)

    // block id of (a, b) in the final pattern, -1 if absent
    int block_id(int a, int b) const;
};

struct Symbolic {
    int64_t n = 0;
    int depth = 0;
    int nlevels = 0;
    ivec leaf_ptr;      // leaf c holds leaf_dofs[leaf_ptr[c] .. leaf_ptr[c+1])
    i64vec leaf_dofs;   // ascending global ids per leaf (one system's analysis only)
    ivec cluster_of;    // leaf of every unknown
    ivec local_of;      // position of every unknown in its leaf
    std::vector<LevelSymbolic> levels;
};

// Build the whole symbolic analysis.  Returns 0 or a negative HS_ERR_* code.
int build_symbolic(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int nx, int ny, int nz,
                   int leaf, Symbolic& out);

// First level whose clusters all neighbour each other in processing order
// (factored densely; every later level of the system is empty).  The root
// level (one cluster) always qualifies.
int complete_level(const Symbolic& S);

// Several independent systems analysed as one block-diagonal system: a
// forest whose trees are the systems' cluster trees, all with their leaves
// on level 0.  Trees are placed by descending last level, so the systems
// present on a level are a prefix of the placement and the children of
// cluster p are 2p and 2p + 1 on every level.  Every per-system array
// (colours, processing order, neighbours, fill partners, pattern) is the
// system's own, shifted; the processing order of a colour lists the systems
// in placement order.  The combined analysis keeps leaf_ptr, cluster_of and
// local_of (leaf_dofs stays empty: nothing downstream reads it).
struct Forest {
    int nsys = 0;
    std::vector<int> sys;                  // placement -> system (caller's index)
    std::vector<int> last;                 // per placement: last level present
    std::vector<int> dense;                // per placement: complete level
    std::vector<int64_t> row_off;          // per system (caller's order): first unknown, nsys + 1 entries
    std::vector<std::vector<int>> cl_off;  // per level: first cluster of every present placement (+ end)
};
// parts[i] is system i's analysis (consumed).  With keep_empty_levels the
// levels after a system's complete level are kept (empty clusters), else
// each tree ends at its complete level.
void combine_symbolic(std::vector<Symbolic>& parts, bool keep_empty_levels, Symbolic& out, Forest& F);

}  // namespace hs
