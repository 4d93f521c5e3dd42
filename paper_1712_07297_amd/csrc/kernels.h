// Host-side launch interface of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device_common.h"

namespace hs {

// Work lists of one colour (device pointers).  Every cluster of the colour
// contributes its neighbour entries, fill entries and Schur output tiles; the
// kernels find their cluster by binary search over the prefix arrays.
struct ColourDev {
    int n = 0;                        // clusters in the colour
    const int* clist = nullptr;       // [n] clusters, processing order
    const int* nbr_pre = nullptr;     // [n+1] prefix of neighbour counts
    const int* fill_pre = nullptr;    // [n+1] prefix of fill-partner counts
    const int64_t* tile_pre = nullptr;// [n+1] prefix of Schur output tiles (capacity)
    int nbr_total = 0;
    int fill_total = 0;
    int64_t tile_total = 0;
    int panels = 0;                   // column panels per neighbour / partner block (capacity)
    int max_m = 0;                    // largest cluster of the colour
    int max_nbr_m = 0;                // largest neighbour or fill partner of a cluster of the colour
    int f32 = 0;                      // the clusters' blocks and records are float32 (else float64)
    // solve lists: the neighbours of every cluster cut into groups of
    // consecutive entries (one backward partial per group)
    const int* grp_pre = nullptr;     // [n+1] prefix of group counts
    const int* grp_e0 = nullptr;      // [grp_total] first neighbour entry of the group
    const int* grp_e1 = nullptr;      // [grp_total] one past its last entry
    int grp_total = 0;
    int fwd_split = 0;                // forward step in two launches (own products, then neighbour updates):
                                      // 1 always, 2 for at most split_nrhs_max right-hand sides
    int split_nrhs_max = 1;
    int max_nt = 0;                   // most neighbour rows (current sizes) of a cluster of the colour
    int apply_wave = 0;               // one right-hand side: own products one wave per cluster (m <= 128)
                                      // in colours of at least this many clusters (0: never)
};
// neighbour groups of the backward sweep: at most this many columns of E_R
// (unless one neighbour alone is wider) and this many entries
constexpr int SOLVE_GROUP_COLS = 256;
constexpr int SOLVE_GROUP_ENTRIES = 32;

// ---- factorization, one colour at a time
// with_offsets: the Gram launch also computes nbr_noff / ntot / fcols (one
// extra workgroup per cluster); otherwise launch_offsets computes them, before
// launch_pivot.
void launch_gram(const LevelDev& L, const ColourDev& C, hipStream_t st, bool with_offsets);
void launch_offsets(const LevelDev& L, const ColourDev& C, hipStream_t st);
// Truncated Householder QR with column pivoting of F^T (rank and P R_k^T)
// for the clusters of the colour that have fill; needs the offsets (fcols).
void launch_qrcp(const LevelDev& L, const ColourDev& C, hipStream_t st);
void launch_pivot(const LevelDev& L, const ColourDev& C, hipStream_t st);
void launch_fill_update(const LevelDev& L, const ColourDev& C, hipStream_t st);
void launch_nbr_update(const LevelDev& L, const ColourDev& C, hipStream_t st);
// both in one launch (they touch disjoint blocks)
void launch_fill_nbr_update(const LevelDev& L, const ColourDev& C, hipStream_t st);
// column panel width used by the fill / neighbour updates for clusters up to max_m
int panel_width(int max_m);
void launch_schur(const LevelDev& L, const ColourDev& C, hipStream_t st);

// ---- level set-up
// Scatter the CSR values into the level-0 block store.
// Blocks of cluster c are float32 where f32[c] != 0, else float64.
void launch_assemble0(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                      const int* cluster_of, const int* local_of, const int* m, const int* pat_ptr, const int* pat,
                      const int64_t* blk_off, void* blocks, const int* f32, hipStream_t st);
// Gather the coarse blocks of the children into the parent level: parent
// block b = (P, Q) of the next level's pattern takes the children's blocks
// (2P + i, 2Q + j) found in the previous level's pattern.  Element types per
// cluster on either side (f32_prev / f32_next).
void launch_merge(int nblk_next, const int* pat_ptr_next, const int* pat_next, int ncl_next,
                  const int* pat_ptr_prev, const int* pat_prev, int ncl_prev, const int* k_prev, const int* m_prev,
                  const int64_t* blk_off_prev, const void* blocks_prev, const int* f32_prev, const int* m_next,
                  const int64_t* blk_off_next, void* blocks_next, const int* f32_next, hipStream_t st);
// Per level: block ids of (s, s), (s, a), (a, s), (s, t), (t, s) for the
// neighbours a and fill partners t of every cluster, and their
// processed-before flags (pos = processing position).
void launch_level_ids(int ncl, const int* nbr_ptr, const int* nbr_id, const int* fill_ptr, const int* fill_id,
                      const int* pos, const int* pat_ptr, const int* pat, int* diag_blk, int* nbr_before,
                      int* nbr_bsa, int* nbr_bas, int* fill_before, int* fill_bst, int* fill_bts, hipStream_t st);
// Zero `bytes` bytes (a multiple of 4) from p.
void launch_fill_zero(void* p, int64_t bytes, hipStream_t st);
// System i's CSR copied into a block-diagonal one: its n_i + 1 row pointers
// (from 0) are shifted by nnz_off and its column indices by row_off.
void launch_shift_csr(int64_t n_i, int64_t nnz_i, int64_t row_off, int64_t nnz_off, int64_t* row_ptr,
                      int32_t* col_idx, hipStream_t st);
// pair_blk[pair_base[s] + i nb + j] = block id of (a_i, a_j) for the
// neighbours a_0 .. a_{nb-1} of every cluster s (binary search in the level's
// block pattern pat_ptr / pat).
void launch_pair_blocks(int ncl, const int* nbr_ptr, const int* nbr_id, const int* pat_ptr, const int* pat,
                        const int64_t* pair_base, int* pair_blk, hipStream_t st);
// Dense level (complete cluster graph): assemble D (N x N, ld N) from the
// block store, unpivoted blocked LU in place, per-cluster operators into the
// records, with panels of `panel` columns (16..128).  inv: 2 * 128 * 128
// doubles of workspace; flag: device int, set to 1 on a zero or non-finite
// pivot.
// The clusters are c0 .. c0 + ncl - 1 of the level (one system); their blocks
// are pattern entries b0 .. b0 + nblk - 1; m, off, ncap, rec_off point at
// cluster c0's entry; m_host / off_host are local to the range.
int dense_level_factor(double* D, int64_t N, const int* pat_ptr, const int* pat, int c0, int b0, const int* m,
                       const int64_t* off, const int64_t* blk_off, const double* blocks, int ncl, int nblk,
                       double* inv, int* flag, const int* ncap, const int64_t* rec_off, double* rec,
                       const std::vector<int>& m_host, const std::vector<int64_t>& off_host, int panel,
                       hipStream_t st);

// ---- solve (Alg. 2)
struct SolveLevelDev {
    int ncl;
    const int* m;
    const int* k;
    const int* nbr_ptr;
    const int* nbr_id;
    const int* nbr_before;
    const int* nbr_noff;
    const int* ntot;
    const int* ncap;
    const int64_t* rec_off;
    const double* rec;   // records: float64, or float32 for the clusters of a float32 list
    const int64_t* seg;  // [ncl+1] offset of every cluster segment (units of unknowns)
};
// z_s = T_L' y_s for the clusters of a colour (deferred: z_s = y_s)
void launch_apply_fwd_t(const SolveLevelDev& S, const ColourDev& C, const double* y, double* z, int nrhs,
                        hipStream_t st);
// both steps above in one launch (when their LDS fits), bit for bit the same
void launch_apply_fwd(const SolveLevelDev& S, const ColourDev& C, double* y, double* z, int nrhs, hipStream_t st);
// neighbours: y_a (or z_a's coarse part) -= E_L[a] z_s[:f]
void launch_apply_fwd_u(const SolveLevelDev& S, const ColourDev& C, double* y, double* z, int nrhs, int max_m,
                        hipStream_t st);
// part[g] = sum over the neighbours a of group g of E_R[:, a] x_a (current
// values); part_off per group in units of f (times nrhs)
void launch_apply_bwd_acc(const SolveLevelDev& S, const ColourDev& C, const double* z, const double* out,
                          double* part, const int64_t* part_off, int nrhs, hipStream_t st);
// out_s = T_R' [z_f - sum_g part[g]; z_c], the groups of s in order
void launch_apply_bwd_t(const SolveLevelDev& S, const ColourDev& C, const double* z, double* out,
                        const double* part, const int64_t* part_off, int nrhs, hipStream_t st);
// next-level y = coarse parts of z (parent = left child then right child)
void launch_to_coarse(const SolveLevelDev& S, const int64_t* seg_next, int ncl_next, const double* z, double* ynext,
                      int nrhs, hipStream_t st);
// coarse parts of z = next-level out
void launch_from_coarse(const SolveLevelDev& S, const int64_t* seg_next, int ncl_next, const double* outnext,
                        double* z, int nrhs, hipStream_t st);
// level-0 vector <-> global vector (cluster_of / local_of: leaf and position of every unknown)
void launch_scatter_rhs(int64_t n, const int* cluster_of, const int* local_of, const int64_t* seg, const int* m,
                        const double* B, int64_t ldb, double* y, int nrhs, hipStream_t st);
void launch_gather_sol(int64_t n, const int* cluster_of, const int* local_of, const int64_t* seg, const int* m,
                       const double* out, double* X, int64_t ldx, int nrhs, hipStream_t st);

// ---- Krylov building blocks (float64, n x nrhs column major).  A vector
// stacks the unknowns of independent systems; every per-system quantity is
// formed in an order fixed by that system alone: chunks of KRY_CHUNK rows
// counted from the system's first row, each reduced by one workgroup, chunk
// results added in chunk order.  Per-system scalars are indexed by the lane
// l = s + nsys * c (system s, column c).
constexpr int KRY_CHUNK = 4096;
struct SegDev {
    int nsys = 0;
    int nchunks = 0;
    const int64_t* row_off = nullptr;    // [nsys+1]
    const int* chunk_sys = nullptr;      // [nchunks]
    const int64_t* chunk_r0 = nullptr;   // [nchunks] first row of the chunk
    const int* sys_chunk0 = nullptr;     // [nsys+1] first chunk of every system
};
void launch_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val, const double* X,
                 int64_t ldx, double* Y, int64_t ldy, int nrhs, hipStream_t st);
// out[v * L + l] = sum over system s's rows i of a_v[i, c] b[i, c], with
// a_v = a + v * vstride (v < nvec) and L = nsys * nrhs; part holds
// nvec * nrhs * nchunks doubles.
void launch_sdots(const SegDev& G, int nvec, const double* a, int64_t vstride, int64_t lda, const double* b,
                  int64_t ldb, int nrhs, double* part, double* out, hipStream_t st);
// y[:, c] = alpha[l] x[:, c] + beta[l] y[:, c] on system s's rows (a zero
// coefficient never reads its operand)
void launch_saxpby(const SegDev& G, const double* alpha, const double* x, int64_t ldx, const double* beta, double* y,
                   int64_t ldy, int nrhs, hipStream_t st);
// y[:, c] = beta[l] y[:, c] + sum_{v < nvec} coef[v * L + l] a_v[:, c] (v ascending)
void launch_scomb(const SegDev& G, int nvec, const double* coef, const double* a, int64_t vstride, int64_t lda,
                  const double* beta, double* y, int64_t ldy, int nrhs, hipStream_t st);
// y = x - y (elementwise, n x nrhs)
void launch_xmy(int64_t n, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t st);
void launch_copy(int64_t n, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t st);

}  // namespace hs
