/*
 * hs.h -- C ABI of the hierarchical low-rank elimination solver for one AMD
 * MI355X (gfx950).
 *
 * The method is the sparse hierarchical factorization of Chen, Pouransari,
 * Rajamanickam, Boman and Darve, "A distributed-memory hierarchical solver for
 * general sparse linear systems" (arXiv 1712.07297):
 *   - Sec. 2.1: for every cluster s of unknowns, the fill blocks A_sw are
 *     compressed to tolerance eps (Eq. lra), the sparsification operator E_s
 *     (Eq. scaling) splits s into fine and coarse unknowns, the elimination
 *     operator G_s (Eq. elim) eliminates the fine unknowns with a Schur
 *     complement update of the neighbour blocks, and P_s (Eq. perm) moves the
 *     coarse unknowns last;
 *   - Alg. 1: all clusters of a level are processed, the coarse unknowns of
 *     sibling clusters form the next level, recursively;
 *   - Alg. 2: the factorization is applied by forward and backward
 *     substitution;
 *   - Sec. 5: it is used as a direct solver (small eps) or as a preconditioner
 *     for CG (symmetric positive definite A) or GMRES (general A).
 *
 * Conventions shared by every entry point:
 *   - Matrices are square, CSR with int64 row pointers, int32 column indices
 *     (sorted, unique within a row, in range) and float64 values.
 *   - Unknowns are the points of an nx*ny*nz grid, index x + nx*(y + ny*z),
 *     and the geometry is used to build the cluster tree (recursive
 *     bisection), or, with dim = 0, the graph of A is bisected instead.
 *   - Dense right-hand sides and solutions are column major, n rows, leading
 *     dimension >= n, float64.
 *   - Every function returns 0 on success, a negative HS_ERR_* code on error,
 *     or a positive HS_WARN_* code when the result is usable but incomplete.
 *     No function throws.  hs_last_error() returns a message for the calling
 *     thread's last failure.
 *   - "Device pointer" means memory allocated on the current HIP device;
 *     "host pointer" means ordinary host memory.  All work is ordered on the
 *     HIP stream passed in (NULL = the default stream); functions that return
 *     host-visible results (ranks, iteration counts) synchronise that stream.
 *   - The library allocates its own device memory (factor storage,
 *     workspaces) with HIP's stream-ordered allocator on the stream of the
 *     call (the device's default memory pool, whose release threshold it
 *     raises so that freed memory is kept for reuse rather than unmapped),
 *     unless hs_set_allocator() installs another allocator.  It never frees or writes caller buffers other than the
 *     documented outputs.
 */
#ifndef HS_H_
#define HS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define HS_OK 0
#define HS_ERR_ARG (-1)         /* null pointer, negative size, bad option */
#define HS_ERR_PATTERN (-2)     /* unsorted / duplicate / out-of-range CSR index */
#define HS_ERR_GEOMETRY (-3)    /* n != nx*ny*nz (dim 1..3), or dim outside 0..3 */
#define HS_ERR_BREAKDOWN (-4)   /* zero or non-finite pivot in an unpivoted LU */
#define HS_ERR_NOMEM (-5)       /* device allocation failed or above the cap */
#define HS_ERR_HIP (-6)         /* a HIP runtime call failed */
#define HS_ERR_UNSUPPORTED (-7) /* a cluster larger than the kernels support */
#define HS_ERR_NODEVICE (-8)    /* no gfx950 device visible */
#define HS_WARN_NOT_CONVERGED 1 /* Krylov solver hit maxit; X holds the last iterate */

/* ---- inputs ----------------------------------------------------------- */

/* Sparse matrix in CSR form.  All arrays are owned by the caller and only
 * read.  on_device = 0: host pointers; 1: device pointers. */
typedef struct hs_csr {
    int64_t n;
    int64_t nnz;
    const int64_t* row_ptr; /* n + 1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t* col_idx; /* nnz entries */
    const double* val;      /* nnz entries */
    int32_t on_device;
} hs_csr;

/* Grid of the unknowns (lexicographic, x fastest), dim = 1, 2 or 3: the
 * cluster tree bisects the grid box.  dim = 0: no grid (nx, ny, nz ignored);
 * the cluster tree bisects the graph of A + A^T instead (Alg. 1, "Partition
 * the graph of A"): every set is put in breadth-first order from a
 * pseudo-peripheral vertex (connected components by their lowest vertex,
 * neighbours in ascending order) and its first half forms the left child. */
typedef struct hs_geometry {
    int32_t dim;
    int32_t nx, ny, nz;
} hs_geometry;

#define HS_FP64 0  /* everything in float64 */
#define HS_MIXED 1 /* float32 storage of the fine levels' blocks and records,
                      Schur products on the bfloat16 units (three-part split,
                      float32 accumulation); float64 on the coarse levels and
                      in every Krylov vector */

/* Options of the factorization.
 *   eps         relative truncation tolerance of the fill compression
 *               (Eq. lra): a pivot R_jj of the rank-revealing QR (column
 *               pivoting over the unknowns of the cluster) is kept while
 *               |R_jj| > eps |R_11|.  eps = 0 selects the exact mode, in which
 *               a cluster with fill is passed whole to the next level.  Two
 *               routes compute that QR: for eps >= 1e-5 without a rank cap the
 *               pivoted Cholesky factorization of the Gram matrix F F^T (one
 *               pass over F; its pivots R_jj^2 carry an absolute rounding
 *               error near u |R_11|^2, u = 2^-53, so ratios |R_jj| / |R_11|
 *               are resolved to about u / (2 eps^2), 5e-7 at eps = 1e-5);
 *               below 1e-5, or with fixed_rank > 0, the Householder QR with
 *               column pivoting of F^T itself (resolved to about u / eps).
 *               hs_config_set("compression" / "qrcp_below_eps") moves the
 *               switch.
 *   fixed_rank  if > 0, additionally cap every rank at this value (the fixed
 *               rank K of Sec. 5.1).
 *   leaf_size   target number of unknowns per leaf cluster (> 0).
 *   precision   HS_FP64 or HS_MIXED.  In the mixed form the level blocks and
 *               factor records of a system's level are float32 when the
 *               level has more than coarse_fp64_dofs unknowns of that system
 *               and is not its complete (dense) level; the Schur update
 *               (Eq. elim) on those levels splits E_L and E_R into three
 *               bfloat16 parts each and accumulates the six products down to
 *               2^-24 in float32 on the matrix cores; the per-cluster dense
 *               algebra still runs in float64 registers; the result is a
 *               preconditioner for float64 CG / GMRES (Sec. 5).
 *   symmetric   1: A is symmetric (one-sided compression, V_R = V_L);
 *               0: general A (row and column fill compressed together);
 *               -1: detect from the values.
 *   coarse_fp64_dofs  mixed form only: a system's levels with at most this
 *               many unknowns keep float64 storage (0 selects 16384).
 *   pivoting    0: A_ss and F_ff are factored by LU without pivoting (the
 *               nonsymmetric counterpart of the Cholesky factor of Eq. elim);
 *               1: by LU with partial pivoting inside each cluster (P A = L U:
 *               at step j the lowest row at or below j whose |entry| is within
 *               1e-10 of the column's largest), for indefinite systems whose
 *               blocks have small or zero leading pivots (the extension to
 *               indefinite matrices of Sec. 6); the stored operators become
 *               L^{-1} P and U^{-1}.  Complete levels then run through the
 *               per-cluster kernels too (no dense level factorization), so
 *               every cluster must stay within the 512-unknown limit
 *               (HS_ERR_UNSUPPORTED otherwise).  Other values: HS_ERR_ARG. */
typedef struct hs_opts {
    double eps;
    int32_t fixed_rank;
    int32_t leaf_size;
    int32_t precision;
    int32_t symmetric;
    int32_t keep_levels; /* 1: keep a host copy of every level's starting matrix
                            (test hook, see hs_factor_level_matrix); 0: off */
    int32_t coarse_fp64_dofs;
    int32_t pivoting;
} hs_opts;

/* Opaque factorization; device resident; owned by the library until hs_free. */
typedef struct hs_factor_s* hs_factor_t;

/* Summary of a factorization (host struct filled by hs_factor_info). */
typedef struct hs_info {
    int32_t nlevels;
    int32_t ncolors_total;     /* colour batches over all levels */
    int64_t n;
    int64_t coarse_dofs[64];   /* unknowns left after each level (sum of ranks) */
    int32_t level_clusters[64];
    int32_t level_colors[64];
    int32_t max_cluster;       /* largest cluster size met */
    int32_t breakdown_level;   /* -1, or the level / cluster of a breakdown */
    int32_t breakdown_cluster;
    double factor_flops;       /* algorithmic flops of the factorization */
    double apply_flops_per_rhs;/* algorithmic flops of one forward+backward solve */
    double factor_bytes;       /* bytes of the stored factor records */
    double symbolic_seconds;   /* host time of the symbolic analysis */
    double numeric_seconds;    /* wall time of the numeric factorization */
    double device_bytes;       /* device memory the factorization holds now (records,
                                  metadata, its copy of A, solve / Krylov workspaces) */
    double peak_device_bytes;  /* largest device memory it has held (hs_factor's level
                                  block stores and workspaces included) */
} hs_info;

/* ---- entry points -------------------------------------------------------- */

/* Factor A (Alg. 1 with the low-rank elimination of Sec. 2.1).
 * A: host or device CSR (see hs_csr); geom: grid of the unknowns; opts: see
 * hs_opts.  On success *F_out receives a new factorization that keeps its own
 * device copy of A (for the Krylov solvers).  Synchronises the stream once per
 * level to size the next level (ranks decide the sizes).  The symbolic
 * analysis runs on the host: a device-resident pattern is copied through a
 * pinned host staging buffer that the library grows on demand (to 1.25 times
 * the largest pattern seen) and keeps until the process ends; a call that
 * finds it in use on another thread copies through pageable memory.
 * Errors: HS_ERR_ARG, HS_ERR_PATTERN, HS_ERR_GEOMETRY, HS_ERR_BREAKDOWN (the
 * failing level and cluster are in hs_factor_info of the partial factor,
 * which is then freed; *F_out is set to NULL), HS_ERR_NOMEM, HS_ERR_HIP,
 * HS_ERR_UNSUPPORTED (a cluster above the supported size). */
int hs_factor(const hs_csr* A, const hs_geometry* geom, const hs_opts* opts, void* hip_stream,
              hs_factor_t* F_out);

/* Factor nsys independent systems A[i] (grid geom[i]) together, as the one
 * block-diagonal system that stacks them in the given order (Alg. 1 on the
 * forest of their cluster trees, leaves of every system on level 0): each
 * kernel launch of a level and colour (Sec. 3.4) covers the clusters of
 * every system, and the stream is synchronised once per level of the
 * deepest system.  The result is one factorization of n = sum of the A[i].n
 * unknowns; hs_solve / hs_pcg / hs_gmres take right-hand sides that stack
 * the systems' rows in the same order, and the Krylov solvers keep one
 * recurrence and one stopping test per system and column.  Every system's
 * factor and Krylov numbers are those of hs_factor on that system alone
 * (the same kernels on the same data in the same order; the work of other
 * systems only shares the launches) whenever both take the same kernel
 * variants: a level that the batch's systems together crowd (at least
 * crowded_min clusters per colour, hs_config_set) takes the crowded variants,
 * which a lone system's sparser level may not, and the two then agree up to
 * rounding.  A batch containing a nonsymmetric system factors every system
 * in the general form when opts->symmetric is -1.  A[i] and geom[i] as for hs_factor (host and device
 * CSR may be mixed); nsys >= 1.  Errors as hs_factor, with the failing
 * system named in hs_last_error(). */
int hs_factor_batch(int32_t nsys, const hs_csr* A, const hs_geometry* geom, const hs_opts* opts,
                    void* hip_stream, hs_factor_t* F_out);

/* Systems of a factorization: *nsys (1 for hs_factor) and, if row_off is not
 * NULL, the first row of every system in the stacked vectors (host array of
 * nsys + 1 entries; row_off[nsys] = n). */
int hs_factor_systems(hs_factor_t F, int32_t* nsys, int64_t* row_off);

/* Apply the factorization once (Alg. 2): X = A_fac^{-1} B.
 * B, X: device pointers, n x nrhs column major with leading dimensions ldb,
 * ldx >= n; B is not modified; X may alias B only if ldx == ldb.  Stream
 * ordered, no synchronisation. */
int hs_solve(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
             void* hip_stream);

/* Allocation-free variant of hs_solve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, result and stream ordering as
 * hs_solve (X = A_fac^{-1} B, Alg. 2, the same kernels in the same order, so
 * the same numbers bit for bit), but the level vectors and partial sums of the
 * sweeps live in a fixed device array of the library instead of buffers it
 * allocates: 64 MiB (HS_NOALLOC_SCRATCH_BYTES) on every GPU the library runs
 * on, held from when the library's code is loaded on that GPU until the
 * process ends.  The call allocates and frees no device memory, launches its
 * kernels one by one on hip_stream (no graph of its own, no events) and does
 * not synchronise.  The first call with a device current looks up that
 * device's array (hipGetSymbolAddress); F must live on the current device.
 * Columns are processed in passes of as many as fit: one column needs
 * 8 (3 n_l summed over the levels + the largest backward-partial buffer + 1)
 * bytes, about 24 bytes per unknown for a 3D Poisson factorization.
 * Errors: HS_ERR_ARG as hs_solve; HS_ERR_NOMEM when one column does not fit
 * in the array (nothing is launched; hs_solve has no such limit).  Every call
 * on one GPU shares that GPU's array and leaves its contents behind (each
 * call writes everything it reads): calls that overlap in time on one GPU,
 * from other streams or threads, race and must be serialised by the caller. */
#define HS_NOALLOC_SCRATCH_BYTES (64u << 20)
int hs_solve_noalloc(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                     void* hip_stream);

/* Preconditioned conjugate gradients (symmetric positive definite A), one
 * recurrence per system and right-hand side (lane l = s + nsys * c), x0 = 0,
 * float64, preconditioner = the factorization (Sec. 5.1).  Iterates until
 * ||b - A x||_2 <= tol ||b||_2 on every lane (norms over the lane's system)
 * or maxit iterations; a lane that meets tol is left as it is.  With a mixed
 * factorization the flexible (Polak-Ribiere) beta is used.  B, X device
 * pointers as in hs_solve.  iters_out (host, may be NULL): iterations taken
 * (largest over the lanes); relres_out (host, nsys * nrhs entries, may be
 * NULL): final true relative residual of every lane.  Returns
 * HS_WARN_NOT_CONVERGED if some lane missed tol. */
int hs_pcg(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
           double tol, int32_t maxit, int32_t* iters_out, double* relres_out, void* hip_stream);

/* Right-preconditioned restarted GMRES(restart), x0 = 0, float64, for
 * general A (Sec. 5.2): the Krylov basis is orthonormalised by classical
 * Gram-Schmidt applied twice, one recurrence per lane as in hs_pcg, all lanes
 * advanced together; a lane whose residual estimate meets tol stops
 * extending its basis and updates x at the end of the cycle.  Same arguments
 * and stopping rule as hs_pcg (iters_out: inner iterations of the slowest
 * lane). */
int hs_gmres(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
             double tol, int32_t maxit, int32_t restart, int32_t* iters_out, double* relres_out,
             void* hip_stream);

/* Fill *out (host) with a summary of F. */
int hs_factor_info(hs_factor_t F, hs_info* out);

/* Copy the ranks (coarse sizes after elimination) of the clusters of one level
 * into ranks (host, room for hs_info.level_clusters[level] entries). */
int hs_factor_ranks(hs_factor_t F, int32_t level, int32_t* ranks);

/* Copy the cluster sizes at the start of a level (host array, as above). */
int hs_factor_sizes(hs_factor_t F, int32_t level, int32_t* sizes);

/* Copy one level's starting matrix, assembled densely in cluster order, to
 * out (host, column major, dim x dim with dim = sum of the level's sizes).
 * Needs opts.keep_levels = 1 at hs_factor time; HS_ERR_ARG otherwise. */
int hs_factor_level_matrix(hs_factor_t F, int32_t level, double* out, int64_t dim);

/* Copy one stored operator of cluster `cluster` at `level` to out (host,
 * column major, cap doubles available); *rows / *cols receive its shape.
 *   which = 0: T_L' = diag(L_f^{-1}, I) [V_L U]^T A_ss^{-1}      (m x m)
 *   which = 1: T_R' = A_ss^{-1} [V_R U] diag(U_f^{-1}, I)         (m x m)
 *   which = 2: E_R  = L_f^{-1} V_L^T A_ss^{-1} A_sn                (f x n_tot)
 *   which = 3: E_L  = A_ns A_ss^{-1} V_R U_f^{-1}                  (n_tot x f)
 * (Sec. 2.1: E_s of Eq. scaling folded with G_s of Eq. elim; a cluster
 * without fill has V = I, U empty, so T_L' = L^{-1}, T_R' = U^{-1}.)  A
 * cluster that kept all its unknowns (k = m) has no operator: shape 0 x 0.
 * Synchronises the device. */
int hs_factor_record(hs_factor_t F, int32_t level, int32_t cluster, int32_t which, double* out, int64_t cap,
                     int64_t* rows, int64_t* cols);

/* ---- symbolic analysis (host only, no device needed) ------------------ */

/* The integer part of the method: cluster tree by recursive bisection of the
 * grid (Alg. 1 "Partition the graph of A"), block pattern A_B per level
 * (Eq. quotient), distance-2 colouring and processing order (Sec. 3.4), and
 * the fill partners w(s) of every cluster (Sec. 2.3).  A must be a host CSR. */
typedef struct hs_symbolic_s* hs_symbolic_t;

int hs_symbolic_create(const hs_csr* A_host, const hs_geometry* geom, int32_t leaf_size,
                       hs_symbolic_t* S_out);
/* Number of levels and of clusters / colours of one level. */
int hs_symbolic_levels(hs_symbolic_t S, int32_t* nlevels);
int hs_symbolic_level(hs_symbolic_t S, int32_t level, int32_t* nclusters, int32_t* ncolors,
                      int64_t* nadj, int64_t* nfill, int64_t* npattern);
/* Leaf (level-0 cluster) of every unknown and position inside it (n each). */
int hs_symbolic_leaves(hs_symbolic_t S, int32_t* leaf_of_dof, int32_t* local_of_dof);
/* Per-level arrays (host, sized from hs_symbolic_level):
 *   colors[nclusters], order[nclusters] (processing order),
 *   adj_ptr[nclusters+1], adj[nadj]       neighbours at the level start,
 *   fill_ptr[nclusters+1], fill[nfill]    fill partners w(s) when s is processed,
 *   pat_ptr[nclusters+1], pat[npattern]   block pattern after the level (A_B^2).
 * Any pointer may be NULL. */
int hs_symbolic_arrays(hs_symbolic_t S, int32_t level, int32_t* colors, int32_t* order,
                       int32_t* adj_ptr, int32_t* adj, int32_t* fill_ptr, int32_t* fill,
                       int32_t* pat_ptr, int32_t* pat);
void hs_symbolic_free(hs_symbolic_t S);

/* ---- tracing ----------------------------------------------------------- */

/* Per-kernel-family timing with HIP events recorded on the stream of each
 * call (a tracing aid; off by default).  Kernel families: "gram", "pivot"
 * (pivot-block kernel on float64 levels), "pivot_f32" (on float32 levels,
 * mixed form), "fill", "nbr", "schur" (Schur updates of float64 levels),
 * "schur_f32" (Schur updates of float32 levels, mixed form), "merge",
 * "apply", "spmv", "dense".  While enabled, every launch of a family is
 * bracketed by two events; intervals are read back at the next
 * synchronisation of the library.  Host families (wall time of the
 * factorization's host steps, one count per step): "host_symbolic",
 * "host_plan" (per-level work lists and offsets), "host_upload",
 * "host_alloc", "host_sync" (the per-level rank read-back, which waits for
 * the level's kernels, and the wait before the children's blocks are freed),
 * "host_solve_plan".  hs_profile_read returns, for one family since the last
 * reset: launches, summed seconds, and the algorithmic bytes and flops of
 * those launches, counted from the sizes the kernels worked on (b = bytes per
 * stored element, 8 or 4):
 *   "schur", "schur_f32": per cluster 2 f n_tot^2 flops and
 *       b (2 f n_tot + 2 n_tot^2) bytes (Eq. elim);
 *   "pivot", "pivot_f32": per cluster with f > 0, 2/3 m^3 flops (LU of
 *       A_ss), plus with fill (0 < k < m) s (2 m^2 k + 4 m k f) + 2 m^2 f +
 *       2 m f^2 + 2/3 f^3 + 2 m k^2 (X = A_ss^{-1} U and the complement, once
 *       per side s = 1 or 2; A_ss^{-1} V; F_ff and its LU; C, Eqs. scaling and
 *       elim); bytes 3 b m^2 (A_ss read, T_L' and T_R' written), plus
 *       8 m^2 + b k^2 with fill (Gram matrix read, C written).
 * Unknown family: HS_ERR_ARG. */
int hs_profile_enable(int32_t enable);
/* Time only the listed families while profiling is on (comma-separated
 * names; NULL or "" = all).  Untimed launches run as without profiling (the
 * solve's level sweeps from their captured graph unless "apply" is timed).
 * Unknown name: HS_ERR_ARG. */
int hs_profile_select(const char* families);
int hs_profile_reset(void);
int hs_profile_read(const char* family, int64_t* launches, double* seconds, double* bytes, double* flops);

/* Release F's solve and Krylov work vectors (the next hs_solve / hs_pcg /
 * hs_gmres allocates them again), keeping the factorization itself; for a
 * resident factorization between uses.  Stream ordered on hip_stream. */
int hs_factor_trim(hs_factor_t F, void* hip_stream);

/* Release F and all its device memory.  NULL is ignored. */
void hs_free(hs_factor_t F);

/* ---- serving ------------------------------------------------------------ */

/* A request loop for a stream of solve requests on one GPU (the factorization
 * of Sec. 2 as preconditioner of CG / GMRES, Sec. 5), with continuous
 * batching: worker threads, each with its own HIP stream, take the oldest
 * waiting request and every other waiting request that fits with it, as long
 * as the device memory they need fits under the cap:
 *   - requests whose operator (op_key) has a resident factorization reuse it
 *     (only the Krylov solve runs);
 *   - new operators of the batch are factored together (hs_factor_batch),
 *     and the resulting factorization stays resident for later requests
 *     until it is evicted (least recently used, only when idle, only when
 *     memory is needed);
 *   - requests that arrive while others run are admitted as soon as a worker
 *     and the memory are free, so their work overlaps on the device.
 * Every result equals that of hs_factor (+ hs_pcg for symmetric operators,
 * hs_gmres(restart 30) otherwise) on the request alone: batched systems get
 * the same kernels in the same order and one Krylov recurrence per system
 * and column (up to rounding where the batch crowds a level that the lone
 * system does not, as for hs_factor_batch).  The memory of a new factorization is estimated as its
 * unknowns times the largest peak bytes per unknown seen so far for the same
 * grid dimension and precision (before the first: 16 KB / unknown), plus the
 * Krylov work vectors. */
typedef struct hs_server_s* hs_server_t;

typedef struct hs_server_opts {
    double hbm_cap_bytes;   /* device memory the server may hold: resident factors plus work
                               in flight (> 0) */
    int32_t workers;        /* batches in flight at once, one stream each (0: 2) */
    int32_t max_batch;      /* most requests in one batch (0: 32) */
    int32_t max_new_ops;    /* most new operators factored together (0: 8) */
} hs_server_opts;

typedef struct hs_result {
    int32_t status;         /* HS_OK, HS_WARN_NOT_CONVERGED, or the HS_ERR_* of the failing call */
    int32_t iterations;     /* Krylov iterations of the request's batch */
    double relres;          /* largest true relative residual over the request's columns */
    double latency_s;       /* submission to completion */
    double queue_s;         /* submission to the start of its batch */
    int32_t reused;         /* 1 if the operator's factorization was resident */
    int32_t batch_size;     /* requests in its batch */
} hs_result;

typedef struct hs_server_stats {
    int64_t submitted, completed, failed;
    int64_t batches;        /* batches started */
    int64_t reused;         /* requests served by a resident factorization */
    int64_t factored_ops;   /* operators factored */
    int64_t evictions;
    double p50_latency_s, p99_latency_s, mean_queue_s;
    double unknowns_per_s;  /* sum of n * nrhs over completed requests / span from the first
                               submission to the last completion */
    double requests_per_s;
    double held_bytes;      /* now: resident factors + reservations of running batches */
    double peak_held_bytes;
} hs_server_stats;

/* Start a server on the current HIP device. */
int hs_server_create(const hs_server_opts* opts, hs_server_t* S_out);

/* Queue one request: solve A X = B to relative residual tol (maxit
 * iterations at most).  op_key names the operator: requests with the same
 * key must pass the same matrix and options (the resident factorization is
 * reused without checking).  A, B, X: device or host CSR as hs_csr, B and X
 * device pointers, n x nrhs column major (ld n), caller-owned and untouched
 * by the caller until the request completes; opts->symmetric must be 0 or 1
 * (it selects GMRES or CG).  *ticket receives the request's id.  Errors:
 * HS_ERR_ARG (bad argument; nothing queued). */
int hs_submit(hs_server_t S, int64_t op_key, const hs_csr* A, const hs_geometry* geom, const hs_opts* opts,
              int32_t nrhs, const double* B, double* X, double tol, int32_t maxit, int64_t* ticket);

/* *done = 1 once the request has completed (its X written). */
int hs_poll(hs_server_t S, int64_t ticket, int32_t* done);

/* Block until the request completes; *out receives its result (may be NULL).
 * A ticket can be waited for once; afterwards it is unknown (HS_ERR_ARG). */
int hs_wait(hs_server_t S, int64_t ticket, hs_result* out);

/* Counters and latency percentiles over the completed requests. */
int hs_server_stats_get(hs_server_t S, hs_server_stats* out);

/* Finish every queued request, stop the workers, free the resident
 * factorizations.  NULL is ignored. */
void hs_server_destroy(hs_server_t S);

/* Install a stream-ordered device allocator for all library-owned memory of
 * later factorizations (their level stores, records, workspaces and solve
 * vectors).  alloc_fn(bytes, hip_stream, ctx) returns device memory that the
 * library uses on hip_stream (the stream of the call that needs it), or NULL
 * (HS_ERR_NOMEM); free_fn(ptr, hip_stream, ctx) takes it back, hip_stream
 * being the stream it was allocated for.  Before free_fn the library has put
 * every use of the buffer on that stream, or synchronised the device, so an
 * allocator that gives the block to later work on the same stream without a
 * wait (PyTorch's caching allocator does) is safe.  Each buffer goes back to
 * the allocator that gave it.  NULLs: back to the built-in allocator (HIP's
 * stream-ordered pool).  Both functions or neither, else HS_ERR_ARG; while
 * any factorization exists, HS_ERR_ARG. */
int hs_set_allocator(void* (*alloc_fn)(size_t, void*, void*), void (*free_fn)(void*, void*, void*), void* ctx);

/* ---- kernel-variant thresholds ----------------------------------------- */

/* Several steps have kernel variants that compute the same numbers (up to
 * rounding) and differ only in where their working data lives, how the work
 * is split, or (rank revelation) how accurately ill-conditioned fill is
 * resolved; thresholds pick one.  These calls read and lower the thresholds for
 * the whole process (test hooks, so that every variant runs on inputs small
 * enough for a CPU reference, and a tuning aid).  A factorization copies the
 * values when hs_factor / hs_factor_batch starts; later changes do not touch
 * it.  Parameters (default, allowed range):
 *   pivot_lds_max    128, 0..128   the pivot-block kernel keeps its working
 *                                  matrix in LDS while the colour's largest
 *                                  cluster is at most this size
 *   trinv8_max       128, 0..128   triangular inverses (Eq. elim) on the
 *                                  matrix cores with 8 blocks of 16 up to
 *                                  this cluster size,
 *   trinv12_max      192, 0..192   with 12 blocks up to this size (working
 *                                  matrix in memory only), per-wave
 *                                  substitution beyond
 *   qr_reg1_max      64, 0..64     complement of A_ss^{-1} U (Eq. scaling):
 *   qr_reg2_max      128, 0..128   Householder QR in registers with one / two
 *                                  row slots per lane up to this cluster size
 *                                  (for at most 64 coarse unknowns), in
 *                                  memory beyond
 *   wy_max           128, 0..128   its Q formed through the compact WY form
 *                                  while the coarse size is at most this
 *   gram_splits_max  256, 1..256   partial sums of the fill's Gram matrix
 *                                  (Eq. lra) per cluster at most
 *   schur_ptab_max   256, 0..256   Schur tile (Eq. elim): block pointers of
 *                                  its neighbour pairs staged in LDS while
 *                                  there are at most this many
 *   schur_noff_max   1024, 0..1024 Schur tile: neighbour offsets staged in
 *                                  LDS while there are at most this many
 *   cholqr           1, 0..1       basis U of the fill by Cholesky QR (0:
 *                                  always Householder QR)
 *   crowded_min      512, 0..2^30  a level whose colours hold at least this
 *                                  many clusters on average is crowded: its
 *                                  pivot kernel takes the three settings below
 *                                  in place of gram_splits_max, wy_max and
 *                                  cholqr (bound by throughput, not by the
 *                                  latency of one cluster's chain)
 *   gram_splits_crowded  4, 1..256 Gram partials per cluster on a crowded level
 *   wy_max_crowded   0, 0..128     wy_max on a crowded level
 *   cholqr_crowded   0, 0..1       cholqr on a crowded level
 *   dense_panel      128, 16..128  panel width of the dense LU of a complete
 *                                  level (Alg. 1, final dense factorization)
 *   apply_fwd        0, 0..2       forward step of the solve (Alg. 2) per
 *                                  colour: 1 one launch whose neighbour
 *                                  workgroups each form z_s[:f] again; 2 two
 *                                  launches (z_s once, then the neighbour
 *                                  updates); 0 two launches where the first
 *                                  would re-read more than twice T_L' and
 *                                  the solve has at most apply_split_nrhs_max
 *                                  right-hand sides
 *   apply_split_nrhs_max  1, 0..2^20  see apply_fwd
 *   apply_wave       1024, 0..2^30 with one right-hand side, the own
 *                                  products of a colour of at least this many
 *                                  clusters, each of at most 128 unknowns, run
 *                                  one wave per cluster (the same sums in the
 *                                  same order; 0: always the 64-row workgroup
 *                                  form)
 *   compression      0, 0..2       rank revelation (Eq. lra): 0 the
 *                                  pivoted QR of F^T under a rank cap or
 *                                  below qrcp_below_eps, else the Gram
 *                                  route; 1 always the pivoted QR; 2 always
 *                                  the Gram route
 *   qrcp_below_eps   1e-5, 0..1    the switch of compression = 0
 *   noalloc_scratch_max  HS_NOALLOC_SCRATCH_BYTES, 0..that   bytes of its
 *                                  device array hs_solve_noalloc may use
 *                                  (read at every call)
 * Errors: HS_ERR_ARG (unknown name, value outside its range, or a fraction
 * for an integer parameter; nothing changed). */
int hs_config_set(const char* name, double value);
int hs_config_get(const char* name, double* value);
/* Every parameter back to its default. */
int hs_config_reset(void);

/* Message describing the calling thread's last failure ("" if none). */
const char* hs_last_error(void);

/* Human-readable name of a status code. */
const char* hs_strerror(int code);

/* Library version string. */
const char* hs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HS_H_ */
