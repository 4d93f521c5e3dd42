// Device-side building blocks shared by the factorization and solve kernels:
// the per-level descriptor and cooperative (whole-workgroup) dense routines.
//
// All matrices are column major.  The cooperative routines take generic
// pointers so the same code works on LDS-resident working matrices (small
// clusters) and on L2-resident global workspaces (large clusters).  Every
// thread of the workgroup must call them (they contain barriers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace hs {

constexpr int WG = 256;       // threads of a per-cluster workgroup
constexpr int LDS_M = 128;    // clusters up to this size keep their working matrix in LDS
constexpr int PANEL = 32;     // column panel of the neighbour / fill update kernels
constexpr int SCHUR_T = 64;   // output tile of the Schur-complement GEMM
constexpr int MAX_M = 512;    // largest cluster the kernels accept
// Fill whose largest row norm is at most this fraction of ||A_ss||_F is the
// rounding noise of earlier Schur updates and is treated as zero; levels
// stored in float32 (mixed form) carry float32 rounding noise.
constexpr double FILL_NOISE_FLOOR = 1e-12;
constexpr double FILL_NOISE_FLOOR_F32 = 1e-6;

// Pointers into LDS carry their address space: routines instantiated for
// them compile to ds_* instructions rather than generic (flat) accesses.
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(1))) double glb_f64;  // global memory
typedef __attribute__((address_space(1))) float glb_f32;
__device__ inline lds_f64* to_lds(double* p) { return (lds_f64*)p; }
__device__ inline lds_i32* to_lds(int* p) { return (lds_i32*)p; }

// Size thresholds that choose between kernel variants computing the same
// numbers (they differ in where the working data lives and how the work is
// split).  The defaults are the production choices; hs_config_set() lowers
// them so that every variant can be run on small inputs.  All are clamped to
// the compile-time capacities below.
struct Knobs {
    int pivot_lds_max;    // pivot kernel: working matrix in LDS while the colour's largest cluster <= this
    int trinv8_max;       // triangular inverses on the matrix cores (8 blocks of 16) up to this size
    int trinv12_max;      // ... with 12 blocks up to this size (global-memory pivot kernel); beyond:
                          // per-wave substitution
    int qr_reg1_max;      // complement: Householder QR in registers, one row slot per lane, up to this m
    int qr_reg2_max;      // ... two row slots per lane up to this m (both for k <= 64); else in memory
    int wy_max;           // complement's Q formed through the compact WY form while k <= this
    int gram_splits_max;  // Gram partial sums of one cluster at most (fill partners per workgroup beyond)
    int schur_ptab_max;   // Schur tile: block pointers of its neighbour pairs in LDS while their count <= this
    int schur_noff_max;   // Schur tile: packed neighbour offsets in LDS while the neighbours <= this
    int cholqr;           // 1: basis U by Cholesky QR (Householder when ill conditioned); 0: Householder
    int qrcp;             // 1: rank and U by Householder QR with column pivoting of F^T (not the Gram route)
};

// Per-level view of the factorization state (device pointers).
struct LevelDev {
    int ncl;
    int symmetric;
    double eps;
    int fixed_rank;
    int pivoting;             // 1: LU of A_ss and F_ff with partial pivoting inside the cluster
    int gram_splits;          // Gram partial slots per cluster workspace (largest of the level)
    const int* m;             // [ncl] sizes at the start of the level
    int* k;                   // [ncl] coarse sizes after elimination (rank)
    int* flag;                // [ncl] 1 = breakdown in an unpivoted LU
    const int64_t* blk_off;   // [nblk] offset of every block in units of its element type
                              // (capacity m_a x m_b, ld m_a)
    double* blocks;           // storage of every cluster's blocks: float64, or float32 for the
                              // clusters of a system whose level is stored in float32 (mixed form)
    const int* diag_blk;      // [ncl] block id of (s, s)
    const int* nbr_ptr;       // [ncl+1] neighbours n(s)
    const int* nbr_id;
    const int* nbr_before;    // neighbour processed before s (then it has its coarse size)
    const int* nbr_bsa;       // block id of (s, a)
    const int* nbr_bas;       // block id of (a, s)
    int* nbr_noff;            // packed offset of a inside E_L / E_R (written by k_offsets)
    int* ntot;                // [ncl] sum of the current neighbour sizes (written by k_offsets)
    int* fcols;               // [ncl] sum of the current fill-partner sizes (written by k_offsets)
    const int* ncap;          // [ncl] sum of the neighbours' level-start sizes (record capacity)
    const int* fill_ptr;      // [ncl+1] fill partners w(s)
    const int* fill_id;
    const int* fill_before;
    const int* fill_bst;      // block id of (s, t)
    const int* fill_bts;      // block id of (t, s)
    const int64_t* pair_base; // [ncl] index of pair (0,0) of s in pair_blk
    const int* pair_blk;      // block id of (a_i, a_j) at pair_base[s] + i*nb + j
    const int64_t* rec_off;   // [ncl] record: T_L' (m^2), T_R' (m^2), E_R (m x ncap, ld m), E_L (ncap x m, ld ncap)
    double* rec;              // same element type as the cluster's blocks (offsets in its units)
    const int64_t* ws_off;    // [ncl] per-colour workspace of every cluster
    double* ws;
    Knobs kn;
};

// Workspace slots of a cluster (each m x m, column major, ld m).
enum WsSlot { WS_AINV = 0, WS_LINV, WS_UINV, WS_U, WS_X, WS_SL, WS_SR, WS_TL, WS_TR, WS_CU, WS_UC, WS_SCR, WS_GP };
__host__ __device__ inline int64_t ws_slots(int gram_splits) { return WS_GP + gram_splits; }
// Gram partial sums of a cluster with nf fill partners: one partner per
// workgroup up to max_splits (at most GRAM_SPLITS_MAX), then consecutive
// partners share a workgroup.  A function of the cluster alone, so the
// sums are formed in the same order whatever else shares the launch.
constexpr int GRAM_SPLITS_MAX = 256;
__host__ __device__ inline int gram_splits_of(int nf, int max_splits) {
    const int cap = max_splits < 1 ? 1 : (max_splits > GRAM_SPLITS_MAX ? GRAM_SPLITS_MAX : max_splits);
    return nf < 1 ? 1 : (nf > cap ? cap : nf);
}

__device__ inline int cur_size(const LevelDev& L, int a, int before) { return before ? L.k[a] : L.m[a]; }
// Block id / record of cluster s in its storage type T (offsets count elements of T).
template <class T>
__device__ inline T* blk_t(const LevelDev& L, int id) {
    return reinterpret_cast<T*>(L.blocks) + L.blk_off[id];
}
template <class T>
__device__ inline T* rec_t(const LevelDev& L, int s) {
    return reinterpret_cast<T*>(L.rec) + L.rec_off[s];
}

// ---------------------------------------------------------------- reductions

// Wave-wide reductions over DPP lane permutations (every lane active): swaps
// inside quads, then the half-row and row mirrors leave each row of 16 lanes
// with its row total; the four row totals are combined from lanes 0, 16, 32
// and 48.  Every lane gets the same result.
template <int CTRL>
__device__ inline double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double readlane_d(double v, int l) {  // value of v in lane l (l uniform)
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_QUAD_1032 = 0xB1, DPP_QUAD_2301 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141;

__device__ inline double wave_sum(double v) {
    v += dpp_d<DPP_QUAD_1032>(v);
    v += dpp_d<DPP_QUAD_2301>(v);
    v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_d<DPP_ROW_MIRROR>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_d<DPP_QUAD_1032>(v));
    v = fmax(v, dpp_d<DPP_QUAD_2301>(v));
    v = fmax(v, dpp_d<DPP_ROW_HALF_MIRROR>(v));
    v = fmax(v, dpp_d<DPP_ROW_MIRROR>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ inline int wave_min_int(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, DPP_QUAD_1032, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, DPP_QUAD_2301, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROW_MIRROR, 0xF, 0xF, false));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Exclusive prefix sum of v over the workgroup in thread order; *total gets
// the sum (the same in every thread).  buf: blockDim.x ints of LDS.  Starts
// with a barrier, so it may be called in a loop.
template <class PI>
__device__ inline int block_scan_excl(int v, PI buf, int* total) {
    const int tid = threadIdx.x, n = blockDim.x;
    __syncthreads();
    buf[tid] = v;
    __syncthreads();
    int before = 0, tot = 0;
    for (int i = 0; i < n; ++i) {  // the same address in every lane: broadcast reads
        const int t = buf[i];
        before += i < tid ? t : 0;
        tot += t;
    }
    *total = tot;
    return before;
}

// Block-wide reductions (blockDim.x a multiple of 64, <= 1024); red has >= 16 slots.
template <class PR>
__device__ inline double block_sum(double v, PR red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += red[i];
    __syncthreads();
    return r;
}
template <class PR>
__device__ inline double block_max(double v, PR red) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, red[i]);
    __syncthreads();
    return r;
}
template <class PR>
__device__ inline int block_min_int(int v, PR red) {
    v = wave_min_int(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    int r = red[0];
    for (int i = 1; i < nw; ++i) r = min(r, red[i]);
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ cooperative copy
// Columns over waves, rows over lanes (no integer division in the loops).

// Workgroup copy of n elements: st(e, ld(e)) for e < n.  Every thread has
// U loads in flight before it stores any (a loop of load-store pairs would
// wait out the full memory latency once per element).  The loads are
// unconditional (the index is clamped), so they issue back to back.
template <int U = 8, class LD, class ST>
__device__ inline void wg_stage(int n, const LD& ld, const ST& st) {
    if (n <= 0) return;
    for (int b = threadIdx.x; b < n; b += blockDim.x * U) {
        decltype(ld(0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(min(b + u * (int)blockDim.x, n - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = b + u * (int)blockDim.x;
            if (e < n) st(e, v[u]);
        }
    }
}

// acc + sum_{l < n} a[l * as] * b(l), added in ascending l with fused
// multiply-adds; the loads of a (memory) are issued eight at a time.
template <class TA, class FB>
__device__ inline double dot_batched(int n, const TA* a, int64_t as, const FB& b, double acc) {
    int l = 0;
    for (; l + 8 <= n; l += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = (double)a[(int64_t)(l + u) * as];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(t[u], b(l + u), acc);
    }
    for (; l < n; ++l) acc = fma((double)a[(int64_t)l * as], b(l), acc);
    return acc;
}

template <class PS, class PD>
__device__ inline void wg_copy(int M, int N, PS src, int lds, PD dst, int ldd) {
    if (M <= 0 || N <= 0) return;
    if (lds == M && ldd == M) {  // both packed: one contiguous range
        wg_stage(M * N, [&](int e) { return src[e]; }, [&](int e, auto v) { dst[e] = v; });
        return;
    }
    wg_stage(
        M * N, [&](int e) { return src[(e % M) + (int64_t)(e / M) * lds]; },
        [&](int e, auto v) { dst[(e % M) + (int64_t)(e / M) * ldd] = v; });
}
template <class PD>
__device__ inline void wg_zero(int M, int N, PD dst, int ldd) {
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int j = threadIdx.x >> 6; j < N; j += nw)
        for (int i = lane; i < M; i += 64) dst[i + (int64_t)j * ldd] = 0.0;
}

// ------------------------------------------------------- staged products
// Operands in memory pass through LDS in tiles of at most TILE_BYTES (read
// once, coalesced, many loads in flight), so long dot products read LDS and
// not memory; a thread holds at most OUT_PER_THREAD running sums.
constexpr int TILE_BYTES = 32768;
constexpr int OUT_PER_THREAD = 4;
constexpr int OUT_CAP = OUT_PER_THREAD * WG;

// out(i, r) = sum_{l < K} A(i, l) X(l, r) for i < R, r < nrhs, every sum taken
// from zero in ascending l.  la(i, l) loads A from memory: the tile is
// fetched with i varying fastest, or with l fastest when ACOL (A stored with
// consecutive l adjacent), so the loads coalesce either way.  lx(l, r) reads
// X (LDS), store(i, r, v) receives each result once.  abuf: TILE_BYTES of
// LDS.  Ends with a barrier.
template <class T, bool ACOL = false, class LA, class LX, class ST>
__device__ void wg_rows_times(int R, int K, int nrhs, const LA& la, const LX& lx, T* abuf, const ST& store) {
    const int tid = threadIdx.x;
    const int RR = min(nrhs, OUT_CAP);
    const int RJ = max(1, min(R, OUT_CAP / max(RR, 1)));
    constexpr int ABUF_N = TILE_BYTES / (int)sizeof(T);
    for (int r0 = 0; r0 < nrhs; r0 += RR) {
        const int rr = min(RR, nrhs - r0);
        for (int i0 = 0; i0 < R; i0 += RJ) {
            const int rj = min(RJ, R - i0);
            const int CC = max(1, min(K, ABUF_N / rj));
            double acc[OUT_PER_THREAD];
#pragma unroll
            for (int t = 0; t < OUT_PER_THREAD; ++t) acc[t] = 0.0;
            for (int l0 = 0; l0 < K; l0 += CC) {
                const int cc = min(CC, K - l0);
                __syncthreads();
                if constexpr (ACOL)
                    wg_stage(
                        rj * cc, [&](int e) { return (T)la(i0 + e / cc, l0 + e % cc); },
                        [&](int e, T v) { abuf[(e / cc) + (e % cc) * rj] = v; });
                else
                    wg_stage(
                        rj * cc, [&](int e) { return (T)la(i0 + e % rj, l0 + e / rj); },
                        [&](int e, T v) { abuf[e] = v; });
                __syncthreads();
#pragma unroll
                for (int t = 0; t < OUT_PER_THREAD; ++t) {
                    const int x = tid + t * WG;
                    if (x < rj * rr) {
                        const int i = x % rj, r = r0 + x / rj;
                        double a = acc[t];
#pragma unroll 4
                        for (int l = 0; l < cc; ++l) a = fma((double)abuf[i + l * rj], lx(l0 + l, r), a);
                        acc[t] = a;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < OUT_PER_THREAD; ++t) {
                const int x = tid + t * WG;
                if (x < rj * rr) store(i0 + x % rj, r0 + x / rj, acc[t]);
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ MFMA tile core
// One 64 x 64 tile of D = Left (64 x K) * Right (K x 64) on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64): 4 waves as 2 x 2 quarters of 32 x 32, each
// quarter 2 x 2 blocks of 16 x 16.  The MFMA computes the transposed block
// (Right^T Left^T) so that lane l % 16 indexes rows of D: the epilogue then
// touches 16 consecutive rows of a column per group of lanes (coalesced for
// column-major outputs).  Lane layout of the instruction: operand a of lane l
// is row l%16, k l/16; operand b of lane l is k l/16, column l%16; result
// element r of lane l is row l/16 + 4r, column l%16.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int MT = 64, MKC = 16;
struct MfmaSmem {
    double a[MKC][MT + 1];  // a[k][row] = Left(row, k)
    double b[MKC][MT + 1];  // b[k][col] = Right(k, col)
};
typedef __attribute__((address_space(3))) MfmaSmem lds_smem;
__device__ inline lds_smem* to_lds(MfmaSmem* p) { return (lds_smem*)p; }

// la(r, k) / lb(k, c) return the operand element or 0 outside the matrix.
// Accumulates into acc (acc += Left * Right).  With PART, only the first rv
// rows and cv columns of the tile are wanted: a wave then skips the
// matrix-core work of its 16 x 16 blocks that lie wholly beyond them (the
// skip is uniform per wave; skipped accumulators keep their values).
template <bool PART = false, class LoadL, class LoadR>
__device__ inline void mfma_tile64_acc(int K, const LoadL& la, const LoadR& lb, lds_smem* sm, v4d acc[2][2],
                                       int rv = MT, int cv = MT) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    // 3: 2 x 2 blocks wanted, 2: 1 x 2, 1: 2 x 1, 0: 1 x 1, -1: none
    const int shape =
        PART ? ((wm < rv && wn < cv) ? ((wm + 16 < rv) ? 1 : 0) + ((wn + 16 < cv) ? 2 : 0) : -1) : 3;
    // each thread stages 4 elements of each operand per K chunk; the next
    // chunk is fetched into registers while the matrix cores work on this one
    constexpr int PER = MT * MKC / WG;
    double ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + t * WG;
            const int r = e % MT, kk = e / MT;
            ra[t] = (k0 + kk < K) ? la(r, k0 + kk) : 0.0;
            const int kb = e % MKC, c = e / MKC;
            rb[t] = (k0 + kb < K) ? lb(k0 + kb, c) : 0.0;
        }
    };
    // straight-line matrix-core code for an NI x NJ block shape
    auto steps = [&](auto NI, auto NJ) {
#pragma unroll
        for (int ks = 0; ks < MKC; ks += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < NI; ++i) av[i] = sm->a[ks + lk][wm + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < NJ; ++j) bv[j] = sm->b[ks + lk][wn + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[i][j], 0, 0, 0);
        }
    };
    using one = std::integral_constant<int, 1>;
    using two = std::integral_constant<int, 2>;
    if (K > 0) fetch(0);
    for (int k0 = 0; k0 < K; k0 += MKC) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + t * WG;
            sm->a[e / MT][e % MT] = ra[t];
            sm->b[e % MKC][e / MKC] = rb[t];
        }
        __syncthreads();
        if (k0 + MKC < K) fetch(k0 + MKC);
        if constexpr (!PART) {
#pragma unroll
            for (int ks = 0; ks < MKC; ks += 4) {
                double av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) av[i] = sm->a[ks + lk][wm + 16 * i + lr];
#pragma unroll
                for (int j = 0; j < 2; ++j) bv[j] = sm->b[ks + lk][wn + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[i][j], 0, 0, 0);
            }
        } else if (shape == 3) {
            steps(two{}, two{});
        } else if (shape == 2) {
            steps(one{}, two{});
        } else if (shape == 1) {
            steps(two{}, one{});
        } else if (shape == 0) {
            steps(one{}, one{});
        }
    }
}

__device__ inline void mfma_zero(v4d acc[2][2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
}

// acc = Left * Right.
template <bool PART = false, class LoadL, class LoadR>
__device__ inline void mfma_tile64(int K, const LoadL& la, const LoadR& lb, lds_smem* sm, v4d acc[2][2], int rv = MT,
                                   int cv = MT) {
    mfma_zero(acc);
    mfma_tile64_acc<PART>(K, la, lb, sm, acc, rv, cv);
}

// Visit the tile's results: f(row, col, value), row/col within the 64 x 64 tile.
template <class Fn>
__device__ inline void mfma_tile64_store(const v4d acc[2][2], const Fn& f) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) f(wm + 16 * i + lr, wn + 16 * j + lk + 4 * r, acc[i][j][r]);
}

// As mfma_tile64_store, with the running index idx in [0, 16) of the entry
// within the lane (compile-time after unrolling).
template <class Fn>
__device__ inline void mfma_tile64_visit(const v4d acc[2][2], const Fn& f) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) f((i * 2 + j) * 4 + r, wm + 16 * i + lr, wn + 16 * j + lk + 4 * r, acc[i][j][r]);
}

// ------------------------------------------------- BF16 tile core (mixed form)
// One 64 x 64 tile of D = Left (64 x K) * Right (K x 64) on the BF16 matrix
// cores with FP32 accumulation (v_mfma_f32_16x16x16_bf16): 4 waves as 2 x 2
// quarters of 32 x 32, each 2 x 2 blocks of 16 x 16.  Instruction layout:
// operand a of lane l holds A[l%16][4(l/16) + i], operand b holds
// B[4(l/16) + i][l%16] (i = 0..3), result r of lane l is D[4(l/16) + r][l%16].
// As in the FP64 core the transposed block is computed, so lane l%16 indexes
// rows of D.  Every float operand is split into three BF16 parts
// x = hi + mid + lo (8 + 8 + 8 significand bits, nearest-even rounding at each
// step) and the six products whose parts sum to at most 2 are accumulated, so
// the tile carries float32 accuracy on the BF16 units.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
constexpr int NSPLIT = 3;
struct MfmaSmemB {
    unsigned short a[NSPLIT][MKC][MT + 2];  // a[part][k][row] = Left(row, k)
    unsigned short b[NSPLIT][MKC][MT + 2];  // b[part][k][col] = Right(k, col)
};
typedef __attribute__((address_space(3))) MfmaSmemB lds_smemb;
__device__ inline lds_smemb* to_lds(MfmaSmemB* p) { return (lds_smemb*)p; }

__device__ inline unsigned short bf16_rne(float x) {
    const unsigned int u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <class LoadL, class LoadR>
__device__ inline void mfma_tile64_bf16(int K, const LoadL& la, const LoadR& lb, lds_smemb* sm, v4f acc[2][2]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    constexpr int PER = MT * MKC / WG;
    float ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + t * WG;
            const int r = e % MT, kk = e / MT;
            ra[t] = (k0 + kk < K) ? (float)la(r, k0 + kk) : 0.f;
            const int kb = e % MKC, c = e / MKC;
            rb[t] = (k0 + kb < K) ? (float)lb(k0 + kb, c) : 0.f;
        }
    };
    auto split = [](float x, unsigned short* h) {
#pragma unroll
        for (int q = 0; q < NSPLIT; ++q) {
            h[q] = bf16_rne(x);
            x -= bf16_to_f32(h[q]);
        }
    };
    if (K > 0) fetch(0);
    for (int k0 = 0; k0 < K; k0 += MKC) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + t * WG;
            unsigned short ha[NSPLIT], hb[NSPLIT];
            split(ra[t], ha);
            split(rb[t], hb);
#pragma unroll
            for (int q = 0; q < NSPLIT; ++q) {
                sm->a[q][e / MT][e % MT] = ha[q];
                sm->b[q][e % MKC][e / MKC] = hb[q];
            }
        }
        __syncthreads();
        if (k0 + MKC < K) fetch(k0 + MKC);
        v4s av[NSPLIT][2], bv[NSPLIT][2];
#pragma unroll
        for (int q = 0; q < NSPLIT; ++q)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    av[q][i][u] = (short)sm->a[q][4 * lk + u][wm + 16 * i + lr];
                    bv[q][i][u] = (short)sm->b[q][4 * lk + u][wn + 16 * i + lr];
                }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // smallest terms first: (lo,hi) (hi,lo) (mid,mid) (mid,hi) (hi,mid) (hi,hi)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[2][j], av[0][i], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[0][j], av[2][i], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[1][j], av[1][i], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[1][j], av[0][i], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[0][j], av[1][i], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv[0][j], av[0][i], acc[i][j], 0, 0, 0);
            }
    }
}

// Visit the BF16 tile's results: f(idx, row, col, value), idx in [0, 16).
template <class Fn>
__device__ inline void mfma_tile64_bf16_visit(const v4f acc[2][2], const Fn& f) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) f((i * 2 + j) * 4 + r, wm + 16 * i + lr, wn + 16 * j + 4 * lk + r, acc[i][j][r]);
}

// ------------------------------------------------------------ cooperative GEMM
// C (M x N) = alpha op(A) op(B) + beta C; op(A) is M x K, op(B) is K x N, on
// the FP64 matrix cores, 64 x 64 tiles.  beta == 0 never reads C.
typedef MfmaSmem GemmSmem;

template <bool TA, bool TB, class PA, class PB, class PC>
__device__ void wg_gemm(int M, int N, int K, double alpha, PA A, int lda, PB B, int ldb, double beta, PC C, int ldc,
                        lds_smem* sm) {
    for (int r0 = 0; r0 < M; r0 += MT)
        for (int c0 = 0; c0 < N; c0 += MT) {
            v4d acc[2][2];
            mfma_tile64<true>(
                K,
                [&](int r, int k) {
                    const int gr = r0 + r;
                    return gr < M ? (TA ? A[k + (int64_t)gr * lda] : A[gr + (int64_t)k * lda]) : 0.0;
                },
                [&](int k, int c) {
                    const int gc = c0 + c;
                    return gc < N ? (TB ? B[gc + (int64_t)k * ldb] : B[k + (int64_t)gc * ldb]) : 0.0;
                },
                sm, acc, M - r0, N - c0);
            if (beta == 0.0) {
                mfma_tile64_store(acc, [&](int r, int c, double v) {
                    const int gr = r0 + r, gc = c0 + c;
                    if (gr < M && gc < N) C[gr + (int64_t)gc * ldc] = alpha * v;
                });
            } else {  // read all 16 old values of the lane, then write
                double old[16];
                mfma_tile64_visit(acc, [&](int idx, int r, int c, double) {
                    const int gr = r0 + r, gc = c0 + c;
                    old[idx] = (gr < M && gc < N) ? C[gr + (int64_t)gc * ldc] : 0.0;
                });
                mfma_tile64_visit(acc, [&](int idx, int r, int c, double v) {
                    const int gr = r0 + r, gc = c0 + c;
                    if (gr < M && gc < N) C[gr + (int64_t)gc * ldc] = fma(alpha, v, beta * old[idx]);
                });
            }
        }
    __syncthreads();
}

// C = Left * Right over 64 x 64 output tiles with caller-supplied loaders
// la(r, k), lb(k, c) (global indices, 0 outside) and store(r, c, v).
template <class LA, class LB, class ST>
__device__ void wg_gemm_fn(int M, int N, int K, const LA& la, const LB& lb, lds_smem* sm, const ST& store) {
    for (int r0 = 0; r0 < M; r0 += MT)
        for (int c0 = 0; c0 < N; c0 += MT) {
            v4d acc[2][2];
            mfma_tile64<true>(
                K, [&](int r, int k) { return r0 + r < M ? la(r0 + r, k) : 0.0; },
                [&](int k, int c) { return c0 + c < N ? lb(k, c0 + c) : 0.0; }, sm, acc, M - r0, N - c0);
            mfma_tile64_store(acc, [&](int r, int c, double v) {
                if (r0 + r < M && c0 + c < N) store(r0 + r, c0 + c, v);
            });
        }
    __syncthreads();
}

// ---------------------------------------------------- LU without pivoting
// In place Doolittle LU of the M x M matrix W (ld ldw), one barrier per
// elimination step: the multipliers of column j are formed on the fly by the
// threads of the trailing update and stored one step later, when nothing
// reads the column any more.  Returns false on a zero or non-finite pivot
// (every thread reads the same pivot, so every thread returns the same).
template <class PW>
__device__ inline bool wg_lu_nopiv(PW W, int M, int ldw) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        const double p = W[j + (int64_t)j * ldw];
        if (p == 0.0 || !isfinite(p)) return false;
        const double inv = 1.0 / p;
        if (j > 0) {
            const double ip = 1.0 / W[(j - 1) + (int64_t)(j - 1) * ldw];
            for (int i = j + tid; i < M; i += blockDim.x) W[i + (int64_t)(j - 1) * ldw] *= ip;
        }
        for (int r0 = j + 1; r0 < M; r0 += 64) {
            const int i = r0 + lane;
            if (i >= M) break;
            const double l = W[i + (int64_t)j * ldw] * inv;
#pragma unroll 4
            for (int c = j + 1 + wv; c < M; c += nw)
                W[i + (int64_t)c * ldw] = fma(-l, W[j + (int64_t)c * ldw], W[i + (int64_t)c * ldw]);
        }
        __syncthreads();
    }
    return true;
}

// Blocked LU without pivoting for M <= 192: 16-wide panels.
// The panel is factored by wave 0 in registers (the same operations, in the
// same order, as the unblocked routine); then U_12 = L_11^{-1} A_12 and
// A_22 -= L_21 U_12 run as 16 x 16 blocks on the matrix cores, spread over
// the waves.  scr holds 256 doubles of LDS, flag one int.  Returns false on a
// zero or non-finite pivot (every thread returns the same).
// x[s] for a uniform slot index s < NS <= 3, by value (keeps x in registers).
template <int NS>
__device__ inline double pick(const double* x, int s) {
    if constexpr (NS == 1) return x[0];
    else if constexpr (NS == 2) return s == 0 ? x[0] : x[1];
    else return s == 0 ? x[0] : (s == 1 ? x[1] : x[2]);
}

template <class PW>
__device__ __attribute__((noinline)) void tri16_lower_unit_inverse(PW W, int ldw, int b0, lds_f64* scr) {
    const int c = threadIdx.x & 63;
    if (c >= 16) return;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
#pragma unroll
        for (int r = j + 1; r < 16; ++r) x[r] = fma(-W[(b0 + r) + (int64_t)(b0 + j) * ldw], x[j], x[r]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) scr[r + 16 * c] = x[r];
}

template <int NS, class PW>
__device__ inline bool wg_lu_blocked_ns(PW W, int M, int ldw, lds_f64* scr, lds_i32* flag) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int p = 0; p < M; p += 16) {
        const int pw = min(16, M - p);
        if (wv == 0) {  // panel: rows p..M-1, columns p..p+pw-1
            double x[16][NS];
#pragma unroll
            for (int c = 0; c < 16; ++c)
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int i = s * 64 + lane;
                    x[c][s] = (c < pw && i < M) ? W[i + (int64_t)(p + c) * ldw] : 0.0;
                }
            bool ok = true;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int col = p + j, sj = col >> 6, lj = col & 63;
                if (ok && j < pw) {
                    const double piv = readlane_d(pick<NS>(x[j], sj), lj);
                    ok = (piv != 0.0 && isfinite(piv));
                    const double inv = 1.0 / piv;
                    double l[NS];
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const int i = s * 64 + lane;
                        l[s] = (ok && i > col) ? x[j][s] * inv : 0.0;
                        x[j][s] = (i > col) ? l[s] : x[j][s];
                    }
#pragma unroll
                    for (int c = j + 1; c < 16; ++c) {
                        const double u = readlane_d(pick<NS>(x[c], sj), lj);
#pragma unroll
                        for (int s = 0; s < NS; ++s) x[c][s] = fma(-l[s], u, x[c][s]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (!ok) {
                if (lane == 0) *flag = 1;
            } else {
#pragma unroll
                for (int c = 0; c < 16; ++c)
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        const int i = s * 64 + lane;
                        if (c < pw && i >= p && i < M) W[i + (int64_t)(p + c) * ldw] = x[c][s];
                    }
            }
        }
        __syncthreads();
        if (*flag) return false;
        const int q = p + pw, n2 = M - q;
        if (n2 <= 0) break;
        if (wv == 0) tri16_lower_unit_inverse(W, ldw, p, scr);
        __syncthreads();
        const int nbc = (n2 + 15) >> 4;
        for (int cb = wv; cb < nbc; cb += nw) {  // U_12 = L_11^{-1} A_12
            const int c0 = q + 16 * cb;
            const bool cin = c0 + lr < M;
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r] = scr[lr + 16 * (4 * r + lk)];
                b[r] = cin ? W[(p + 4 * r + lk) + (int64_t)(c0 + lr) * ldw] : 0.0;
            }
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[r], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (cin) W[(p + lk + 4 * r) + (int64_t)(c0 + lr) * ldw] = acc[r];
        }
        __syncthreads();
        for (int b = wv; b < nbc * nbc; b += nw) {  // A_22 -= L_21 U_12
            const int rb = b % nbc, cb = b / nbc;
            const int r0 = q + 16 * rb, c0 = q + 16 * cb;
            const bool cin = c0 + lr < M, rin = r0 + lr < M;
            v4d acc;
            double a[4], bb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + lk + 4 * r;
                acc[r] = (row < M && cin) ? W[row + (int64_t)(c0 + lr) * ldw] : 0.0;
                a[r] = rin ? -W[(r0 + lr) + (int64_t)(p + 4 * r + lk) * ldw] : 0.0;
                bb[r] = cin ? W[(p + 4 * r + lk) + (int64_t)(c0 + lr) * ldw] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], bb[r], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + lk + 4 * r;
                if (row < M && cin) W[row + (int64_t)(c0 + lr) * ldw] = acc[r];
            }
        }
        __syncthreads();
    }
    return true;
}

// Unpivoted LU: blocked on the matrix cores (BLK, M <= 128) or the unblocked
// routine.
template <bool BLK, class PW>
__device__ inline bool wg_lu(PW W, int M, int ldw, lds_f64* scr, lds_i32* flag) {
    if constexpr (BLK) {
        if (M <= 64) return wg_lu_blocked_ns<1, PW>(W, M, ldw, scr, flag);
        if (M <= 128) return wg_lu_blocked_ns<2, PW>(W, M, ldw, scr, flag);
        if (M <= 192) return wg_lu_blocked_ns<3, PW>(W, M, ldw, scr, flag);
    }
    return wg_lu_nopiv(W, M, ldw);
}

// ------------------------------------------------------- triangular inverses
// One wave computes two columns (c0, c1) of the inverse by substitution in
// its registers: row i = 64 s + lane lives in slot s.  The two columns share
// the loads of the triangle and give the wave two independent chains.

// Triangle columns are read U at a time, double buffered: the loads of the
// next group are in flight while the current group is applied.
template <int NS>
struct TriBuf {
    static constexpr int U = NS <= 2 ? 4 : (NS <= 4 ? 2 : 1);
    double v[U][NS];
    double d[U];  // reciprocals of the diagonal entries (upper triangle only)
};

// Columns of L^{-1}, L = unit lower triangle of W.
template <int NS, class PW, class PO>
__device__ inline void wave_inv_lower_unit(PW W, int M, int ldw, int c0, int c1, PO out, int ldo) {
    constexpr int U = TriBuf<NS>::U;
    const int lane = threadIdx.x & 63;
    double x[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        x[s] = (s * 64 + lane == c0) ? 1.0 : 0.0;
        y[s] = (s * 64 + lane == c1) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
        const int j0 = max(c0, sb * 64), j1 = min(M, sb * 64 + 64);
        // entries L[i, jj] below the diagonal of columns jj in [j, j + U)
        auto load = [&](TriBuf<NS>& b, int j) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j + u;
                auto colj = W + (int64_t)min(jj, M - 1) * ldw;
#pragma unroll
                for (int s = sb; s < NS; ++s) {
                    const int i = s * 64 + lane;
                    b.v[u][s] = (jj < j1 && i > jj && i < M) ? colj[i] : 0.0;
                }
            }
        };
        auto apply = [&](const TriBuf<NS>& b, int j) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j + u;
                if (jj < j1) {
                    const double xj = readlane_d(x[sb], jj - sb * 64);
                    const double yj = readlane_d(y[sb], jj - sb * 64);
#pragma unroll
                    for (int s = sb; s < NS; ++s) {
                        x[s] = fma(-b.v[u][s], xj, x[s]);
                        y[s] = fma(-b.v[u][s], yj, y[s]);
                    }
                }
            }
        };
        TriBuf<NS> ba, bb;
        if (j0 < j1) load(ba, j0);
        for (int j = j0; j < j1; j += 2 * U) {
            if (j + U < j1) load(bb, j + U);
            apply(ba, j);
            if (j + U < j1) {
                if (j + 2 * U < j1) load(ba, j + 2 * U);
                apply(bb, j + U);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i < M) {
            out[i + (int64_t)c0 * ldo] = x[s];
            if (c1 < M) out[i + (int64_t)c1 * ldo] = y[s];
        }
    }
}

// Columns of U^{-1}, U = upper triangle of W (with its diagonal); c0 < c1.
template <int NS, class PW, class PO>
__device__ inline void wave_inv_upper(PW W, int M, int ldw, int c0, int c1, PO out, int ldo) {
    constexpr int U = TriBuf<NS>::U;
    const int lane = threadIdx.x & 63;
    const int ctop = c1 < M ? c1 : c0;
    double x[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        x[s] = (s * 64 + lane == c0) ? 1.0 : 0.0;
        y[s] = (s * 64 + lane == c1) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int sb = NS - 1; sb >= 0; --sb) {
        const int jt = min(ctop, sb * 64 + 63), jb = sb * 64;
        // column jj (descending from j): entries above the diagonal, and the diagonal
        auto load = [&](TriBuf<NS>& b, int j) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j - u;
                auto colj = W + (int64_t)max(jj, 0) * ldw;
                b.d[u] = (jj >= jb) ? 1.0 / colj[max(jj, 0)] : 1.0;  // reciprocal, off the chain
#pragma unroll
                for (int s = 0; s <= sb; ++s) {
                    const int i = s * 64 + lane;
                    b.v[u][s] = (jj >= jb && i < jj) ? colj[i] : 0.0;
                }
            }
        };
        auto apply = [&](const TriBuf<NS>& b, int j) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j - u;
                if (jj >= jb) {
                    const double xj = readlane_d(x[sb], jj - jb) * b.d[u];
                    const double yj = readlane_d(y[sb], jj - jb) * b.d[u];
                    if (lane == jj - jb) {
                        x[sb] = xj;
                        y[sb] = yj;
                    }
#pragma unroll
                    for (int s = 0; s <= sb; ++s) {
                        x[s] = fma(-b.v[u][s], xj, x[s]);
                        y[s] = fma(-b.v[u][s], yj, y[s]);
                    }
                }
            }
        };
        TriBuf<NS> ba, bb;
        if (jt >= jb) load(ba, jt);
        for (int j = jt; j >= jb; j -= 2 * U) {
            if (j - U >= jb) load(bb, j - U);
            apply(ba, j);
            if (j - U >= jb) {
                if (j - 2 * U >= jb) load(ba, j - 2 * U);
                apply(bb, j - U);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i < M) {
            out[i + (int64_t)c0 * ldo] = x[s];
            if (c1 < M) out[i + (int64_t)c1 * ldo] = y[s];
        }
    }
}

template <bool UPPER, int NS, class PW, class PO>
__device__ inline void wg_trinv_ns(PW W, int M, int ldw, PO out, int ldo) {
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wv; c < M; c += 2 * nw) {
        if (UPPER)
            wave_inv_upper<NS, PW, PO>(W, M, ldw, c, c + nw, out, ldo);
        else
            wave_inv_lower_unit<NS, PW, PO>(W, M, ldw, c, c + nw, out, ldo);
    }
}

template <bool UPPER, class PW, class PO>
__device__ inline void wg_trinv(PW W, int M, int ldw, PO out, int ldo) {
    switch ((M + 63) >> 6) {
        case 0: break;
        case 1: wg_trinv_ns<UPPER, 1, PW, PO>(W, M, ldw, out, ldo); break;
        case 2: wg_trinv_ns<UPPER, 2, PW, PO>(W, M, ldw, out, ldo); break;
        case 3: wg_trinv_ns<UPPER, 3, PW, PO>(W, M, ldw, out, ldo); break;
        case 4: wg_trinv_ns<UPPER, 4, PW, PO>(W, M, ldw, out, ldo); break;
        case 5: wg_trinv_ns<UPPER, 5, PW, PO>(W, M, ldw, out, ldo); break;
        case 6: wg_trinv_ns<UPPER, 6, PW, PO>(W, M, ldw, out, ldo); break;
        case 7: wg_trinv_ns<UPPER, 7, PW, PO>(W, M, ldw, out, ldo); break;
        default: wg_trinv_ns<UPPER, 8, PW, PO>(W, M, ldw, out, ldo); break;
    }
    __syncthreads();
}

// Blocked triangular inverse on the FP64 matrix cores, M <= 16 NBMAX (NBMAX =
// 8 or 12 blocks of 16).  The native result layout of v_mfma_f64_16x16x4f64 (lane l,
// element r holds D[l/16 + 4r][l%16]) is its B-operand layout for the k-chunk
// 4r, so a wave keeps one block column of the inverse in accumulators and
// feeds finished blocks straight back as operands.
//   lower (unit):  X_JJ = L_JJ^{-1}, X_IJ = -X_II sum_{J<=l<I} L_Il X_lJ  (I > J)
//   upper:         X_JJ = U_JJ^{-1}, X_IJ = -X_II sum_{I<l<=J} U_Il X_lJ  (I < J)
// Block columns are independent: wave w takes J = w, w + 4, ...  The 16 x 16
// diagonal inverses go first, one 16-lane group per block, into scr
// (NBMAX x 256 doubles of LDS).  Padding beyond M is the identity.
constexpr int TRI_MFMA_MAX = 128;  // with 8 blocks
constexpr int TRI_MFMA_MAX12 = 192;  // with 12 blocks

// Inverses of the 16 x 16 diagonal blocks, one 16-lane group per block,
// column c of block g into scr[g * 256 + 16 c ...].
template <bool UPPER, class PW>
__device__ __attribute__((noinline)) void diag_block_inverses(PW W, int M, int ldw, lds_f64* scr) {
    const int tid = threadIdx.x;
    const int nb = (M + 15) >> 4;
    const int g = tid >> 4, c = tid & 15;
    if (g >= nb) return;
    const int b0 = 16 * g;
    auto T = [&](int r, int j) -> double {
        const int gr = b0 + r, gj = b0 + j;
        if (gr >= M || gj >= M) return (r == j) ? 1.0 : 0.0;
        return W[gr + (int64_t)gj * ldw];
    };
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == c) ? 1.0 : 0.0;
    if (!UPPER) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
#pragma unroll
            for (int r = j + 1; r < 16; ++r) x[r] = fma(-T(r, j), x[j], x[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int j = 15; j >= 0; --j) {
            x[j] = x[j] / T(j, j);
#pragma unroll
            for (int r = 0; r < j; ++r) x[r] = fma(-T(r, j), x[j], x[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) scr[g * 256 + r + 16 * c] = x[r];
}

template <bool UPPER, int NBMAX, class PW, class PO>
__device__ inline void wg_trinv_mfma(PW W, int M, int ldw, PO out, int ldo, lds_f64* scr) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    const int nb = (M + 15) >> 4;
    diag_block_inverses<UPPER, PW>(W, M, ldw, scr);
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    v4d ident;
#pragma unroll
    for (int r = 0; r < 4; ++r) ident[r] = (lk + 4 * r == lr) ? 1.0 : 0.0;
    const v4d zero = {0.0, 0.0, 0.0, 0.0};
    for (int J = wv; J < nb; J += nw) {
        v4d X[NBMAX];
#pragma unroll
        for (int ii = 0; ii < NBMAX; ++ii) {
            const int I = UPPER ? NBMAX - 1 - ii : ii;  // the order in which blocks become available
            if (I >= nb || (UPPER ? I > J : I < J)) continue;
            v4d S = (I == J) ? ident : zero;
#pragma unroll
            for (int l = 0; l < NBMAX; ++l) {
                if (l >= nb || (UPPER ? (l <= I || l > J) : (l < J || l >= I))) continue;
                const int gr = 16 * I + lr;
                auto colp = W + gr + (int64_t)(16 * l + lk) * ldw;
                double a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = (gr < M && 16 * l + 4 * r + lk < M) ? -colp[(int64_t)(4 * r) * ldw] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) S = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], X[l][r], S, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            v4d acc = zero;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(scr[I * 256 + lr + 16 * (4 * r + lk)], S[r], acc, 0, 0, 0);
            X[I] = acc;
        }
#pragma unroll
        for (int I = 0; I < NBMAX; ++I) {
            if (I >= nb) continue;
            const bool nz = UPPER ? I <= J : I >= J;
            const int col = 16 * J + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * I + lk + 4 * r;
                if (row < M && col < M) out[row + (int64_t)col * ldo] = nz ? X[I][r] : 0.0;
            }
        }
    }
    __syncthreads();
}

// out = L^{-1}, L = unit lower triangle of W.  MODE 1: matrix cores with 8
// blocks (M <= 128), 2: with 12 blocks (M <= 192, scr of 12 x 256), 0:
// per-wave substitution, -1: matrix cores when M <= 128.
template <int MODE = -1, class PW, class PO>
__device__ inline void wg_trinv_lower_unit(PW W, int M, int ldw, PO out, int ldo, lds_f64* scr) {
    if (MODE == 1 || (MODE == -1 && M <= TRI_MFMA_MAX))
        wg_trinv_mfma<false, 8, PW, PO>(W, M, ldw, out, ldo, scr);
    else if (MODE == 2)
        wg_trinv_mfma<false, 12, PW, PO>(W, M, ldw, out, ldo, scr);
    else
        wg_trinv<false, PW, PO>(W, M, ldw, out, ldo);
}
// out = U^{-1}, U = upper triangle of W (with diagonal).
template <int MODE = -1, class PW, class PO>
__device__ inline void wg_trinv_upper(PW W, int M, int ldw, PO out, int ldo, lds_f64* scr) {
    if (MODE == 1 || (MODE == -1 && M <= TRI_MFMA_MAX))
        wg_trinv_mfma<true, 8, PW, PO>(W, M, ldw, out, ldo, scr);
    else if (MODE == 2)
        wg_trinv_mfma<true, 12, PW, PO>(W, M, ldw, out, ldo, scr);
    else
        wg_trinv<true, PW, PO>(W, M, ldw, out, ldo);
}

// ----------------------------------------------------------- Householder QR
// Reflector of column jj of A (rows jj..M-1) by one wave, LAPACK larfg
// convention: H = I - tau v v^T, v(jj) = 1, beta = -sign(alpha) ||x||, tau = 0
// when the part below the diagonal is zero.  Lane l handles rows jj + l + 64 t
// (the mapping of the trailing update, so every lane reads what it wrote).
template <class PA, class PT>
__device__ inline void wave_reflector(PA A, int M, int jj, int lda, PT tau_sh) {
    const int lane = threadIdx.x & 63;
    auto col = A + (int64_t)jj * lda;
    double part = 0.0, alpha = 0.0;
    for (int i = jj + lane; i < M; i += 64) {
        const double v = col[i];
        if (i == jj)
            alpha = v;
        else
            part = fma(v, v, part);
    }
    const double xn2 = wave_sum(part);
    alpha = readlane_d(alpha, 0);
    double tau = 0.0, beta = alpha;
    if (xn2 != 0.0) {
        const double nrm = hypot(alpha, sqrt(xn2));
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        const double scale = 1.0 / (alpha - beta);
        for (int i = jj + lane; i < M; i += 64)
            if (i > jj) col[i] *= scale;
    }
    if (lane == 0) {
        col[jj] = beta;
        tau_sh[jj] = tau;
    }
}

// In place QR of A (M x K, K <= M, ld lda): R on and above the diagonal,
// reflectors below it, tau in tau_sh (shared, K entries).  The trailing update
// of step j gives one column per wave (lanes over rows); the wave that updates
// column j + 1 then forms its reflector, so each step needs one barrier.
template <class PA, class PT>
__device__ inline void wg_house_qr(PA A, int M, int K, int lda, PT tau_sh) {
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (K > 0 && wv == 0) wave_reflector(A, M, 0, lda, tau_sh);
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        const double tau = tau_sh[j];
        auto v = A + (int64_t)j * lda;
        for (int c = j + 1 + wv; c < K; c += nw) {
            if (tau != 0.0) {
                auto col = A + (int64_t)c * lda;
                double part = 0.0;
                for (int i = j + 1 + lane; i < M; i += 64) part = fma(v[i], col[i], part);
                const double cj = col[j];
                const double w = tau * (cj + wave_sum(part));
                if (lane == 0) col[j] = cj - w;
                for (int i = j + 1 + lane; i < M; i += 64) col[i] = fma(-w, v[i], col[i]);
            }
            if (c == j + 1) wave_reflector(A, M, j + 1, lda, tau_sh);
        }
        __syncthreads();
    }
}

// The same QR with the columns held in registers (M <= 64 NS, K <= 64):
// column c lives in wave c % 4, lane l holding rows l + 64 q.  Step j: the
// wave holding column j forms its reflector (LAPACK larfg convention, as
// wave_reflector), stores the finished column to A and publishes v (zero
// above row j, one at it) and tau; after one barrier every wave applies the
// reflector to its later columns, whose sums are independent so their
// reductions overlap.  v alternates between two halves of vsh (2 M doubles),
// so one barrier per step suffices.
template <int NS, class PA, class PT>
__device__ __attribute__((noinline)) void wg_house_qr_reg(PA A, int M, int K, int lda, PT tau_sh, lds_f64* vsh) {
    constexpr int NW = WG / 64, CW = 64 / NW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double x[CW][NS];
#pragma unroll
    for (int t = 0; t < CW; ++t) {
        const int c = wv + NW * t;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int i = lane + 64 * q;
            x[t][q] = (c < K && i < M) ? (double)A[i + (int64_t)c * lda] : 0.0;
        }
    }
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        lds_f64* v = vsh + (j & 1) * M;
        if (wv == j % NW) {
            const int ot = j / NW;
#pragma unroll
            for (int t = 0; t < CW; ++t) {
                if (t != ot) continue;
                double part = 0.0, alpha = 0.0;
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int i = lane + 64 * q;
                    if (i == j) alpha = x[t][q];
                    if (i > j && i < M) part = fma(x[t][q], x[t][q], part);
                }
                const double xn2 = wave_sum(part);
                alpha = wave_sum(alpha);  // one lane holds it, the others add zeros
                double tau = 0.0, beta = alpha, scale = 0.0;
                if (xn2 != 0.0) {
                    const double nrm = hypot(alpha, sqrt(xn2));
                    beta = (alpha >= 0.0) ? -nrm : nrm;
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int i = lane + 64 * q;
                    if (i >= M) continue;
                    double val = x[t][q], vi = 0.0;
                    if (i == j) {
                        val = beta;
                        vi = 1.0;
                    } else if (i > j) {
                        val = x[t][q] * scale;
                        vi = val;
                    }
                    A[i + (int64_t)j * lda] = val;
                    v[i] = vi;
                }
                if (lane == 0) tau_sh[j] = tau;
            }
        }
        __syncthreads();
        const double tau = tau_sh[j];
        if (tau == 0.0) continue;
        double vq[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int i = lane + 64 * q;
            vq[q] = i < M ? (double)v[i] : 0.0;
        }
        double w[CW];
#pragma unroll
        for (int t = 0; t < CW; ++t) {
            double part = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) part = fma(vq[q], x[t][q], part);
            w[t] = part;
        }
#pragma unroll
        for (int t = 0; t < CW; ++t) {
            const int c = wv + NW * t;
            const double wt = (c > j && c < K) ? tau * wave_sum(w[t]) : 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) x[t][q] = fma(-wt, vq[q], x[t][q]);
        }
    }
    __syncthreads();
}

// Columns [c0, c0 + nq) of Q = H_0 H_1 ... H_{K-1} (M x M) from the reflectors
// left in A by wg_house_qr, into Q (ld ldq).  With flip, column c < K is
// negated where R_cc < 0 (the orthonormal factor with a positive diagonal).
// One wave per pair of columns (the second one only with hb), in registers;
// no barriers inside.
template <int NS, class PA, class PT, class PQ>
__device__ inline void wave_form_q(PA A, int M, int K, int lda, PT tau_sh, int ca, int cb, bool hb, bool flip, PQ Qa,
                                   PQ Qb) {
    const int lane = threadIdx.x & 63;
    double x[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        x[s] = (s * 64 + lane == ca) ? 1.0 : 0.0;
        y[s] = (hb && s * 64 + lane == cb) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int sb = NS - 1; sb >= 0; --sb) {
        const int jt = min(K - 1, sb * 64 + 63);
        for (int j = jt; j >= sb * 64; --j) {
            const double tau = tau_sh[j];
            if (tau == 0.0) continue;
            auto v = A + (int64_t)j * lda;
            double px = 0.0, py = 0.0;
#pragma unroll
            for (int s = sb; s < NS; ++s) {
                const int i = s * 64 + lane;
                if (i > j && i < M) {
                    const double vi = v[i];
                    px = fma(vi, x[s], px);
                    py = fma(vi, y[s], py);
                }
            }
            const double wx = tau * (readlane_d(x[sb], j - sb * 64) + wave_sum(px));
            const double wy = tau * (readlane_d(y[sb], j - sb * 64) + wave_sum(py));
            if (lane == j - sb * 64) {
                x[sb] -= wx;
                y[sb] -= wy;
            }
#pragma unroll
            for (int s = sb; s < NS; ++s) {
                const int i = s * 64 + lane;
                if (i > j && i < M) {
                    const double vi = v[i];
                    x[s] = fma(-wx, vi, x[s]);
                    y[s] = fma(-wy, vi, y[s]);
                }
            }
        }
    }
    const double sa = (flip && ca < K && A[ca + (int64_t)ca * lda] < 0.0) ? -1.0 : 1.0;
    const double sbn = (hb && flip && cb < K && A[cb + (int64_t)cb * lda] < 0.0) ? -1.0 : 1.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * 64 + lane;
        if (i < M) {
            Qa[i] = sa * x[s];
            if (hb) Qb[i] = sbn * y[s];
        }
    }
}

template <int NS, class PA, class PT, class PQ>
__device__ inline void wg_form_q_ns(PA A, int M, int K, int lda, PT tau_sh, int c0, int nq, bool flip, PQ Q, int ldq) {
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wv; c < nq; c += 2 * nw) {
        const int c2 = c + nw;
        const bool hb = c2 < nq;
        wave_form_q<NS, PA, PT, PQ>(A, M, K, lda, tau_sh, c0 + c, c0 + c2, hb, flip, Q + (int64_t)c * ldq,
                                    Q + (int64_t)(hb ? c2 : c) * ldq);
    }
}

template <class PA, class PT, class PQ>
__device__ inline void wg_house_form_q(PA A, int M, int K, int lda, PT tau_sh, int c0, int nq, PQ Q, int ldq,
                                       bool flip = false) {
    switch ((M + 63) >> 6) {
        case 0: break;
        case 1: wg_form_q_ns<1, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 2: wg_form_q_ns<2, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 3: wg_form_q_ns<3, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 4: wg_form_q_ns<4, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 5: wg_form_q_ns<5, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 6: wg_form_q_ns<6, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        case 7: wg_form_q_ns<7, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
        default: wg_form_q_ns<8, PA, PT, PQ>(A, M, K, lda, tau_sh, c0, nq, flip, Q, ldq); break;
    }
    __syncthreads();
}

// Columns [c0, c0 + nq) of Q = H_0 ... H_{K-1} from the reflectors left in A
// (ld lda) by wg_house_qr, through the compact WY form Q = I - Y T Y^T (Y unit
// lower trapezoidal; T upper triangular with T^{-1} = diag(1/tau) +
// strict_upper(Y^T Y), the UT-transform identity; a reflector with tau = 0 is
// the identity and gets a zero row and column in T):
//   G = Y^T Y;  T = (diag(1/tau) + strict_upper(G))^{-1};  Z = T Y[c0:c0+nq, :]^T;
//   Q[:, cols] = E - Y Z.
// K <= 128.  Gs, Ts (K x K) and Zs (K x nq) are global scratch, scr 8 x 256
// doubles of LDS.  With flip, column c < K is negated where R_cc < 0.
template <class PA, class PT, class PQ>
__device__ void wg_house_form_q_wy(PA A, int M, int K, int lda, PT tau_sh, int c0, int nq, PQ Q, int ldq, bool flip,
                                   double* Gs, double* Ts, double* Zs, lds_smem* sm, lds_f64* scr) {
    auto Y = [&](int i, int j) -> double { return i == j ? 1.0 : (i > j ? (double)A[i + (int64_t)j * lda] : 0.0); };
    wg_gemm_fn(K, K, M, [&](int r, int k) { return Y(k, r); }, [&](int k, int c) { return Y(k, c); }, sm,
               [&](int r, int c, double v) { Gs[r + (int64_t)c * K] = v; });
    {
        const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
        for (int j = threadIdx.x >> 6; j < K; j += nw) {
            const bool zj = tau_sh[j] == 0.0;
            for (int i = lane; i <= j; i += 64) {
                double& g = Gs[i + (int64_t)j * K];
                if (i == j)
                    g = zj ? 1.0 : 1.0 / tau_sh[j];
                else if (zj || tau_sh[i] == 0.0)
                    g = 0.0;
            }
        }
    }
    __syncthreads();
    wg_trinv_upper<1>(Gs, K, K, Ts, K, scr);
    for (int j = threadIdx.x; j < K; j += blockDim.x)
        if (tau_sh[j] == 0.0) Ts[j + (int64_t)j * K] = 0.0;
    __syncthreads();
    wg_gemm_fn(K, nq, K, [&](int r, int k) { return Ts[r + (int64_t)k * K]; }, [&](int k, int c) { return Y(c0 + c, k); },
               sm, [&](int r, int c, double v) { Zs[r + (int64_t)c * K] = v; });
    wg_gemm_fn(M, nq, K, [&](int r, int k) { return Y(r, k); }, [&](int k, int c) { return Zs[k + (int64_t)c * K]; }, sm,
               [&](int r, int c, double v) {
                   const int col = c0 + c;
                   double q = (r == col ? 1.0 : 0.0) - v;
                   if (flip && col < K && A[col + (int64_t)col * lda] < 0.0) q = -q;
                   Q[r + (int64_t)c * ldq] = q;
               });
}

}  // namespace hs
