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

namespace hs {

constexpr int WG = 256;       // threads of a per-cluster workgroup
constexpr int LDS_M = 128;    // clusters up to this size keep their working matrix in LDS
constexpr int PANEL = 32;     // column panel of the neighbour / fill update kernels
constexpr int SCHUR_T = 64;   // output tile of the Schur-complement GEMM
constexpr int MAX_M = 512;    // largest cluster the kernels accept
// Fill whose largest row norm is at most this fraction of ||A_ss||_F is the
// rounding noise of earlier Schur updates and is treated as zero.
constexpr double FILL_NOISE_FLOOR = 1e-12;

// Per-level view of the factorization state (device pointers).
struct LevelDev {
    int ncl;
    int symmetric;
    double eps;
    int fixed_rank;
    int gram_splits;
    const int* m;             // [ncl] sizes at the start of the level
    int* k;                   // [ncl] coarse sizes after elimination (rank)
    int* flag;                // [ncl] 1 = breakdown in an unpivoted LU
    const int64_t* blk_off;   // [nblk] element offset of every block (capacity m_a x m_b, ld m_a)
    double* blocks;
    const int* diag_blk;      // [ncl] block id of (s, s)
    const int* nbr_ptr;       // [ncl+1] neighbours n(s)
    const int* nbr_id;
    const int* nbr_before;    // neighbour processed before s (then it has its coarse size)
    const int* nbr_bsa;       // block id of (s, a)
    const int* nbr_bas;       // block id of (a, s)
    int* nbr_noff;            // packed offset of a inside E_L / E_R (written by the pivot kernel)
    int* ntot;                // [ncl] sum of the current neighbour sizes (written by the pivot kernel)
    const int* ncap;          // [ncl] sum of the neighbours' level-start sizes (record capacity)
    const int* fill_ptr;      // [ncl+1] fill partners w(s)
    const int* fill_id;
    const int* fill_before;
    const int* fill_bst;      // block id of (s, t)
    const int* fill_bts;      // block id of (t, s)
    const int64_t* pair_base; // [ncl] index of pair (0,0) of s in pair_blk
    const int* pair_blk;      // block id of (a_i, a_j) at pair_base[s] + i*nb + j
    const int64_t* rec_off;   // [ncl] record: T_L' (m^2), T_R' (m^2), E_R (m x ncap, ld m), E_L (ncap x m, ld ncap)
    double* rec;
    const int64_t* ws_off;    // [ncl] per-colour workspace of every cluster
    double* ws;
};

// Workspace slots of a cluster (each m x m, column major, ld m).
enum WsSlot { WS_AINV = 0, WS_LINV, WS_UINV, WS_U, WS_X, WS_SL, WS_SR, WS_TL, WS_TR, WS_CU, WS_UC, WS_SCR, WS_GP };
__host__ __device__ inline int64_t ws_slots(int gram_splits) { return WS_GP + gram_splits; }

__device__ inline int cur_size(const LevelDev& L, int a, int before) { return before ? L.k[a] : L.m[a]; }
__device__ inline double* blk_ptr(const LevelDev& L, int id) { return L.blocks + L.blk_off[id]; }

// ---------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_min_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide reductions (blockDim.x a multiple of 64, <= 1024); red has >= 16 slots.
__device__ inline double block_sum(double v, double* red) {
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
__device__ inline double block_max(double v, double* red) {
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
__device__ inline int block_min_int(int v, int* red) {
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

__device__ inline void wg_copy(int M, int N, const double* src, int lds, double* dst, int ldd) {
    for (int64_t e = threadIdx.x; e < (int64_t)M * N; e += blockDim.x) {
        int i = (int)(e % M), j = (int)(e / M);
        dst[i + (int64_t)j * ldd] = src[i + (int64_t)j * lds];
    }
}
__device__ inline void wg_zero(int M, int N, double* dst, int ldd) {
    for (int64_t e = threadIdx.x; e < (int64_t)M * N; e += blockDim.x) {
        int i = (int)(e % M), j = (int)(e / M);
        dst[i + (int64_t)j * ldd] = 0.0;
    }
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

// la(r, k) / lb(k, c) return the operand element or 0 outside the matrix.
template <class LoadL, class LoadR>
__device__ inline void mfma_tile64(int K, const LoadL& la, const LoadR& lb, MfmaSmem* sm, v4d acc[2][2]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += MKC) {
        __syncthreads();
        for (int e = tid; e < MT * MKC; e += WG) {
            const int r = e % MT, kk = e / MT;
            sm->a[kk][r] = (k0 + kk < K) ? la(r, k0 + kk) : 0.0;
            const int kb = e % MKC, c = e / MKC;
            sm->b[kb][c] = (k0 + kb < K) ? lb(k0 + kb, c) : 0.0;
        }
        __syncthreads();
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
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[i][j], 0, 0, 0);
        }
    }
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

// ------------------------------------------------------------ cooperative GEMM
// C (M x N) = alpha op(A) op(B) + beta C; op(A) is M x K, op(B) is K x N, on
// the FP64 matrix cores, 64 x 64 tiles.  beta == 0 never reads C.
typedef MfmaSmem GemmSmem;

template <bool TA, bool TB>
__device__ void wg_gemm(int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb,
                        double beta, double* C, int ldc, GemmSmem* sm) {
    for (int r0 = 0; r0 < M; r0 += MT)
        for (int c0 = 0; c0 < N; c0 += MT) {
            v4d acc[2][2];
            mfma_tile64(
                K,
                [&](int r, int k) {
                    const int gr = r0 + r;
                    return gr < M ? (TA ? A[k + (int64_t)gr * lda] : A[gr + (int64_t)k * lda]) : 0.0;
                },
                [&](int k, int c) {
                    const int gc = c0 + c;
                    return gc < N ? (TB ? B[gc + (int64_t)k * ldb] : B[k + (int64_t)gc * ldb]) : 0.0;
                },
                sm, acc);
            mfma_tile64_store(acc, [&](int r, int c, double v) {
                const int gr = r0 + r, gc = c0 + c;
                if (gr < M && gc < N) {
                    double* p = C + gr + (int64_t)gc * ldc;
                    *p = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * *p);
                }
            });
        }
    __syncthreads();
}

// ---------------------------------------------------- LU without pivoting
// In place Doolittle LU of the M x M matrix W (ld ldw).  Returns false on a
// zero or non-finite pivot (every thread gets the same answer).
__device__ inline bool wg_lu_nopiv(double* W, int M, int ldw, int* flag_sh) {
    const int tid = threadIdx.x;
    if (tid == 0) *flag_sh = 0;
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        const double p = W[j + (int64_t)j * ldw];
        if (p == 0.0 || !isfinite(p)) {
            if (tid == 0) *flag_sh = 1;
        }
        __syncthreads();
        if (*flag_sh) return false;
        const double inv = 1.0 / p;
        for (int i = j + 1 + tid; i < M; i += blockDim.x) W[i + (int64_t)j * ldw] *= inv;
        __syncthreads();
        const int n = M - j - 1;
        for (int64_t e = tid; e < (int64_t)n * n; e += blockDim.x) {
            int i = j + 1 + (int)(e % n), c = j + 1 + (int)(e / n);
            W[i + (int64_t)c * ldw] -= W[i + (int64_t)j * ldw] * W[j + (int64_t)c * ldw];
        }
        __syncthreads();
    }
    return true;
}

// out = L^{-1}, L = unit lower triangle of W.  One column of the inverse per thread.
__device__ inline void wg_trinv_lower_unit(const double* W, int M, int ldw, double* out, int ldo) {
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        double* x = out + (int64_t)c * ldo;
        for (int i = 0; i < c; ++i) x[i] = 0.0;
        x[c] = 1.0;
        for (int i = c + 1; i < M; ++i) {
            double s = 0.0;
            for (int j = c; j < i; ++j) s = fma(W[i + (int64_t)j * ldw], x[j], s);
            x[i] = -s;
        }
    }
    __syncthreads();
}

// out = U^{-1}, U = upper triangle of W (with diagonal).
__device__ inline void wg_trinv_upper(const double* W, int M, int ldw, double* out, int ldo) {
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        double* x = out + (int64_t)c * ldo;
        for (int i = c + 1; i < M; ++i) x[i] = 0.0;
        for (int i = c; i >= 0; --i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int j = i + 1; j <= c; ++j) s = fma(-W[i + (int64_t)j * ldw], x[j], s);
            x[i] = s / W[i + (int64_t)i * ldw];
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------- Householder QR
// In place QR of A (M x K, K <= M) with reflectors H_j = I - tau_j v_j v_j^T,
// v_j(0) = 1, beta_j = -sign(alpha) ||x|| (LAPACK larfg convention, tau = 0
// when the part below the diagonal is zero).  R on and above the diagonal,
// v below it; tau in tau_sh (shared, K entries).
__device__ inline void wg_house_qr(double* A, int M, int K, int lda, double* tau_sh, double* red) {
    const int tid = threadIdx.x;
    for (int j = 0; j < K; ++j) {
        double part = 0.0;
        for (int i = j + 1 + tid; i < M; i += blockDim.x) {
            double v = A[i + (int64_t)j * lda];
            part = fma(v, v, part);
        }
        const double xn2 = block_sum(part, red);
        const double alpha = A[j + (int64_t)j * lda];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (xn2 != 0.0) {
            const double nrm = hypot(alpha, sqrt(xn2));
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        __syncthreads();
        if (xn2 != 0.0)
            for (int i = j + 1 + tid; i < M; i += blockDim.x) A[i + (int64_t)j * lda] *= scale;
        if (tid == 0) tau_sh[j] = tau;
        __syncthreads();
        if (tid == 0) A[j + (int64_t)j * lda] = beta;
        // apply H_j to the trailing columns: one column per thread
        if (tau != 0.0)
            for (int c = j + 1 + tid; c < K; c += blockDim.x) {
                double* col = A + (int64_t)c * lda;
                const double* v = A + (int64_t)j * lda;
                double w = col[j];
                for (int i = j + 1; i < M; ++i) w = fma(v[i], col[i], w);
                w *= tau;
                col[j] -= w;
                for (int i = j + 1; i < M; ++i) col[i] = fma(-w, v[i], col[i]);
            }
        __syncthreads();
    }
}

// Q columns [c0, c0 + nq) of Q = H_0 H_1 ... H_{K-1} (M x M) from the
// reflectors left in A by wg_house_qr; written to Q (ld ldq), one column per thread.
__device__ inline void wg_house_form_q(const double* A, int M, int K, int lda, const double* tau_sh, int c0, int nq,
                                       double* Q, int ldq) {
    for (int c = threadIdx.x; c < nq; c += blockDim.x) {
        double* q = Q + (int64_t)c * ldq;
        for (int i = 0; i < M; ++i) q[i] = (i == c0 + c) ? 1.0 : 0.0;
        for (int j = K - 1; j >= 0; --j) {
            const double tau = tau_sh[j];
            if (tau == 0.0) continue;
            const double* v = A + (int64_t)j * lda;
            double w = q[j];
            for (int i = j + 1; i < M; ++i) w = fma(v[i], q[i], w);
            w *= tau;
            q[j] -= w;
            for (int i = j + 1; i < M; ++i) q[i] = fma(-w, v[i], q[i]);
        }
    }
    __syncthreads();
}

}  // namespace hs
