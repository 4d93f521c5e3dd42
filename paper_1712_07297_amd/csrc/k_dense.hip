// Dense levels.  When every cluster of a level neighbours every other one,
// no cluster has fill (Sec. 2.3: fill needs a pair at distance two), so every
// cluster is eliminated exactly by a block LU step and the level is the
// "small enough" case of Alg. 1, factored by the conventional dense
// factorization: here an unpivoted LU of the whole level matrix in
// processing order, blocked with panels of at most 128 columns (128 by
// default; narrower panels run the same kernels on smaller matrices).  The
// per-cluster operators of the solve (T_L' = L_ss^{-1}, T_R' = U_ss^{-1},
// E_R = U[s, later], E_L = L[later, s]) are then cut out of the factors.
#include <algorithm>
#include <vector>

#include "device_common.h"
#include "kernels.h"

namespace hs {

constexpr int DNB = 128;  // widest panel (layout of the diagonal inverses)

// D[o_a + i, o_b + j] = B(a, b)[i, j] for every block of the clusters
// c0 .. c0 + ncl - 1 (pattern entries from b0; a, c local to the range).
__global__ void k_dense_assemble(const int* __restrict__ pat_ptr, const int* __restrict__ pat, int c0, int b0,
                                 const int* __restrict__ m, const int64_t* __restrict__ off,
                                 const int64_t* __restrict__ blk_off, const double* __restrict__ blocks,
                                 double* __restrict__ D, int64_t ldd, int ncl) {
    const int b = b0 + blockIdx.x;
    // row cluster of block b: last a with pat_ptr[c0 + a] <= b
    int lo = 0, hi = ncl;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pat_ptr[c0 + mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    const int a = lo, c = pat[b] - c0;
    const int ma = m[a], mc = m[c];
    const double* src = blocks + blk_off[b];
    double* dst = D + off[a] + off[c] * ldd;
    for (int x = threadIdx.x; x < ma * mc; x += blockDim.x) {
        const int i = x % ma, j = x / ma;
        dst[i + (int64_t)j * ldd] = src[i + (int64_t)j * ma];
    }
}

// LU of the diagonal block D[p:p+nb, p:p+nb] in LDS; writes the factors back
// and L11^{-1}, U11^{-1} (nb x nb, ld DNB) to inv.
__global__ void __launch_bounds__(WG) k_dense_diag(double* __restrict__ D, int64_t ldd, int p, int nb,
                                                   double* __restrict__ inv, int* __restrict__ flag) {
    extern __shared__ double Wd[];  // nb x nb
    __shared__ double scr_d[8 * 256];
    lds_f64* W = to_lds(Wd);
    double* dp = D + p + (int64_t)p * ldd;
    wg_copy(nb, nb, dp, (int)ldd, W, nb);
    __syncthreads();
    __shared__ int fl;
    if (!wg_lu<true>(W, nb, nb, to_lds(scr_d), to_lds(&fl))) {
        if (threadIdx.x == 0) *flag = 1;
        return;
    }
    wg_copy(nb, nb, W, nb, dp, (int)ldd);
    __syncthreads();
    wg_trinv_lower_unit<1>(W, nb, nb, inv, DNB, to_lds(scr_d));
    wg_trinv_upper<1>(W, nb, nb, inv + DNB * DNB, DNB, to_lds(scr_d));
}

// Panel updates, in place: column chunks of U12 = L11^{-1} D[p:p+nb, chunk]
// (blockIdx.x < nchunks) and row chunks of L21 = D[chunk, p:p+nb] U11^{-1}.
__global__ void __launch_bounds__(WG) k_dense_panels(double* __restrict__ D, int64_t ldd, int N, int p, int nb,
                                                     const double* __restrict__ inv, const int* __restrict__ flag) {
    __shared__ MfmaSmem sm;
    if (*flag) return;
    const int nchunks = (N - p - nb + MT - 1) / MT;
    const bool colpanel = (int)blockIdx.x < nchunks;
    const int q0 = p + nb + (colpanel ? blockIdx.x : blockIdx.x - nchunks) * MT;
    const double* Linv = inv;
    const double* Uinv = inv + DNB * DNB;
    // both 64-wide halves are computed before either is stored: each half
    // reads the whole panel it overwrites
    v4d acc[2][2][2];
    const int halves = (nb + MT - 1) / MT;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h >= halves) break;
        const int hh = h * MT, hw = min(MT, nb - hh);
        if (colpanel)
            mfma_tile64<true>(
                nb, [&](int r, int k) { return (r < hw) ? Linv[(hh + r) + (int64_t)k * DNB] : 0.0; },
                [&](int k, int c) { return (q0 + c < N) ? D[(p + k) + (int64_t)(q0 + c) * ldd] : 0.0; }, to_lds(&sm),
                acc[h], hw, N - q0);
        else
            mfma_tile64<true>(
                nb, [&](int r, int k) { return (q0 + r < N) ? D[(q0 + r) + (int64_t)(p + k) * ldd] : 0.0; },
                [&](int k, int c) { return (c < hw) ? Uinv[k + (int64_t)(hh + c) * DNB] : 0.0; }, to_lds(&sm), acc[h],
                N - q0, hw);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h >= halves) break;
        const int hh = h * MT, hw = min(MT, nb - hh);
        if (colpanel)
            mfma_tile64_store(acc[h], [&](int r, int c, double v) {
                if (r < hw && q0 + c < N) D[(p + hh + r) + (int64_t)(q0 + c) * ldd] = v;
            });
        else
            mfma_tile64_store(acc[h], [&](int r, int c, double v) {
                if (q0 + r < N && c < hw) D[(q0 + r) + (int64_t)(p + hh + c) * ldd] = v;
            });
    }
}

// Trailing update D[p+nb:, p+nb:] -= L21 U12.
__global__ void __launch_bounds__(WG) k_dense_trailing(double* __restrict__ D, int64_t ldd, int N, int p, int nb,
                                                       const int* __restrict__ flag) {
    __shared__ MfmaSmem sm;
    if (*flag) return;
    const int q = p + nb;
    const int tiles = (N - q + MT - 1) / MT;
    const int r0 = q + (blockIdx.x % tiles) * MT, c0 = q + (blockIdx.x / tiles) * MT;
    v4d acc[2][2];
    mfma_tile64<true>(
        nb, [&](int r, int k) { return (r0 + r < N) ? D[(r0 + r) + (int64_t)(p + k) * ldd] : 0.0; },
        [&](int k, int c) { return (c0 + c < N) ? D[(p + k) + (int64_t)(c0 + c) * ldd] : 0.0; }, to_lds(&sm), acc,
        N - r0, N - c0);
    mfma_tile64_store(acc, [&](int r, int c, double v) {
        if (r0 + r < N && c0 + c < N) D[(r0 + r) + (int64_t)(c0 + c) * ldd] -= v;
    });
}

// Per-cluster operators from the factors: T_L' = inverse of the unit lower
// diagonal block, T_R' = inverse of the upper diagonal block (one workgroup
// per cluster, L2-resident).
__global__ void __launch_bounds__(WG) k_dense_inverses(const double* __restrict__ D, int64_t ldd,
                                                       const int* __restrict__ m, const int64_t* __restrict__ off,
                                                       const int64_t* __restrict__ rec_off, double* __restrict__ rec) {
    __shared__ double scr_d[8 * 256];
    const int s = blockIdx.x;
    const int M = m[s];
    if (M == 0) return;
    const double* dd = D + off[s] + off[s] * ldd;
    double* TL = rec + rec_off[s];
    double* TR = TL + (int64_t)M * M;
    wg_trinv_lower_unit(dd, M, (int)ldd, TL, M, to_lds(scr_d));
    wg_trinv_upper(dd, M, (int)ldd, TR, M, to_lds(scr_d));
}

// E_R = U[s, later] (M x nt, ld M) and E_L = L[later, s] (nt x M, ld ncap).
__global__ void k_dense_couplings(const double* __restrict__ D, int64_t ldd, int N, const int* __restrict__ m,
                                  const int64_t* __restrict__ off, const int* __restrict__ ncap,
                                  const int64_t* __restrict__ rec_off, double* __restrict__ rec, int s) {
    const int M = m[s];
    const int64_t o = off[s], nt = N - o - M;
    const int64_t MM = (int64_t)M * M;
    double* ER = rec + rec_off[s] + 2 * MM;
    double* EL = ER + (int64_t)M * ncap[s];
    const int64_t tot = (int64_t)M * nt;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < tot; x += (int64_t)gridDim.x * blockDim.x) {
        // E_R: element (i, j), i fastest
        const int64_t i = x % M, j = x / M;
        ER[i + j * M] = D[(o + i) + (o + M + j) * ldd];
        // E_L: element (j2, i2), j2 fastest
        const int64_t j2 = x % nt, i2 = x / nt;
        EL[j2 + i2 * ncap[s]] = D[(o + M + j2) + (o + i2) * ldd];
    }
}

int dense_level_factor(double* D, int64_t N, const int* pat_ptr, const int* pat, int c0, int b0, const int* m,
                       const int64_t* off, const int64_t* blk_off, const double* blocks, int ncl, int nblk,
                       double* inv, int* flag, const int* ncap, const int64_t* rec_off, double* rec,
                       const std::vector<int>& m_host, const std::vector<int64_t>& off_host, int panel, hipStream_t st) {
    const int pw = std::max(16, std::min(DNB, panel));
    launch_fill_zero(D, N * N * (int64_t)sizeof(double), st);
    if (nblk > 0)
        hipLaunchKernelGGL(k_dense_assemble, dim3(nblk), dim3(256), 0, st, pat_ptr, pat, c0, b0, m, off, blk_off,
                           blocks, D, (int64_t)N, ncl);
    for (int64_t p = 0; p < N; p += pw) {
        const int nb = (int)std::min<int64_t>(pw, N - p);
        hipLaunchKernelGGL(k_dense_diag, dim3(1), dim3(WG), (size_t)nb * nb * sizeof(double), st, D, (int64_t)N, (int)p,
                           nb, inv, flag);
        const int64_t rest = N - p - nb;
        if (rest <= 0) break;
        const int chunks = (int)((rest + MT - 1) / MT);
        hipLaunchKernelGGL(k_dense_panels, dim3(2 * chunks), dim3(WG), 0, st, D, (int64_t)N, (int)N, (int)p, nb, inv,
                           flag);
        hipLaunchKernelGGL(k_dense_trailing, dim3((unsigned)((int64_t)chunks * chunks)), dim3(WG), 0, st, D,
                           (int64_t)N, (int)N, (int)p, nb, flag);
    }
    hipLaunchKernelGGL(k_dense_inverses, dim3(ncl), dim3(WG), 0, st, D, (int64_t)N, m, off, rec_off, rec);
    for (int s = 0; s < ncl; ++s) {
        const int64_t M = m_host[s];
        const int64_t nt = N - off_host[s] - M;
        if (M == 0 || nt == 0) continue;
        const int64_t tot = M * nt;
        const unsigned g = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
        hipLaunchKernelGGL(k_dense_couplings, dim3(g), dim3(256), 0, st, D, (int64_t)N, (int)N, m, off, ncap, rec_off,
                           rec, s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace hs
