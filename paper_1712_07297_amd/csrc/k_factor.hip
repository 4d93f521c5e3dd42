// Factorization kernels: one level of the hierarchical solver, one colour at a
// time (clusters of one colour are more than two apart in A_B, Sec. 2.3, so
// every kernel below runs all of them at once without write conflicts).
//
// Per cluster s with m unknowns, k coarse unknowns and f = m - k fine ones:
//   gram      G = F F^T, F = [A_s,w ...] (+ [A_w,s^T ...] when A is
//             nonsymmetric): the fill blocks of s (Eq. lra), partial sums over
//             slices of the fill partners;
//   pivot     LU of A_ss with explicit L^{-1}, U^{-1}, A_ss^{-1}; the
//             row-pivoted truncated QR of F^T computed as a pivoted Cholesky
//             of G; U; V_L (V_R) = complement of A_ss^{-1} U (A_ss^{-T} U);
//             T_L = [V_L U]^T A_ss^{-1}, T_R = A_ss^{-1} [V_R U] (the two
//             halves of E_s, Eq. scaling); F_ff = V_L^T A_ss^{-1} V_R = L_f U_f
//             (Eq. elim); folded operators T_L' = diag(L_f^{-1}, I) T_L,
//             T_R' = T_R diag(U_f^{-1}, I); C = U^T A_ss^{-1} U;
//   fill      coarse fill blocks C Z (Eq. scaling), Z = U^T F;
//   nbr       [E_R; B_cn] = T_L' A_sn and [E_L, B_nc] = A_ns T_R';
//   schur     A_ab -= E_L[a] E_R[b] for every ordered neighbour pair (Eq. elim).
// A cluster without fill keeps E_s = I (Sec. 2.2): T_L' = L^{-1}, T_R' = U^{-1}.
// Blocks of a processed cluster keep its coarse rows / columns first.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace hs {

__device__ inline int find_cluster(const int* pre, int n, int q) {
    // largest ci with pre[ci] <= q (pre ascending, pre[0] = 0)
    int lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}
__device__ inline int find_cluster64(const int64_t* pre, int n, int64_t q) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Packed offsets of every cluster's current neighbour sizes inside E_L / E_R
// (nbr_noff) and their sum (ntot): a prefix sum over the neighbour list, a
// workgroup's width at a time; and the sum of its current fill-partner sizes
// (fcols).  One workgroup per cluster of the colour, either in a launch of
// its own or as the last column of the Gram launch's grid (the Gram partials
// neither read nor write these arrays).
__device__ void offsets_body(const LevelDev& L, int s, lds_i32* buf) {
    const int tid = threadIdx.x;
    const int e0 = L.nbr_ptr[s], ne = L.nbr_ptr[s + 1] - e0;
    int carry = 0;
    for (int b = 0; b < ne; b += blockDim.x) {
        const int e = b + tid;
        const int v = e < ne ? cur_size(L, L.nbr_id[e0 + e], L.nbr_before[e0 + e]) : 0;
        int tot;
        const int ex = block_scan_excl(v, buf, &tot);
        if (e < ne) L.nbr_noff[e0 + e] = carry + ex;
        carry += tot;
    }
    if (tid == 0) L.ntot[s] = carry;
    const int f0 = L.fill_ptr[s], nf = L.fill_ptr[s + 1] - f0;
    int fc = 0;
    for (int b = 0; b < nf; b += blockDim.x) {
        const int e = b + tid;
        const int v = e < nf ? cur_size(L, L.fill_id[f0 + e], L.fill_before[f0 + e]) : 0;
        int tot;
        (void)block_scan_excl(v, buf, &tot);
        fc += tot;
    }
    if (tid == 0) L.fcols[s] = fc;
}

__global__ void __launch_bounds__(WG) k_offsets(LevelDev L, const int* __restrict__ clist) {
    __shared__ int buf[WG];
    offsets_body(L, clist[blockIdx.x], to_lds(buf));
}

// ============================================================== Gram partials

// G_split = sum over the split's fill partners t of B(s,t) B(s,t)^T (and, for
// a general matrix, + B(t,s)^T B(t,s)): the Gram matrix F F^T of the fill
// (Eq. lra) in gram_splits_of(nf) partial sums.  Each 64 x 64 tile of the partial is
// accumulated over all partners of the split in registers and stored once.
template <class T>
__global__ void __launch_bounds__(WG) k_gram(LevelDev L, const int* __restrict__ clist, int with_offsets) {
    __shared__ GemmSmem sm;
    __shared__ int obuf[WG];
    const int s = clist[blockIdx.y];
    const int split = blockIdx.x;
    if (with_offsets && split == (int)gridDim.x - 1) {
        offsets_body(L, s, to_lds(obuf));
        return;
    }
    const int M = L.m[s];
    if (M == 0) return;
    double* Gp = L.ws + L.ws_off[s] + (int64_t)(WS_GP + split) * M * M;
    const int f0 = L.fill_ptr[s], nf = L.fill_ptr[s + 1] - f0;
    const int splits = gram_splits_of(nf, L.kn.gram_splits_max);
    if (split >= splits) return;
    const int chunk = (nf + splits - 1) / splits;
    const int e0 = f0 + split * chunk, e1 = min(f0 + nf, e0 + chunk);
    lds_smem* sm_l = to_lds(&sm);
    for (int r0 = 0; r0 < M; r0 += MT)
        for (int c0 = 0; c0 < M; c0 += MT) {
            v4d acc[2][2];
            mfma_zero(acc);
            for (int e = e0; e < e1; ++e) {
                const int t = L.fill_id[e];
                const int ct = cur_size(L, t, L.fill_before[e]);
                if (ct == 0) continue;
                const T* Bst = blk_t<T>(L, L.fill_bst[e]);  // M x ct, ld M
                mfma_tile64_acc<true>(
                    ct, [&](int r, int k) { return r0 + r < M ? Bst[(r0 + r) + (int64_t)k * M] : 0.0; },
                    [&](int k, int c) { return c0 + c < M ? Bst[(c0 + c) + (int64_t)k * M] : 0.0; }, sm_l, acc, M - r0,
                    M - c0);
                if (!L.symmetric) {
                    const int mt = L.m[t];
                    const T* Bts = blk_t<T>(L, L.fill_bts[e]);  // ct x M, ld m_t
                    mfma_tile64_acc<true>(
                        ct, [&](int r, int k) { return r0 + r < M ? Bts[k + (int64_t)(r0 + r) * mt] : 0.0; },
                        [&](int k, int c) { return c0 + c < M ? Bts[k + (int64_t)(c0 + c) * mt] : 0.0; }, sm_l, acc,
                        M - r0, M - c0);
                }
            }
            mfma_tile64_store(acc, [&](int r, int c, double v) {
                if (r0 + r < M && c0 + c < M) Gp[(r0 + r) + (int64_t)(c0 + c) * M] = v;
            });
        }
}

// Partial 0 += partials 1 .. splits-1 (in that order), one entry per thread.
__global__ void k_gram_reduce(LevelDev L, const int* __restrict__ clist) {
    const int s = clist[blockIdx.y];
    const int M = L.m[s];
    const int64_t MM = (int64_t)M * M;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MM) return;
    const int splits = gram_splits_of(L.fill_ptr[s + 1] - L.fill_ptr[s], L.kn.gram_splits_max);
    double* G = L.ws + L.ws_off[s] + WS_GP * MM;
    double g = G[e];
    int sp = 1;
    for (; sp + 8 <= splits; sp += 8) {  // eight loads in flight, added in order
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = G[(sp + u) * MM + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) g += t[u];
    }
    for (; sp < splits; ++sp) g += G[sp * MM + e];
    G[e] = g;
}

void launch_gram(const LevelDev& L, const ColourDev& C, hipStream_t st, bool with_offsets) {
    if (C.n == 0) return;
    const dim3 grid(L.gram_splits + (with_offsets ? 1 : 0), C.n);
    if (C.f32)
        hipLaunchKernelGGL(k_gram<float>, grid, dim3(WG), 0, st, L, C.clist, (int)with_offsets);
    else
        hipLaunchKernelGGL(k_gram<double>, grid, dim3(WG), 0, st, L, C.clist, (int)with_offsets);
    const int64_t mm = (int64_t)C.max_m * C.max_m;
    if (L.gram_splits > 1 && mm > 0) {
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((mm + 255) / 256), C.n), dim3(256), 0, st, L, C.clist);
    }
}

// ============================================================== pivot kernel

// Pivoted Cholesky of the Gram matrix W (M x M, symmetric, ld M), i.e. the
// column-pivoted QR of F^T: pivot = largest remaining diagonal, ties within a
// relative 1e-10 go to the lowest current position, rows / columns exchanged
// physically; stop at the first chosen pivot d_j <= eps^2 d_0 (that is
// |R_jj| <= eps |R_11|) or at fixed_rank.  On return the first k columns of W
// hold the factor in the exchanged order and perm[i] is the unknown at
// position i.  The pivot search runs on one wave; the trailing update forms
// the scaled column on the fly and stores it after the update.
template <class PW, class PI, class PD>
__device__ int wg_pivoted_cholesky(PW W, int M, double eps, int fixed_rank, PI perm, PD d, PI isc) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    for (int i = tid; i < M; i += blockDim.x) {
        perm[i] = i;
        d[i] = W[i + (int64_t)i * M];
    }
    __syncthreads();
    double d0 = 0.0;
    int kk = 0;
    for (int j = 0; j < M; ++j) {
        if (wv == 0) {
            double mx = -1.0;
            for (int i = j + lane; i < M; i += 64) mx = fmax(mx, d[i]);
            mx = wave_max(mx);
            const double thr = (1.0 - 1e-10) * mx;
            int cand = M;
            for (int i = j + lane; i < M; i += 64)
                if (d[i] >= thr) {
                    cand = i;
                    break;
                }
            cand = wave_min_int(cand);
            if (lane == 0) isc[0] = (mx > 0.0) ? cand : -1;
        }
        __syncthreads();
        const int p = isc[0];
        if (p < 0) break;
        const double dj = d[p];
        if (j == 0) d0 = dj;
        if (dj <= eps * eps * d0) break;
        if (fixed_rank > 0 && j >= fixed_rank) break;
        if (p != j) {
            for (int c = tid; c < M; c += blockDim.x) {
                const double t = W[j + (int64_t)c * M];
                W[j + (int64_t)c * M] = W[p + (int64_t)c * M];
                W[p + (int64_t)c * M] = t;
            }
            __syncthreads();
            for (int r = tid; r < M; r += blockDim.x) {
                const double t = W[r + (int64_t)j * M];
                W[r + (int64_t)j * M] = W[r + (int64_t)p * M];
                W[r + (int64_t)p * M] = t;
            }
            if (tid == 0) {
                const int ti = perm[j];
                perm[j] = perm[p];
                perm[p] = ti;
                const double td = d[j];
                d[j] = d[p];
                d[p] = td;
            }
            __syncthreads();
        }
        const double ljj = sqrt(W[j + (int64_t)j * M]);
        const double inv = 1.0 / ljj;
        for (int r0 = j + 1; r0 < M; r0 += 64) {
            const int i = r0 + lane;
            if (i >= M) break;
            const double li = W[i + (int64_t)j * M] * inv;
            for (int c = j + 1 + wv; c < M; c += nw)
                W[i + (int64_t)c * M] = fma(-li, W[c + (int64_t)j * M] * inv, W[i + (int64_t)c * M]);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < M; i += blockDim.x) {
            W[i + (int64_t)j * M] *= inv;
            d[i] = W[i + (int64_t)i * M];
        }
        if (tid == 0) W[j + (int64_t)j * M] = ljj;
        kk = j + 1;
        __syncthreads();
    }
    __syncthreads();
    return kk;
}

// The same factorization, left-looking, for a Gram matrix held in LDS with
// M <= 128: nothing is exchanged physically.  Every wave keeps a replica of
// the remaining diagonal and of the current positions (lane l, slot s: the
// unknown l + 64 s) and finds the pivot itself, so a step needs one barrier.
// Column j is formed for every row u as W(u, p_j) - sum_{i<j} L(u, i) L(p_j, i)
// in the same order of fused multiply-adds as the right-looking update and is
// stored over column p_j of W, which no later step reads: the factor, the
// pivots and the stopping decisions are bit for bit those of the routine
// above.  piv[j] is the unknown chosen at step j, pos[u] the final position
// of unknown u.
template <class PW, class PI>
__device__ int wg_pivoted_cholesky_ll(PW W, int M, double eps, int fixed_rank, PI piv, PI pos) {
    const int tid = threadIdx.x, lane = tid & 63;
    double dr[2];
    int pr[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        const int u = lane + 64 * sl;
        dr[sl] = u < M ? W[u + (int64_t)u * M] : 0.0;
        pr[sl] = u;
    }
    double d0 = 0.0;
    int kk = 0;
    for (int j = 0; j < M; ++j) {
        if (j > 0) {  // the previous column updates the remaining diagonal
            const int pc = piv[j - 1];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int u = lane + 64 * sl;
                if (u < M && pr[sl] >= j) {
                    const double l = W[u + (int64_t)pc * M];
                    dr[sl] = fma(-l, l, dr[sl]);
                }
            }
        }
        double mx = -1.0;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
            if (lane + 64 * sl < M && pr[sl] >= j) mx = fmax(mx, dr[sl]);
        mx = wave_max(mx);
        if (!(mx > 0.0)) break;
        const double thr = (1.0 - 1e-10) * mx;
        int cand = M;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
            if (lane + 64 * sl < M && pr[sl] >= j && dr[sl] >= thr) cand = min(cand, pr[sl]);
        const int p = wave_min_int(cand);
        int up = M, uj = M;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const int u = lane + 64 * sl;
            if (u < M && pr[sl] == p) up = u;
            if (u < M && pr[sl] == j) uj = u;
        }
        up = wave_min_int(up);
        uj = wave_min_int(uj);
        const double dj = readlane_d(up < 64 ? dr[0] : dr[1], up & 63);
        if (j == 0) d0 = dj;
        if (dj <= eps * eps * d0) break;
        if (fixed_rank > 0 && j >= fixed_rank) break;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {  // exchange positions j and p
            const int u = lane + 64 * sl;
            if (u == up) pr[sl] = j;
            else if (u == uj) pr[sl] = p;
        }
        if (tid == 0) piv[j] = up;
        const double ljj = sqrt(dj);
        const double inv = 1.0 / ljj;
        if (tid < M) {
            const int u = tid;
            double c = W[u + (int64_t)up * M];
#pragma unroll 4
            for (int i = 0; i < j; ++i) {
                const int pi = piv[i];
                c = fma(-W[u + (int64_t)pi * M], W[up + (int64_t)pi * M], c);
            }
            W[u + (int64_t)up * M] = (u == up) ? ljj : c * inv;
        }
        kk = j + 1;
        __syncthreads();
    }
    if (tid < 64) {
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
            if (lane + 64 * sl < M) pos[lane + 64 * sl] = pr[sl];
    }
    __syncthreads();
    return kk;
}

// Orthonormal factor Q (M x k, positive diagonal R) of X = Q R by Cholesky
// QR: G = Y^T Y = R^T R, R = D^{-1/2} U_G from the unpivoted LU G = L_G U_G
// (D = diag U_G), Y <- Y R^{-1}.  One pass leaves an orthogonality error of
// about u cond(X)^2 = u pmax/pmin (Gram pivots); it suffices while
// pmin/pmax >= one_pass, else a second pass brings it to u.  Beyond cond(X) ~ 1e7
// (pmin < 1e-14 pmax) it returns false and leaves the caller to use
// Householder QR.  G is a k x k scratch, T1 an M x k and T2 a k x k global
// scratch.
constexpr double CHOLQR_ONE_PASS = 1e-6;  // one pass while cond(X) <= 1e3 (error ~ 1e-10)
// Clusters stored in float32 keep the orthogonality error of one pass below
// the rounding of their stored operators (6e-8) while cond(X) <= 1e4, which
// covers every truncation at eps >= 1e-4 (the kept pivots stay above eps^2).
constexpr double CHOLQR_ONE_PASS_F32 = 1e-8;

template <class PG>
__device__ bool wg_cholqr2(const double* X, int M, int k, PG G, double* T1, double* T2, double* Q, lds_smem* sm,
                           lds_f64* scr, lds_f64* red, lds_i32* flag, double one_pass) {
    const double* src = X;
    bool last = false;
    for (int pass = 0; pass < 2 && !last; ++pass) {
        wg_gemm<true, false>(k, k, M, 1.0, src, M, src, M, 0.0, G, k, sm);
        if (!wg_lu<true>(G, k, k, scr, flag)) return false;
        double pmax = 0.0, nmin = -INFINITY;
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            const double d = G[i + (int64_t)i * k];
            pmax = fmax(pmax, d);
            nmin = fmax(nmin, -d);
        }
        pmax = block_max(pmax, red);
        const double pmin = -block_max(nmin, red);
        if (!(pmin > 1e-14 * pmax)) return false;
        last = pass == 1 || pmin >= one_pass * pmax;
        double* dst = last ? Q : T1;
        if (k <= TRI_MFMA_MAX)
            wg_trinv_upper<1>(G, k, k, T2, k, scr);
        else
            wg_trinv_upper<0>(G, k, k, T2, k, scr);
        const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
        for (int j = threadIdx.x >> 6; j < k; j += nw) {
            const double sj = sqrt(G[j + (int64_t)j * k]);
            for (int i = lane; i <= j; i += 64) T2[i + (int64_t)j * k] *= sj;
        }
        __syncthreads();
        wg_gemm<false, false>(M, k, k, 1.0, src, M, T2, k, 0.0, dst, M, sm);
        src = dst;
    }
    return true;
}

// Householder complement: Q columns [K, M) of the QR of X (M x K, ld M) into
// V (ld ldv), Q formed through its compact WY form (scratch: three global
// M x M slots).  X is destroyed.  The QR keeps X in registers when it fits
// (M <= 128, K <= 64); scr then holds the published reflectors.  Which form
// runs is set by the size thresholds of kn (all give the same reflectors).
template <class PX, class PV, class PT>
__device__ void wg_complement(PX X, int M, int K, PV V, int ldv, PT tau_sh, double* s1, double* s2, double* s3,
                              lds_smem* sm, lds_f64* scr, const Knobs& kn) {
    if (K <= 64 && M <= min(64, kn.qr_reg1_max))
        wg_house_qr_reg<1>(X, M, K, M, tau_sh, scr);
    else if (K <= 64 && M <= min(128, kn.qr_reg2_max))
        wg_house_qr_reg<2>(X, M, K, M, tau_sh, scr);
    else
        wg_house_qr(X, M, K, M, tau_sh);
    if (K <= min(TRI_MFMA_MAX, kn.wy_max))
        wg_house_form_q_wy(X, M, K, M, tau_sh, K, M - K, V, ldv, false, s1, s2, s3, sm, scr);
    else
        wg_house_form_q(X, M, K, M, tau_sh, K, M - K, V, ldv);
}

// LU with partial pivoting of the M x M matrix W (ld ldw), in place, P W = L U
// with L unit lower: at step j the lowest row at or below j whose |entry| is
// within 1e-10 of the column's largest (one wave searches), rows exchanged
// across the whole matrix, the column divided by the pivot and the trailing
// block updated.  perm[i] = original row of row i.  False (nothing else
// changed) at a zero or non-finite pivot.
template <class PW>
__device__ bool wg_lu_partial(PW W, int M, int ldw, lds_i32* perm, lds_i32* ctl) {
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int u = tid; u < M; u += nth) perm[u] = u;
    for (int j = 0; j < M; ++j) {
        if (tid < 64) {
            double mx = 0.0;
            bool bad = false;
            for (int i = j + tid; i < M; i += 64) {
                const double a = fabs(W[i + (int64_t)j * ldw]);
                bad |= !(a <= 1.7976931348623157e308);  // NaN or infinite
                mx = fmax(mx, a);
            }
            mx = wave_max(mx);
            const double thr = (1.0 - 1e-10) * mx;
            int cand = M;
            for (int i = j + tid; i < M; i += 64)
                if (fabs(W[i + (int64_t)j * ldw]) >= thr) {
                    cand = i;
                    break;
                }
            cand = wave_min_int(cand);
            const int anybad = __builtin_amdgcn_readfirstlane(wave_min_int(bad ? 0 : 1) == 0);
            if (tid == 0) {
                ctl[0] = cand;
                ctl[1] = (mx > 0.0 && !anybad && cand < M) ? 0 : 1;
            }
        }
        __syncthreads();
        if (ctl[1]) return false;
        const int piv = ctl[0];
        if (piv != j) {
            for (int c = tid; c < M; c += nth) {
                const double a = W[j + (int64_t)c * ldw];
                W[j + (int64_t)c * ldw] = W[piv + (int64_t)c * ldw];
                W[piv + (int64_t)c * ldw] = a;
            }
            if (tid == 0) {
                const int t = perm[j];
                perm[j] = perm[piv];
                perm[piv] = t;
            }
        }
        __syncthreads();
        const double p = W[j + (int64_t)j * ldw];
        for (int i = j + 1 + tid; i < M; i += nth) W[i + (int64_t)j * ldw] /= p;
        __syncthreads();
        const int r = M - j - 1;
        for (int e = tid; e < r * r; e += nth) {
            const int i = j + 1 + e % r, c = j + 1 + e / r;
            W[i + (int64_t)c * ldw] -= W[i + (int64_t)j * ldw] * W[j + (int64_t)c * ldw];
        }
        __syncthreads();
    }
    return true;
}

// dst (n x n, ld ldd) = src (ld lds) with its columns permuted: dst[:, perm[i]]
// = src[:, i]; the inverse of a pivoted L times P, from the inverse of L.
template <class PD>
__device__ void wg_permute_columns(int n, const double* src, int lds, const lds_i32* perm, PD dst, int ldd) {
    __syncthreads();
    for (int x = threadIdx.x; x < n * n; x += blockDim.x) {
        const int r = x % n, i = x / n;
        dst[r + (int64_t)perm[i] * ldd] = src[r + (int64_t)i * lds];
    }
    __syncthreads();
}

// Per-cluster elimination operators.  The working M x M matrix W lives in
// LDS when the colour's largest cluster fits (lds_m), else in the cluster's
// L2-resident workspace; every dense step below reuses it in turn.
// One workgroup per CU: with 512 registers per lane (256 of them
// accumulation registers) the kernel keeps every value in registers; with
// two workgroups per CU it spilled 20-160 registers per lane to scratch
// memory, and builds that spilled more than about 30 gave wrong factors at
// random clusters of large launches (see the tests that check the compiled
// kernel spills nothing).
template <bool INLDS, class T>
__global__ void __launch_bounds__(WG, 1) k_pivot(LevelDev L, const int* __restrict__ clist) {
    extern __shared__ double dyn[];  // INLDS: M * M doubles (largest M of the colour); else 12 x 256
    __shared__ GemmSmem sm;
    __shared__ double red[16];
    __shared__ int isc[4];
    __shared__ int perm[MAX_M];
    __shared__ int pos_sh[LDS_M];
    __shared__ double dsh[MAX_M];
    __shared__ int fcols_sh;

    const int s = clist[blockIdx.x];
    const int tid = threadIdx.x;
    const int M = L.m[s];

    // the number of fill columns (counted, like the packed neighbour offsets,
    // by the offsets workgroups of an earlier launch of the colour) and, on
    // the pivoted-QR route, the rank that k_qrcp found
    __shared__ int kq_sh;
    if (tid == 0) {
        fcols_sh = L.fcols[s];
        kq_sh = L.k[s];
    }
    __syncthreads();
    if (M == 0) {
        if (tid == 0) L.k[s] = 0;
        return;
    }
    const int64_t MM = (int64_t)M * M;
    double* ws = L.ws + L.ws_off[s];
    double* Ainv = ws + WS_AINV * MM;
    double* Linv = ws + WS_LINV * MM;
    double* Uinv = ws + WS_UINV * MM;
    double* Umat = ws + WS_U * MM;
    double* X = ws + WS_X * MM;
    double* SL = ws + WS_SL * MM;
    double* SR = ws + WS_SR * MM;
    double* TL = ws + WS_TL * MM;
    double* TR = ws + WS_TR * MM;
    double* CU = ws + WS_CU * MM;
    double* UC = ws + WS_UC * MM;
    auto W = [&] {
        if constexpr (INLDS)
            return to_lds(dyn);
        else
            return ws + WS_SCR * MM;
    }();
    lds_f64* red_l = to_lds(red);
    lds_f64* dsh_l = to_lds(dsh);
    lds_smem* sm_l = to_lds(&sm);
    // block scratch: the GEMM staging area (2080 doubles) when the working
    // matrix is in LDS, else 12 x 256 doubles of dynamic LDS
    lds_f64* scr = INLDS ? (lds_f64*)sm_l : to_lds(dyn);
    // triangular inverses: matrix cores with 8 blocks up to 128 (always in
    // the LDS kernel, whose clusters are at most 128), 12 blocks up to 192,
    // per-wave substitution beyond (chosen by M and the thresholds alone)
    const int tri = INLDS ? 1
                          : (M <= min(TRI_MFMA_MAX, L.kn.trinv8_max)
                                 ? 1
                                 : (M <= min(TRI_MFMA_MAX12, L.kn.trinv12_max) ? 2 : 0));
    auto inv_lower = [&](auto Wp, int n, auto out) {
        if (tri == 1)
            wg_trinv_lower_unit<1>(Wp, n, M, out, M, scr);
        else if (tri == 2)
            wg_trinv_lower_unit<2>(Wp, n, M, out, M, scr);
        else
            wg_trinv_lower_unit<0>(Wp, n, M, out, M, scr);
    };
    auto inv_upper = [&](auto Wp, int n, auto out) {
        if (tri == 1)
            wg_trinv_upper<1>(Wp, n, M, out, M, scr);
        else if (tri == 2)
            wg_trinv_upper<2>(Wp, n, M, out, M, scr);
        else
            wg_trinv_upper<0>(Wp, n, M, out, M, scr);
    };
    T* TLp = rec_t<T>(L, s);
    T* TRp = TLp + MM;
    T* Bss = blk_t<T>(L, L.diag_blk[s]);

    // ---- 1. rank of the fill (Eq. lra)
    int kk;
    if (fcols_sh == 0) {
        kk = 0;
    } else if (L.eps == 0.0) {
        kk = M;  // exact mode
    } else if (L.kn.qrcp) {
        // rank and P R_k^T (X slot) from k_qrcp; U = the orthonormal factor of
        // X with a positive diagonal, by Householder QR (X has the condition
        // number |R_11| / |R_kk|, up to 1 / eps)
        kk = kq_sh;
        if (kk > 0 && kk < M) {
            wg_copy(M, kk, X, M, W, M);
            wg_house_qr(W, M, kk, M, dsh_l);
            wg_house_form_q(W, M, kk, M, dsh_l, 0, kk, Umat, M, true);
        }
    } else {
        double ass2 = 0.0;  // ||A_ss||_F^2 (noise floor of the fill)
        wg_stage((int)MM, [&](int e) { return (double)Bss[e]; }, [&](int, double v) { ass2 = fma(v, v, ass2); });
        ass2 = block_sum(ass2, red_l);
        // W = the Gram matrix (partials already summed into the first slot)
        const double* Gp = ws + WS_GP * MM;
        wg_stage((int)MM, [&](int e) { return Gp[e]; }, [&](int e, double v) { W[e] = v; });
        __syncthreads();
        // fill at the rounding level of A_ss is noise: treat it as zero
        double dmax = 0.0;
        for (int i = tid; i < M; i += blockDim.x) dmax = fmax(dmax, W[i + (int64_t)i * M]);
        dmax = block_max(dmax, red_l);
        constexpr double floor_ = std::is_same<T, float>::value ? FILL_NOISE_FLOOR_F32 : FILL_NOISE_FLOOR;
        if (dmax <= floor_ * floor_ * ass2)
            kk = 0;
        else if constexpr (INLDS)
            kk = wg_pivoted_cholesky_ll(W, M, L.eps, L.fixed_rank, to_lds(perm), to_lds(pos_sh));
        else
            kk = wg_pivoted_cholesky(W, M, L.eps, L.fixed_rank, to_lds(perm), dsh_l, to_lds(isc));
        if (kk > 0 && kk < M) {
            // P R_k^T in the unknowns' order (through X), then its orthonormal
            // factor U with a positive diagonal
            const int lane = tid & 63, nw = blockDim.x >> 6;
            if constexpr (INLDS) {  // column j sits over column piv[j] of W
                for (int j = tid >> 6; j < kk; j += nw)
                    for (int u = lane; u < M; u += 64)
                        X[u + (int64_t)j * M] = (pos_sh[u] >= j) ? W[u + (int64_t)perm[j] * M] : 0.0;
            } else {
                for (int j = tid >> 6; j < kk; j += nw)
                    for (int i = lane; i < M; i += 64)
                        X[perm[i] + (int64_t)j * M] = (i >= j) ? W[i + (int64_t)j * M] : 0.0;
            }
            __syncthreads();
            bool done = false;
            if (L.kn.cholqr)
                done = wg_cholqr2(X, M, kk, W, Linv, Uinv, Umat, sm_l, scr, red_l, to_lds(isc + 1),
                              std::is_same<T, float>::value ? CHOLQR_ONE_PASS_F32 : CHOLQR_ONE_PASS);
            if (!done) {
                wg_copy(M, kk, X, M, W, M);
                wg_house_qr(W, M, kk, M, dsh_l);
                wg_house_form_q(W, M, kk, M, dsh_l, 0, kk, Umat, M, true);
            }
        }
    }
    if (tid == 0) L.k[s] = kk;
    if (kk == M) return;  // nothing eliminated

    // ---- 2. A_ss = L U (P A_ss = L U with pivoting) and its inverse factors
    wg_copy(M, M, Bss, M, W, M);
    lds_i32* lu_perm = to_lds(perm);  // the Cholesky pivots above are no longer needed
    const bool lu_ok =
        L.pivoting ? wg_lu_partial(W, M, M, lu_perm, to_lds(isc + 1)) : wg_lu<true>(W, M, M, scr, to_lds(isc + 1));
    if (!lu_ok) {
        if (tid == 0) {
            L.flag[s] = 1;
            L.k[s] = M;  // leave the cluster untouched
        }
        return;
    }
    if (kk == 0) {  // E_s = I: one block LU step
        if (L.pivoting) {  // T_L' = L^{-1} P
            inv_lower(W, M, Linv);
            wg_permute_columns(M, Linv, M, lu_perm, TLp, M);
        } else {
            inv_lower(W, M, TLp);
        }
        inv_upper(W, M, TRp);
        return;
    }
    if (L.pivoting) {  // L^{-1} P, formed in the A^{-1} slot first
        inv_lower(W, M, Ainv);
        wg_permute_columns(M, Ainv, M, lu_perm, Linv, M);
    } else {
        inv_lower(W, M, Linv);
    }
    inv_upper(W, M, Uinv);
    wg_gemm<false, false>(M, M, M, 1.0, Uinv, M, Linv, M, 0.0, Ainv, M, sm_l);
    const int f = M - kk;

    // ---- 3. sparsification operator E_s (Eq. scaling)
    // S_L = [V_L U], V_L the complement of A^{-1} U
    wg_gemm<false, false>(M, kk, M, 1.0, Ainv, M, Umat, M, 0.0, W, M, sm_l);
    wg_complement(W, M, kk, SL, M, dsh_l, Linv, Uinv, X, sm_l, scr, L.kn);
    wg_copy(M, kk, Umat, M, SL + (int64_t)f * M, M);
    __syncthreads();
    if (L.symmetric) {
        wg_copy(M, M, SL, M, SR, M);
    } else {
        wg_gemm<true, false>(M, kk, M, 1.0, Ainv, M, Umat, M, 0.0, W, M, sm_l);  // A^{-T} U
        wg_complement(W, M, kk, SR, M, dsh_l, Linv, Uinv, X, sm_l, scr, L.kn);
        wg_copy(M, kk, Umat, M, SR + (int64_t)f * M, M);
    }
    __syncthreads();
    wg_gemm<true, false>(M, M, M, 1.0, SL, M, Ainv, M, 0.0, TL, M, sm_l);   // T_L = S_L^T A^{-1}
    wg_gemm<false, false>(M, M, M, 1.0, Ainv, M, SR, M, 0.0, TR, M, sm_l);  // T_R = A^{-1} S_R

    // ---- 4. elimination operator G_s (Eq. elim): F_ff = T_L[:f] S_R[:, :f] = L_f U_f
    wg_gemm<false, false>(f, f, M, 1.0, TL, M, SR, M, 0.0, W, M, sm_l);
    const bool ff_ok =
        L.pivoting ? wg_lu_partial(W, f, M, lu_perm, to_lds(isc + 1)) : wg_lu<true>(W, f, M, scr, to_lds(isc + 1));
    if (!ff_ok) {
        if (tid == 0) {
            L.flag[s] = 2;
            L.k[s] = M;
        }
        return;
    }
    if (L.pivoting) {  // L_f^{-1} P_f, formed in the C U^T slot first (written in step 5)
        inv_lower(W, f, CU);
        wg_permute_columns(f, CU, M, lu_perm, Linv, M);
    } else {
        inv_lower(W, f, Linv);
    }
    inv_upper(W, f, Uinv);
    // T_L' = [L_f^{-1} T_L[:f, :]; T_L[f:, :]],  T_R' = [T_R[:, :f] U_f^{-1}, T_R[:, f:]]
    wg_gemm<false, false>(f, M, f, 1.0, Linv, M, TL, M, 0.0, TLp, M, sm_l);
    wg_copy(kk, M, TL + f, M, TLp + f, M);
    wg_gemm<false, false>(M, f, f, 1.0, TR, M, Uinv, M, 0.0, TRp, M, sm_l);
    wg_copy(M, kk, TR + (int64_t)f * M, M, TRp + (int64_t)f * M, M);

    // ---- 5. coarse block C = U^T A^{-1} U = T_L[f:] S_R[:, f:] into (s, s); C U^T and U C
    wg_gemm<false, false>(kk, kk, M, 1.0, TL + f, M, SR + (int64_t)f * M, M, 0.0, W, M, sm_l);
    wg_copy(kk, kk, W, M, Bss, M);
    wg_gemm<false, true>(kk, M, kk, 1.0, W, M, Umat, M, 0.0, CU, M, sm_l);   // C U^T (k x m)
    wg_gemm<false, false>(M, kk, kk, 1.0, Umat, M, W, M, 0.0, UC, M, sm_l);  // U C (m x k)
}

void launch_offsets(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.n == 0) return;
    hipLaunchKernelGGL(k_offsets, dim3(C.n), dim3(WG), 0, st, L, C.clist);
}

void launch_pivot(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.n == 0) return;
    const size_t shmem = (size_t)C.max_m * C.max_m * sizeof(double);
    if (C.max_m <= min(LDS_M, L.kn.pivot_lds_max)) {
        if (C.f32)
            hipLaunchKernelGGL((k_pivot<true, float>), dim3(C.n), dim3(WG), shmem, st, L, C.clist);
        else
            hipLaunchKernelGGL((k_pivot<true, double>), dim3(C.n), dim3(WG), shmem, st, L, C.clist);
    } else {
        const size_t scr_bytes = 12 * 256 * sizeof(double);
        if (C.f32)
            hipLaunchKernelGGL((k_pivot<false, float>), dim3(C.n), dim3(WG), scr_bytes, st, L, C.clist);
        else
            hipLaunchKernelGGL((k_pivot<false, double>), dim3(C.n), dim3(WG), scr_bytes, st, L, C.clist);
    }
}

// ================================================== pivoted Householder QR
// Rank revelation by the truncated Householder QR with column pivoting of
// F^T itself (Eq. lra, reading R4), for a rank cap or a small eps, where the
// Gram route cannot resolve the weakest kept directions.  F (M x ncol: the
// fill blocks B(s, t), then for a general matrix the B(t, s)^T) is gathered
// into the cluster's workspace behind its slots, column major, ld M.  The
// columns of F^T are the unknowns of s (rows of F) and its rows are the
// columns of F, so a reflector of step j acts on columns j.. of F:
//   norms  n_u = sum_{c >= j} F(u, c)^2, recomputed every step;
//   pivot  the lowest position whose norm is within a relative 1e-10 of the
//          largest (positions are exchanged as the pivots are chosen);
//   stop   at the first |R_jj| <= eps |R_11|, at fixed_rank, or when every
//          remaining norm is zero;
//   H_j    LAPACK's larfg convention on x = F(u_p, j..); w_u = v^T F(u, j..),
//          F(u, j..) -= tau w_u v; row u_p becomes (beta, 0, ...);
//   sign   column j negated when beta < 0, so that R_jj > 0.
// Afterwards F(u, j) = R(j, position of u) for j < k: the first k columns of
// F are P R_k^T, written to the X slot; k goes to L.k[s].  Rows are spread
// over the threads (RR rows at a time, GG column groups), every sum over the
// column groups is added in group order.
// One workgroup of QR_WG threads per cluster: the rows of F over lanes, its
// columns over QR_WG / m groups (more threads per row shorten the per-thread
// sums over the fill columns, the latency of every step).
constexpr int QR_WG = 1024;
constexpr int QR_PART = QR_WG;
template <class T>
__global__ void __launch_bounds__(QR_WG) k_qrcp(LevelDev L, const int* __restrict__ clist) {
    __shared__ int perm[MAX_M];     // position -> unknown
    __shared__ int posof[MAX_M];    // unknown -> position
    __shared__ double nrm[MAX_M];   // remaining norms of the unknowns
    __shared__ double wt[MAX_M];    // tau w_u of the current step
    __shared__ double part[QR_PART];
    __shared__ double red[16];
    __shared__ int ctl[4];          // pivot position, stop flag
    const int s = clist[blockIdx.x];
    const int tid = threadIdx.x;
    const int M = L.m[s];
    const int fc = L.fcols[s];
    if (M == 0 || fc == 0 || L.eps <= 0.0) return;
    const int ncol = L.symmetric ? fc : 2 * fc;
    const int64_t MM = (int64_t)M * M;
    double* ws = L.ws + L.ws_off[s];
    double* X = ws + WS_X * MM;
    double* Fw = ws + ws_slots(L.gram_splits) * MM;  // M x ncol, ld M
    lds_f64* red_l = to_lds(red);
    // ---- gather F
    {
        const int f0 = L.fill_ptr[s], nf = L.fill_ptr[s + 1] - f0;
        int coff = 0;
        for (int e = f0; e < f0 + nf; ++e) {
            const int t = L.fill_id[e];
            const int ct = cur_size(L, t, L.fill_before[e]);
            if (ct == 0) continue;
            const T* Bst = blk_t<T>(L, L.fill_bst[e]);  // M x ct, ld M
            double* dst = Fw + (int64_t)coff * M;
            wg_stage(M * ct, [&](int x) { return (double)Bst[x]; }, [&](int x, double v) { dst[x] = v; });
            if (!L.symmetric) {
                const int mt = L.m[t];
                const T* Bts = blk_t<T>(L, L.fill_bts[e]);  // ct x M, ld m_t
                double* dst2 = Fw + (int64_t)(fc + coff) * M;
                wg_stage(
                    M * ct, [&](int x) { return (double)Bts[(x / M) + (int64_t)(x % M) * mt]; },
                    [&](int x, double v) { dst2[x] = v; });
            }
            coff += ct;
        }
    }
    // ||A_ss||_F^2 for the noise floor (reading R12)
    double ass2 = 0.0;
    {
        const T* Bss = blk_t<T>(L, L.diag_blk[s]);
        wg_stage((int)MM, [&](int e) { return (double)Bss[e]; }, [&](int, double v) { ass2 = fma(v, v, ass2); });
        ass2 = block_sum(ass2, red_l);
    }
    __syncthreads();
    const int RR = M < QR_WG ? M : QR_WG;   // rows per pass
    const int GG = QR_WG / RR;           // column groups
    const int r = tid % RR, g = tid / RR;
    const bool active = g < GG;
    // norms of every row over columns >= c0, summed over the groups in order
    auto row_norms = [&](int c0) {
        for (int u0 = 0; u0 < M; u0 += RR) {
            const int u = u0 + r;
            if (active && u < M) {
                double acc = 0.0;
#pragma unroll 8
                for (int c = c0 + g; c < ncol; c += GG) {
                    const double v = Fw[u + (int64_t)c * M];
                    acc = fma(v, v, acc);
                }
                part[g * RR + r] = acc;
            }
            __syncthreads();
            if (g == 0 && u < M) {
                double sum = 0.0;
                for (int q = 0; q < GG; ++q) sum += part[q * RR + r];
                nrm[u] = sum;
            }
            __syncthreads();
        }
    };
    for (int u = tid; u < M; u += QR_WG) {
        perm[u] = u;
        posof[u] = u;
    }
    row_norms(0);
    double dmax = 0.0;
    for (int u = tid; u < M; u += QR_WG) dmax = fmax(dmax, nrm[u]);
    dmax = block_max(dmax, red_l);
    constexpr double floor_ = std::is_same<T, float>::value ? FILL_NOISE_FLOOR_F32 : FILL_NOISE_FLOOR;
    int kk = 0;
    if (!(dmax <= floor_ * floor_ * ass2)) {
        double r11 = 0.0;
        const int jmax = min(ncol, M);
        for (int j = 0; j < jmax; ++j) {
            // ---- pivot: lowest position within 1e-10 of the largest norm
            if (tid < 64) {
                double mx = -1.0;
                for (int q = j + tid; q < M; q += 64) mx = fmax(mx, nrm[perm[q]]);
                mx = wave_max(mx);
                const double thr = (1.0 - 1e-10) * mx;
                int cand = M;
                for (int q = j + tid; q < M; q += 64)
                    if (nrm[perm[q]] >= thr) {
                        cand = q;
                        break;
                    }
                cand = wave_min_int(cand);
                if (tid == 0) {
                    int stop = !(mx > 0.0);
                    if (!stop) {
                        const double rjj = sqrt(nrm[perm[cand]]);
                        if (j == 0) r11 = rjj;
                        stop = (rjj <= L.eps * r11) || (L.fixed_rank > 0 && j >= L.fixed_rank);
                    }
                    ctl[0] = cand;
                    ctl[1] = stop;
                    if (!stop && cand != j) {  // exchange positions j and cand
                        const int a = perm[j], b = perm[cand];
                        perm[j] = b;
                        perm[cand] = a;
                        posof[b] = j;
                        posof[a] = cand;
                    }
                }
            }
            __syncthreads();
            if (ctl[1]) break;
            const int up = perm[j];
            // ---- reflector of x = F(up, j..ncol)
            double xn2 = 0.0;
            for (int c = j + 1 + tid; c < ncol; c += QR_WG) {
                const double v = Fw[up + (int64_t)c * M];
                xn2 = fma(v, v, xn2);
            }
            xn2 = block_sum(xn2, red_l);
            const double alpha = Fw[up + (int64_t)j * M];
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (xn2 != 0.0) {
                const double nrm2 = hypot(alpha, sqrt(xn2));
                beta = (alpha >= 0.0) ? -nrm2 : nrm2;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            if (xn2 != 0.0)
                for (int c = j + 1 + tid; c < ncol; c += QR_WG) Fw[up + (int64_t)c * M] *= scale;  // v(c), v(j) = 1
            __syncthreads();
            // ---- w_u = v^T F(u, j..) for the rows still unpivoted, then the update
            if (tau != 0.0) {
                for (int u0 = 0; u0 < M; u0 += RR) {
                    const int u = u0 + r;
                    const bool live = active && u < M && posof[u] > j;
                    if (active && u < M) {
                        double acc = 0.0;
                        if (live) {
                            if (g == 0) acc = Fw[u + (int64_t)j * M];
#pragma unroll 8
                            for (int c = j + 1 + g; c < ncol; c += GG)
                                acc = fma(Fw[up + (int64_t)c * M], Fw[u + (int64_t)c * M], acc);
                        }
                        part[g * RR + r] = acc;
                    }
                    __syncthreads();
                    if (g == 0 && u < M) {
                        double sum = 0.0;
                        for (int q = 0; q < GG; ++q) sum += part[q * RR + r];
                        wt[u] = (posof[u] > j) ? tau * sum : 0.0;
                    }
                    __syncthreads();
                }
                // the update, with each row's remaining norm over columns >= j + 1
                // summed as it is written (same columns, order and grouping as
                // row_norms, so the same bits); eight columns' loads are issued
                // before their stores
                for (int u0 = 0; u0 < M; u0 += RR) {
                    const int u = u0 + r;
                    double acc = 0.0;
                    if (active && u < M && posof[u] > j) {
                        const double w = wt[u];
                        if (g == 0) Fw[u + (int64_t)j * M] -= w;
                        int c = j + 1 + g;
                        for (; c + 7 * GG < ncol; c += 8 * GG) {
                            double pv[8], fv[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                pv[q] = Fw[up + (int64_t)(c + q * GG) * M];
                                fv[q] = Fw[u + (int64_t)(c + q * GG) * M];
                            }
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const double nv = fma(-w, pv[q], fv[q]);
                                Fw[u + (int64_t)(c + q * GG) * M] = nv;
                                acc = fma(nv, nv, acc);
                            }
                        }
                        for (; c < ncol; c += GG) {
                            const double nv = fma(-w, Fw[up + (int64_t)c * M], Fw[u + (int64_t)c * M]);
                            Fw[u + (int64_t)c * M] = nv;
                            acc = fma(nv, nv, acc);
                        }
                    }
                    if (active && u < M) part[g * RR + r] = acc;
                    __syncthreads();
                    if (g == 0 && u < M) {  // rows already pivoted: unused
                        double sum = 0.0;
                        for (int q = 0; q < GG; ++q) sum += part[q * RR + r];
                        nrm[u] = sum;
                    }
                    __syncthreads();
                }
            }
            // ---- the pivot row becomes (beta, 0, ...); R_jj > 0
            for (int c = j + 1 + tid; c < ncol; c += QR_WG) Fw[up + (int64_t)c * M] = 0.0;
            if (tid == 0) Fw[up + (int64_t)j * M] = beta;
            __syncthreads();
            if (beta < 0.0)
                for (int u = tid; u < M; u += QR_WG) Fw[u + (int64_t)j * M] = -Fw[u + (int64_t)j * M];
            kk = j + 1;
            __syncthreads();
            if (tau == 0.0) row_norms(j + 1);  // else summed during the update
        }
    }
    // ---- P R_k^T into the X slot; the rank for the pivot kernel
    if (kk > 0 && kk < M)
        wg_stage(M * kk, [&](int x) { return Fw[x]; }, [&](int x, double v) { X[x] = v; });
    if (tid == 0) L.k[s] = kk;
}

void launch_qrcp(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.n == 0 || C.fill_total == 0) return;
    if (C.f32)
        hipLaunchKernelGGL(k_qrcp<float>, dim3(C.n), dim3(QR_WG), 0, st, L, C.clist);
    else
        hipLaunchKernelGGL(k_qrcp<double>, dim3(C.n), dim3(QR_WG), 0, st, L, C.clist);
}

// ============================================================ fill update
// Coarse fill blocks (Eq. scaling): B(s^c, t) = C U^T B(s, t) and
// B(t, s^c) = B(s, t)^T U C (symmetric) or B(t, s) U C (general); one column
// panel of one partner block per workgroup, read before written (in place).
int panel_width(int max_m) {
    int pw = max_m > 0 ? 4096 / max_m : PANEL;
    return pw < 1 ? 1 : (pw > PANEL ? PANEL : pw);
}

template <class T>
__device__ void fill_update_body(const LevelDev& L, const ColourDev& C, int pw, int q) {
    extern __shared__ double dyn[];
    const int ci = find_cluster(C.fill_pre, C.n, q);
    const int s = C.clist[ci];
    const int e = L.fill_ptr[s] + (q - C.fill_pre[ci]);
    const int M = L.m[s];
    const int kk = L.k[s];
    if (kk == 0 || kk == M) return;
    const int t = L.fill_id[e];
    const int ct = cur_size(L, t, L.fill_before[e]);
    const int c0 = blockIdx.x * pw;
    const int w = min(pw, ct - c0);
    if (w <= 0) return;
    const int64_t MM = (int64_t)M * M;
    const double* ws = L.ws + L.ws_off[s];
    const double* CU = ws + WS_CU * MM;
    const double* UC = ws + WS_UC * MM;
    T* Bst = blk_t<T>(L, L.fill_bst[e]);
    T* Bts = blk_t<T>(L, L.fill_bts[e]);
    const int mt = L.m[t];
    double* P1 = dyn;                    // M x w (ld M): B(s, t)[:, panel]
    double* P2 = dyn + (int64_t)M * pw;  // w x M (ld pw): B(t, s)[panel, :]
    wg_stage(
        M * w, [&](int x) { return (double)Bst[(x % M) + (int64_t)(c0 + x / M) * M]; },
        [&](int x, double v) { P1[x] = v; });
    if (!L.symmetric)
        wg_stage(
            M * w, [&](int x) { return (double)Bts[(c0 + x % w) + (int64_t)(x / w) * mt]; },
            [&](int x, double v) { P2[(x % w) + (x / w) * pw] = v; });
    __syncthreads();
    // many workgroups run at once here: the operator columns come straight
    // from memory (L2), not through a staged tile
    for (int x = threadIdx.x; x < kk * w; x += blockDim.x) {
        int i = x % kk, j = x / kk;
        const double a = dot_batched(M, CU + i, M, [&](int l) { return P1[l + j * M]; }, 0.0);
        const double b = dot_batched(
            M, UC + (int64_t)i * M, 1, [&](int l) { return L.symmetric ? P1[l + j * M] : P2[j + l * pw]; }, 0.0);
        Bst[i + (int64_t)(c0 + j) * M] = (T)a;
        Bts[(c0 + j) + (int64_t)i * mt] = (T)b;
    }
}

template <class T>
__global__ void __launch_bounds__(WG) k_fill_update(LevelDev L, ColourDev C, int pw) {
    fill_update_body<T>(L, C, pw, blockIdx.y);
}

void launch_fill_update(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.fill_total == 0 || C.panels == 0) return;
    const int pw = panel_width(C.max_m);
    const size_t shmem = (size_t)2 * C.max_m * pw * sizeof(double);
    if (C.f32)
        hipLaunchKernelGGL(k_fill_update<float>, dim3(C.panels, C.fill_total), dim3(WG), shmem, st, L, C, pw);
    else
        hipLaunchKernelGGL(k_fill_update<double>, dim3(C.panels, C.fill_total), dim3(WG), shmem, st, L, C, pw);
}

// ======================================================== neighbour update
// [E_R; B(s^c, a)] = T_L' B(s, a) and [E_L[a], B(a, s^c)] = B(a, s) T_R',
// one column panel of one neighbour per workgroup (in place on the blocks).
template <class T>
__device__ void nbr_update_body(const LevelDev& L, const ColourDev& C, int pw, int q) {
    extern __shared__ double dyn[];
    const int ci = find_cluster(C.nbr_pre, C.n, q);
    const int s = C.clist[ci];
    const int e = L.nbr_ptr[s] + (q - C.nbr_pre[ci]);
    const int M = L.m[s];
    const int kk = L.k[s];
    if (M == 0 || kk == M) return;
    const int f = M - kk;
    const int a = L.nbr_id[e];
    const int ca = cur_size(L, a, L.nbr_before[e]);
    const int c0 = blockIdx.x * pw;
    const int w = min(pw, ca - c0);
    if (w <= 0) return;
    const int64_t MM = (int64_t)M * M;
    const int ncap = L.ncap[s];
    const T* TLp = rec_t<T>(L, s);
    const T* TRp = TLp + MM;
    T* ER = rec_t<T>(L, s) + 2 * MM;     // f x ntot, ld M
    T* EL = ER + (int64_t)M * ncap;      // ntot x f, ld ncap
    const int off = L.nbr_noff[e];
    T* Bsa = blk_t<T>(L, L.nbr_bsa[e]);
    T* Bas = blk_t<T>(L, L.nbr_bas[e]);
    const int ma = L.m[a];
    double* P1 = dyn;                     // M x w
    double* P2 = dyn + (int64_t)M * pw;   // w x M (ld pw)
    wg_stage(
        M * w, [&](int x) { return (double)Bsa[(x % M) + (int64_t)(c0 + x / M) * M]; },
        [&](int x, double v) { P1[x] = v; });
    wg_stage(
        M * w, [&](int x) { return (double)Bas[(c0 + x % w) + (int64_t)(x / w) * ma]; },
        [&](int x, double v) { P2[(x % w) + (x / w) * pw] = v; });
    __syncthreads();
    for (int x = threadIdx.x; x < M * w; x += blockDim.x) {
        int i = x % M, j = x / M;
        const double acc = dot_batched(M, TLp + i, M, [&](int l) { return P1[l + j * M]; }, 0.0);
        if (i < f)
            ER[i + (int64_t)(off + c0 + j) * M] = (T)acc;
        else
            Bsa[(i - f) + (int64_t)(c0 + j) * M] = (T)acc;
    }
    for (int x = threadIdx.x; x < M * w; x += blockDim.x) {
        int j = x % w, c = x / w;
        const double acc = dot_batched(M, TRp + (int64_t)c * M, 1, [&](int l) { return P2[j + l * pw]; }, 0.0);
        if (c < f)
            EL[(off + c0 + j) + (int64_t)c * ncap] = (T)acc;
        else
            Bas[(c0 + j) + (int64_t)(c - f) * ma] = (T)acc;
    }
}

template <class T>
__global__ void __launch_bounds__(WG) k_nbr_update(LevelDev L, ColourDev C, int pw) {
    nbr_update_body<T>(L, C, pw, blockIdx.y);
}

// Both updates of a colour in one launch: rows below fill_total of the grid
// are fill-partner panels, the rest neighbour panels.  They touch disjoint
// blocks (fill partners are not neighbours), so they may run side by side.
template <class T>
__global__ void __launch_bounds__(WG) k_fill_nbr_update(LevelDev L, ColourDev C, int pw) {
    const int q = blockIdx.y;
    if (q < C.fill_total)
        fill_update_body<T>(L, C, pw, q);
    else
        nbr_update_body<T>(L, C, pw, q - C.fill_total);
}

void launch_fill_nbr_update(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.fill_total + C.nbr_total == 0 || C.panels == 0) return;
    const int pw = panel_width(C.max_m);
    const size_t shmem = (size_t)2 * C.max_m * pw * sizeof(double);
    const dim3 grid(C.panels, C.fill_total + C.nbr_total);
    if (C.f32)
        hipLaunchKernelGGL(k_fill_nbr_update<float>, grid, dim3(WG), shmem, st, L, C, pw);
    else
        hipLaunchKernelGGL(k_fill_nbr_update<double>, grid, dim3(WG), shmem, st, L, C, pw);
}

void launch_nbr_update(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.nbr_total == 0 || C.panels == 0) return;
    const int pw = panel_width(C.max_m);
    const size_t shmem = (size_t)2 * C.max_m * pw * sizeof(double);
    if (C.f32)
        hipLaunchKernelGGL(k_nbr_update<float>, dim3(C.panels, C.nbr_total), dim3(WG), shmem, st, L, C, pw);
    else
        hipLaunchKernelGGL(k_nbr_update<double>, dim3(C.panels, C.nbr_total), dim3(WG), shmem, st, L, C, pw);
}

// ============================================================ Schur update
// A_ab -= E_L[a] E_R[b] for all neighbour pairs of s, computed as the single
// product E_L E_R (ntot x ntot, inner dimension f) in 64 x 64 tiles whose
// epilogue scatters every entry into its block (Eq. elim).
constexpr int PTAB = 256;      // block-pointer table of a Schur tile (row x column neighbours)
constexpr int NOFF_LDS = 1024;  // neighbour offsets staged in LDS up to this many neighbours
struct SchurMaps {
    int noff[NOFF_LDS];  // packed offsets of the neighbours (when nb <= NOFF_LDS)
    int rblk[SCHUR_T];   // neighbour index of every tile row (-1 = none)
    int rloc[SCHUR_T];
    int cblk[SCHUR_T];
    int cloc[SCHUR_T];
    double* ptab[PTAB];  // block (bi0 + i, bj0 + j) at ptab[i * nbj + j]
    int ldtab[SCHUR_T];  // leading dimension of row neighbour bi0 + i
};

template <class PN>
__device__ inline void map_rows(PN noff, int nb, int r0, int nt, int* nbr_of, int* loc_of) {
    for (int r = threadIdx.x; r < SCHUR_T; r += blockDim.x) {
        const int g = r0 + r;
        int idx = -1, loc = 0;
        if (g < nt) {
            // last neighbour whose packed offset is <= g
            int lo = 0, hi = nb;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (noff[mid] <= g)
                    lo = mid;
                else
                    hi = mid;
            }
            idx = lo;
            loc = g - noff[lo];
        }
        nbr_of[r] = idx;
        loc_of[r] = loc;
    }
}

// At most 102 registers per lane (five waves per SIMD): the float kernel then
// fits 79 without spilling and runs six workgroups per CU, the double one
// five; the update is bound by the latency of its scattered loads and
// stores, so more resident waves serve it better than more registers.
template <class T>
__global__ void __launch_bounds__(WG, 5) k_schur(LevelDev L, ColourDev C) {
    constexpr bool F64 = std::is_same<T, double>::value;
    __shared__ std::conditional_t<F64, MfmaSmem, MfmaSmemB> sm;
    __shared__ SchurMaps mp;
    const int64_t q = blockIdx.x;
    const int ci = find_cluster64(C.tile_pre, C.n, q);
    const int s = C.clist[ci];
    const int M = L.m[s];
    const int kk = L.k[s];
    const int f = M - kk;
    if (M == 0 || f == 0) return;
    const int ncap = L.ncap[s];
    const int nt = L.ntot[s];
    const int tpr = (ncap + SCHUR_T - 1) / SCHUR_T;
    const int64_t t = q - C.tile_pre[ci];
    const int r0 = (int)(t / tpr) * SCHUR_T, c0 = (int)(t % tpr) * SCHUR_T;
    if (r0 >= nt || c0 >= nt) return;
    const int64_t MM = (int64_t)M * M;
    const T* ER = rec_t<T>(L, s) + 2 * MM;  // f x ntot, ld M
    const T* EL = ER + (int64_t)M * ncap;   // ntot x f, ld ncap
    const int e0 = L.nbr_ptr[s], nb = L.nbr_ptr[s + 1] - e0;
    if (nb <= min(NOFF_LDS, L.kn.schur_noff_max)) {
        for (int x = threadIdx.x; x < nb; x += blockDim.x) mp.noff[x] = L.nbr_noff[e0 + x];
        __syncthreads();
        map_rows(to_lds(mp.noff), nb, r0, nt, mp.rblk, mp.rloc);
        map_rows(to_lds(mp.noff), nb, c0, nt, mp.cblk, mp.cloc);
    } else {
        map_rows(L.nbr_noff + e0, nb, r0, nt, mp.rblk, mp.rloc);
        map_rows(L.nbr_noff + e0, nb, c0, nt, mp.cblk, mp.cloc);
    }
    auto la = [&](int r, int k) { return (r0 + r < nt && k < f) ? EL[(r0 + r) + (int64_t)k * ncap] : (T)0; };
    auto lb = [&](int k, int c) { return (c0 + c < nt && k < f) ? ER[k + (int64_t)(c0 + c) * M] : (T)0; };
    std::conditional_t<F64, v4d, v4f> acc[2][2];
    if constexpr (F64)
        mfma_tile64(f, la, lb, to_lds(&sm), acc);
    else
        mfma_tile64_bf16(f, la, lb, to_lds(&sm), acc);
    __syncthreads();
    const int64_t pb = L.pair_base[s];
    // neighbour ranges covered by the tile; the block pointers of every
    // (row neighbour, column neighbour) pair go to LDS once
    const int nr = min(SCHUR_T, nt - r0), nc = min(SCHUR_T, nt - c0);
    const int bi0 = mp.rblk[0], bj0 = mp.cblk[0];
    const int nbi = mp.rblk[nr - 1] - bi0 + 1, nbj = mp.cblk[nc - 1] - bj0 + 1;
    const bool table = nbi * nbj <= min(PTAB, L.kn.schur_ptab_max);
    if (table) {
        for (int x = threadIdx.x; x < nbi * nbj; x += blockDim.x) {
            const int i = x / nbj, j = x % nbj;
            mp.ptab[x] = (double*)blk_t<T>(L, L.pair_blk[pb + (int64_t)(bi0 + i) * nb + (bj0 + j)]);
        }
        for (int i = threadIdx.x; i < nbi; i += blockDim.x) mp.ldtab[i] = L.m[L.nbr_id[e0 + bi0 + i]];
    }
    __syncthreads();
    // every entry of the tile has its own address: all 16 targets of a lane
    // are read before any is written back
    using GT = std::conditional_t<F64, glb_f64, glb_f32>;
    GT* dst[16];
    auto addr = [&](int idx, int r, int c, double) {
        const int bi = mp.rblk[r], bj = mp.cblk[c];
        T* p = nullptr;
        if (bi >= 0 && bj >= 0) {
            if (table) {
                const int i = bi - bi0;
                p = (T*)mp.ptab[i * nbj + (bj - bj0)] + mp.rloc[r] + (int64_t)mp.cloc[c] * mp.ldtab[i];
            } else {
                const int a = L.nbr_id[e0 + bi];
                p = blk_t<T>(L, L.pair_blk[pb + (int64_t)bi * nb + bj]) + mp.rloc[r] + (int64_t)mp.cloc[c] * L.m[a];
            }
        }
        dst[idx] = (GT*)p;
    };
    if constexpr (F64)
        mfma_tile64_visit(acc, addr);
    else
        mfma_tile64_bf16_visit(acc, addr);
    T old[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) old[x] = dst[x] ? *dst[x] : (T)0;
    auto upd = [&](int idx, int, int, double v) {
        if (dst[idx]) *dst[idx] = old[idx] - (T)v;
    };
    if constexpr (F64)
        mfma_tile64_visit(acc, upd);
    else
        mfma_tile64_bf16_visit(acc, upd);
}

void launch_schur(const LevelDev& L, const ColourDev& C, hipStream_t st) {
    if (C.tile_total == 0) return;
    if (C.f32)
        hipLaunchKernelGGL(k_schur<float>, dim3((unsigned)C.tile_total), dim3(WG), 0, st, L, C);
    else
        hipLaunchKernelGGL(k_schur<double>, dim3((unsigned)C.tile_total), dim3(WG), 0, st, L, C);
}

// ================================================================ assembly

__global__ void k_assemble0(int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                            const double* __restrict__ val, const int* __restrict__ cluster_of,
                            const int* __restrict__ local_of, const int* __restrict__ m,
                            const int* __restrict__ pat_ptr, const int* __restrict__ pat,
                            const int64_t* __restrict__ blk_off, void* __restrict__ blocks,
                            const int* __restrict__ f32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = cluster_of[i], li = local_of[i];
    const int lo0 = pat_ptr[ci], hi0 = pat_ptr[ci + 1];
    const bool single = f32[ci] != 0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int j = col_idx[e];
        const int cj = cluster_of[j], lj = local_of[j];
        int lo = lo0, hi = hi0;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (pat[mid] < cj)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int64_t x = blk_off[lo] + li + (int64_t)lj * m[ci];
        if (single)
            static_cast<float*>(blocks)[x] = (float)val[e];
        else
            static_cast<double*>(blocks)[x] = val[e];
    }
}

void launch_assemble0(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                      const int* cluster_of, const int* local_of, const int* m, const int* pat_ptr, const int* pat,
                      const int64_t* blk_off, void* blocks, const int* f32, hipStream_t st) {
    if (n == 0) return;
    const int bs = 256;
    hipLaunchKernelGGL(k_assemble0, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, n, row_ptr, col_idx, val,
                       cluster_of, local_of, m, pat_ptr, pat, blk_off, blocks, f32);
}

// Position of block (a, b) in a level's pattern (rows sorted), -1 if absent.
__device__ inline int pat_find(const int* __restrict__ pat_ptr, const int* __restrict__ pat, int a, int b) {
    int lo = pat_ptr[a], hi = pat_ptr[a + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pat[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < end && pat[lo] == b) ? lo : -1;
}

// Parent block (P, Q) = [[B(l_P, l_Q), B(l_P, r_Q)], [B(r_P, l_Q), B(r_P, r_Q)]]
// of the children's coarse blocks (Alg. 1 "Extract A_c").
template <class TS, class TD>
__device__ void merge_block(int b, int P, int Q, const int* __restrict__ pat_ptr_prev,
                            const int* __restrict__ pat_prev, int ncl_prev, const int* __restrict__ k_prev,
                            const int* __restrict__ m_prev, const int64_t* __restrict__ blk_off_prev,
                            const TS* __restrict__ blocks_prev, const int* __restrict__ m_next,
                            const int64_t* __restrict__ blk_off_next, TD* __restrict__ blocks_next) {
    const int ldn = m_next[P];
    TD* dst = blocks_next + blk_off_next[b];
    for (int h = 0; h < 4; ++h) {
        const int a = 2 * P + (h >> 1), c = 2 * Q + (h & 1);
        if (a >= ncl_prev || c >= ncl_prev) continue;
        const int src = pat_find(pat_ptr_prev, pat_prev, a, c);
        if (src < 0) continue;
        const int roff = (h >> 1) ? k_prev[2 * P] : 0;
        const int coff = (h & 1) ? k_prev[2 * Q] : 0;
        const int ka = k_prev[a], kc = k_prev[c];
        const TS* sp = blocks_prev + blk_off_prev[src];
        const int lds = m_prev[a];
        if (ka == 0) continue;
        // one wave per parent block: four loads in flight per lane
        const int tot = ka * kc, lane = threadIdx.x & 63;
        for (int x0 = lane; x0 < tot; x0 += 4 * 64) {
            TS v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = min(x0 + u * 64, tot - 1);
                v[u] = sp[(x % ka) + (int64_t)(x / ka) * lds];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = x0 + u * 64;
                if (x < tot) dst[(roff + x % ka) + (int64_t)(coff + x / ka) * ldn] = (TD)v[u];
            }
        }
    }
}

// One wave per parent block (four per workgroup); its row P by binary search
// over the pattern's row pointers.  Element types per cluster on either side
// (a system's children and parent may differ).
__global__ void k_merge(const int* __restrict__ pat_ptr_next, const int* __restrict__ pat_next, int ncl_next,
                        const int* __restrict__ pat_ptr_prev, const int* __restrict__ pat_prev, int ncl_prev,
                        const int* __restrict__ k_prev, const int* __restrict__ m_prev,
                        const int64_t* __restrict__ blk_off_prev, const void* __restrict__ blocks_prev,
                        const int* __restrict__ f32_prev, const int* __restrict__ m_next,
                        const int64_t* __restrict__ blk_off_next, void* __restrict__ blocks_next,
                        const int* __restrict__ f32_next) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= pat_ptr_next[ncl_next]) return;
    int lo = 0, hi = ncl_next;  // last P with pat_ptr_next[P] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pat_ptr_next[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    const int P = lo, Q = pat_next[b];
    const bool s32 = f32_prev[2 * P] != 0, d32 = f32_next[P] != 0;
#define HS_MERGE(TS, TD)                                                                                             \
    merge_block<TS, TD>(b, P, Q, pat_ptr_prev, pat_prev, ncl_prev, k_prev, m_prev, blk_off_prev,                      \
                        static_cast<const TS*>(blocks_prev), m_next, blk_off_next, static_cast<TD*>(blocks_next))
    if (s32 && d32)
        HS_MERGE(float, float);
    else if (s32)
        HS_MERGE(float, double);
    else if (d32)
        HS_MERGE(double, float);
    else
        HS_MERGE(double, double);
#undef HS_MERGE
}

void launch_merge(int nblk_next, const int* pat_ptr_next, const int* pat_next, int ncl_next,
                  const int* pat_ptr_prev, const int* pat_prev, int ncl_prev, const int* k_prev, const int* m_prev,
                  const int64_t* blk_off_prev, const void* blocks_prev, const int* f32_prev, const int* m_next,
                  const int64_t* blk_off_next, void* blocks_next, const int* f32_next, hipStream_t st) {
    if (nblk_next == 0) return;
    hipLaunchKernelGGL(k_merge, dim3((nblk_next + 3) / 4), dim3(256), 0, st, pat_ptr_next, pat_next, ncl_next, pat_ptr_prev,
                       pat_prev, ncl_prev, k_prev, m_prev, blk_off_prev, blocks_prev, f32_prev, m_next, blk_off_next,
                       blocks_next, f32_next);
}

// Block ids of (s, s), of (s, a) and (a, s) for every neighbour a and of
// (s, t) and (t, s) for every fill partner t, and whether a / t is processed
// before s; one workgroup per cluster.
__global__ void k_level_ids(const int* __restrict__ nbr_ptr, const int* __restrict__ nbr_id,
                            const int* __restrict__ fill_ptr, const int* __restrict__ fill_id,
                            const int* __restrict__ pos, const int* __restrict__ pat_ptr,
                            const int* __restrict__ pat, int* __restrict__ diag_blk, int* __restrict__ nbr_before,
                            int* __restrict__ nbr_bsa, int* __restrict__ nbr_bas, int* __restrict__ fill_before,
                            int* __restrict__ fill_bst, int* __restrict__ fill_bts) {
    const int s = blockIdx.x;
    if (threadIdx.x == 0) diag_blk[s] = pat_find(pat_ptr, pat, s, s);
    for (int e = nbr_ptr[s] + threadIdx.x; e < nbr_ptr[s + 1]; e += blockDim.x) {
        const int a = nbr_id[e];
        nbr_before[e] = pos[a] < pos[s];
        nbr_bsa[e] = pat_find(pat_ptr, pat, s, a);
        nbr_bas[e] = pat_find(pat_ptr, pat, a, s);
    }
    for (int e = fill_ptr[s] + threadIdx.x; e < fill_ptr[s + 1]; e += blockDim.x) {
        const int t = fill_id[e];
        fill_before[e] = pos[t] < pos[s];
        fill_bst[e] = pat_find(pat_ptr, pat, s, t);
        fill_bts[e] = pat_find(pat_ptr, pat, t, s);
    }
}

void launch_level_ids(int ncl, const int* nbr_ptr, const int* nbr_id, const int* fill_ptr, const int* fill_id,
                      const int* pos, const int* pat_ptr, const int* pat, int* diag_blk, int* nbr_before,
                      int* nbr_bsa, int* nbr_bas, int* fill_before, int* fill_bst, int* fill_bts, hipStream_t st) {
    if (ncl == 0) return;
    hipLaunchKernelGGL(k_level_ids, dim3(ncl), dim3(64), 0, st, nbr_ptr, nbr_id, fill_ptr, fill_id, pos, pat_ptr, pat,
                       diag_blk, nbr_before, nbr_bsa, nbr_bas, fill_before, fill_bst, fill_bts);
}

__global__ void k_pair_blocks(const int* __restrict__ nbr_ptr, const int* __restrict__ nbr_id,
                              const int* __restrict__ pat_ptr, const int* __restrict__ pat,
                              const int64_t* __restrict__ pair_base, int* __restrict__ pair_blk) {
    const int s = blockIdx.x;
    const int e0 = nbr_ptr[s], nb = nbr_ptr[s + 1] - e0;
    int* out = pair_blk + pair_base[s];
    for (int x = threadIdx.x; x < nb * nb; x += blockDim.x) {
        const int a = nbr_id[e0 + x / nb], b = nbr_id[e0 + x % nb];
        int lo = pat_ptr[a], hi = pat_ptr[a + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pat[mid] < b)
                lo = mid + 1;
            else
                hi = mid;
        }
        out[x] = (lo < pat_ptr[a + 1] && pat[lo] == b) ? lo : -1;
    }
}

void launch_pair_blocks(int ncl, const int* nbr_ptr, const int* nbr_id, const int* pat_ptr, const int* pat,
                        const int64_t* pair_base, int* pair_blk, hipStream_t st) {
    if (ncl == 0) return;
    hipLaunchKernelGGL(k_pair_blocks, dim3(ncl), dim3(256), 0, st, nbr_ptr, nbr_id, pat_ptr, pat, pair_base, pair_blk);
}

__global__ void k_fill_zero(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
    const int64_t n = bytes / 4;
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, n);
}

__global__ void k_shift_csr(int64_t n_i, int64_t nnz_i, int64_t row_off, int64_t nnz_off, int64_t* __restrict__ row_ptr,
                            int32_t* __restrict__ col_idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n_i; i += stride) row_ptr[i] += nnz_off;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz_i; e += stride)
        col_idx[e] += (int32_t)row_off;
}

void launch_shift_csr(int64_t n_i, int64_t nnz_i, int64_t row_off, int64_t nnz_off, int64_t* row_ptr,
                      int32_t* col_idx, hipStream_t st) {
    if (row_off == 0 && nnz_off == 0) return;
    const int64_t work = std::max(n_i + 1, nnz_i);
    const unsigned g = (unsigned)std::min<int64_t>((work + 255) / 256, 8192);
    hipLaunchKernelGGL(k_shift_csr, dim3(g), dim3(256), 0, st, n_i, nnz_i, row_off, nnz_off, row_ptr, col_idx);
}

}  // namespace hs
