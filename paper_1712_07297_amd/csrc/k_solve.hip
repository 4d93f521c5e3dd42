// Solve kernels (Alg. 2) and float64 Krylov building blocks.
//
// Level vectors hold one segment per cluster, the segment of cluster s being
// an m_s x nrhs column-major block at offset seg[s] * nrhs.  Forward
// substitution applies W_s = P_s G_s E_s cluster by cluster in processing
// order: z_s = T_L' y_s (fine unknowns first, coarse last) and every
// neighbour's current unknowns lose E_L[a] z_s[:f].  Backward substitution
// runs in reverse: out_s = T_R' [z_f - sum_a E_R[:, a] x_a ; x_c].  A
// neighbour processed before s is represented by its coarse part.
#include "device_common.h"
#include "kernels.h"

namespace hs {

template <class T>
__device__ inline const T* srec(const SolveLevelDev& S, int s) {
    return reinterpret_cast<const T*>(S.rec) + S.rec_off[s];
}

__device__ inline int find_pre(const int* pre, int n, int q) {
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

template <class T>
__device__ inline T* tile_buf(double* after) {
    return reinterpret_cast<T*>(after);
}

// ---------------------------------------------------------------- forward

// rows of a cluster's own products per workgroup (the split forward step
// and the backward step)
constexpr int UROWS = 64;

// z_s = T_L' y_s, rows r0 .. r0 + 63 of cluster s = clist[blockIdx.y] per
// workgroup (blockIdx.x = r0 / 64); every row's sum runs over the whole of
// y_s in ascending order, so the rows do not depend on the chunking.
template <class T>
__global__ void __launch_bounds__(WG) k_apply_fwd_t(SolveLevelDev S, ColourDev C, const double* __restrict__ y,
                                                    double* __restrict__ z, int nrhs) {
    extern __shared__ double ys[];  // max_m x nrhs, then the operand tile
    const int s = C.clist[blockIdx.y];
    const int M = S.m[s];
    const int r0 = blockIdx.x * UROWS;
    if (r0 >= M) return;
    const int nr = min(UROWS, M - r0);
    const int kk = S.k[s];
    const double* ysrc = y + S.seg[s] * nrhs;
    double* zdst = z + S.seg[s] * nrhs;
    const int tot = M * nrhs;
    if (kk == M) {
        wg_stage(
            nr * nrhs, [&](int x) { return ysrc[r0 + x % nr + (x / nr) * M]; },
            [&](int x, double v) { zdst[r0 + x % nr + (x / nr) * M] = v; });
        return;
    }
    wg_stage(tot, [&](int x) { return ysrc[x]; }, [&](int x, double v) { ys[x] = v; });
    const T* TL = srec<T>(S, s) + r0;
    wg_rows_times<T>(
        nr, M, nrhs, [&](int i, int l) { return TL[i + (int64_t)l * M]; }, [&](int l, int r) { return ys[l + r * M]; },
        tile_buf<T>(ys + (size_t)C.max_m * nrhs), [&](int i, int r, double v) { zdst[r0 + i + r * M] = v; });
}

static size_t tile_shmem(size_t doubles) { return doubles * sizeof(double) + TILE_BYTES; }

// One right-hand side, clusters of at most WAVE_MAXM unknowns and a colour
// of at least apply_wave clusters: one wave per cluster (four clusters per
// workgroup), lane l holding rows l and l + 64.  A wave waits for one memory
// round trip per WAVE_LD columns, so the form pays where a launch holds
// thousands of clusters (throughput), not on sparse levels (latency).  The operator is read straight from memory, a batch of WAVE_LD
// columns in flight per lane (consecutive lanes read consecutive rows of a
// column), and the vector entry of column l is broadcast from the lane that
// holds it; every row's sum is taken from zero in ascending l with one fma
// per column, the order of the workgroup form, so both give the same bits.
constexpr int WAVE_MAXM = 128;
constexpr int WAVE_LD = 8;

// out(i) = sum_l Op(i, l) v(l) for the rows i = lane, lane + 64 < M; v(l) is
// v0 of lane l (l < 64) or v1 of lane l - 64.
template <class T>
__device__ inline void wave_rows_times(const T* __restrict__ op, int M, double v0, double v1, double& a0,
                                       double& a1) {
    const int lane = threadIdx.x & 63;
    const bool ok0 = lane < M, ok1 = lane + 64 < M;
    a0 = 0.0;
    a1 = 0.0;
    int l = 0;
    for (; l + WAVE_LD <= M; l += WAVE_LD) {
        T t0[WAVE_LD], t1[WAVE_LD];
#pragma unroll
        for (int u = 0; u < WAVE_LD; ++u) {
            const T* col = op + (int64_t)(l + u) * M;
            t0[u] = ok0 ? col[lane] : T(0);
            t1[u] = ok1 ? col[lane + 64] : T(0);
        }
#pragma unroll
        for (int u = 0; u < WAVE_LD; ++u) {
            const int lu = l + u;
            const double vl = lu < 64 ? readlane_d(v0, lu) : readlane_d(v1, lu - 64);
            a0 = fma((double)t0[u], vl, a0);
            a1 = fma((double)t1[u], vl, a1);
        }
    }
    for (; l < M; ++l) {
        const T* col = op + (int64_t)l * M;
        const double vl = l < 64 ? readlane_d(v0, l) : readlane_d(v1, l - 64);
        a0 = fma((double)(ok0 ? col[lane] : T(0)), vl, a0);
        a1 = fma((double)(ok1 ? col[lane + 64] : T(0)), vl, a1);
    }
}

// z_s = T_L' y_s (one right-hand side), one wave per cluster.
template <class T>
__global__ void __launch_bounds__(WG) k_apply_fwd_t_wave(SolveLevelDev S, ColourDev C, const double* __restrict__ y,
                                                         double* __restrict__ z) {
    const int ci = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    if (ci >= C.n) return;
    const int lane = threadIdx.x & 63;
    const int s = C.clist[ci];
    const int M = S.m[s];
    const double* ys = y + S.seg[s];
    double* zs = z + S.seg[s];
    const double y0 = lane < M ? ys[lane] : 0.0;
    const double y1 = lane + 64 < M ? ys[lane + 64] : 0.0;
    double a0 = y0, a1 = y1;
    if (S.k[s] != M) wave_rows_times<T>(srec<T>(S, s), M, y0, y1, a0, a1);
    if (lane < M) zs[lane] = a0;
    if (lane + 64 < M) zs[lane + 64] = a1;
}

void launch_apply_fwd_t(const SolveLevelDev& S, const ColourDev& C, const double* y, double* z, int nrhs,
                        hipStream_t st) {
    if (C.n == 0) return;
    if (nrhs == 1 && C.apply_wave > 0 && C.n >= C.apply_wave && C.max_m <= WAVE_MAXM) {
        const dim3 wgrid((C.n + WG / 64 - 1) / (WG / 64));
        if (C.f32)
            hipLaunchKernelGGL(k_apply_fwd_t_wave<float>, wgrid, dim3(WG), 0, st, S, C, y, z);
        else
            hipLaunchKernelGGL(k_apply_fwd_t_wave<double>, wgrid, dim3(WG), 0, st, S, C, y, z);
        return;
    }
    const size_t sh = tile_shmem((size_t)C.max_m * nrhs);
    const dim3 grid(std::max(1, (C.max_m + UROWS - 1) / UROWS), C.n);
    if (C.f32)
        hipLaunchKernelGGL(k_apply_fwd_t<float>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
    else
        hipLaunchKernelGGL(k_apply_fwd_t<double>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
}

// Neighbour updates of the split forward step: y_a (or z_a's coarse part) -=
// E_L[a] z_s[:f], one thread per neighbour row (rows row0 .. row0 + 255 of
// cluster s = clist[blockIdx.y], packed in the order of s's neighbour list,
// blockIdx.x = row0 / 256).  A row's sum runs over j ascending from zero, as
// in the one-launch form, so both give the same bits; consecutive threads
// read consecutive rows of each column of E_L.
constexpr int NB_TAB = 512;  // neighbour entries of a cluster looked up in LDS

template <class T>
__global__ void __launch_bounds__(WG) k_apply_fwd_u(SolveLevelDev S, ColourDev C, double* __restrict__ y,
                                                    double* __restrict__ z, int nrhs) {
    extern __shared__ double zf[];  // f x nrhs
    __shared__ int noff_sh[NB_TAB];
    const int s = C.clist[blockIdx.y];
    const int M = S.m[s];
    const int f = M - S.k[s];
    if (M == 0 || f == 0) return;
    const int row0 = blockIdx.x * WG;
    const int nt = S.ntot[s];
    if (row0 >= nt) return;
    const int e0 = S.nbr_ptr[s], ne = S.nbr_ptr[s + 1] - e0;
    const double* zs = z + S.seg[s] * nrhs;
    wg_stage(
        f * nrhs, [&](int x) { return zs[(x % f) + (x / f) * M]; }, [&](int x, double v) { zf[x] = v; });
    const bool in_lds = ne <= NB_TAB;
    if (in_lds)
        for (int q = threadIdx.x; q < ne; q += blockDim.x) noff_sh[q] = S.nbr_noff[e0 + q];
    __syncthreads();
    const int i = row0 + threadIdx.x;
    if (i >= nt) return;
    // the entry holding packed row i: the last e with noff[e] <= i (entries
    // with no rows share their offset with the next one, which holds i)
    int lo = 0, hi = ne;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((in_lds ? noff_sh[mid] : S.nbr_noff[e0 + mid]) <= i)
            lo = mid;
        else
            hi = mid;
    }
    const int e = e0 + lo;
    const int a = S.nbr_id[e];
    const int before = S.nbr_before[e];
    const int ma = S.m[a];
    const int ca = before ? S.k[a] : ma;
    const int li = i - (in_lds ? noff_sh[lo] : S.nbr_noff[e]);
    double* tgt = (before ? z + S.seg[a] * nrhs + (ma - ca) : y + S.seg[a] * nrhs) + li;  // ld ma
    const int ncap = S.ncap[s];
    const T* EL = srec<T>(S, s) + 2 * (int64_t)M * M + (int64_t)M * ncap + i;  // row i, ld ncap
    for (int r0 = 0; r0 < nrhs; r0 += 4) {
        const int rr = min(4, nrhs - r0);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (rr == 1) {
#pragma unroll 8
            for (int jj = 0; jj < f; ++jj) acc[0] = fma((double)EL[(int64_t)jj * ncap], zf[jj + r0 * f], acc[0]);
        } else {
#pragma unroll 4
            for (int jj = 0; jj < f; ++jj) {
                const double av = (double)EL[(int64_t)jj * ncap];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < rr) acc[t] = fma(av, zf[jj + (r0 + t) * f], acc[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < rr) tgt[(int64_t)(r0 + t) * ma] -= acc[t];
    }
}

void launch_apply_fwd_u(const SolveLevelDev& S, const ColourDev& C, double* y, double* z, int nrhs, int max_m,
                        hipStream_t st) {
    if (C.nbr_total == 0 || C.max_nt == 0) return;
    (void)max_m;
    const size_t sh = (size_t)C.max_m * nrhs * sizeof(double);
    const dim3 grid((C.max_nt + WG - 1) / WG, C.n);
    if (C.f32)
        hipLaunchKernelGGL(k_apply_fwd_u<float>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
    else
        hipLaunchKernelGGL(k_apply_fwd_u<double>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
}

// Forward step of a colour in one launch: workgroups (x, q) for q below the
// neighbour count update neighbour rows, each forming the z_s[:f] it needs
// itself (the same products, in the same order, as the cluster's own
// workgroup, so every copy is bit for bit the same); workgroups q = nbr_total
// + i write z_i = T_L' y_i for cluster i of the colour.  Clusters of a colour
// are more than two apart, so no workgroup reads what another writes.
template <class T>
__global__ void __launch_bounds__(WG) k_apply_fwd(SolveLevelDev S, ColourDev C, double* __restrict__ y,
                                                  double* __restrict__ z, int nrhs) {
    extern __shared__ double ys[];  // max_m x nrhs, then z_f (max_m x nrhs), then the operand tile
    const int q = blockIdx.y;
    const bool own = q >= C.nbr_total;
    if (own && blockIdx.x > 0) return;
    const int ci = own ? q - C.nbr_total : find_pre(C.nbr_pre, C.n, q);
    const int s = C.clist[ci];
    const int M = S.m[s];
    if (M == 0) return;
    const int kk = S.k[s];
    const int f = M - kk;
    const double* ysrc = y + S.seg[s] * nrhs;
    const int tot = M * nrhs;
    const size_t cap = (size_t)C.max_m * nrhs;
    const T* TL = srec<T>(S, s);
    if (own) {
        double* zdst = z + S.seg[s] * nrhs;
        if (kk == M) {
            wg_stage(tot, [&](int x) { return ysrc[x]; }, [&](int x, double v) { zdst[x] = v; });
            return;
        }
        wg_stage(tot, [&](int x) { return ysrc[x]; }, [&](int x, double v) { ys[x] = v; });
        wg_rows_times<T>(
            M, M, nrhs, [&](int i, int l) { return TL[i + (int64_t)l * M]; }, [&](int l, int r) { return ys[l + r * M]; },
            tile_buf<T>(ys + 2 * cap), [&](int i, int r, double v) { zdst[i + r * M] = v; });
        return;
    }
    if (f == 0) return;
    const int e = S.nbr_ptr[s] + (q - C.nbr_pre[ci]);
    const int a = S.nbr_id[e];
    const int before = S.nbr_before[e];
    const int ma = S.m[a];
    const int ca = before ? S.k[a] : ma;
    const int r0 = blockIdx.x * UROWS;
    if (r0 >= ca) return;
    const int nr = min(UROWS, ca - r0);
    double* zf = ys + cap;
    wg_stage(tot, [&](int x) { return ysrc[x]; }, [&](int x, double v) { ys[x] = v; });
    wg_rows_times<T>(
        f, M, nrhs, [&](int i, int l) { return TL[i + (int64_t)l * M]; }, [&](int l, int r) { return ys[l + r * M]; },
        tile_buf<T>(ys + 2 * cap), [&](int i, int r, double v) { zf[i + r * f] = v; });
    const int ncap = S.ncap[s];
    const T* EL = srec<T>(S, s) + 2 * (int64_t)M * M + (int64_t)M * ncap + S.nbr_noff[e] + r0;  // ld ncap
    double* tgt = (before ? z + S.seg[a] * nrhs + (ma - ca) : y + S.seg[a] * nrhs) + r0;    // ld ma
    wg_rows_times<T>(
        nr, f, nrhs, [&](int i, int j) { return EL[i + (int64_t)j * ncap]; }, [&](int j, int r) { return zf[j + r * f]; },
        tile_buf<T>(ys + 2 * cap), [&](int i, int r, double v) { tgt[i + (int64_t)r * ma] -= v; });
}

// LDS of the one-launch forward step; above FWD_FUSED_MAX_LDS the two
// kernels run instead.
constexpr size_t FWD_FUSED_MAX_LDS = 150 * 1024;

void launch_apply_fwd(const SolveLevelDev& S, const ColourDev& C, double* y, double* z, int nrhs, hipStream_t st) {
    if (C.n == 0) return;
    const size_t sh = tile_shmem(2 * (size_t)C.max_m * nrhs);
    // fwd_split: 1 always two launches, 2 two launches for at most
    // split_nrhs_max right-hand sides (the one-launch form's re-formed z_s
    // costs less than the second launch once the right-hand sides share it)
    const bool split = C.fwd_split == 1 || (C.fwd_split == 2 && nrhs <= C.split_nrhs_max);
    if (split || sh > FWD_FUSED_MAX_LDS) {
        launch_apply_fwd_t(S, C, y, z, nrhs, st);
        launch_apply_fwd_u(S, C, y, z, nrhs, C.max_nbr_m, st);
        return;
    }
    const int chunks = std::max(1, (C.max_nbr_m + UROWS - 1) / UROWS);
    const dim3 grid(chunks, C.nbr_total + C.n);
    if (C.f32)
        hipLaunchKernelGGL(k_apply_fwd<float>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
    else
        hipLaunchKernelGGL(k_apply_fwd<double>, grid, dim3(WG), sh, st, S, C, y, z, nrhs);
}

// --------------------------------------------------------------- backward

// part = E_R[:, cols] x over the group's columns: the four waves take four
// consecutive slices of the columns, each lane one row of E_R (consecutive
// lanes read consecutive rows of a column), and the four slice sums are added
// in slice order.  The x values of the group are gathered into LDS first.
constexpr int BWD_XCOLS = 512;   // columns of x held in LDS per pass (times RC right-hand sides)

template <class T, int RC>
__global__ void __launch_bounds__(WG) k_apply_bwd_acc(SolveLevelDev S, ColourDev C, const double* __restrict__ z,
                                                      const double* __restrict__ out, double* __restrict__ part,
                                                      const int64_t* __restrict__ part_off, int nrhs) {
    __shared__ double xs[RC * BWD_XCOLS];
    __shared__ double red[3][64][RC];
    __shared__ int tab_c[SOLVE_GROUP_ENTRIES + 1];
    __shared__ int tab_ld[SOLVE_GROUP_ENTRIES];
    __shared__ const double* tab_src[SOLVE_GROUP_ENTRIES];
    const int g = blockIdx.x;
    const int ci = find_pre(C.grp_pre, C.n, g);
    const int s = C.clist[ci];
    const int M = S.m[s];
    const int f = M - S.k[s];
    if (M == 0 || f == 0) return;
    const int e0 = C.grp_e0[g], e1 = C.grp_e1[g], ne = e1 - e0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < ne) {
        const int e = e0 + tid;
        const int a = S.nbr_id[e];
        const int ma = S.m[a];
        const int before = S.nbr_before[e];
        const int ca = before ? S.k[a] : ma;
        tab_c[tid + 1] = S.nbr_noff[e] - S.nbr_noff[e0] + ca;
        tab_ld[tid] = ma;
        tab_src[tid] = before ? z + S.seg[a] * nrhs + (ma - ca) : out + S.seg[a] * nrhs;
    }
    if (tid == 0) tab_c[0] = 0;
    __syncthreads();
    const int ncols = tab_c[ne];
    const T* ER = srec<T>(S, s) + 2 * (int64_t)M * M + (int64_t)S.nbr_noff[e0] * M;  // ld M
    double* dst = part + part_off[g] * nrhs;                                           // f x nrhs
    for (int r0 = 0; r0 < nrhs; r0 += RC) {
        const int rr = min(RC, nrhs - r0);
        for (int j0 = 0; j0 < f; j0 += 64) {
            const int j = j0 + lane;
            double acc[RC];
#pragma unroll
            for (int t = 0; t < RC; ++t) acc[t] = 0.0;
            for (int c0 = 0; c0 < ncols; c0 += BWD_XCOLS) {
                const int cc = min(BWD_XCOLS, ncols - c0);
                __syncthreads();
                for (int x = tid; x < cc * rr; x += WG) {
                    const int c = c0 + x % cc, r = r0 + x / cc;
                    int lo = 0, hi = ne;  // the entry holding column c: tab_c[lo] <= c < tab_c[lo + 1]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (tab_c[mid] <= c)
                            lo = mid;
                        else
                            hi = mid;
                    }
                    xs[x] = tab_src[lo][(c - tab_c[lo]) + (int64_t)r * tab_ld[lo]];
                }
                __syncthreads();
                // this wave's slice of the pass's columns
                const int q0 = (int)(((int64_t)cc * w) / 4), q1 = (int)(((int64_t)cc * (w + 1)) / 4);
                if (j < f) {
                    const T* col = ER + j + (int64_t)c0 * M;
                    if (rr == 1) {
#pragma unroll 8
                        for (int q = q0; q < q1; ++q) acc[0] = fma((double)col[(int64_t)q * M], xs[q], acc[0]);
                    } else {
#pragma unroll 4
                        for (int q = q0; q < q1; ++q) {
                            const double av = (double)col[(int64_t)q * M];
#pragma unroll
                            for (int t = 0; t < RC; ++t)
                                if (t < rr) acc[t] = fma(av, xs[q + t * cc], acc[t]);
                        }
                    }
                }
            }
            if (w > 0)
#pragma unroll
                for (int t = 0; t < RC; ++t) red[w - 1][lane][t] = acc[t];
            __syncthreads();
            if (w == 0 && j < f)
#pragma unroll
                for (int t = 0; t < RC; ++t)
                    if (t < rr)
                        dst[j + (int64_t)(r0 + t) * f] =
                            ((acc[t] + red[0][lane][t]) + red[1][lane][t]) + red[2][lane][t];
            __syncthreads();
        }
    }
}

void launch_apply_bwd_acc(const SolveLevelDev& S, const ColourDev& C, const double* z, const double* out,
                          double* part, const int64_t* part_off, int nrhs, hipStream_t st) {
    if (C.grp_total == 0) return;
    // right-hand sides per pass over E_R: eight where there are more than
    // four (E_R read once for up to eight), else four (half the LDS)
    const dim3 g(C.grp_total);
    if (nrhs > 4) {
        if (C.f32)
            hipLaunchKernelGGL((k_apply_bwd_acc<float, 8>), g, dim3(WG), 0, st, S, C, z, out, part, part_off, nrhs);
        else
            hipLaunchKernelGGL((k_apply_bwd_acc<double, 8>), g, dim3(WG), 0, st, S, C, z, out, part, part_off, nrhs);
    } else {
        if (C.f32)
            hipLaunchKernelGGL((k_apply_bwd_acc<float, 4>), g, dim3(WG), 0, st, S, C, z, out, part, part_off, nrhs);
        else
            hipLaunchKernelGGL((k_apply_bwd_acc<double, 4>), g, dim3(WG), 0, st, S, C, z, out, part, part_off, nrhs);
    }
}

constexpr int BWD_POFF = 512;

// out_s = T_R' v_s, v_s = [z_f - sum of the partials; z_c], rows r0 .. r0 + 63
// per workgroup (blockIdx.x = r0 / 64, blockIdx.y = cluster of the colour);
// every workgroup of a cluster forms the whole of v_s the same way.
template <class T>
__global__ void __launch_bounds__(WG) k_apply_bwd_t(SolveLevelDev S, ColourDev C, const double* __restrict__ z,
                                                    double* __restrict__ out, const double* __restrict__ part,
                                                    const int64_t* __restrict__ part_off, int nrhs) {
    extern __shared__ double vs[];  // max_m x nrhs, then the operand tile
    const int ci = blockIdx.y;
    const int s = C.clist[ci];
    const int M = S.m[s];
    const int r0 = blockIdx.x * UROWS;
    if (r0 >= M) return;
    const int nr = min(UROWS, M - r0);
    const int kk = S.k[s];
    const int f = M - kk;
    const double* zs = z + S.seg[s] * nrhs;
    double* os = out + S.seg[s] * nrhs;
    const int tot = M * nrhs;
    if (f == 0) {
        wg_stage(
            nr * nrhs, [&](int x) { return zs[r0 + x % nr + (x / nr) * M]; },
            [&](int x, double v) { os[r0 + x % nr + (x / nr) * M] = v; });
        return;
    }
    // partials of the neighbour groups: offsets staged in LDS, the loads of
    // one element issued eight at a time
    __shared__ int64_t poff[BWD_POFF];
    const int q0 = C.grp_pre[ci], q1 = C.grp_pre[ci + 1];
    for (int q0c = q0; q0c < q1 || q0c == q0; q0c += BWD_POFF) {
        const int nq = min(BWD_POFF, q1 - q0c);
        __syncthreads();
        for (int q = threadIdx.x; q < nq; q += blockDim.x) poff[q] = part_off[q0c + q] * nrhs;
        __syncthreads();
        for (int x = threadIdx.x; x < tot; x += blockDim.x) {
            const int i = x % M, r = x / M;
            double v = (q0c == q0) ? zs[x] : vs[x];
            if (i < f) {
                const double* pp = part + i + r * f;
                int q = 0;
                for (; q + 8 <= nq; q += 8) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) t[u] = pp[poff[q + u]];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v -= t[u];
                }
                for (; q < nq; ++q) v -= pp[poff[q]];
            }
            vs[x] = v;
        }
        if (q1 - q0c <= BWD_POFF) break;
    }
    const T* TR = srec<T>(S, s) + (int64_t)M * M + r0;  // T_R', from row r0
    wg_rows_times<T>(
        nr, M, nrhs, [&](int i, int l) { return TR[i + (int64_t)l * M]; }, [&](int l, int r) { return vs[l + r * M]; },
        tile_buf<T>(vs + (size_t)C.max_m * nrhs), [&](int i, int r, double v) { os[r0 + i + r * M] = v; });
}

// out_s = T_R' [z_f - sum of the neighbour-group partials ; z_c] (one
// right-hand side), one wave per cluster; the partials are subtracted in
// group order, WAVE_LD loads in flight, as in the workgroup form.
template <class T>
__global__ void __launch_bounds__(WG) k_apply_bwd_t_wave(SolveLevelDev S, ColourDev C, const double* __restrict__ z,
                                                         double* __restrict__ out, const double* __restrict__ part,
                                                         const int64_t* __restrict__ part_off) {
    const int ci = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    if (ci >= C.n) return;
    const int lane = threadIdx.x & 63;
    const int s = C.clist[ci];
    const int M = S.m[s];
    const int f = M - S.k[s];
    const double* zs = z + S.seg[s];
    double* os = out + S.seg[s];
    double v0 = lane < M ? zs[lane] : 0.0;
    double v1 = lane + 64 < M ? zs[lane + 64] : 0.0;
    if (f > 0) {
        const bool p0 = lane < f, p1 = lane + 64 < f;
        const int q0 = C.grp_pre[ci], q1 = C.grp_pre[ci + 1];
        int q = q0;
        for (; q + WAVE_LD <= q1; q += WAVE_LD) {
            double t0[WAVE_LD], t1[WAVE_LD];
#pragma unroll
            for (int u = 0; u < WAVE_LD; ++u) {
                const double* pp = part + part_off[q + u];
                t0[u] = p0 ? pp[lane] : 0.0;
                t1[u] = p1 ? pp[lane + 64] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < WAVE_LD; ++u) {
                v0 -= t0[u];
                v1 -= t1[u];
            }
        }
        for (; q < q1; ++q) {
            const double* pp = part + part_off[q];
            if (p0) v0 -= pp[lane];
            if (p1) v1 -= pp[lane + 64];
        }
        double a0, a1;
        wave_rows_times<T>(srec<T>(S, s) + (int64_t)M * M, M, v0, v1, a0, a1);
        v0 = a0;
        v1 = a1;
    }
    if (lane < M) os[lane] = v0;
    if (lane + 64 < M) os[lane + 64] = v1;
}

void launch_apply_bwd_t(const SolveLevelDev& S, const ColourDev& C, const double* z, double* out,
                        const double* part, const int64_t* part_off, int nrhs, hipStream_t st) {
    if (C.n == 0) return;
    if (nrhs == 1 && C.apply_wave > 0 && C.n >= C.apply_wave && C.max_m <= WAVE_MAXM) {
        const dim3 wgrid((C.n + WG / 64 - 1) / (WG / 64));
        if (C.f32)
            hipLaunchKernelGGL(k_apply_bwd_t_wave<float>, wgrid, dim3(WG), 0, st, S, C, z, out, part, part_off);
        else
            hipLaunchKernelGGL(k_apply_bwd_t_wave<double>, wgrid, dim3(WG), 0, st, S, C, z, out, part, part_off);
        return;
    }
    const size_t sh = tile_shmem((size_t)C.max_m * nrhs);
    const dim3 grid(std::max(1, (C.max_m + UROWS - 1) / UROWS), C.n);
    if (C.f32)
        hipLaunchKernelGGL(k_apply_bwd_t<float>, grid, dim3(WG), sh, st, S, C, z, out, part, part_off, nrhs);
    else
        hipLaunchKernelGGL(k_apply_bwd_t<double>, grid, dim3(WG), sh, st, S, C, z, out, part, part_off, nrhs);
}

// ---------------------------------------------------------- level transfer

__global__ void k_to_coarse(SolveLevelDev S, const int64_t* __restrict__ seg_next, int ncl_next,
                            const double* __restrict__ z, double* __restrict__ ynext, int nrhs, int from) {
    const int P = blockIdx.x;
    const int l = 2 * P, r = 2 * P + 1;
    const int kl = S.k[l], kr = (r < S.ncl) ? S.k[r] : 0;
    const int mp = kl + kr;
    double* yp = ynext + seg_next[P] * nrhs;
    for (int x = threadIdx.x; x < mp * nrhs; x += blockDim.x) {
        const int i = x % mp, c = x / mp;
        int cl = l, ii = i;
        if (i >= kl) {
            cl = r;
            ii = i - kl;
        }
        const int mc = S.m[cl];
        double* zc = const_cast<double*>(z) + S.seg[cl] * nrhs + (mc - S.k[cl]) + ii + (int64_t)c * mc;
        if (from)
            *zc = yp[x];
        else
            yp[x] = *zc;
    }
}

void launch_to_coarse(const SolveLevelDev& S, const int64_t* seg_next, int ncl_next, const double* z, double* ynext,
                      int nrhs, hipStream_t st) {
    if (ncl_next == 0) return;
    hipLaunchKernelGGL(k_to_coarse, dim3(ncl_next), dim3(256), 0, st, S, seg_next, ncl_next, z, ynext, nrhs, 0);
}

void launch_from_coarse(const SolveLevelDev& S, const int64_t* seg_next, int ncl_next, const double* outnext,
                        double* z, int nrhs, hipStream_t st) {
    if (ncl_next == 0) return;
    hipLaunchKernelGGL(k_to_coarse, dim3(ncl_next), dim3(256), 0, st, S, seg_next, ncl_next, z,
                       const_cast<double*>(outnext), nrhs, 1);
}

__global__ void k_scatter_gather(int64_t n, const int* __restrict__ cluster_of, const int* __restrict__ local_of,
                                 const int64_t* __restrict__ seg, const int* __restrict__ m, double* g, int64_t ldg,
                                 double* v, int nrhs, int to_level) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cluster_of[i], li = local_of[i], mc = m[c];
    double* base = v + seg[c] * nrhs + li;
    for (int r = 0; r < nrhs; ++r) {
        if (to_level)
            base[(int64_t)r * mc] = g[i + r * ldg];
        else
            g[i + r * ldg] = base[(int64_t)r * mc];
    }
}

void launch_scatter_rhs(int64_t n, const int* cluster_of, const int* local_of, const int64_t* seg, const int* m,
                        const double* B, int64_t ldb, double* y, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cluster_of, local_of,
                       seg, m, const_cast<double*>(B), ldb, y, nrhs, 1);
}

void launch_gather_sol(int64_t n, const int* cluster_of, const int* local_of, const int64_t* seg, const int* m,
                       const double* out, double* X, int64_t ldx, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cluster_of, local_of,
                       seg, m, X, ldx, const_cast<double*>(out), nrhs, 0);
}

}  // namespace hs
