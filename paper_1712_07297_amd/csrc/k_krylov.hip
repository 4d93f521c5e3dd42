// Krylov building blocks of Sec. 5 (CG for symmetric positive definite A,
// GMRES otherwise; float64).  A vector stacks the unknowns of one or more
// independent systems.  Sparse products go row by row; dot products and
// vector updates are per system, over chunks of KRY_CHUNK rows counted from
// the system's first row: one workgroup reduces a chunk in a fixed tree and
// the chunk sums of a system are added in chunk order, so a system's numbers
// do not depend on the systems stacked with it.
#include "device_common.h"
#include "kernels.h"

namespace hs {

constexpr int KRY_WG = 256;
constexpr int KRY_T = KRY_CHUNK / KRY_WG;  // rows per thread

__global__ void __launch_bounds__(KRY_WG) k_spmv(int64_t n, const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col_idx, const double* __restrict__ val,
                                                 const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                                 int64_t ldy, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    for (int r = 0; r < nrhs; ++r) {
        const double* x = X + r * ldx;
        double acc = 0.0;
        for (int64_t e = e0; e < e1; ++e) acc = fma(val[e], x[col_idx[e]], acc);
        Y[i + r * ldy] = acc;
    }
}

void launch_spmv(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val, const double* X,
                 int64_t ldx, double* Y, int64_t ldy, int nrhs, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)((n + KRY_WG - 1) / KRY_WG)), dim3(KRY_WG), 0, st, n, row_ptr, col_idx,
                       val, X, ldx, Y, ldy, nrhs);
}

// One chunk of one column: its rows of b stay in registers while the nvec
// vectors a_v stream past.
__global__ void __launch_bounds__(KRY_WG) k_sdots_part(SegDev G, int nvec, const double* __restrict__ a,
                                                       int64_t vstride, int64_t lda, const double* __restrict__ b,
                                                       int64_t ldb, double* __restrict__ part) {
    __shared__ double red[16];
    const int q = blockIdx.x, c = blockIdx.y, nrhs = gridDim.y;
    const int s = G.chunk_sys[q];
    const int64_t r0 = G.chunk_r0[q];
    const int64_t r1 = min(r0 + (int64_t)KRY_CHUNK, G.row_off[s + 1]);
    double bv[KRY_T];
#pragma unroll
    for (int t = 0; t < KRY_T; ++t) {
        const int64_t i = r0 + threadIdx.x + KRY_WG * t;
        bv[t] = i < r1 ? b[i + c * ldb] : 0.0;
    }
    for (int v = 0; v < nvec; ++v) {
        const double* av = a + v * vstride + c * lda;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < KRY_T; ++t) {
            const int64_t i = r0 + threadIdx.x + KRY_WG * t;
            if (i < r1) acc = fma(av[i], bv[t], acc);
        }
        acc = block_sum(acc, to_lds(red));
        if (threadIdx.x == 0) part[((int64_t)v * nrhs + c) * G.nchunks + q] = acc;
    }
}

// out[v * L + s + nsys c] = the system's chunk sums in chunk order.
__global__ void k_sdots_final(SegDev G, int nvec, int nrhs, const double* __restrict__ part, double* __restrict__ out) {
    const int64_t L = (int64_t)G.nsys * nrhs;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nvec * L) return;
    const int v = (int)(x / L);
    const int l = (int)(x % L);
    const int s = l % G.nsys, c = l / G.nsys;
    const double* p = part + ((int64_t)v * nrhs + c) * G.nchunks;
    double acc = 0.0;
    const int q1 = G.sys_chunk0[s + 1];
    int q = G.sys_chunk0[s];
    for (; q + 8 <= q1; q += 8) {  // eight loads in flight, added in chunk order
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = p[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t[u];
    }
    for (; q < q1; ++q) acc += p[q];
    out[x] = acc;
}

void launch_sdots(const SegDev& G, int nvec, const double* a, int64_t vstride, int64_t lda, const double* b,
                  int64_t ldb, int nrhs, double* part, double* out, hipStream_t st) {
    if (nvec <= 0 || G.nchunks == 0) return;
    hipLaunchKernelGGL(k_sdots_part, dim3(G.nchunks, nrhs), dim3(KRY_WG), 0, st, G, nvec, a, vstride, lda, b, ldb,
                       part);
    const int64_t tot = (int64_t)nvec * G.nsys * nrhs;
    hipLaunchKernelGGL(k_sdots_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, G, nvec, nrhs, part, out);
}

__global__ void __launch_bounds__(KRY_WG) k_saxpby(SegDev G, const double* __restrict__ alpha,
                                                   const double* __restrict__ x, int64_t ldx,
                                                   const double* __restrict__ beta, double* __restrict__ y,
                                                   int64_t ldy) {
    const int q = blockIdx.x, c = blockIdx.y;
    const int s = G.chunk_sys[q];
    const int l = s + G.nsys * c;
    const double al = alpha[l], be = beta[l];
    const int64_t r0 = G.chunk_r0[q];
    const int64_t r1 = min(r0 + (int64_t)KRY_CHUNK, G.row_off[s + 1]);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += KRY_WG) {
        double v = 0.0;
        if (al != 0.0) v = al * x[i + c * ldx];
        if (be != 0.0) v = fma(be, y[i + c * ldy], v);
        y[i + c * ldy] = v;
    }
}

void launch_saxpby(const SegDev& G, const double* alpha, const double* x, int64_t ldx, const double* beta, double* y,
                   int64_t ldy, int nrhs, hipStream_t st) {
    if (G.nchunks == 0) return;
    hipLaunchKernelGGL(k_saxpby, dim3(G.nchunks, nrhs), dim3(KRY_WG), 0, st, G, alpha, x, ldx, beta, y, ldy);
}

__global__ void __launch_bounds__(KRY_WG) k_scomb(SegDev G, int nvec, const double* __restrict__ coef,
                                                  const double* __restrict__ a, int64_t vstride, int64_t lda,
                                                  const double* __restrict__ beta, double* __restrict__ y,
                                                  int64_t ldy) {
    const int q = blockIdx.x, c = blockIdx.y, nrhs = gridDim.y;
    const int s = G.chunk_sys[q];
    const int64_t L = (int64_t)G.nsys * nrhs;
    const int l = s + G.nsys * c;
    const double be = beta[l];
    const int64_t r0 = G.chunk_r0[q];
    const int64_t r1 = min(r0 + (int64_t)KRY_CHUNK, G.row_off[s + 1]);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += KRY_WG) {
        double v = be != 0.0 ? be * y[i + c * ldy] : 0.0;
        for (int k = 0; k < nvec; ++k) {
            const double cf = coef[k * L + l];
            if (cf != 0.0) v = fma(cf, a[k * vstride + i + c * lda], v);
        }
        y[i + c * ldy] = v;
    }
}

void launch_scomb(const SegDev& G, int nvec, const double* coef, const double* a, int64_t vstride, int64_t lda,
                  const double* beta, double* y, int64_t ldy, int nrhs, hipStream_t st) {
    if (G.nchunks == 0) return;
    hipLaunchKernelGGL(k_scomb, dim3(G.nchunks, nrhs), dim3(KRY_WG), 0, st, G, nvec, coef, a, vstride, lda, beta, y,
                       ldy);
}

__global__ void __launch_bounds__(KRY_WG) k_xmy(int64_t n, const double* __restrict__ x, int64_t ldx,
                                                double* __restrict__ y, int64_t ldy, int nrhs, int copy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < nrhs; ++r) y[i + r * ldy] = copy ? x[i + r * ldx] : x[i + r * ldx] - y[i + r * ldy];
}

void launch_xmy(int64_t n, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_xmy, dim3((unsigned)((n + KRY_WG - 1) / KRY_WG)), dim3(KRY_WG), 0, st, n, x, ldx, y, ldy,
                       nrhs, 0);
}

void launch_copy(int64_t n, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_xmy, dim3((unsigned)((n + KRY_WG - 1) / KRY_WG)), dim3(KRY_WG), 0, st, n, x, ldx, y, ldy,
                       nrhs, 1);
}

}  // namespace hs
