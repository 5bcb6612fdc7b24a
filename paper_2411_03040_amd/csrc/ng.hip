// Ng acceleration on the device (FP64), Section "Adaptive Ng-acceleration"
// and its appendix: c = (R R^T)^-1 1 / (1^T (R R^T)^-1 1), n* = sum_k c_k
// y_{k+1}, residuals r_k = y_{k+1} - y_k.
//
// The Gram matrix G = R R^T is kept on the device and grown by one row per
// appended iterate (the new residual against all stored ones), so an
// adaptive step that forms a prediction after every iteration streams each
// residual once instead of rebuilding G.  Dot products are block partial
// sums reduced in a fixed order (deterministic).  The (N-1) x (N-1) solve is
// one thread's Gaussian elimination with partial pivoting; the combination
// is a streaming kernel that also flags negative predictions.

#include "mgx_internal.h"

namespace mgx {

constexpr int kNgThreads = 256;
constexpr int kNgKMax = kNgMaxHist;  // residuals <= 31

int ng_gram_blocks(int64_t n)
{
    int64_t b = (n + kNgThreads * 4 - 1) / (kNgThreads * 4);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

// Append: dst_y = src, dst_r = src - prev, partial[block][a] = sum r_a . r_new
// over this block's elements for a < K (K counts the new residual).
__global__ __launch_bounds__(kNgThreads) void k_ng_append(int64_t n, int K, const double *src,
                                                        const double *prev, double *dst_y,
                                                        double *dst_r,
                                                        const PtrTable r_ptrs,
                                                        double *partial)
{
    double acc[kNgKMax];
#pragma unroll
    for (int a = 0; a < kNgKMax; a++) acc[a] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = src[i];
        const double rn = v - prev[i];
        dst_y[i] = v;
        dst_r[i] = rn;
#pragma unroll
        for (int a = 0; a < kNgKMax; a++) {
            if (a < K - 1) acc[a] += r_ptrs.p[a][i] * rn;
        }
        if (K - 1 < kNgKMax) {
#pragma unroll
            for (int a = 0; a < kNgKMax; a++)
                if (a == K - 1) acc[a] += rn * rn;
        }
    }
    __shared__ double red[kNgThreads];
    for (int a = 0; a < K; a++) {
        red[threadIdx.x] = acc[a];
        __syncthreads();
        for (int s = kNgThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kNgKMax + a] = red[0];
        __syncthreads();
    }
}

// Sum the block partials of column a (one workgroup per a, fixed order:
// strided per-thread sums, then a tree) into row/column K-1 of G.
__global__ __launch_bounds__(kNgThreads) void k_ng_grow(int K, const double *partial,
                                                      int nblocks, double *G)
{
    const int a = blockIdx.x;
    __shared__ double red[kNgThreads];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kNgThreads) s += partial[(size_t)b * kNgKMax + a];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = kNgThreads / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        G[a * kNgKMax + (K - 1)] = red[0];
        G[(K - 1) * kNgKMax + a] = red[0];
    }
}

// Drop the oldest residual: G <- G[1:, 1:].
__global__ void k_ng_shift(int K, double *G)
{
    if (threadIdx.x != 0) return;
    for (int i = 0; i < K - 1; i++)
        for (int j = 0; j < K - 1; j++) G[i * kNgKMax + j] = G[(i + 1) * kNgKMax + (j + 1)];
}

// c = G^-1 1 / 1^T G^-1 1; status 0 ok, -1 singular (pivot below 1e-14 max G_kk).
__global__ void k_ng_solve(int K, const double *G, double *coef, int *status)
{
    if (threadIdx.x != 0) return;
    __shared__ double A[kNgKMax * (kNgKMax + 1)];
    const int K1 = K + 1;
    double gmax = 0.0;
    for (int i = 0; i < K; i++) {
        for (int j = 0; j < K; j++) A[i * K1 + j] = G[i * kNgKMax + j];
        A[i * K1 + K] = 1.0;
        if (G[i * kNgKMax + i] > gmax) gmax = G[i * kNgKMax + i];
    }
    int st = 0;
    for (int k = 0; k < K && st == 0; k++) {
        int piv = k;
        for (int i = k + 1; i < K; i++)
            if (fabs(A[i * K1 + k]) > fabs(A[piv * K1 + k])) piv = i;
        if (!(fabs(A[piv * K1 + k]) > 1e-14 * gmax)) {
            st = -1;
            break;
        }
        if (piv != k)
            for (int j = 0; j <= K; j++) {
                const double t = A[k * K1 + j];
                A[k * K1 + j] = A[piv * K1 + j];
                A[piv * K1 + j] = t;
            }
        for (int i = k + 1; i < K; i++) {
            const double f = A[i * K1 + k] / A[k * K1 + k];
            for (int j = k; j <= K; j++) A[i * K1 + j] -= f * A[k * K1 + j];
        }
    }
    if (st == 0) {
        double c[kNgKMax];
        double sum = 0.0;
        for (int i = K - 1; i >= 0; i--) {
            double s = A[i * K1 + K];
            for (int j = i + 1; j < K; j++) s -= A[i * K1 + j] * c[j];
            c[i] = s / A[i * K1 + i];
        }
        for (int i = 0; i < K; i++) sum += c[i];
        for (int i = 0; i < K; i++) coef[i] = c[i] / sum;
    }
    *status = st;
}

// out = sum_k c_k y_{k+1}; neg |= any(out < 0).  y_ptrs[k] = y_{k+1}.
__global__ __launch_bounds__(kNgThreads) void k_ng_combine(int64_t n, int K,
                                                         const PtrTable y_ptrs,
                                                         const double *coef, const int *status,
                                                         double *out, int *neg)
{
    if (*status != 0) return;
    double c[kNgKMax];
#pragma unroll
    for (int k = 0; k < kNgKMax; k++) c[k] = (k < K) ? coef[k] : 0.0;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kNgKMax; k++)
            if (k < K) s += c[k] * y_ptrs.p[k][i];
        out[i] = s;
        bad |= (s < 0.0);
    }
    if (bad) atomicOr(neg, 1);
}

hipError_t launch_ng_append(int64_t n, int K, const double *src, const double *prev,
                            double *dst_y, double *dst_r, const PtrTable &r_ptrs,
                            double *partial, double *G, hipStream_t s)
{
    const int nb = ng_gram_blocks(n);
    k_ng_append<<<nb, kNgThreads, 0, s>>>(n, K, src, prev, dst_y, dst_r, r_ptrs, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ng_grow<<<K, kNgThreads, 0, s>>>(K, partial, nb, G);
    return hipGetLastError();
}

hipError_t launch_ng_shift(int K, double *G, hipStream_t s)
{
    k_ng_shift<<<1, 64, 0, s>>>(K, G);
    return hipGetLastError();
}

hipError_t launch_ng_predict(int64_t n, int K, const double *G, const PtrTable &y_ptrs,
                             double *coef, int *status, double *out, int *neg, hipStream_t s)
{
    k_ng_solve<<<1, 64, 0, s>>>(K, G, coef, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = ng_gram_blocks(n);
    k_ng_combine<<<nb, kNgThreads, 0, s>>>(n, K, y_ptrs, coef, status, out, neg);
    return hipGetLastError();
}

}  // namespace mgx
