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

// ---------------------------------------------------------------------------
// The prediction without device allocation (mgx_ng_predict_noalloc): the
// iterates stay where the caller keeps them, and everything else the
// kernels need -- the Gram rows' block partial sums, the Gram matrix, the
// solve's status and the negative-entry flag -- lives in one fixed area
// compiled into the library.  Each GPU the library runs on holds its own
// copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
// ---------------------------------------------------------------------------
namespace mgx {

constexpr int kScratchPartial = 1024 * kNgKMax;     // block partials (max blocks x columns)
constexpr int kScratchG = kNgKMax * kNgKMax;        // Gram matrix
constexpr int kScratchDoubles = kScratchPartial + kScratchG + 32;  // + 256 bytes of flags
static __device__ __align__(256) double scratch[kScratchDoubles];

// Row j of the Gram matrix from the iterates themselves: r_j = y_{j+1} - y_j
// against r_a = y_{a+1} - y_a (a <= j), block partials as k_ng_append forms
// them (same residual arithmetic, same per-thread order, same tree), so the
// matrix is the one the context's incremental path builds.
__global__ __launch_bounds__(kNgThreads) void k_ng_gram_row(int64_t n, int j, const PtrTable y,
                                                          double *partial)
{
    double acc[kNgKMax];
#pragma unroll
    for (int a = 0; a < kNgKMax; a++) acc[a] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double rn = y.p[j + 1][i] - y.p[j][i];
#pragma unroll
        for (int a = 0; a < kNgKMax; a++) {
            if (a < j) acc[a] += (y.p[a + 1][i] - y.p[a][i]) * rn;
        }
#pragma unroll
        for (int a = 0; a < kNgKMax; a++)
            if (a == j) acc[a] += rn * rn;
    }
    __shared__ double red[kNgThreads];
    for (int a = 0; a <= j; a++) {
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

// flags[0]: Gram solve status, flags[1]: negative entry seen
__global__ void k_noalloc_clear(int *flags)
{
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

__global__ void k_noalloc_status(const int *flags, int *status_out)
{
    if (threadIdx.x == 0) *status_out = (flags[0] == 0 && flags[1] == 0) ? 1 : 0;
}

}  // namespace mgx

#include <mutex>

#include "../../include/mgx.h"

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices];  // per device: the address of `scratch` there
}  // namespace

// message of the last failed call without a context (mgx_last_error(NULL))
namespace mgxh {
extern thread_local std::string g_create_error;
}

extern "C" mgx_status mgx_ng_predict_noalloc(int device, void *stream,
                                             const double *const *iterates, int nhist, int64_t n,
                                             double *prediction, double *coef, int *status)
{
    using namespace mgx;
    std::string &err = mgxh::g_create_error;
    err.clear();
    if (nhist < 2 || nhist > kNgMaxHist) {
        err = "nhist must be 2.." + std::to_string(kNgMaxHist) + " (fixed scratch area)";
        return MGX_EINVAL;
    }
    if (n < 1 || !iterates || !prediction || !coef || !status) {
        err = "n >= 1 and non-NULL iterates, prediction, coef and status required";
        return MGX_EINVAL;
    }
    for (int k = 0; k < nhist; k++)
        if (!iterates[k]) {
            err = "NULL iterate pointer";
            return MGX_EINVAL;
        }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
        device >= kMaxDevices) {
        err = "no such HIP device";
        return MGX_EINVAL;
    }
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        err = "hipSetDevice failed";
        return MGX_EHIP;
    }
    mgx_status rc = MGX_OK;
    double *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e == hipSuccess && p)
                g_scratch[device] = (double *)p;
            else
                err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        }
        base = g_scratch[device];
    }
    if (!base) rc = MGX_EHIP;
    if (rc == MGX_OK) {
        hipStream_t s = (hipStream_t)stream;
        double *partial = base;
        double *G = base + kScratchPartial;
        int *flags = (int *)(base + kScratchPartial + kScratchG);
        PtrTable y{};
        for (int k = 0; k < nhist; k++) y.p[k] = iterates[k];
        PtrTable yt{};
        for (int k = 0; k + 1 < nhist; k++) yt.p[k] = iterates[k + 1];
        const int K = nhist - 1;
        const int nb = ng_gram_blocks(n);
        hipError_t e = hipSuccess;
        k_noalloc_clear<<<1, 64, 0, s>>>(flags);
        e = hipGetLastError();
        for (int j = 0; j < K && e == hipSuccess; j++) {
            k_ng_gram_row<<<nb, kNgThreads, 0, s>>>(n, j, y, partial);
            e = hipGetLastError();
            if (e == hipSuccess) {
                k_ng_grow<<<j + 1, kNgThreads, 0, s>>>(j + 1, partial, nb, G);
                e = hipGetLastError();
            }
        }
        if (e == hipSuccess) e = launch_ng_predict(n, K, G, yt, coef, flags, prediction, flags + 1, s);
        if (e == hipSuccess) {
            k_noalloc_status<<<1, 64, 0, s>>>(flags, status);
            e = hipGetLastError();
        }
        if (e != hipSuccess) {
            err = std::string("HIP: ") + hipGetErrorString(e);
            rc = MGX_EHIP;
        }
    }
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    return rc;
}
