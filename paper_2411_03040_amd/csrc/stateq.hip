// Statistical equilibrium, LTE populations and convergence measure (FP64).
//
// Rates with the approximate operator (accelerated Lambda-iteration,
// Rybicki & Hummer 1991):
//   J_eff = Jbar - Lstar S_old
//   R_ul = A (1 - Lstar) + B_ul J_eff + C_ul,   R_lu = B_lu J_eff + C_lu
//   C_ul = n_coll K0 sqrt(T / 100 K),  C_lu = C_ul (g_u / g_l) exp(-(E_u - E_l) / k T)
// Rate matrix M_ij = R_{j->i}, M_ii = -sum_j R_{i->j}; row 0 replaced by
// sum_i f_i = 1; Gaussian elimination with partial pivoting.
//
// Launch shape: one wave64 per point.  Each wave keeps its (nlev x nlev+1)
// augmented matrix in LDS; lanes own rows during elimination (the pivot row
// is an LDS broadcast) and columns while assembling the diagonal.  The pivot
// search is a cross-lane max with the lowest row index winning ties.  The
// work is far below the formal solution's (levels^3 per point against
// rays x bins x points-per-ray), so this favours simplicity over peak rate.

#include "mgx_internal.h"

namespace mgx {

__global__ void k_reset_counters(Counters *c, int with_masing)
{
    if (threadIdx.x == 0) {
        if (with_masing) c->masing = 0;
        c->singular = 0;
        c->nonfinite = 0;
        c->change_bits = 0;
    }
}

hipError_t launch_reset_counters(Counters *c, hipStream_t s, bool with_masing)
{
    k_reset_counters<<<1, 64, 0, s>>>(c, with_masing ? 1 : 0);
    return hipGetLastError();
}

__global__ void k_lte(int N, int nlev, const double *T, const double *E, const double *g,
                      double *pops)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double z = 0.0;
    for (int i = 0; i < nlev; i++) {
        const double v = g[i] * exp(-E[i] / (kKB * T[p]));
        pops[(int64_t)p * nlev + i] = v;
        z += v;
    }
    for (int i = 0; i < nlev; i++) pops[(int64_t)p * nlev + i] /= z;
}

hipError_t launch_lte(int N, int nlev, const double *T, const double *E, const double *g,
                      double *pops, hipStream_t s)
{
    k_lte<<<(N + 255) / 256, 256, 0, s>>>(N, nlev, T, E, g, pops);
    return hipGetLastError();
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *bits, double v)
{
    // non-negative doubles (and NaN, which sorts above +inf) order like their bits
    atomicMax(bits, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double o = __shfl_xor(v, m, 64);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

// One group of G lanes per point (G the smallest of 8, 16, 32, 64 that is at
// least the level count, so a wave solves 64 / G points side by side); the
// point's rate matrix sits in LDS, row i belongs to lane i of the group.
// Gaussian elimination with partial pivoting (largest magnitude, ties to
// the lower row), then back substitution; singular systems keep the old
// populations and are counted.
__global__ __launch_bounds__(256) void k_stateq(StateqArgs a)
{
    extern __shared__ double sm[];
    if (a.active && !a.active[a.model]) return;  // uniform over the grid
    const int L = a.nlev, L1 = L + 1, G = a.group;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / G, gl = lane - grp * G;
    const int ppw = 64 / G;
    double *M = sm + ((size_t)wid * ppw + grp) * L * L1;
    const int p = (blockIdx.x * a.wpb + wid) * ppw + grp;
    const bool valid = p < a.N;
    const int pp = valid ? p : 0;

    for (int i = gl; i < L * L1; i += G) M[i] = 0.0;
    __syncthreads();
    if (valid) {
        for (int t = gl; t < a.nlines; t += G) {
            const int u = a.up[t], lw = a.lo[t];
            const int64_t pl = (int64_t)pp * a.nlines + t;
            const double Ls = a.L[pl];
            const double Jeff = a.J[pl] - Ls * a.S64[pl];
            M[lw * L1 + u] = a.A[t] * (1.0 - Ls) + a.Bul[t] * Jeff;
            M[u * L1 + lw] = a.Blu[t] * Jeff;
        }
    }
    __syncthreads();
    if (valid) {
        const double T = a.T[pp];
        const double sq = sqrt(T / 100.0);
        for (int t = gl; t < a.ncoll_tr; t += G) {
            const int u = a.cu[t], lw = a.cl[t];
            const double Cul = a.ncoll[pp] * a.K0[t] * sq;
            const double Clu = Cul * (a.g[u] / a.g[lw]) * exp(-(a.E[u] - a.E[lw]) / (kKB * T));
            M[lw * L1 + u] += Cul;
            M[u * L1 + lw] += Clu;
        }
    }
    __syncthreads();
    if (gl < L) {
        double s = 0.0;
        for (int j = 0; j < L; j++)
            if (j != gl) s += M[j * L1 + gl];
        M[gl * L1 + gl] = -s;
    }
    __syncthreads();
    if (gl < L) {
        M[gl] = 1.0;                                 // row 0: sum f = 1
        M[gl * L1 + L] = (gl == 0) ? 1.0 : 0.0;      // right-hand side
    }
    __syncthreads();

    bool singular = false;  // uniform over the group
    for (int k = 0; k < L; k++) {
        double v = (gl >= k && gl < L) ? fabs(M[gl * L1 + k]) : -1.0;
        int idx = gl;
        for (int m = G >> 1; m >= 1; m >>= 1) {
            const double ov = __shfl_xor(v, m, G);
            const int oi = __shfl_xor(idx, m, G);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        if (!(v >= 1e-300)) singular = true;
        if (!singular && idx != k) {
            for (int j = gl; j <= L; j += G) {
                const double t = M[k * L1 + j];
                M[k * L1 + j] = M[idx * L1 + j];
                M[idx * L1 + j] = t;
            }
        }
        __syncthreads();
        if (!singular && gl > k && gl < L) {
            const double fct = M[gl * L1 + k] / M[k * L1 + k];
            for (int j = k; j <= L; j++) M[gl * L1 + j] -= fct * M[k * L1 + j];
        }
        __syncthreads();
    }
    for (int i = L - 1; i >= 0; i--) {
        if (!singular && gl == i) M[i * L1 + L] /= M[i * L1 + i];
        __syncthreads();
        if (!singular && gl < i) M[gl * L1 + L] -= M[gl * L1 + i] * M[i * L1 + L];
        __syncthreads();
    }

    double ch = 0.0;
    if (valid && gl < L) {
        const int64_t pi = (int64_t)p * L + gl;
        const double old = a.pops_old[pi];
        double nw = singular ? old : M[gl * L1 + L];
        if (!isfinite(nw)) {
            atomicAdd(&a.cnt->nonfinite, 1ull);
        }
        a.pops_new[pi] = nw;
        const double den = nw > a.pop_floor ? nw : a.pop_floor;
        ch = fabs(nw - old) / den;
    }
    if (valid && gl == 0 && singular) atomicAdd(&a.cnt->singular, 1ull);
    ch = wave_max(ch);
    if (lane == 0) atomic_max_nonneg(&a.cnt->change_bits, ch);
}

int stateq_group(int nlev)
{
    return nlev <= 8 ? 8 : nlev <= 16 ? 16 : nlev <= 32 ? 32 : 64;
}

hipError_t launch_stateq(const StateqArgs &a, hipStream_t s)
{
    if (a.group != stateq_group(a.nlev) || a.wpb < 1) return hipErrorInvalidValue;
    const int ppw = 64 / a.group;
    const size_t per_wave = sizeof(double) * a.nlev * (a.nlev + 1) * ppw;
    const int64_t per_block = (int64_t)a.wpb * ppw;
    const int blocks = (int)((a.N + per_block - 1) / per_block);
    if (blocks == 0) return hipSuccess;
    k_stateq<<<blocks, 64 * a.wpb, per_wave * a.wpb, s>>>(a);
    return hipGetLastError();
}

__global__ void k_rel_change(int64_t n, const double *a, const double *b, double floor_,
                             unsigned long long *bits)
{
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double den = a[i] > floor_ ? a[i] : floor_;
        const double d = fabs(a[i] - b[i]) / den;
        m = (d > m || d != d) ? d : m;
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(bits, m);
}

hipError_t launch_rel_change(int64_t n, const double *a, const double *b, double floor_,
                             unsigned long long *bits, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_rel_change<<<blocks, 256, 0, s>>>(n, a, b, floor_, bits);
    return hipGetLastError();
}

__global__ void k_copy(int64_t n, const double *src, double *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(int64_t n, const double *src, double *dst, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_copy<<<blocks, 256, 0, s>>>(n, src, dst);
    return hipGetLastError();
}

__global__ void k_copy_if_active(int64_t n, const double *src, double *dst, const int *active,
                                 int model)
{
    if (!active[model]) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy_if_active(int64_t n, const double *src, double *dst, const int *active,
                                 int model, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_copy_if_active<<<blocks, 256, 0, s>>>(n, src, dst, active, model);
    return hipGetLastError();
}

// per-model max relative change (IEEE bits in each model's counters) -> out[m],
// and a failure flag -> out[M + m]: 1 singular system, 2 non-finite result
__global__ void k_gather_changes(int M, Counters *const *cnt, double *out)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const Counters *c = cnt[m];
    out[m] = __longlong_as_double((long long)c->change_bits);
    out[M + m] = c->singular ? 1.0 : (c->nonfinite ? 2.0 : 0.0);
}

hipError_t launch_gather_changes(int M, Counters *const *cnt, double *out, hipStream_t s)
{
    k_gather_changes<<<(M + 255) / 256, 256, 0, s>>>(M, cnt, out);
    return hipGetLastError();
}

}  // namespace mgx
