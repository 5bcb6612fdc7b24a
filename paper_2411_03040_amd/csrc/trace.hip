// Ray tracing on the device (gfx950).
//
// Neighbour walk on the point cloud: from the current point step to the
// listed neighbour that lies further along the ray and is closest to the
// ray line; ties go to the earlier neighbour-list entry; stop after stepping
// onto a boundary point or when no neighbour lies further along.  Spherical
// shells (dim 1): crossings of every shell with r^2 > b^2 beyond the origin,
// in path order, until a boundary shell.  Traces are compared bit for bit
// with an independent CPU walk, so every multiply and add here rounds on its
// own (no contraction) and is evaluated in a fixed order.
//
// Launch shape (point cloud): one group of 16 lanes per walk, four walks per
// wave64.  At each step the 16 lanes test up to 16 neighbour candidates at
// once (coalesced CSR read, independent position gathers) and reduce the
// lexicographic minimum of (squared distance to the ray line, list
// position) with cross-lane shuffles, so a step costs one gather round trip
// instead of k sequential ones.
#pragma clang fp contract(off)

#include <hipcub/hipcub.hpp>

#include "mgx_internal.h"

namespace mgx {

__global__ void k_point_widths(int N, const double *__restrict__ T,
                               const double *__restrict__ vturb2, double mass,
                               double *__restrict__ b2, double *__restrict__ b,
                               float *__restrict__ bf, float *__restrict__ ibf_scaled,
                               double *__restrict__ bd, double *__restrict__ ibd)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const double v2 = ((2.0 * kKB) * T[p]) / mass + vturb2[p];
    const double bb = sqrt(v2);
    b2[p] = v2;
    b[p] = bb;
    bf[p] = (float)bb;
    // exp(-x^2) = exp2(-(x sqrt(log2 e))^2): fold sqrt(log2 e) into 1/b
    ibf_scaled[p] = (float)(sqrt(kLog2e) / bb);
    bd[p] = bb;
    ibd[p] = 1.0 / bb;
}

hipError_t launch_point_widths(int N, const double *T, const double *vturb2, double mass,
                               double *b2, double *b, float *bf, float *ibf_scaled,
                               double *bd, double *ibd, hipStream_t s)
{
    k_point_widths<<<(N + 255) / 256, 256, 0, s>>>(N, T, vturb2, mass, b2, b, bf, ibf_scaled,
                                                  bd, ibd);
    return hipGetLastError();
}

// Branch rule shared by both trace shapes: semi-analytic iff the projected
// velocity difference across the segment is at least thr averaged widths,
// compared in squares: d^2 >= thr^2 (b0^2 + b1^2) / 2.
__device__ __forceinline__ bool use_semi(double dv0, double b20, double dv1, double b21,
                                         double thr)
{
    const double d = dv1 - dv0;
    return d * d >= (thr * thr) * ((b20 + b21) * 0.5);
}

template <bool FILL>
__device__ __forceinline__ void emit(const TraceArgs &a, int64_t pos, int j, double Z,
                                     double dv, double Zprev, double dvprev, double b2prev,
                                     unsigned long long &nsemi)
{
    if (!FILL) return;
    const double b2j = a.b2[j];
    const bool semi = use_semi(dvprev, b2prev, dv, b2j, a.thr);
    a.r_idx[pos] = j;
    a.r_Z[pos] = Z;
    a.r_dv[pos] = dv;
    a.r_dx[pos] = Z - Zprev;
    a.r_ibb[pos] = 1.0 / sqrt((b2prev + b2j) * 0.5);
    a.r_semi[pos] = semi ? 1 : 0;
    nsemi += semi ? 1 : 0;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_trace3d(TraceArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = gid >> 4;
    const int l16 = threadIdx.x & 15;
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (w >= nwalk) return;  // uniform across the 16-lane group
    const int o = (int)(w / a.R);
    const int r = (int)(w - (int64_t)o * a.R);
    const double nx = a.ray_dir[3 * r + 0];
    const double ny = a.ray_dir[3 * r + 1];
    const double nz = a.ray_dir[3 * r + 2];
    const double xo = a.x[o], yo = a.y[o], zo = a.z[o];
    const double vxo = a.vx[o], vyo = a.vy[o], vzo = a.vz[o];
    int c = o;
    double Zc = 0.0, dvc = 0.0, b2c = FILL ? a.b2[o] : 0.0;
    int64_t n = 0;
    const int64_t base = FILL ? a.off[w] : 0;
    unsigned long long nsemi = 0;
    for (;;) {
        const int q0 = a.nbs_off[c], q1 = a.nbs_off[c + 1];
        double bd2 = INFINITY, bZ = 0.0;
        int bq = 0x7fffffff, bj = -1;
        for (int qb = q0; qb < q1; qb += 16) {
            const int q = qb + l16;
            if (q < q1) {
                const int j = a.nbs[q];
                const double ddx = a.x[j] - xo;
                const double ddy = a.y[j] - yo;
                const double ddz = a.z[j] - zo;
                const double Zj = (ddx * nx + ddy * ny) + ddz * nz;
                if (Zj > Zc) {
                    const double ex = ddx - Zj * nx;
                    const double ey = ddy - Zj * ny;
                    const double ez = ddz - Zj * nz;
                    const double d2 = (ex * ex + ey * ey) + ez * ez;
                    if (d2 < bd2) {
                        bd2 = d2;
                        bq = q;
                        bj = j;
                        bZ = Zj;
                    }
                }
            }
        }
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) {
            const double od2 = __shfl_xor(bd2, m, 16);
            const int oq = __shfl_xor(bq, m, 16);
            const int oj = __shfl_xor(bj, m, 16);
            const double oZ = __shfl_xor(bZ, m, 16);
            if (od2 < bd2 || (od2 == bd2 && oq < bq)) {
                bd2 = od2;
                bq = oq;
                bj = oj;
                bZ = oZ;
            }
        }
        if (bj < 0) {
            if (FILL && l16 == 0 && !a.bdy[c]) atomicAdd(&a.cnt->holes, 1ull);
            break;
        }
        const double dv = ((a.vx[bj] - vxo) * nx + (a.vy[bj] - vyo) * ny) + (a.vz[bj] - vzo) * nz;
        if (l16 == 0) emit<FILL>(a, base + n, bj, bZ, dv, Zc, dvc, b2c, nsemi);
        n++;
        c = bj;
        Zc = bZ;
        dvc = dv;
        if (FILL) b2c = a.b2[c];
        if (a.bdy[c]) break;
    }
    if (l16 == 0) {
        if (!FILL) a.counts[w] = n;
        if (FILL && nsemi) atomicAdd(&a.cnt->semi, nsemi);
    }
}

// Spherical shells: one thread per (origin, mu).
template <bool FILL>
__global__ __launch_bounds__(256) void k_trace1d(TraceArgs a)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (w >= nwalk) return;
    const int o = (int)(w / a.R);
    const int r = (int)(w - (int64_t)o * a.R);
    const int N = a.N;
    const double mu = a.ray_dir[3 * r + 0];
    const double ro = a.x[o];
    const double so = ro * mu;
    double b2 = ro * ro - so * so;
    if (b2 < 0.0) b2 = 0.0;
    const double vo = a.vx[o];
    int64_t n = 0;
    const int64_t base = FILL ? a.off[w] : 0;
    double Zp = 0.0, dvp = 0.0, b2p = FILL ? a.b2[o] : 0.0;
    unsigned long long nsemi = 0;
    auto rec = [&](int k, double s) {
        const double Z = s - so;
        const double dv = a.vx[k] * (s / a.x[k]) - vo * mu;
        emit<FILL>(a, base + n, k, Z, dv, Zp, dvp, b2p, nsemi);
        n++;
        Zp = Z;
        dvp = dv;
        if (FILL) b2p = a.b2[k];
    };
    bool done = false;
    if (mu >= 0.0) {
        for (int k = o + 1; k < N && !done; k++) {
            rec(k, sqrt(a.x[k] * a.x[k] - b2));
            done = a.bdy[k] != 0;
        }
    } else if (o != 0) {
        int k = o - 1;
        while (!done && k >= 0 && a.x[k] * a.x[k] > b2) {
            rec(k, -sqrt(a.x[k] * a.x[k] - b2));
            done = a.bdy[k] != 0;
            k--;
        }
        for (int kk = k + 1; kk < N && !done; kk++) {
            rec(kk, sqrt(a.x[kk] * a.x[kk] - b2));
            done = a.bdy[kk] != 0;
        }
    }
    if (!FILL) a.counts[w] = n;
    if (FILL && nsemi) atomicAdd(&a.cnt->semi, nsemi);
}

hipError_t launch_trace(const TraceArgs &a, bool fill, hipStream_t s)
{
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (a.dim == 1) {
        const int64_t blocks = (nwalk + 255) / 256;
        if (fill)
            k_trace1d<true><<<blocks, 256, 0, s>>>(a);
        else
            k_trace1d<false><<<blocks, 256, 0, s>>>(a);
    } else {
        const int64_t blocks = (nwalk * 16 + 255) / 256;
        if (fill)
            k_trace3d<true><<<blocks, 256, 0, s>>>(a);
        else
            k_trace3d<false><<<blocks, 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

// Convert the double-precision trace into the packed records of the solve.
template <typename T>
__global__ void k_pack(int64_t n, const int32_t *__restrict__ idx,
                       const uint8_t *__restrict__ semi, const double *__restrict__ dx,
                       const double *__restrict__ dv, const double *__restrict__ ibb,
                       double inv_L, Rec<T> *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec<T> r;
    r.ps = idx[i] | (semi[i] ? (int32_t)0x80000000u : 0);
    r.dx = (T)(dx[i] * inv_L);
    r.dv = (T)dv[i];
    r.ibb = (T)ibb[i];
    out[i] = r;
}

template <>
__global__ void k_pack<double>(int64_t n, const int32_t *__restrict__ idx,
                               const uint8_t *__restrict__ semi, const double *__restrict__ dx,
                               const double *__restrict__ dv, const double *__restrict__ ibb,
                               double inv_L, Rec<double> *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec<double> r;
    r.ps = idx[i] | (semi[i] ? (int32_t)0x80000000u : 0);
    r.pad = 0;
    r.dx = dx[i] * inv_L;
    r.dv = dv[i];
    r.ibb = ibb[i];
    out[i] = r;
}

hipError_t launch_pack_trace(int64_t n, const int32_t *idx, const uint8_t *semi,
                             const double *dx, const double *dv, const double *ibb,
                             double inv_L, bool fp32, void *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (fp32)
        k_pack<float><<<blocks, 256, 0, s>>>(n, idx, semi, dx, dv, ibb, inv_L,
                                            (Rec<float> *)out);
    else
        k_pack<double><<<blocks, 256, 0, s>>>(n, idx, semi, dx, dv, ibb, inv_L,
                                             (Rec<double> *)out);
    return hipGetLastError();
}

}  // namespace mgx

// Exclusive scan of walk lengths into record offsets (hipCUB device scan).
extern "C" hipError_t mgx_internal_scan(int64_t *counts, int64_t *offsets, int64_t n,
                                        void **tmp, size_t *tmp_bytes, hipStream_t s)
{
    size_t need = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, need, counts, offsets, n, s);
    if (e != hipSuccess) return e;
    if (need > *tmp_bytes) {
        if (*tmp) (void)hipFree(*tmp);
        *tmp = nullptr;
        e = hipMalloc(tmp, need);
        if (e != hipSuccess) {
            *tmp_bytes = 0;
            return e;
        }
        *tmp_bytes = need;
    }
    return hipcub::DeviceScan::ExclusiveSum(*tmp, need, counts, offsets, n, s);
}
