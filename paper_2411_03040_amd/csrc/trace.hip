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
                                     unsigned long long &nsemi, double b2j)
{
    if (!FILL) return;
    const bool semi = use_semi(dvprev, b2prev, dv, b2j, a.thr);
    a.r_idx[pos] = j;
    a.r_Z[pos] = Z;
    a.r_dv[pos] = dv;
    // the segment length, or for a semi-analytic segment the lane-independent
    // factor of its optical depth, dx sqrt(pi)/4 / (dv_prev - dv) (the solve
    // needs nothing else of its length)
    a.r_dx[pos] = semi ? (Z - Zprev) * (kSqrtPi / 4.0) / (dvprev - dv) : Z - Zprev;
    a.r_ibb[pos] = 1.0 / sqrt((b2prev + b2j) * 0.5);
    a.r_semi[pos] = semi ? 1 : 0;
    nsemi += semi ? 1 : 0;
}

// MODE 0: lengths and holes; 1: records at CSR offsets; 2: lengths, holes and
// the chosen points in fixed slots (see launch_trace).
template <int MODE>
__global__ __launch_bounds__(256) void k_trace3d(TraceArgs a)
{
    constexpr bool FILL = MODE == 1;
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
                const double4 pj = a.p4[j];
                const double ddx = pj.x - xo;
                const double ddy = pj.y - yo;
                const double ddz = pj.z - zo;
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
            if (!FILL && l16 == 0 && !a.bdy[c]) atomicAdd(&a.cnt->holes, 1ull);
            break;
        }
        const double4 vj = a.v4[bj];
        const double dv = ((vj.x - vxo) * nx + (vj.y - vyo) * ny) + (vj.z - vzo) * nz;
        if (l16 == 0) emit<FILL>(a, base + n, bj, bZ, dv, Zc, dvc, b2c, nsemi, vj.w);
        if (MODE == 2 && l16 == 0 && n < a.cap) a.slot[w * a.cap + n] = bj;
        n++;
        c = bj;
        Zc = bZ;
        dvc = dv;
        if (FILL) b2c = vj.w;
        if (a.bdy[c]) break;
    }
    if (l16 == 0) {
        if (!FILL) a.counts[w] = n;
        if (MODE == 2) atomicMax(a.maxn, (unsigned long long)n);
        if (FILL && nsemi) atomicAdd(&a.cnt->semi, nsemi);
    }
}

// Records of walks kept in slots: 16 lanes per walk, lane l writes records
// l, l + 16, ...; each record needs only its point and the one before it
// (the origin for the first), whose projections are recomputed with the
// walk's own expressions, so the records equal the searching pass's bit for
// bit.
__global__ __launch_bounds__(256) void k_trace_emit(TraceArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = gid >> 4;
    const int l16 = threadIdx.x & 15;
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (w >= nwalk) return;
    const int o = (int)(w / a.R);
    const int r = (int)(w - (int64_t)o * a.R);
    const double nx = a.ray_dir[3 * r + 0];
    const double ny = a.ray_dir[3 * r + 1];
    const double nz = a.ray_dir[3 * r + 2];
    const double xo = a.x[o], yo = a.y[o], zo = a.z[o];
    const double vxo = a.vx[o], vyo = a.vy[o], vzo = a.vz[o];
    const int64_t n = a.counts[w], base = a.off[w];
    const int32_t *sl = a.slot + w * a.cap;
    auto point = [&](int j, double &Z, double &dv, double &b2) {
        const double4 pj = a.p4[j];
        const double ddx = pj.x - xo;
        const double ddy = pj.y - yo;
        const double ddz = pj.z - zo;
        Z = (ddx * nx + ddy * ny) + ddz * nz;
        const double4 vj = a.v4[j];
        dv = ((vj.x - vxo) * nx + (vj.y - vyo) * ny) + (vj.z - vzo) * nz;
        b2 = vj.w;
    };
    unsigned long long nsemi = 0;
    for (int64_t k = l16; k < n; k += 16) {
        double Zp = 0.0, dvp = 0.0, b2p = a.b2[o];
        if (k > 0) point(sl[k - 1], Zp, dvp, b2p);
        const int j = sl[k];
        double Z, dv, b2;
        point(j, Z, dv, b2);
        emit<true>(a, base + k, j, Z, dv, Zp, dvp, b2p, nsemi, b2);
    }
    for (int m = 8; m >= 1; m >>= 1) nsemi += __shfl_xor(nsemi, m, 16);
    if (l16 == 0 && nsemi) atomicAdd(&a.cnt->semi, nsemi);
}

hipError_t launch_trace_emit(const TraceArgs &a, hipStream_t s)
{
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (a.dim != 3 || a.cap < 1) return hipErrorInvalidValue;
    const int64_t blocks = (nwalk * 16 + 255) / 256;
    k_trace_emit<<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
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
        emit<FILL>(a, base + n, k, Z, dv, Zp, dvp, b2p, nsemi, FILL ? a.b2[k] : 0.0);
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

hipError_t launch_trace(const TraceArgs &a, TraceMode mode, hipStream_t s)
{
    const int64_t nwalk = (int64_t)a.N * a.R;
    if (a.dim == 1) {
        if (mode == TraceMode::slots) return hipErrorInvalidValue;
        const int64_t blocks = (nwalk + 255) / 256;
        if (mode == TraceMode::fill)
            k_trace1d<true><<<blocks, 256, 0, s>>>(a);
        else
            k_trace1d<false><<<blocks, 256, 0, s>>>(a);
    } else {
        const int64_t blocks = (nwalk * 16 + 255) / 256;
        if (mode == TraceMode::slots && a.cap < 1) return hipErrorInvalidValue;
        if (mode == TraceMode::fill)
            k_trace3d<1><<<blocks, 256, 0, s>>>(a);
        else if (mode == TraceMode::slots)
            k_trace3d<2><<<blocks, 256, 0, s>>>(a);
        else
            k_trace3d<0><<<blocks, 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

// {vx, vy, vz, b^2} per point for the walk step (one 32-byte load).
__global__ void k_pack_vel4(int N, const double *vel, const double *b2, double4 *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] = make_double4(vel[i], vel[(size_t)N + i], vel[2 * (size_t)N + i], b2[i]);
}

hipError_t launch_pack_vel4(int N, const double *vel, const double *b2, double4 *out,
                            hipStream_t s)
{
    k_pack_vel4<<<(N + 255) / 256, 256, 0, s>>>(N, vel, b2, out);
    return hipGetLastError();
}

// Convert the double-precision trace into the packed records of the solve,
// with the point's widths from the solve-precision per-point tables.
template <typename T>
__global__ void k_pack(int64_t n, const int32_t *__restrict__ idx,
                       const uint8_t *__restrict__ semi, const T *__restrict__ bpt,
                       const T *__restrict__ ibpt, const double *__restrict__ dx,
                       const double *__restrict__ dv, const double *__restrict__ ibb,
                       double inv_L, Rec<T> *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = idx[i];
    Rec<T> r;
    r.ps = p | (semi[i] ? (int32_t)0x80000000u : 0);
    if constexpr (sizeof(T) == 8) r.pad = 0;
    r.dx = (T)(dx[i] * inv_L);
    r.ibb = (T)ibb[i];
    r.b = bpt[p];
    r.dv = (T)dv[i];
    r.ib = ibpt[p];
    out[i] = r;
}

hipError_t launch_pack_trace(int64_t n, const int32_t *idx, const uint8_t *semi,
                             const void *bpt, const void *ibpt, const double *dx,
                             const double *dv, const double *ibb, double inv_L, bool fp32,
                             void *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (fp32)
        k_pack<float><<<blocks, 256, 0, s>>>(n, idx, semi, (const float *)bpt,
                                            (const float *)ibpt, dx, dv, ibb, inv_L,
                                            (Rec<float> *)out);
    else
        k_pack<double><<<blocks, 256, 0, s>>>(n, idx, semi, (const double *)bpt,
                                             (const double *)ibpt, dx, dv, ibb, inv_L,
                                             (Rec<double> *)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Image geometry: projections on the image basis, the projected extent, the
// entry point of every pixel ray and the pixel walks.  The same products and
// sums in the same order as the CPU definition.
// ---------------------------------------------------------------------------
__global__ void k_render_project(RenderGeom g)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.N) return;
    const double xj = g.x[j], yj = g.y[j], zj = g.z[j];
    g.u[j] = (xj * g.e1[0] + yj * g.e1[1]) + zj * g.e1[2];
    g.v[j] = (xj * g.e2[0] + yj * g.e2[1]) + zj * g.e2[2];
    g.Z[j] = (xj * g.d[0] + yj * g.d[1]) + zj * g.d[2];
    g.w[j] = (g.vx[j] * g.d[0] + g.vy[j] * g.d[1]) + g.vz[j] * g.d[2];
}

// order-preserving map of a double to unsigned 64 bits
__device__ __forceinline__ unsigned long long ordered(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double unordered(unsigned long long k)
{
    const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// min / max of u and v over all points (exact operations: any order gives
// the same result).  Blocks reduce their share, then combine through atomic
// min / max on order-preserving keys held in the ext slots; a last one-thread
// kernel turns the keys back into doubles.
__global__ void k_render_extent_init(unsigned long long *key)
{
    if (threadIdx.x == 0) {
        key[0] = ~0ull;  // min u
        key[1] = 0ull;   // max u
        key[2] = ~0ull;  // min v
        key[3] = 0ull;   // max v
    }
}

__global__ void k_render_extent(int N, const double *u, const double *v, unsigned long long *key)
{
    __shared__ double r[4][256];
    double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < N; j += gridDim.x * 256) {
        a = fmin(a, u[j]);
        b = fmax(b, u[j]);
        c = fmin(c, v[j]);
        d = fmax(d, v[j]);
    }
    r[0][threadIdx.x] = a;
    r[1][threadIdx.x] = b;
    r[2][threadIdx.x] = c;
    r[3][threadIdx.x] = d;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) {
            r[0][threadIdx.x] = fmin(r[0][threadIdx.x], r[0][threadIdx.x + m]);
            r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + m]);
            r[2][threadIdx.x] = fmin(r[2][threadIdx.x], r[2][threadIdx.x + m]);
            r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + m]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&key[0], ordered(r[0][0]));
        atomicMax(&key[1], ordered(r[1][0]));
        atomicMin(&key[2], ordered(r[2][0]));
        atomicMax(&key[3], ordered(r[3][0]));
    }
}

__global__ void k_render_extent_final(unsigned long long *key)
{
    if (threadIdx.x < 4) {
        const double x = unordered(key[threadIdx.x]);
        ((double *)key)[threadIdx.x] = x;
    }
}

struct PixGrid {
    double umin, vmin, du, dv, R2;
};

__device__ __forceinline__ PixGrid pix_grid(const RenderGeom &g)
{
    PixGrid p;
    p.umin = g.ext[0];
    p.vmin = g.ext[2];
    p.du = (g.ext[1] - g.ext[0]) / g.npx;
    p.dv = (g.ext[3] - g.ext[2]) / g.npy;
    double R = p.du > p.dv ? p.du : p.dv;
    if (g.h > R) R = g.h;
    p.R2 = R * R;
    return p;
}

// Entry search, scattered from the boundary points: every boundary point
// offers its Z to the pixels whose line passes within R of it (exact test
// as in the CPU definition); pass 0 keeps the smallest Z per pixel, pass 1
// the smallest point index among those with exactly that Z.
__global__ void k_render_entry(RenderGeom g, int pass)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.N || !g.bdy[j]) return;
    const PixGrid P = pix_grid(g);
    const double uj = g.u[j], vj = g.v[j], Zj = g.Z[j];
    const double R = sqrt(P.R2);
    int ix0 = (int)floor((uj - R - P.umin) / P.du - 0.5) - 1;
    int ix1 = (int)floor((uj + R - P.umin) / P.du - 0.5) + 1;
    int iy0 = (int)floor((vj - R - P.vmin) / P.dv - 0.5) - 1;
    int iy1 = (int)floor((vj + R - P.vmin) / P.dv - 0.5) + 1;
    ix0 = max(ix0, 0);
    iy0 = max(iy0, 0);
    ix1 = min(ix1, g.npx - 1);
    iy1 = min(iy1, g.npy - 1);
    const unsigned long long kz = ordered(Zj);
    for (int iy = iy0; iy <= iy1; iy++) {
        const double vc = P.vmin + (iy + 0.5) * P.dv;
        for (int ix = ix0; ix <= ix1; ix++) {
            const double uc = P.umin + (ix + 0.5) * P.du;
            const double a = uj - uc, b = vj - vc;
            const double r2 = a * a + b * b;
            if (!(r2 <= P.R2)) continue;
            const int pix = iy * g.npx + ix;
            if (pass == 0)
                atomicMin(&g.key[pix], kz);
            else if (g.key[pix] == kz)
                atomicMin(&g.entry[pix], j);
        }
    }
}

__global__ void k_render_entry_init(int npix, unsigned long long *key, int32_t *entry)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    key[i] = ~0ull;
    entry[i] = 0x7fffffff;
}

hipError_t launch_render_geometry(RenderGeom &g, hipStream_t s)
{
    const int npix = g.npx * g.npy;
    k_render_project<<<(g.N + 255) / 256, 256, 0, s>>>(g);
    unsigned long long *key = (unsigned long long *)g.ext;
    const int eblocks = std::min(1024, std::max(1, (g.N + 255) / 256));
    k_render_extent_init<<<1, 64, 0, s>>>(key);
    k_render_extent<<<eblocks, 256, 0, s>>>(g.N, g.u, g.v, key);
    k_render_extent_final<<<1, 64, 0, s>>>(key);
    k_render_entry_init<<<(npix + 255) / 256, 256, 0, s>>>(npix, g.key, g.entry);
    k_render_entry<<<(g.N + 255) / 256, 256, 0, s>>>(g, 0);
    k_render_entry<<<(g.N + 255) / 256, 256, 0, s>>>(g, 1);
    return hipGetLastError();
}

// Pixel walk: 16 lanes per pixel as in the ray trace, distances measured
// from the pixel line; the entry point is the first record.
// MODE 0: lengths only; 1: walks at CSR offsets; 2: walks in fixed slots of
// g.cap points (longer walks are cut there but their full lengths recorded,
// with the longest in *g.maxn, so the caller can redo them exactly).
template <int MODE>
__global__ __launch_bounds__(256) void k_render_walk(RenderGeom g)
{
    constexpr bool FILL = MODE != 0;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pix = gid >> 4;
    const int l16 = threadIdx.x & 15;
    const int npix = g.npx * g.npy;
    if (pix >= npix) return;
    const int e = g.entry[pix];
    int64_t n = 0;
    if (e != 0x7fffffff) {
        const PixGrid P = pix_grid(g);
        const int ix = (int)(pix % g.npx), iy = (int)(pix / g.npx);
        const double uc = P.umin + (ix + 0.5) * P.du, vc = P.vmin + (iy + 0.5) * P.dv;
        const int64_t base = MODE == 1 ? g.off[pix] : MODE == 2 ? pix * g.cap : 0;
        const int64_t lim = MODE == 2 ? g.cap : INT64_MAX;
        if (FILL && l16 == 0) g.walk[base] = e;
        n = 1;
        int c = e;
        double Zc = g.Z[e];
        for (;;) {
            const int q0 = g.nbs_off[c], q1 = g.nbs_off[c + 1];
            double bd = INFINITY, bZ = 0.0;
            int bq = 0x7fffffff, bj = -1;
            for (int qb = q0; qb < q1; qb += 16) {
                const int q = qb + l16;
                if (q < q1) {
                    const int j = g.nbs[q];
                    const double Zj = g.Z[j];
                    if (Zj > Zc) {
                        const double a = g.u[j] - uc, b = g.v[j] - vc;
                        const double r2 = a * a + b * b;
                        if (r2 < bd) {
                            bd = r2;
                            bq = q;
                            bj = j;
                            bZ = Zj;
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 8; m >= 1; m >>= 1) {
                const double od = __shfl_xor(bd, m, 16);
                const int oq = __shfl_xor(bq, m, 16);
                const int oj = __shfl_xor(bj, m, 16);
                const double oZ = __shfl_xor(bZ, m, 16);
                if (od < bd || (od == bd && oq < bq)) {
                    bd = od;
                    bq = oq;
                    bj = oj;
                    bZ = oZ;
                }
            }
            if (bj < 0) break;
            if (FILL && l16 == 0 && n < lim) g.walk[base + n] = bj;
            n++;
            c = bj;
            Zc = bZ;
        }
    }
    if (MODE != 1 && l16 == 0) g.counts[pix] = n;
    if (MODE == 2 && l16 == 0) atomicMax(g.maxn, (unsigned long long)n);
}

hipError_t launch_render_walk(const RenderGeom &g, WalkMode mode, hipStream_t s)
{
    const int64_t npix = (int64_t)g.npx * g.npy;
    const int64_t blocks = (npix * 16 + 255) / 256;
    if (mode == WalkMode::capped && g.cap < 1) return hipErrorInvalidValue;
    if (mode == WalkMode::count)
        k_render_walk<0><<<blocks, 256, 0, s>>>(g);
    else if (mode == WalkMode::fill)
        k_render_walk<1><<<blocks, 256, 0, s>>>(g);
    else
        k_render_walk<2><<<blocks, 256, 0, s>>>(g);
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
