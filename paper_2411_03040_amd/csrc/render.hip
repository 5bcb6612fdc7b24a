// Synthetic images: intensity along every pixel walk, for every
// observer-frame frequency (the API's image call).
//
// Along the walk of a pixel (entry point first), with w = d.v the velocity
// towards the observer and nu' = nu (1 - w / c) the comoving frequency, every
// line adds its opacity chi^ij phi(nu') and emissivity S chi^ij phi(nu'); the
// offset from line centre is formed in velocity units,
//   x = (c (nu - nu_l) / nu_l - (nu / nu_l) w) / b.
// Segment optical depths use the trapezoidal rule on the summed opacity or,
// where the projected velocity changes by at least the branch threshold in
// averaged widths, the semi-analytic form line by line.  The intensity starts
// at the CMB (comoving frequency of the entry point) and is propagated with a
// source function linear in optical depth:
//   I1 = I0 e^-t + S0 ((1 - e^-t)/t - e^-t) + S1 (1 - (1 - e^-t)/t),
// with a short series for small t.
//
// Launch shape: lanes are frequencies; one pixel per group of
// ceil(nfreq / 64) waves, several pixels per 256-thread block when nfreq
// <= 128.  The walk's point data are read by all lanes of a pixel at once
// (one broadcast per wave).

#include "mgx_internal.h"

namespace mgx {

template <typename T>
struct RM;
template <>
struct RM<float> {
    static __device__ __forceinline__ float ex(float x) { return __expf(x); }
    static __device__ __forceinline__ float em1(float x) { return expm1f(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float erfc_(float x) { return erfcf(x); }
    static constexpr float series_below = 0.1f;
};
template <>
struct RM<double> {
    static __device__ __forceinline__ double ex(double x) { return exp(x); }
    static __device__ __forceinline__ double em1(double x) { return expm1(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double erfc_(double x) { return erfc(x); }
    static constexpr double series_below = 1e-4;
};

template <typename T>
__device__ __forceinline__ T erf_diff_r(T a, T b)
{
    const T ea = RM<T>::erfc_(fabs(a));
    const T eb = RM<T>::erfc_(fabs(b));
    if (a >= (T)0 && b >= (T)0) return ea - eb;
    if (a <= (T)0 && b <= (T)0) return eb - ea;
    const T t = (T)2 - ea - eb;
    return (b > a) ? t : -t;
}

template <typename T>
__device__ __forceinline__ void lin_weights(T t, T &att, T &w0, T &w1)
{
    if (t < RM<T>::series_below) {
        att = RM<T>::ex(-t);
        const T t2 = t * t, t3 = t2 * t, t4 = t3 * t, t5 = t4 * t;
        w0 = t / 2 - t2 / 3 + t3 / 8 - t4 / 30 + t5 / 144;
        w1 = t / 2 - t2 / 6 + t3 / 24 - t4 / 120 + t5 / 720;
        return;
    }
    const T em = RM<T>::em1(-t);
    const T a = -em / t;
    att = (T)1 + em;
    w0 = a - att;
    w1 = (T)1 - a;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_render_integrate(RenderArgs<T> a, int lanes_per_pixel,
                                                         int pix_per_block)
{
    const int t = threadIdx.x;
    const int pix = blockIdx.x * pix_per_block + t / lanes_per_pixel;
    const int f = t % lanes_per_pixel;
    const int npix = a.npx * a.npy;
    if (pix >= npix || f >= a.nfreq) return;
    const int nl = a.nlines;
    const double nu = (a.nfreq == 1) ? a.f_min
                                     : a.f_min + (a.f_max - a.f_min) * f / (a.nfreq - 1);
    const double f_mid = 0.5 * (a.f_min + a.f_max);
    const int64_t o0 = a.off[pix], n = a.off[pix + 1] - o0;
    float *out = a.img + (int64_t)pix * a.nfreq + f;
    auto planck_n = [&](double nup) -> double {  // B_nu(Tcmb) / I_img
        const double r = nup / f_mid;
        return r * r * r / expm1(kH * nup / (kKB * a.Tcmb));
    };
    if (n == 0) {
        *out = (float)(planck_n(nu) * a.I_img);
        return;
    }
    const T spi4 = (T)(kSqrtPi / 4.0);
    const double thr2 = a.thr * a.thr;
    T I = (T)0, chi0 = (T)0, S0 = (T)0;
    int p0 = -1;
    double w0d = 0.0;
    for (int64_t k = 0; k < n; k++) {
        const int p = a.walk[o0 + k];
        const double wd = a.w[p];
        const T ib = (T)a.ib[p];
        // opacity (sum over lines) and source function: the profile-weighted
        // mean of the line source functions with weights relative to the
        // nearest line, exp(-(x_l^2 - x_min^2)), so S keeps its value where
        // every profile underflows
        T chi1 = (T)0, x2min = (T)INFINITY;
        for (int l = 0; l < nl; l++) {
            const double nul = a.nu_line[l];
            const T x = (T)(kC * (nu - nul) / nul - (nu / nul) * wd) * ib;
            const T x2 = x * x;
            x2min = x2 < x2min ? x2 : x2min;
            chi1 += a.chi[(int64_t)p * nl + l] * RM<T>::ex(-x2);
        }
        T sw = (T)0, sws = (T)0;
        for (int l = 0; l < nl; l++) {
            const double nul = a.nu_line[l];
            const T x = (T)(kC * (nu - nul) / nul - (nu / nul) * wd) * ib;
            // chi' already holds the profile's 1 / dnu = c / (nu_l b)
            const T wt = a.chi[(int64_t)p * nl + l] * RM<T>::ex(-(x * x - x2min));
            sw += wt;
            sws += wt * a.S[(int64_t)p * nl + l] * (T)(a.Iref[l] / a.I_img);
        }
        const T S1 = sw > (T)0 ? sws / sw : (T)0;
        if (k == 0) {
            I = (T)planck_n(nu * (1.0 - wd / kC));
        } else {
            const double dd = wd - w0d;
            const bool semi = dd * dd >= thr2 * ((a.b2[p0] + a.b2[p]) * 0.5);
            const T dx = (T)((a.Z[p] - a.Z[p0]) * a.inv_L);
            T dt = (T)0;
            if (semi) {
                const T ibb = (T)(1.0 / sqrt((a.b2[p0] + a.b2[p]) * 0.5));
                const T b0 = (T)a.b[p0], b1 = (T)a.b[p];
                for (int l = 0; l < nl; l++) {
                    const double nul = a.nu_line[l];
                    const double cd = kC * (nu - nul) / nul, rr = nu / nul;
                    const T xa = (T)(cd - rr * w0d) * ibb;
                    const T xb = (T)(cd - rr * wd) * ibb;
                    const T dxb = (T)(-rr * dd) * ibb;
                    const T cb = a.chi[(int64_t)p0 * nl + l] * b0 + a.chi[(int64_t)p * nl + l] * b1;
                    dt += dx * cb * spi4 * ibb * erf_diff_r<T>(xa, xb) * RM<T>::rcp(dxb);
                }
            } else {
                dt = dx * (chi0 + chi1) * (T)0.5;
            }
            T att, wa, wb;
            lin_weights<T>(dt, att, wa, wb);
            I = I * att + S0 * wa + S1 * wb;
        }
        chi0 = chi1;
        S0 = S1;
        p0 = p;
        w0d = wd;
    }
    *out = (float)((double)I * a.I_img);
}

template <typename T>
hipError_t launch_render_integrate(const RenderArgs<T> &a, hipStream_t s)
{
    const int lanes = ((a.nfreq + 63) / 64) * 64;
    const int ppb = lanes >= 256 ? 1 : 256 / lanes;
    const int threads = lanes >= 256 ? lanes : 256;
    const int npix = a.npx * a.npy;
    const int blocks = (npix + ppb - 1) / ppb;
    if (threads > 256) {
        // one pixel with more than 256 frequencies: a larger block
        k_render_integrate<T><<<npix, lanes, 0, s>>>(a, lanes, 1);
    } else {
        k_render_integrate<T><<<blocks, threads, 0, s>>>(a, lanes, ppb);
    }
    return hipGetLastError();
}

template hipError_t launch_render_integrate<float>(const RenderArgs<float> &, hipStream_t);
template hipError_t launch_render_integrate<double>(const RenderArgs<double> &, hipStream_t);

}  // namespace mgx
