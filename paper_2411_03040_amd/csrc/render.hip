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
// Launch shape: lanes are frequencies, one wave per 64 frequencies of one
// pixel, up to four waves per block.  The pixel, its walk and every point
// datum are the same for all lanes of a wave: they are read with scalar loads
// into scalar registers, and only the per-frequency arithmetic is per lane.
// Source functions arrive in units of the image's intensity unit, and the
// profile offsets are scaled by sqrt(log2 e) in FP32 so that each Gaussian is
// one base-2 exponential.  Opacities and semi-analytic terms are summed over
// the lines that can reach the image's band (a list the host derives from
// the model's largest speed and width; the others would add exact zeros),
// and on semi-analytic segments lines that lie in one far wing at both ends
// for the whole wave (both erfc exactly zero) are skipped by a wave vote.
// The source-function fallback where every profile underflows still ranks
// all lines.

#include "mgx_internal.h"

namespace mgx {

template <typename T>
struct RM;
template <>
struct RM<float> {
    static __device__ __forceinline__ float ex(float x) { return __expf(x); }
    // Gaussian profiles take offsets pre-scaled by sqrt(log2 e), so that
    // exp(-x^2) is one base-2 exponential of the scaled square
    static constexpr double gauss_k = 1.2011224087864498;  // sqrt(log2 e)
    static __device__ __forceinline__ float gauss(float xs2) { return __builtin_amdgcn_exp2f(-xs2); }
    // e^x - 1 for x <= -0.1 only (the linear-source weights use a series
    // above): exp2 - 1, relative error < 1e-6 there
    static __device__ __forceinline__ float em1(float x)
    {
        return __builtin_amdgcn_exp2f(x * 1.44269504f) - 1.0f;
    }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * rcp(b); }
    // 1 / sqrt(v) of the averaged squared width (the branch rule itself is
    // decided in FP64)
    static __device__ __forceinline__ float rsqrt_w(double v) { return __builtin_amdgcn_rsqf((float)v); }
    // erfc for x >= 0, branch-free (Numerical Recipes' Chebyshev form
    // erfc(x) = t exp(-x^2 + P(t)), t = 1/(1 + x/2), fractional error
    // < 1.2e-7), so the bins of a wave never diverge
    static __device__ __forceinline__ float erfc_(float x)
    {
        const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
        float p = 0.17087277f;
        p = fmaf(p, t, -0.82215223f);
        p = fmaf(p, t, 1.48851587f);
        p = fmaf(p, t, -1.13520398f);
        p = fmaf(p, t, 0.27886807f);
        p = fmaf(p, t, -0.18628806f);
        p = fmaf(p, t, 0.09678418f);
        p = fmaf(p, t, 0.37409196f);
        p = fmaf(p, t, 1.00002368f);
        p = fmaf(p, t, -1.26551223f);
        return t * __expf(fmaf(-x, x, p));
    }
    static constexpr float series_below = 0.1f;
    static constexpr float tiny = 1e-30f;  // smallest opacity sum used as a divisor
    // erfc_ returns exactly 0 beyond this (its exponential is below the
    // smallest denormal)
    static constexpr float erfc_zero = 10.5f;
    // exp2(-y) is exactly zero (below the smallest denormal) for y > 150;
    // squares of offsets carry a relative rounding of at most 6e-8
    static constexpr float weight_zero = 151.0f;
    static constexpr float sq_rel = 2e-7f;
};
template <>
struct RM<double> {
    static __device__ __forceinline__ double ex(double x) { return exp(x); }
    static constexpr double gauss_k = 1.0;
    static __device__ __forceinline__ double gauss(double x2) { return exp(-x2); }
    static __device__ __forceinline__ double em1(double x) { return expm1(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double rsqrt_w(double v) { return 1.0 / sqrt(v); }
    static __device__ __forceinline__ double erfc_(double x) { return erfc(x); }
    static constexpr double series_below = 1e-4;
    static constexpr double tiny = 1e-290;
    // the library erfc is exactly 0 beyond this (erfc(27.3) < 5e-324)
    static constexpr double erfc_zero = 27.5;
    // exp(-y) is exactly zero for y > 745.2
    static constexpr double weight_zero = 746.0;
    static constexpr double sq_rel = 1e-15;
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
        // (coefficients as reciprocal constants: no division per point)
        w0 = t * (T)0.5 - t2 * (T)(1.0 / 3) + t3 * (T)0.125 - t4 * (T)(1.0 / 30) +
             t5 * (T)(1.0 / 144);
        w1 = t * (T)0.5 - t2 * (T)(1.0 / 6) + t3 * (T)(1.0 / 24) - t4 * (T)(1.0 / 120) +
             t5 * (T)(1.0 / 720);
        return;
    }
    const T em = RM<T>::em1(-t);
    const T a = RM<T>::div(-em, t);
    att = (T)1 + em;
    w0 = a - att;
    w1 = (T)1 - a;
}

// Per lane (frequency nu) and line l, the two frequency factors of the
// offset x = (cd - rr w) / b, rr = nu / nu_l and cd = c (nu - nu_l) / nu_l,
// computed once per pixel in double and kept in LDS (each lane reads only
// its own entries).  Lines beyond what LDS holds are computed per point.
template <typename T>
struct LineLane {
    T cd, rr;
};

template <typename T, bool TAB>
__global__ __launch_bounds__(256) void k_render_integrate(RenderArgs<T> a, int nslices)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int t = threadIdx.x;
    const int nl = a.nlines;
    const gptr<double> nu_line = glob(a.nu_line);
    const gptr<int32_t> act = glob(a.act);
    const int nact = a.nact;
    // 64 frequencies of one pixel per wave: the pixel, its walk and every
    // point datum are wave-uniform (scalar registers and loads)
    const int slice =
        __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + t) >> 6));
    const int pix = slice / nslices;
    const int f = (slice - pix * nslices) * 64 + (t & 63);
    const int npix = a.npx * a.npy;
    if (pix >= npix || f >= a.nfreq) return;
    const double nu = (a.nfreq == 1) ? a.f_min
                                     : a.f_min + (a.f_max - a.f_min) * f / (a.nfreq - 1);
    const double f_mid = 0.5 * (a.f_min + a.f_max);
    LineLane<T> *tab = (LineLane<T> *)smem + (size_t)t * nl;
    auto line_lane = [&](int l) -> LineLane<T> {
        LineLane<T> e;
        if (TAB) {
            e = tab[l];
        } else {
            e.cd = (T)(kC * (nu - nu_line[l]) / nu_line[l]);
            e.rr = (T)(nu / nu_line[l]);
        }
        return e;
    };
    if (TAB)
        for (int l = 0; l < nl; l++) {
            LineLane<T> e;
            e.cd = (T)(kC * (nu - nu_line[l]) / nu_line[l]);
            e.rr = (T)(nu / nu_line[l]);
            tab[l] = e;
        }
    const gptr<int64_t> off = glob(a.off), cnt = glob(a.cnt);
    const gptr<int32_t> walk = glob(a.walk);
    const gptr<double> Wv = glob(a.w), Zv = glob(a.Z), bv = glob(a.b), ibv = glob(a.ib);
    const gptr<double> b2v = glob(a.b2);
    const gptr<T> chi = glob(a.chi), Sv = glob(a.S);
    // the pixel's walk: at CSR offsets, or in its slot of cap points
    const int64_t o0 = a.off ? off[pix] : (int64_t)pix * a.cap;
    const int64_t n = a.off ? off[pix + 1] - o0 : cnt[pix];
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
    double w0d = 0.0, Z0 = 0.0, b20 = 0.0;
    // the next walk index is fetched one point ahead
    int p_next = walk[o0];
    for (int64_t k = 0; k < n; k++) {
        const int p = p_next;
        if (k + 1 < n) p_next = walk[o0 + k + 1];
        const double wd = Wv[p];
        const T w = (T)wd;
        const T ibg = (T)(ibv[p] * RM<T>::gauss_k);
        const gptr<T> chi_p = chi + (int64_t)p * nl;
        const gptr<T> S_p = Sv + (int64_t)p * nl;
        // opacity (sum over lines) and the profile-weighted mean of the line
        // source functions, in one pass; where every profile underflows the
        // source function is the same mean with weights relative to the
        // nearest line, exp(-(x_l^2 - x_min^2)) (the limit of eta / chi)
        // (only the lines that can reach the band: the others add exact
        // zeros, in the same order)
        T chi1 = (T)0, sws = (T)0;
        for (int j = 0; j < nact; j++) {
            const int l = act[j];
            const LineLane<T> e = line_lane(l);
            const T x = (e.cd - e.rr * w) * ibg;
            const T c = chi_p[l] * RM<T>::gauss(x * x);
            chi1 += c;
            sws += c * S_p[l];
        }
        T S1;
        if (chi1 > RM<T>::tiny) {
            S1 = RM<T>::div(sws, chi1);
        } else {
            // nearest line (smallest squared offset) and the next nearest
            T x2min = (T)INFINITY, x2sec = (T)INFINITY;
            int lmin = 0;
            for (int l = 0; l < nl; l++) {
                const LineLane<T> e = line_lane(l);
                const T x = (e.cd - e.rr * w) * ibg;
                const T y = x * x;
                if (y < x2min) {
                    x2sec = x2min;
                    x2min = y;
                    lmin = l;
                } else {
                    x2sec = fmin(x2sec, y);
                }
            }
            // Where every other line's relative weight exp(-(y - y_min))
            // underflows to zero, the mean is the nearest line's own,
            // (c S) / c, as the full sum gives it (with a margin for the
            // rounding of the squares); otherwise the full sum.
            if (x2sec - x2min > RM<T>::weight_zero + RM<T>::sq_rel * x2sec) {
                const T c = chi_p[lmin];
                S1 = c > (T)0 ? (c * S_p[lmin]) / c : (T)0;
            } else {
                T sw = (T)0;
                sws = (T)0;
                for (int l = 0; l < nl; l++) {
                    const LineLane<T> e = line_lane(l);
                    const T x = (e.cd - e.rr * w) * ibg;
                    // (clamped: the square of the nearest line's offset may
                    // be fused into this subtraction unrounded, leaving a
                    // residue of either sign, large where the offsets are)
                    const T wt = chi_p[l] * RM<T>::gauss(fmax(x * x - x2min, (T)0));
                    sw += wt;
                    sws += wt * S_p[l];
                }
                // (IEEE division: the weights may be denormal, where the
                // hardware reciprocal flushes to infinity)
                S1 = sw > (T)0 ? sws / sw : (T)0;
            }
        }
        const double Zd = Zv[p], b2d = b2v[p];
        if (k == 0) {
            I = (T)planck_n(nu * (1.0 - wd / kC));
        } else {
            const double dd = wd - w0d;
            const bool semi = dd * dd >= thr2 * ((b20 + b2d) * 0.5);
            const T dx = (T)((Zd - Z0) * a.inv_L);
            T dt = (T)0;
            if (semi) {
                const T ibb = RM<T>::rsqrt_w((b20 + b2d) * 0.5);
                const T b0 = (T)bv[p0], b1 = (T)bv[p];
                const T w0 = (T)w0d;
                const gptr<T> chi_q = chi + (int64_t)p0 * nl;
                const T ddt = (T)dd;
                for (int j = 0; j < nact; j++) {
                    const int l = act[j];
                    const LineLane<T> e = line_lane(l);
                    const T xa = (e.cd - e.rr * w0) * ibb;
                    const T xb = (e.cd - e.rr * w) * ibb;
                    // both ends in the same far wing for every lane of the
                    // wave: both erfc are exactly zero, so is the term
                    const bool far = (xa > RM<T>::erfc_zero && xb > RM<T>::erfc_zero) ||
                                     (xa < -RM<T>::erfc_zero && xb < -RM<T>::erfc_zero);
                    if (__all(far)) continue;
                    const T dxb = -e.rr * ddt * ibb;
                    const T cb = chi_q[l] * b0 + chi_p[l] * b1;
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
        Z0 = Zd;
        b20 = b2d;
    }
    *out = (float)((double)I * a.I_img);
}

template <typename T>
hipError_t launch_render_integrate(const RenderArgs<T> &a, hipStream_t s)
{
    const int nslices = (a.nfreq + 63) / 64;
    const int64_t waves = (int64_t)a.npx * a.npy * nslices;
    const size_t per_thread = sizeof(LineLane<T>) * (size_t)a.nlines;
    // the largest block (256, 128 or 64 threads) whose line tables fit 40 KB
    int threads = 256;
    while (threads > 64 && per_thread * threads > (40u << 10)) threads /= 2;
    const bool tab = per_thread * threads <= (64u << 10);
    const size_t lds = tab ? per_thread * threads : 0;
    const int64_t blocks = (waves * 64 + threads - 1) / threads;
    if (tab)
        k_render_integrate<T, true><<<(unsigned)blocks, threads, lds, s>>>(a, nslices);
    else
        k_render_integrate<T, false><<<(unsigned)blocks, threads, lds, s>>>(a, nslices);
    return hipGetLastError();
}

template hipError_t launch_render_integrate<float>(const RenderArgs<float> &, hipStream_t);
template hipError_t launch_render_integrate<double>(const RenderArgs<double> &, hipStream_t);

}  // namespace mgx
