// Line coefficients and the formal solution on gfx950.
//
// Formal solution (per origin o, ray pair, line l, bin f):
//  * Comoving offset from line centre at a point of the pair grid, in line
//    widths, formed in velocity units so float keeps its digits:
//      x = (x_f b_o + dv + x_f b_o dv / c) / b_point
//    (Doppler shift of the Gaussian profile; line width equation).
//  * Opacity chi = chi^ij phi(nu) with the Gaussian profile; the per-point
//    factor chi^ij / (dnu sqrt(pi)) comes from the line-coefficient table.
//  * Segment optical depth: trapezoidal rule, or the semi-analytic form
//    dtau = dx (chi^ij_0 + chi^ij_1)/2 (erf(x1) - erf(x0)) / (2 dnu_bar
//    (x1 - x0)) where the segment's Doppler shift reaches the threshold
//    (semi-analytic optical depth equation); plus tau_floor, which keeps
//    every segment depth positive.
//  * Second-order Feautrier system on the pair grid, eliminated from both
//    far ends towards the origin with O(1) state per lane.  With the
//    scaled unknowns f_j = F_j / dtau_{j+1/2} and e_j / dtau_{j+1/2} of the
//    Rybicki-Hummer (1991) forward elimination, one step across a point P
//    followed by a segment of depth dt (dm = previous segment, 0 at a far
//    end) reads
//      D  = (dm + dt) / 2,   q = D + g,   inv = 1 / (1 + q dt),
//      g <- q inv,           eps <- (D S_P + eps) inv,
//    started with g = 1, eps = I_boundary (the far-end boundary row folds
//    into the same recursion).  At the origin, with D_o = (dm_- + dm_+)/2,
//      u = (D_o S_o + eps_- + eps_+) / (D_o + g_- + g_+),
//      Lambda*_oo = D_o / (D_o + g_- + g_+);
//    an empty half keeps (dm, g, eps) = (0, 1, I_boundary at the origin), so
//    boundary origins and isolated points need no special case.  The kernel
//    carries h = dt/2 and G = 2g instead of dt and g: D = h_m + h,
//    G <- (2D + G) inv with inv = 1 / (1 + (2D + G) h), one operation fewer
//    per step, and, the factors being powers of two, the same roundings.
//    Two consecutive steps share one reciprocal: the first leaves (G, eps)
//    as a fraction over its denominator 1 + (2D + G) h, the second scales
//    its own terms by that denominator and divides once (the reciprocal is
//    the dearest instruction of the step).
//  * J-bar = sum_pairs 2 w_r sum_f W_f u, Lambda-bar* likewise.
//
// Launch shape: one workgroup per (origin, chunk of lines); one lane per
// (line, bin) of the chunk, so a line's bins sit in adjacent lanes and the
// per-point line data of one record is a broadcast for most of a wave.  The
// workgroup walks the ray pairs of its origin; each pair's records are staged
// in LDS in chunks of CH records per half, farthest first -- per record and
// line the gathered opacity and source factors, per record and bin the
// profile and erf-difference factors, computed once for all lines -- and
// both halves are swept in the same loop (two independent dependency chains
// per lane).
// Reductions over bins happen once per origin in LDS in a fixed order (no
// atomics: bit-reproducible).

#include <cfloat>

#include "mgx_internal.h"

// Multiply-adds are fused only where one source expression writes them, so
// every kernel that inlines the solve (single model, batched) rounds the
// same way and their results agree bit for bit.
#pragma clang fp contract(on)

namespace mgx {

template <typename T>
struct FM;

template <>
struct FM<float> {
    // the profile exp(-x^2) of a (point, bin) as exp2(-xs^2), xs = x sqrt(log2
    // e) (the factor is folded into 1/b)
    static __device__ __forceinline__ float phi_of(float xs)
    {
        return __builtin_amdgcn_exp2f(-(xs * xs));
    }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rcp_ge1(float x) { return __builtin_amdgcn_rcpf(x); }
    // erfc for x >= 0, branch-free, in the product form of Numerical Recipes
    // (Press et al., 2nd ed., Sec. 6.2),
    //   erfc(x) = t exp(-x^2 + P(t)),  t = 1 / (1 + p x),
    // with our own fit (fit_erfc.py in the package reproduces it): p = 0.62
    // and a degree-6 P, fitted for least maximum relative error of erfc on x
    // in [0, 9.6] (2.0e-6 in exact arithmetic; in FP32 the rounding of the
    // exponent argument dominates at large x, as for the published degree-9
    // form; degree 7 reaches 2.8e-7 for one more multiply-add per erfc, which
    // measured 1.5-2.4 % slower for a J-bar error of 2e-7 instead of 8e-7).
    // One reciprocal, one exp2 and six multiply-adds, the same for every
    // lane (the library erfcf branches by argument range, which diverges
    // across the bins of a wave).  Evaluated
    // in base 2: the argument comes scaled by sqrt(log2 e) (xs = x sqrt(log2 e),
    // see erf_scale), P is fitted to log2(erfc(x) / t) + xs^2 directly and
    // p is divided by sqrt(log2 e).
    static constexpr float erf_scale = 1.2011224f;  // sqrt(log2 e)
    static __device__ __forceinline__ float erfc_scaled(float xs)
    {
        const float t = __builtin_amdgcn_rcpf(fmaf(xs, 0.51618386f, 1.0f));
        float p = -0.29999480f;
        p = fmaf(p, t, 1.21250997f);
        p = fmaf(p, t, -1.66093528f);
        p = fmaf(p, t, 0.49260237f);
        p = fmaf(p, t, 0.31400948f);
        p = fmaf(p, t, 1.45791962f);
        p = fmaf(p, t, -1.51611420f);
        return t * __builtin_amdgcn_exp2f(fmaf(-xs, xs, p));
    }
    // e^x - 1 for the CMB boundary intensity: exp2 away from zero, a
    // four-term series below |x| = 0.1 (relative error < 1e-6 on both sides)
    static __device__ __forceinline__ float expm1_(float x)
    {
        const float e = __builtin_amdgcn_exp2f(x * 1.44269504f) - 1.0f;
        const float s = x * fmaf(x, fmaf(x, fmaf(x, 1.0f / 24.0f, 1.0f / 6.0f), 0.5f), 1.0f);
        return fabsf(x) < 0.1f ? s : e;
    }
};

template <>
struct FM<double> {
    static __device__ __forceinline__ double phi_of(double x) { return exp(-(x * x)); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    // 1 / x for x >= 1 (finite or +inf): the hardware estimate refined by two
    // Newton steps (within an ulp; the argument range rules out the
    // operands IEEE division guards against).  An infinite x is clamped to
    // the largest double first, whose reciprocal is subnormal: 0 to within
    // 2^-1022, where the Newton steps on x itself would give NaN.
    static __device__ __forceinline__ double rcp_ge1(double x)
    {
        x = fmin(x, DBL_MAX);
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        r = fma(r, fma(-x, r, 1.0), r);
        return r;
    }
    static constexpr double erf_scale = 1.0;
    // erfc for x >= 0, branch-free: the product form erfc(x) = t exp(P(t) -
    // x^2), t = 1 / (1 + x / 2), with a degree-20 P fitted at 50 digits for
    // x in [0, 26.5] (fit_erfc.py --fp64 reproduces it); the double
    // evaluation is within 8e-14 of erfc there, the rounding of x^2 dominating
    // near the top of the range.  (The library erfc branches by argument
    // range, which diverges across the bins of a wave.)
    static __device__ __forceinline__ double erfc_scaled(double x)
    {
        const double t = rcp_ge1(fma(x, 0.5, 1.0));
        double p = -0.016239501604125413;
        p = fma(p, t, 0.39759805519212382);
        p = fma(p, t, -3.2793542009084606);
        p = fma(p, t, 14.598535839604947);
        p = fma(p, t, -41.377983391993126);
        p = fma(p, t, 80.68994480295521);
        p = fma(p, t, -112.65882633664431);
        p = fma(p, t, 115.01700588295229);
        p = fma(p, t, -87.126719461560256);
        p = fma(p, t, 50.058971529304863);
        p = fma(p, t, -22.629240549741915);
        p = fma(p, t, 8.0951282183331497);
        p = fma(p, t, -2.0788523994433934);
        p = fma(p, t, 0.51027472396717621);
        p = fma(p, t, -0.17288954588737776);
        p = fma(p, t, -0.13329972931773915);
        p = fma(p, t, -0.086941180427807283);
        p = fma(p, t, 0.083402493085032281);
        p = fma(p, t, 0.37499678709769213);
        p = fma(p, t, 1.0000000896502224);
        p = fma(p, t, -1.2655121246141809);
        return t * exp(fma(-x, x, p));
    }

    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
};

// erf(b) - erf(a) from ea = erfc(|a|) and eb = erfc(|b|) (arguments scaled
// by erf_scale): with sa, sb = +-1 the signs of a and b (of their sign bits,
// so -0 counts as negative), erf(x) = s (1 - erfc|x|) gives
//   erf(b) - erf(a) = (sb - sa) + sa ea - sb eb,
// i.e. +-(ea - eb) for equal signs -- no cancellation in the wings -- and
// +-((2 - ea) - eb) for opposite signs (the semi-analytic branch guarantees
// |b - a| is at least about the branch threshold, so that never cancels
// either).  Two multiply-adds, the same for every lane: no divergent branch
// (the sign-dependent forms measured 3 % slower on the clumpy cloud).
template <typename T>
__device__ __forceinline__ T erf_diff(T a, T b, T ea, T eb)
{
    const T sa = copysign((T)1, a), sb = copysign((T)1, b);
    return fma(-sb, eb, fma(sa, ea, sb - sa));
}

// LDS records.  The offset of a (point, bin) from the line centre is formed
// in velocity units, x = (x_f b_o + dv + x_f b_o dv / c) / b, so it does not
// depend on the line: the profile at a point and the semi-analytic optical
// depth's erf difference are the same for every line of the chunk.  The
// staging pass therefore computes them once per (record, bin) and every
// line's lanes read them; the per-point line data is staged per (record,
// line).  Both forms of a segment's half depth are a sum over its two ends of
// the point's line factor chi' times a bin factor,
//   trapezoidal:    h = chi'_P (q phi_P) + chi'_Q (q phi_Q),  q = dx / 4,
//   semi-analytic:  h = chi'_P (b_P W) + chi'_Q (b_Q W),
// with W the segment's erf difference times its factor (below): the point's
// Doppler width b, which the semi-analytic form weights each end's opacity
// with, rides in the bin factor, so a point has one line factor whatever the
// forms of its two segments, and the sweep evaluates one multiply-add, the
// same for every segment.  Segment k runs from record k to record k - 1 (the
// next one towards the origin, or the origin itself):
//  * MetaA (per record): dv, read by the sweep only at a ray's far end (the
//    boundary intensity's comoving frequency).
//  * StageRec (per record, staging only): dv here and at the next record
//    towards the origin (0 at the origin), 1/b here and there (scaled for
//    the profile), 1/b-bar of the segment (times erf_scale), the segment's
//    lane-independent factor (trapezoidal: a quarter of its length;
//    semi-analytic: half of dx sqrt(pi)/4 / (dv_Q - dv_P), which the trace
//    computed in FP64 and stored in place of the length), b here and at the
//    next record towards the origin, the point indices here and at the
//    record beyond (-1 past the far end), and the segment's form.
//  * LineRec (per record and line), two values: the point's line factor
//    chi' and S' at the record beyond (the elimination row of this visit
//    crosses that point).  S' at record 0 of each half, needed only for the
//    row across the last point before the origin, is staged on its own
//    (2 nlc values).
//  * BinRec (per record and bin): the bin factors of the segment that starts
//    here, at its far end (vf, this point) and its near end (vn, the next
//    point): q phi_P and q phi_Q for a trapezoidal segment, b_P W and b_Q W
//    with W = (erf x_Q - erf x_P) times the factor above times 1/k1 for a
//    semi-analytic one (x_Q - x_P = (dv_Q - dv_P) k1 / b-bar: b-bar cancels
//    outside the erf arguments).  In FP32 the profile underflows past ~10
//    widths, where chi' times it is far below the optical-depth floor.
// A sweep element reads 16 bytes of LDS in FP32 (a LineRec and a BinRec),
// against 20 with a line record that carries a point's factor for each of
// its two segments' forms; at 20 the LDS return bandwidth, not the VALU,
// set the sweep's pace (clumpy cloud: 99.7 -> 84.2 ms per FP32 launch with
// the smaller record).
//  (Quarters and halves: the sweep works with half optical depths.)
// Row order, as measured.  FP32 keeps a record's LineRecs (BinRecs)
// adjacent: the sweep steps its pointers by nlc (nb) per record.  FP64 keeps
// a line's (bin's) records adjacent, in rows of an odd number of records so
// the lines and bins one wave reads fall in different banks: the two records
// of an unrolled step share one address with immediate offsets (FP64: 436
// against 473 ms per clumpy-cloud solve; the same order costs FP32 6 %).
// Line gathers a staging thread issues ahead of the bin arithmetic: one in
// FP32 (more raise the staging's register peak above the sweep's), none in
// FP64, whose staging registers would spill.
template <typename T>
constexpr int kLineAhead = sizeof(T) == 4 ? 1 : 0;
template <typename T>
constexpr bool kRowsByRecord = sizeof(T) == 8;
template <typename T>
struct MetaA {
    T dv;
};
template <typename T>
struct StageRec {
    T dv, dvm, ib, ibm, sibb, rw, b, bm;
    int32_t p, pn, semi;  // semi: this record's segment is semi-analytic
};
template <typename T>
struct alignas(2 * sizeof(T)) LineRec {
    T u, Sn;
};
template <typename T>
struct alignas(2 * sizeof(T)) BinRec {
    T vf, vn;
};
struct LDSLayout {
    int ch;                  // records per half
    int ls, le, bs, be;      // LineRec (BinRec) index = line (bin) * ls (bs)
                             // + staged record * le (be)
    size_t st, a, s0, line, bin, total;
};

// Every section starts 16-byte aligned.
template <typename T>
__host__ __device__ inline LDSLayout lds_layout(int ch, int nlc, int nb, int nthreads)
{
    LDSLayout L;
    L.ch = ch;
    const int rows = kRowsByRecord<T> ? 2 * ch + 1 : 2 * ch;
    L.ls = kRowsByRecord<T> ? rows : 1;
    L.le = kRowsByRecord<T> ? 1 : nlc;
    L.bs = kRowsByRecord<T> ? rows : 1;
    L.be = kRowsByRecord<T> ? 1 : nb;
    size_t o = 0;
    L.st = o;
    o += sizeof(StageRec<T>) * 2 * ch;
    o = (o + 15) & ~(size_t)15;
    L.a = o;
    o += sizeof(MetaA<T>) * 2 * ch;
    o = (o + 15) & ~(size_t)15;
    L.s0 = o;
    o += sizeof(T) * 2 * (size_t)nlc;
    o = (o + 15) & ~(size_t)15;
    L.line = o;
    o += sizeof(LineRec<T>) * (size_t)rows * nlc;
    L.bin = o;
    o += sizeof(BinRec<T>) * (size_t)rows * nb;
    const size_t red = sizeof(double) * 2 * nthreads;
    L.total = o > red ? o : red;
    return L;
}

// Trace records are read once per launch: stream them past the L2 (non-
// temporal) so they do not evict the per-point line table the gathers reuse.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i_a8 __attribute__((ext_vector_type(4), aligned(8)));

__device__ __forceinline__ Rec<float> load_stream(gptr<Rec<float>> p)
{
    const v4i v = __builtin_nontemporal_load((gptr<v4i_a8>)p);
    const v2i w = __builtin_nontemporal_load((gptr<v2i>)p + 2);
    Rec<float> r;
    r.ps = v.x;
    r.dx = __int_as_float(v.y);
    r.ibb = __int_as_float(v.z);
    r.b = __int_as_float(v.w);
    r.dv = __int_as_float(w.x);
    r.ib = __int_as_float(w.y);
    return r;
}

__device__ __forceinline__ Rec<double> load_stream(gptr<Rec<double>> p)
{
    const v4i v0 = __builtin_nontemporal_load((gptr<v4i>)p);
    const v4i v1 = __builtin_nontemporal_load((gptr<v4i>)p + 1);
    const v4i v2 = __builtin_nontemporal_load((gptr<v4i>)p + 2);
    Rec<double> r;
    r.ps = v0.x;
    r.pad = 0;
    r.dx = __hiloint2double(v0.w, v0.z);
    r.ibb = __hiloint2double(v1.y, v1.x);
    r.b = __hiloint2double(v1.w, v1.z);
    r.dv = __hiloint2double(v2.y, v2.x);
    r.ib = __hiloint2double(v2.w, v2.z);
    return r;
}

// LDS pointers as 32-bit addresses.  opaque() hides how an address was
// formed: the optimiser would otherwise split a stepped sweep pointer into
// its lane-dependent and uniform parts and add the two at every access
// (ds instructions take no scalar offset), one vector add per read instead
// of one per step.
template <typename X>
using lptr = const __attribute__((address_space(3))) X *;
template <typename X>
__device__ __forceinline__ lptr<X> opaque(const X *p)
{
    uint32_t v = (uint32_t)(uintptr_t)(lptr<X>)p;
    asm volatile("" : "+v"(v));
    return (lptr<X>)(uintptr_t)v;
}

template <typename T>
struct HalfState {
    T G, eps, hm;  // elimination state: 2g, eps, half the previous depth
    T a, vn;       // previous point P: its end's term of the segment from P
                   // towards the origin (u vf) and that segment's near-end
                   // bin factor
    T Dn;          // after the first row of a pair, G and eps hold the
                   // numerators of N / Dn and E / Dn until the second row
                   // divides
};

// Unrolling and occupancy, as measured: the sweep loops take two records
// per step (no register copies between steps).  FP32 launches other than
// one-width models are held to 64 VGPRs (eight waves per SIMD, no spills);
// one-width models keep their 70 (seven waves, which for their 12-wave
// workgroups is the same two workgroups per CU as eight).  Every FP64 launch
// is held to 128 VGPRs (four waves; it needs 123).
// ONE_WIDTH: the model has one Doppler width everywhere (T and v_turb the
// same at every point); it selects only this cap.
template <typename T, bool ONE_WIDTH>
constexpr int kWavesPerEu = sizeof(T) == 4 ? (ONE_WIDTH ? 7 : 8) : 4;

// One origin x line chunk, executed by the whole workgroup (blockDim.x
// threads, at least nlc * nbins).  Shared by the single-model launch and the
// persistent batched launch, so both give bit-identical results.
template <typename T>
__device__ __forceinline__ void solve_origin(const FSArgs<T> &a, const int o, const int chunk,
                                             const int ch, unsigned char *smem)
{
    const int nb = a.nbins, nl = a.nlines, nlc = a.nlc, nth = blockDim.x;
    const int l0 = chunk * nlc;
    const int nl_here = min(nlc, nl - l0);
    const int tid = threadIdx.x;
    const bool active = tid < nl_here * nb;
    const int ll = min(tid / nb, nl_here - 1);
    const int f = tid % nb;
    const int l = l0 + ll;

    const gptr<int64_t> off = glob(a.off);
    const gptr<Rec<T>> rec = glob(a.rec);
    const gptr<int32_t> pair_r = glob(a.pair_r), pair_a = glob(a.pair_a);
    const gptr<double> pair_w = glob(a.pair_w), b64 = glob(a.b64), xf = glob(a.xf);
    const gptr<double> W = glob(a.W), acmb_l = glob(a.acmb), Iref = glob(a.Iref);
    const gptr<T> chi = glob(a.chi), S = glob(a.S), bpt = glob(a.bpt), ibpt = glob(a.ibpt);
    const gptr_mut<double> Jout = glob_mut(a.J), Lout = glob_mut(a.L);

    const LDSLayout LY = lds_layout<T>(ch, nlc, nb, nth);
    StageRec<T> *s_st = (StageRec<T> *)(smem + LY.st);
    MetaA<T> *s_a = (MetaA<T> *)(smem + LY.a);
    LineRec<T> *s_line = (LineRec<T> *)(smem + LY.line);
    T *s_S0 = (T *)(smem + LY.s0);
    BinRec<T> *s_bin = (BinRec<T> *)(smem + LY.bin);

    // per-lane constants (bin f: x_f b_o, k1 = 1 + x_f b_o / c, 1/k1)
    const double bo = b64[o];
    const double xfd = xf[f];
    const double xbd = xfd * bo;
    const T xb = (T)xbd;
    const T k1 = (T)(1.0 + xbd / kC);
    const T ik1 = (T)(1.0 / (1.0 + xbd / kC));
    const T inv_c = (T)(1.0 / kC);
    const T acmb = (T)acmb_l[l];
    const int ldl = a.ldl;
    const int64_t ol = (int64_t)o * ldl + l;
    const T chi_o = chi[ol];
    const T S_o = S[ol];
    const T b_o = bpt[o];
    const T half_floor = (T)(0.5 * a.tau_floor);
    const T half = (T)0.5;

    auto bdy_I = [&](T dv) -> T {
        const T r = k1 * ((T)1 + dv * inv_c);
        return r * r * r * FM<T>::rcp(FM<T>::expm1_(acmb * r));
    };
    // the boundary intensity at the origin (an empty half's)
    const T I_o = bdy_I((T)0);
    // 1/b at the origin (the near end of each half's last segment)
    const T ib_o = ibpt[o];

    // staging columns, fixed per thread so the loops need no division:
    // line li of records le0, le0 + lrows, ...; bin f (the lane's own) of
    // records be0, be0 + brows, ... (threads past the last full row idle)
    const int lrows = nth / nl_here, brows = nth / nb;
    const int li_s = tid % nl_here, le0 = tid / nl_here < lrows ? tid / nl_here : INT_MAX;
    const int be0 = tid / nb < brows ? tid / nb : INT_MAX;

    // one elimination step across the previous point (source SP), h = half
    // the depth of the segment that follows it (q2 = 2q, and q2 h = q dt
    // exactly)
    auto row = [&](HalfState<T> &st, T h, T SP) {
        const T D = st.hm + h;
        const T q2 = D * (T)2 + st.G;
        const T inv = FM<T>::rcp_ge1((T)1 + q2 * h);
        st.G = q2 * inv;
        st.eps = (D * SP + st.eps) * inv;
        st.hm = h;
    };

    // half the optical depth of the segment from the previous point of st
    // (farther out) to Q, whose line factor is uQ: trapezoidal
    //   dt/2 = dx/4 (chi'_P phi_P + chi'_Q phi_Q),
    // semi-analytic
    //   dt/2 = dx sqrt(pi)/8 (chi'_P b_P + chi'_Q b_Q) (erf x_Q - erf x_P) / (b-bar (x_Q - x_P)),
    // both as the far end's term plus uQ times the near-end bin factor.
    // The far end's term carries tau_floor / 2 (visit below).
    auto segment = [&](const HalfState<T> &st, T uQ) -> T {
        return uQ * st.vn + st.a;
    };

    double accJ = 0.0, accL = 0.0;
    const int64_t R = a.R;
    for (int pi = 0; pi < a.npairs; pi++) {
        const int rp = pair_r[pi], rm = pair_a[pi];
        const int64_t offp = off[(int64_t)o * R + rp];
        const int np = (int)(off[(int64_t)o * R + rp + 1] - offp);
        const int64_t offm = off[(int64_t)o * R + rm];
        const int nm = (int)(off[(int64_t)o * R + rm + 1] - offm);

        // Halves by length: A the longer (all of a chunk's records lie
        // inside it), B the shorter.  The minus half is staged first.
        const bool a_minus = nm >= np;
        const int nA = a_minus ? nm : np, nB = a_minus ? np : nm;
        HalfState<T> A, B;
        A.G = B.G = (T)2;
        A.hm = B.hm = (T)0;
        A.eps = B.eps = I_o;  // replaced at the far end of a non-empty half
        A.a = A.vn = (T)0;
        B.a = B.vn = (T)0;

        // point Q (staged record e) of a half: either the far-end boundary
        // intensity or one elimination row
        auto visit = [&](HalfState<T> &s, T dv, auto pl, auto pn, bool far_end) {
            const T u = pl->u, Sn = pl->Sn;
            const T vf = pn->vf, vn = pn->vn;
            if (far_end)
                s.eps = bdy_I(dv);
            else
                row(s, segment(s, u), Sn);
            s.a = u * vf + half_floor;  // one multiply-add
            s.vn = vn;
        };
        // Rows in pairs with one reciprocal.  The rows at records 2j + 1 and
        // 2j of a half form a pair: after the first, (G, eps) is carried as
        // the fraction (N / Dn, E / Dn) whose denominator 1 + q2 h is the one
        // a single row divides by; the second row then gives
        //   N2 = 2 D2 Dn + N,  Dn2 = Dn + N2 h2,  E2 = D2 SP2 Dn + E,
        // and G = N2 / Dn2, eps = E2 / Dn2 (both denominators are >= 1, and
        // their product stays far inside the range for any segment depths
        // a line profile produces).  The row right below a far end at an
        // even record has no partner and divides at once.  Pairs follow
        // the record index, not the staging chunks, so every chunk size
        // gives the same roundings.
        auto first = [&](HalfState<T> &s, auto pl, auto pn) {
            const T u = pl->u, Sn = pl->Sn;
            const T vf = pn->vf, vn = pn->vn;
            const T h = segment(s, u);
            const T D = s.hm + h;
            s.G = D * (T)2 + s.G;
            s.Dn = s.G * h + (T)1;
            s.eps = D * Sn + s.eps;
            s.hm = h;
            s.a = u * vf + half_floor;
            s.vn = vn;
        };
        auto second = [&](HalfState<T> &s, auto pl, auto pn) {
            const T u = pl->u, Sn = pl->Sn;
            const T vf = pn->vf, vn = pn->vn;
            const T h = segment(s, u);
            const T D = s.hm + h;
            const T t = D * s.Dn;
            const T N = t * (T)2 + s.G;
            const T r = FM<T>::rcp_ge1(N * h + s.Dn);
            s.G = N * r;
            s.eps = (t * Sn + s.eps) * r;
            s.hm = h;
            s.a = u * vf + half_floor;
            s.vn = vn;
        };
        // the row at an even record k of a half of n records: the second of
        // a pair, or a single row right below the far end
        auto even_row = [&](HalfState<T> &s, int k, int n, auto pl, auto pn) {
            if (k <= n - 3)
                second(s, pl, pn);
            else
                visit(s, (T)0, pl, pn, false);
        };
        // the row at record k (not a far end)
        auto any_row = [&](HalfState<T> &s, int k, int n, auto pl, auto pn) {
            if (k & 1)
                first(s, pl, pn);
            else
                even_row(s, k, n, pl, pn);
        };

        for (int hi = nA; hi > 0; hi -= ch) {
            const int lo = hi - ch > 0 ? hi - ch : 0;
            // valid records of each half in [lo, hi), packed densely: the
            // minus half first, then the plus half
            const int cm = max(0, min(hi, nm) - lo);
            const int cp = max(0, min(hi, np) - lo);
            const int cnt = cm + cp;
            __syncthreads();
            for (int t = tid; t < cnt; t += nth) {
                const bool plus = t >= cm;
                const int k = lo + (plus ? t - cm : t);
                const int64_t base = plus ? offp : offm;
                const int n = plus ? np : nm;
                const Rec<T> rc = load_stream(rec + base + k);
                const int p = rc.ps & 0x7fffffff;
                const bool semi = rc.ps < 0;
                StageRec<T> sr;
                sr.dv = rc.dv;
                if (k > 0) {
                    sr.dvm = rec[base + k - 1].dv;
                    sr.ibm = rec[base + k - 1].ib;
                    sr.bm = rec[base + k - 1].b;
                } else {  // the origin, dv = 0
                    sr.dvm = (T)0;
                    sr.ibm = ib_o;
                    sr.bm = b_o;
                }
                sr.ib = rc.ib;
                sr.sibb = rc.ibb * (T)FM<T>::erf_scale;
                // semi-analytic: half its lane-independent factor; trapezoidal:
                // a quarter of its length
                sr.rw = semi ? rc.dx * half : rc.dx * (T)0.25;
                sr.b = rc.b;
                sr.p = p;
                sr.pn = k + 1 < n ? rec[base + k + 1].ps & 0x7fffffff : -1;
                sr.semi = semi ? 1 : 0;
                s_st[t] = sr;
                MetaA<T> ma;
                ma.dv = rc.dv;
                s_a[t] = ma;
            }
            __syncthreads();
            // per (record, line): the gathers of the thread's first
            // kLineAhead records are issued before the bin factors below
            // are computed, and stored after them, so that arithmetic
            // covers their latency
            constexpr int kA = kLineAhead<T> > 0 ? kLineAhead<T> : 1;
            T g_chi[kA], g_Sn[kA];
    #pragma unroll
            for (int j = 0; j < kLineAhead<T>; j++) {
                const int e = le0 < cnt ? le0 + j * lrows : cnt;
                if (e < cnt) {
                    const StageRec<T> &sr = s_st[e];
                    const int64_t idx = (int64_t)sr.p * ldl + l0 + li_s;
                    g_chi[j] = chi[idx];
                    g_Sn[j] = sr.pn >= 0 ? S[(int64_t)sr.pn * ldl + l0 + li_s] : (T)0;
                }
            }
            // per (record, bin): the bin factors of the segment towards the
            // origin (P this record, Q the next one)
            for (int e = be0; e < cnt; e += brows) {
                const StageRec<T> &sr = s_st[e];
                const T uP = xb + sr.dv * k1;
                const T uQ = xb + sr.dvm * k1;
                BinRec<T> br;
                if (sr.semi) {
                    const T xP = uP * sr.sibb;
                    const T xQ = uQ * sr.sibb;
                    const T eP = FM<T>::erfc_scaled(fabs(xP));
                    const T eQ = FM<T>::erfc_scaled(fabs(xQ));
                    const T Wd = erf_diff<T>(xP, xQ, eP, eQ) * (sr.rw * ik1);
                    br.vf = Wd * sr.b;
                    br.vn = Wd * sr.bm;
                } else {
                    br.vf = sr.rw * FM<T>::phi_of(uP * sr.ib);
                    br.vn = sr.rw * FM<T>::phi_of(uQ * sr.ibm);
                }
                s_bin[f * LY.bs + e * LY.be] = br;
            }
            auto line_rec = [&](T chi_l, T Sn_l) {
                LineRec<T> lr;
                lr.u = chi_l;
                lr.Sn = Sn_l;
                return lr;
            };
            // S' at record 0 of each half (minus, plus), for the row across
            // the last point before the origin
            auto stage_s0 = [&](int e, const StageRec<T> &sr) {
                const bool mh = e < cm;
                if (lo == 0 && (mh ? e : e - cm) == 0)
                    s_S0[(mh ? 0 : nlc) + li_s] = S[(int64_t)sr.p * ldl + l0 + li_s];
            };
    #pragma unroll
            for (int j = 0; j < kLineAhead<T>; j++) {
                const int e = le0 < cnt ? le0 + j * lrows : cnt;
                if (e < cnt) {
                    s_line[li_s * LY.ls + e * LY.le] = line_rec(g_chi[j], g_Sn[j]);
                    stage_s0(e, s_st[e]);
                }
            }
            // the rest of the thread's records
            for (int e = le0 < cnt ? le0 + kLineAhead<T> * lrows : cnt; e < cnt; e += lrows) {
                const StageRec<T> &sr = s_st[e];
                const int64_t idx = (int64_t)sr.p * ldl + l0 + li_s;
                const T Sn_l = sr.pn >= 0 ? S[(int64_t)sr.pn * ldl + l0 + li_s] : (T)0;
                s_line[li_s * LY.ls + e * LY.le] = line_rec(chi[idx], Sn_l);
                stage_s0(e, sr);
            }
            __syncthreads();
            // record k of half A is staged at eA + k, of half B at eB + k; a
            // lane's line and bin rows of each half, indexed by record
            const int eA = (a_minus ? 0 : cm) - lo, eB = (a_minus ? cm : 0) - lo;
            if constexpr (kRowsByRecord<T>) {
                const LineRec<T> *la = s_line + ll * LY.ls + eA, *lb = s_line + ll * LY.ls + eB;
                const BinRec<T> *na = s_bin + f * LY.bs + eA, *nbr = s_bin + f * LY.bs + eB;
                int k = hi - 1;
                // records beyond the end of B: A alone (its far end first), a
                // pair of rows per step
                if (k >= nB && k == nA - 1) {
                    visit(A, s_a[eA + k].dv, la + k, na + k, true);
                    k--;
                }
                const int kAB = max(lo, nB);
                if (k >= kAB && !(k & 1)) {
                    even_row(A, k, nA, la + k, na + k);
                    k--;
                }
                {
                    // pointers at the lower record of each step: the upper one is
                    // an immediate offset
                    lptr<LineRec<T>> pl = opaque(la + k - 1);
                    lptr<BinRec<T>> pn = opaque(na + k - 1);
                    for (; k > kAB; k -= 2, pl -= 2, pn -= 2) {
                        first(A, pl + 1, pn + 1);
                        second(A, pl, pn);
                    }
                }
                if (k == kAB) {
                    first(A, la + k, na + k);
                    k--;
                }
                // B's far end (A's too when the halves are equally long)
                if (k >= lo && k == nB - 1) {
                    if (k == nA - 1)
                        visit(A, s_a[eA + k].dv, la + k, na + k, true);
                    else
                        any_row(A, k, nA, la + k, na + k);
                    visit(B, s_a[eB + k].dv, lb + k, nbr + k, true);
                    k--;
                }
                if (k >= lo && !(k & 1)) {
                    even_row(A, k, nA, la + k, na + k);
                    even_row(B, k, nB, lb + k, nbr + k);
                    k--;
                }
                {
                    lptr<LineRec<T>> pla = opaque(la + k - 1), plb = opaque(lb + k - 1);
                    lptr<BinRec<T>> pna = opaque(na + k - 1), pnb = opaque(nbr + k - 1);
                    for (; k > lo; k -= 2, pla -= 2, plb -= 2, pna -= 2, pnb -= 2) {
                        first(A, pla + 1, pna + 1);
                        first(B, plb + 1, pnb + 1);
                        second(A, pla, pna);
                        second(B, plb, pnb);
                    }
                }
                if (k == lo) {
                    first(A, la + k, na + k);
                    first(B, lb + k, nbr + k);
                }
            } else {
                int k = hi - 1;
                const LineRec<T> *la = s_line + (eA + k) * nlc + ll;
                const BinRec<T> *na = s_bin + (eA + k) * nb + f;
                // records beyond the end of B: A alone (its far end first)
                if (k >= nB && k == nA - 1) {
                    visit(A, s_a[eA + k].dv, la, na, true);
                    la -= nlc;
                    na -= nb;
                    k--;
                }
                const int kAB = max(lo, nB);
                if (k >= kAB && !(k & 1)) {
                    even_row(A, k, nA, la, na);
                    la -= nlc;
                    na -= nb;
                    k--;
                }
                for (; k > kAB; k -= 2, la -= 2 * nlc, na -= 2 * nb) {
                    first(A, la, na);
                    second(A, la - nlc, na - nb);
                }
                if (k == kAB) {
                    first(A, la, na);
                    la -= nlc;
                    na -= nb;
                    k--;
                }
                const LineRec<T> *lb = s_line + (eB + k) * nlc + ll;
                const BinRec<T> *nbp = s_bin + (eB + k) * nb + f;
                // B's far end (A's too when the halves are equally long)
                if (k >= lo && k == nB - 1) {
                    if (k == nA - 1)
                        visit(A, s_a[eA + k].dv, la, na, true);
                    else
                        any_row(A, k, nA, la, na);
                    visit(B, s_a[eB + k].dv, lb, nbp, true);
                    la -= nlc;
                    lb -= nlc;
                    na -= nb;
                    nbp -= nb;
                    k--;
                }
                if (k >= lo && !(k & 1)) {
                    even_row(A, k, nA, la, na);
                    even_row(B, k, nB, lb, nbp);
                    la -= nlc;
                    lb -= nlc;
                    na -= nb;
                    nbp -= nb;
                    k--;
                }
                for (; k > lo; k -= 2, la -= 2 * nlc, lb -= 2 * nlc, na -= 2 * nb, nbp -= 2 * nb) {
                    first(A, la, na);
                    first(B, lb, nbp);
                    second(A, la - nlc, na - nb);
                    second(B, lb - nlc, nbp - nb);
                }
                if (k == lo) {
                    first(A, la, na);
                    first(B, lb, nbp);
                }
            }
        }
        // last segment of each non-empty half ends at the origin (S' at
        // record 0 of each half, staged with the last chunk)
        if (nA > 0) row(A, segment(A, chi_o), s_S0[(a_minus ? 0 : nlc) + ll]);
        if (nB > 0) row(B, segment(B, chi_o), s_S0[(a_minus ? nlc : 0) + ll]);
        // combine in the order minus, plus
        const HalfState<T> &Hm = a_minus ? A : B, &Hp = a_minus ? B : A;
        const T Do = Hm.hm + Hp.hm;
        const T inv_den = FM<T>::rcp(Do + Hm.G * half + Hp.G * half);
        const T u = (Do * S_o + Hm.eps + Hp.eps) * inv_den;
        const T lam = Do * inv_den;
        const double w = pair_w[pi];
        accJ += w * (double)u;
        accL += w * (double)lam;
    }

    __syncthreads();
    double *s_red = (double *)smem;
    const double Wf = W[f];
    s_red[tid] = active ? Wf * accJ : 0.0;
    s_red[nth + tid] = active ? Wf * accL : 0.0;
    __syncthreads();
    if (tid < nl_here) {
        double sj = 0.0, sl = 0.0;
        for (int ff = 0; ff < nb; ff++) {
            sj += s_red[tid * nb + ff];
            sl += s_red[nth + tid * nb + ff];
        }
        const int64_t out = (int64_t)o * nl + l0 + tid;
        Jout[out] = Iref[l0 + tid] * sj;
        Lout[out] = sl;
    }
}

// Workgroups are dealt round-robin to the XCDs in launch order.  With an
// origin order (given when the line table outgrows an XCD's L2), each XCD
// gets a contiguous run of the origins' Morton order, so the workgroups that
// share an L2 solve neighbouring origins, whose walks gather the same points.
// Smaller tables stay L2-resident anyway and keep the launch order, which
// measured faster there (costs of neighbouring origins are correlated).
constexpr int kXcds = 8;

template <typename T, int MAXT, bool ORDERED, bool ONE_WIDTH>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<T, ONE_WIDTH>)))
void k_formal_solve(FSArgs<T> a, int ch)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (ORDERED) {
        const int G = gridDim.x, b = blockIdx.x;
        const int x = b % kXcds, q = G / kXcds, r = G % kXcds;
        // loaded, so uniform only by construction: say so, or every address
        // derived from the origin becomes per-lane
        const int o = __builtin_amdgcn_readfirstlane(a.order[x * q + min(x, r) + b / kXcds]);
        solve_origin<T>(a, o, blockIdx.y, ch, smem);
    } else {
        solve_origin<T>(a, blockIdx.x, blockIdx.y, ch, smem);
    }
}

// Batched launch: one workgroup per work item (model, origin, line chunk) of
// one lane class, items in the order the tuner picked for the class (longest
// first, so the dispatcher hands out the heavy ones early, or by model and
// Morton origin, so workgroups that share an XCD's L2 gather neighbouring
// points); workgroups past the live item count or of converged
// (inactive) models return at once.  The descriptor of the item's model
// replaces the kernel-argument descriptor of the single-model launch.  (Lane
// classes mix models, so it takes the register cap of models with more than
// one Doppler width.)
template <typename T, int MAXT>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<T, false>)))
void k_formal_solve_batch(const FSArgs<T> *__restrict__ descs, const int4 *__restrict__ items,
                          const int *__restrict__ count, const int *__restrict__ active, int ch)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int it = blockIdx.x;
    if (it >= *count) return;
    const int4 w = items[it];
    if (!active[w.x]) return;
    solve_origin<T>(descs[w.x], w.y, w.z, ch, smem);
}

template <typename T>
size_t formal_solve_lds(int ch, int nlc, int nb, int nthreads)
{
    return lds_layout<T>(ch, nlc, nb, nthreads).total;
}
template size_t formal_solve_lds<float>(int, int, int, int);
template size_t formal_solve_lds<double>(int, int, int, int);

// The LDS a workgroup may take: 160 KiB shared by the workgroups the
// registers let a CU hold (whole workgroups only; measured targets of 28
// waves per CU in FP32 and 12 in FP64, whose four waves per SIMD hold only
// two 5-wave workgroups: a workgroup's waves are spread unevenly over the
// four SIMDs).  The chunk is then the largest that fits, in steps of 8
// records: a record chunk ends in a barrier and a wait on the next chunk's
// gathers that only the CU's other workgroups can cover, so fewer, larger
// chunks matter more than one more resident workgroup (clumpy cloud, two
// 12-wave workgroups per CU: 56 records per half, 109 against 116 ms with
// 32; outflow, five 5-wave workgroups: 32 against 16, 9.1 against 10.5 ms;
// FP64 clumpy cloud, one workgroup per CU with 148 KiB: 56 against 24, 326
// against 359 ms; FP64 outflow, two workgroups: 33.9 against 35.7 ms; with
// two-value line records the clumpy cloud's FP32 chunk reaches 72 records,
// 83.1 against 83.9 ms at 64).
static size_t lds_budget(int nthreads, int target_waves)
{
    const int waves = (nthreads + 63) / 64;
    int wgs = target_waves / waves;
    if (wgs < 1) wgs = 1;
    return (size_t)160 * 1024 / wgs - 1024;
}

template <typename T>
int formal_solve_chunk(int nlc, int nb, int nthreads)
{
    const size_t budget = lds_budget(nthreads, sizeof(T) == 4 ? 28 : 12);
    int ch = 128;
    while (lds_layout<T>(ch, nlc, nb, nthreads).total > budget && ch > 1) ch -= ch > 8 ? 8 : 1;
    return ch;
}
template int formal_solve_chunk<float>(int, int, int);
template int formal_solve_chunk<double>(int, int, int);

template <typename T>
hipError_t launch_formal_solve_batch(const FSArgs<T> *descs, const int4 *items, const int *count,
                                     int blocks, const int *active, int ch, int nthreads,
                                     size_t lds, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    if (ch < 1) return hipErrorInvalidValue;
    if (sizeof(T) == 8 && nthreads <= 512)
        k_formal_solve_batch<T, 512><<<blocks, nthreads, lds, s>>>(descs, items, count, active,
                                                                   ch);
    else
        k_formal_solve_batch<T, 1024><<<blocks, nthreads, lds, s>>>(descs, items, count, active,
                                                                    ch);
    return hipGetLastError();
}
template hipError_t launch_formal_solve_batch<float>(const FSArgs<float> *, const int4 *,
                                                     const int *, int, const int *, int, int,
                                                     size_t, hipStream_t);
template hipError_t launch_formal_solve_batch<double>(const FSArgs<double> *, const int4 *,
                                                      const int *, int, const int *, int, int,
                                                      size_t, hipStream_t);

template <typename T, int MAXT>
static void launch_fs_variant(const FSArgs<T> &a, dim3 grid, size_t lds, int ch, hipStream_t s)
{
    const bool ordered = a.order != nullptr, one = a.one_width != 0;
    if (ordered && one)
        k_formal_solve<T, MAXT, true, true><<<grid, a.nthreads, lds, s>>>(a, ch);
    else if (ordered)
        k_formal_solve<T, MAXT, true, false><<<grid, a.nthreads, lds, s>>>(a, ch);
    else if (one)
        k_formal_solve<T, MAXT, false, true><<<grid, a.nthreads, lds, s>>>(a, ch);
    else
        k_formal_solve<T, MAXT, false, false><<<grid, a.nthreads, lds, s>>>(a, ch);
}

template <typename T>
hipError_t launch_formal_solve(const FSArgs<T> &a, hipStream_t s)
{
    const int ch = formal_solve_chunk<T>(a.nlc, a.nbins, a.nthreads);
    const LDSLayout L = lds_layout<T>(ch, a.nlc, a.nbins, a.nthreads);
    const int nchunks = (a.nlines + a.nlc - 1) / a.nlc;
    dim3 grid(a.N, nchunks);
    // FP64 workgroups of at most 512 threads take the 512-thread bound (the
    // same 128 VGPRs as the 1024 bound under the four-wave cap)
    if constexpr (sizeof(T) == 8) {
        if (a.nthreads <= 512) {
            launch_fs_variant<T, 512>(a, grid, L.total, ch, s);
            return hipGetLastError();
        }
    }
    launch_fs_variant<T, 1024>(a, grid, L.total, ch, s);
    return hipGetLastError();
}

template hipError_t launch_formal_solve<float>(const FSArgs<float> &, hipStream_t);
template hipError_t launch_formal_solve<double>(const FSArgs<double> &, hipStream_t);

// ---------------------------------------------------------------------------
// Per-line constants (Einstein coefficients, scalings) and the bin table.
// ---------------------------------------------------------------------------
__global__ void k_line_table(int nlines, const double *A, const double *nu, const double *g,
                             const int32_t *up, const int32_t *lo, double L_unit, double Tcmb,
                             double *Bul, double *Blu, double *hnu4pi, double *chiscale,
                             double *Iref, double *acmb)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    const double v = nu[l];
    const double bul = A[l] * kC * kC / (2.0 * kH * v * v * v);
    Bul[l] = bul;
    Blu[l] = g[up[l]] / g[lo[l]] * bul;
    hnu4pi[l] = kH * v / (4.0 * kPi);
    // chi' = chi^ij / (dnu sqrt(pi)) * L_unit, dnu = nu b / c
    chiscale[l] = kC / (v * kSqrtPi) * L_unit;
    Iref[l] = 2.0 * kH * v * v * v / (kC * kC);
    acmb[l] = kH * v / (kKB * Tcmb);
}

hipError_t launch_line_table(int nlines, int nlev, const double *A, const double *nu,
                             const double *g, const int32_t *up, const int32_t *lo,
                             double L_unit, double Tcmb, double *Bul, double *Blu,
                             double *hnu4pi, double *chiscale, double *Iref, double *acmb,
                             hipStream_t s)
{
    (void)nlev;
    k_line_table<<<(nlines + 63) / 64, 64, 0, s>>>(nlines, A, nu, g, up, lo, L_unit, Tcmb, Bul,
                                                   Blu, hnu4pi, chiscale, Iref, acmb);
    return hipGetLastError();
}

__global__ void k_bin_table(int nb, double xmax, double *xf, double *W)
{
    __shared__ double e[kMaxBins];
    const int f = threadIdx.x;
    if (f < nb) {
        const double x = (nb == 1) ? 0.0 : -xmax + 2.0 * xmax * f / (nb - 1);
        xf[f] = x;
        e[f] = exp(-x * x);
    }
    __syncthreads();
    if (f < nb) {
        double s = 0.0;
        for (int i = 0; i < nb; i++) s += e[i];
        W[f] = e[f] / s;
    }
}

hipError_t launch_bin_table(int nbins, double xmax, double *xf, double *W, hipStream_t s)
{
    k_bin_table<<<1, kMaxBins, 0, s>>>(nbins, xmax, xf, W);
    return hipGetLastError();
}

// chi^ij = (h nu / 4 pi)(n_l B_lu - n_u B_ul), eta^ij = (h nu / 4 pi) n_u A,
// S = eta^ij / chi^ij; stored as chi' = chi^ij c L_unit / (nu b sqrt(pi)) and
// S / Iref (S / I_img for images) in the solve precision, S in double for
// statistical equilibrium.
__global__ void k_line_coeffs(LineArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)a.N * a.nlines) return;
    const int p = (int)(i / a.nlines);
    const int l = (int)(i - (int64_t)p * a.nlines);
    const double n = a.nspec[p];
    const double nu_ = n * a.pops[(int64_t)p * a.nlev + a.up[l]];
    const double nl_ = n * a.pops[(int64_t)p * a.nlev + a.lo[l]];
    double chi = a.hnu4pi[l] * (nl_ * a.Blu[l] - nu_ * a.Bul[l]);
    const double eta = a.hnu4pi[l] * nu_ * a.A[l];
    if (chi <= a.chi_min) {
        chi = a.chi_min;
        atomicAdd(&a.cnt->masing, 1ull);
    }
    const double S = eta / chi;
    a.S64[i] = S;
    const double chis = chi * a.chiscale[l] / a.b[p];
    const double Ss = S / (a.S_unit > 0.0 ? a.S_unit : a.Iref[l]);
    const int64_t it = (int64_t)p * a.ldt + l;
    if (a.fp32) {
        ((float *)a.chiT)[it] = (float)chis;
        ((float *)a.ST)[it] = (float)Ss;
    } else {
        ((double *)a.chiT)[it] = chis;
        ((double *)a.ST)[it] = Ss;
    }
}

hipError_t launch_line_coeffs(const LineArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.N * a.nlines;
    k_line_coeffs<<<(n + 255) / 256, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mgx
