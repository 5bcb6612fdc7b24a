// Internal declarations of the gfx950 line radiative transfer library.
// Device-state layout, kernel argument blocks and launch wrappers shared by
// the HIP translation units.  Not part of the public ABI (include/mgx.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgx {

// CODATA 2018 exact SI values.
constexpr double kH = 6.62607015e-34;
constexpr double kKB = 1.380649e-23;
constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.7724538509055160273;
constexpr double kLog2e = 1.4426950408889634074;

constexpr int kMaxLevels = 64;
constexpr int kMaxBins = 1024;
constexpr int kNgMaxHist = 32;

// Global-memory pointers.  Every table the kernels read lives in global
// memory; pointers loaded from device memory (the batched launch's
// descriptors) or carried in by-value argument blocks are generic to the
// compiler and would otherwise become flat accesses, which also wait on LDS
// traffic and cannot become scalar loads.
template <typename X>
using gptr = const __attribute__((address_space(1))) X *;
template <typename X>
using gptr_mut = __attribute__((address_space(1))) X *;
template <typename X>
__device__ __forceinline__ gptr<X> glob(const X *p)
{
    return (gptr<X>)p;
}
template <typename X>
__device__ __forceinline__ gptr_mut<X> glob_mut(X *p)
{
    return (gptr_mut<X>)p;
}

// Device counters (reset per pass by k_reset_counters).
struct Counters {
    unsigned long long masing;
    unsigned long long singular;
    unsigned long long nonfinite;
    unsigned long long holes;
    unsigned long long semi;
    unsigned long long change_bits;   // max relative change, as IEEE bits (>= 0)
    unsigned long long pad[2];
};

// Packed trace record used by the formal solution: point index with the
// semi-analytic flag in bit 31; for a trapezoidal segment its length from
// the previous record (or the origin), for a semi-analytic one
// dx sqrt(pi)/4 / (dv_prev - dv) (both scaled by 1/L_unit); 1/b-bar of the
// segment; the point's Doppler width b; the projected velocity difference to
// the origin and the point's 1/b (scaled as the solve's per-point table),
// adjacent so the record after this one reads both with one load.  Carrying
// the point's widths saves the staging a dependent gather.
template <typename T>
struct Rec;
template <>
struct alignas(8) Rec<float> {
    int32_t ps;
    float dx, ibb, b, dv, ib;
};
template <>
struct alignas(16) Rec<double> {
    int32_t ps;
    int32_t pad;
    double dx, ibb, b, dv, ib;
};

struct TraceArgs {
    int dim, N, R;
    const double *x, *y, *z, *vx, *vy, *vz;
    const double4 *p4;     // [N] {x, y, z, 0}: one gather per neighbour candidate
    const double4 *v4;     // [N] {vx, vy, vz, b2}: one load per step
    const int32_t *nbs_off, *nbs;
    const uint8_t *bdy;
    const double *ray_dir;
    const double *b2;      // [N] squared Doppler speed
    double thr;            // branch threshold in line widths
    int64_t *counts;       // count pass: [N R]
    const int64_t *off;    // fill pass: [N R + 1]
    int32_t *r_idx;
    uint8_t *r_semi;
    double *r_Z, *r_dv, *r_dx, *r_ibb;
    Counters *cnt;
    int32_t *slot;             // slot pass: walk w's points at slot[w cap], at most cap
    int64_t cap;
    unsigned long long *maxn;  // slot pass: longest walk (atomic max)
};

template <typename T>
struct FSArgs {
    int N, R, npairs, nlines, nbins, nlc, nthreads;
    const int64_t *off;
    const Rec<T> *rec;
    const int32_t *pair_r, *pair_a;
    const double *pair_w;
    const T *chi, *S;       // [N][ldl] scaled opacity factor and source
    const T *bpt, *ibpt;    // [N] b and (scaled) 1/b in T
    const double *b64;      // [N] b
    const double *xf, *W;   // [nbins]
    const double *acmb;     // [nlines] h nu / (k Tcmb)
    const double *Iref;     // [nlines] 2 h nu^3 / c^2
    double tau_floor;
    double *J, *L;          // [N][nlines]
    const int32_t *order;   // [N] origins in Morton order of their positions
    int one_width;          // every point has the same Doppler width b
    int ldl;                // row stride of chi and S (>= nlines)
};

struct LineArgs {
    int N, nlev, nlines;
    const double *pops, *nspec, *b;
    const int32_t *up, *lo;
    const double *A, *Bul, *Blu, *hnu4pi, *chiscale, *Iref;
    double chi_min;
    double S_unit;          // > 0: the solve-precision S is S / S_unit (images), else S / Iref
    double *S64;            // [N][nlines] physical source function
    void *chiT, *ST;        // [N][ldt] in the solve precision
    int ldt;                // their row stride (>= nlines)
    int fp32;
    Counters *cnt;
};

struct StateqArgs {
    int N, nlev, nlines, ncoll_tr;
    int group, wpb;        // lanes per point (stateq_group), waves per block
    const double *J, *L, *S64;
    const double *T, *ncoll;
    const double *E, *g;
    const int32_t *up, *lo, *cu, *cl;
    const double *A, *Bul, *Blu, *K0;
    const double *pops_old;
    double *pops_new;
    double pop_floor;
    Counters *cnt;
    const int *active;     // batched use: skip when active[model] == 0 (may be NULL)
    int model;
};

// Launch wrappers (return hipError_t of the launch).
hipError_t launch_point_widths(int N, const double *T, const double *vturb2, double mass,
                               double *b2, double *b, float *bf, float *ibf_scaled,
                               double *bd, double *ibd, hipStream_t s);
// Walk lengths (counts) and hole count; records at CSR offsets (off); or, in
// 3D, lengths, holes and the walks' point indices in slots of a.cap, with the
// longest length in *a.maxn.  launch_trace_emit then writes the records of
// walks that fit their slots without searching again.
enum class TraceMode { count, fill, slots };
hipError_t launch_trace(const TraceArgs &a, TraceMode mode, hipStream_t s);
hipError_t launch_trace_emit(const TraceArgs &a, hipStream_t s);
hipError_t launch_pack_vel4(int N, const double *vel, const double *b2, double4 *out,
                            hipStream_t s);
hipError_t launch_pack_trace(int64_t n, const int32_t *idx, const uint8_t *semi,
                             const void *bpt, const void *ibpt, const double *dx, const double *dv, const double *ibb,
                             double inv_L, bool fp32, void *out, hipStream_t s);
hipError_t launch_line_coeffs(const LineArgs &a, hipStream_t s);
template <typename T>
hipError_t launch_formal_solve(const FSArgs<T> &a, hipStream_t s);
// batched: one workgroup per (model, origin, line chunk) item of a lane class
template <typename T>
size_t formal_solve_lds(int ch, int nlc, int nb, int nthreads);
// records per half staged at once: the largest chunk (steps of 8 records,
// at most 128; down to 1 for very wide bin sets) whose LDS fits the share of a
// CU's 160 KiB that the workgroups its registers allow leave each
template <typename T>
int formal_solve_chunk(int nlc, int nb, int nthreads);
template <typename T>
hipError_t launch_formal_solve_batch(const FSArgs<T> *descs, const int4 *items, const int *count,
                                     int blocks, const int *active, int ch, int nthreads,
                                     size_t lds, hipStream_t s);
hipError_t launch_origin_cost(int N, int R, const int64_t *off, int64_t *cost, hipStream_t s);
// order-preserving selection of the items whose model is active; *count on
// the device receives the number kept (tmp: cached scratch, grown as needed)
hipError_t launch_compact_items(const int4 *in, int n, int4 *out, int *count, const int *active,
                                void **tmp, size_t *tmp_bytes, hipStream_t s);
hipError_t launch_copy_if_active(int64_t n, const double *src, double *dst, const int *active,
                                 int model, hipStream_t s);
hipError_t launch_gather_changes(int M, Counters *const *cnt, double *out, hipStream_t s);
hipError_t launch_lte(int N, int nlev, const double *T, const double *E, const double *g,
                      double *pops, hipStream_t s);
int stateq_group(int nlev);  // lanes per point of the statistical-equilibrium kernel
hipError_t launch_stateq(const StateqArgs &a, hipStream_t s);
// with_masing false: keep the masing count of the last line-coefficient pass
// (the statistical-equilibrium step resets only its own counters)
hipError_t launch_reset_counters(Counters *c, hipStream_t s, bool with_masing = true);
hipError_t launch_rel_change(int64_t n, const double *a, const double *b, double floor_,
                             unsigned long long *bits, hipStream_t s);
hipError_t launch_bin_table(int nbins, double xmax, double *xf, double *W, hipStream_t s);
hipError_t launch_line_table(int nlines, int nlev, const double *A, const double *nu,
                             const double *g, const int32_t *up, const int32_t *lo,
                             double L_unit, double Tcmb, double *Bul, double *Blu,
                             double *hnu4pi, double *chiscale, double *Iref, double *acmb,
                             hipStream_t s);
hipError_t launch_copy(int64_t n, const double *src, double *dst, hipStream_t s);

// Synthetic images.  Geometry in FP64 without contraction (bit-exact pixel
// walks); integration in the solve precision.
struct RenderGeom {
    int N, npx, npy;
    double d[3], e1[3], e2[3];
    double h;                  // length scale (bbox diagonal / N^(1/3))
    const double *x, *y, *z, *vx, *vy, *vz;
    const int32_t *nbs_off, *nbs;
    const uint8_t *bdy;
    double *u, *v, *Z, *w;     // [N] projections and d.v
    double *ext;               // [4] umin, umax, vmin, vmax (after reduce)
    unsigned long long *key;   // [npx npy] entry search scratch
    int32_t *entry;            // [npx npy]
    int64_t *counts;           // [npx npy + 1]
    const int64_t *off;        // [npx npy + 1]
    int32_t *walk;             // records
    int64_t cap;               // capped fill: pixel i's walk at walk[i cap], at most cap points
    unsigned long long *maxn;  // capped fill: longest walk (atomic max)
};
hipError_t launch_render_geometry(RenderGeom &g, hipStream_t s);  // project + extent + entry
// walk lengths only (counts), walks at CSR offsets (off), or walks in slots of
// g.cap points with exact lengths in counts and the longest in *maxn
enum class WalkMode { count, fill, capped };
hipError_t launch_render_walk(const RenderGeom &g, WalkMode mode, hipStream_t s);

template <typename T>
struct RenderArgs {
    int npx, npy, nfreq, nlines;
    const int64_t *off;        // CSR offsets of the walks, or null: slots of cap points
    const int64_t *cnt;        // with off null: walk lengths
    int64_t cap;
    const int32_t *walk;
    const double *Z, *w;       // [N] (double; scaled inside)
    const T *chi, *S;          // [N][nlines] scaled opacity factor and S / I_img
    const double *b, *ib;      // [N] b and 1/b
    const double *nu_line;     // [nlines]
    const int32_t *act;        // [nact] lines that can reach the band (others add exact zeros)
    int nact;
    double inv_L, f_min, f_max, Tcmb, I_img;
    double thr;                // branch threshold (widths)
    const double *b2;          // [N] squared Doppler speed (branch rule in FP64)
    float *img;                // [npy][npx][nfreq]
};
template <typename T>
hipError_t launch_render_integrate(const RenderArgs<T> &a, hipStream_t s);

// Ng: incremental Gram matrix, solve, combine.  Pointer tables are passed by
// value (kernel arguments), entry k is residual r_k or iterate y_{k+1}.
struct PtrTable {
    const double *p[kNgMaxHist];
};
int ng_gram_blocks(int64_t n);
hipError_t launch_ng_append(int64_t n, int K, const double *src, const double *prev,
                            double *dst_y, double *dst_r, const PtrTable &r_ptrs,
                            double *partial, double *G, hipStream_t s);
hipError_t launch_ng_shift(int K, double *G, hipStream_t s);
hipError_t launch_ng_predict(int64_t n, int K, const double *G, const PtrTable &y_ptrs,
                             double *coef, int *status, double *out, int *neg, hipStream_t s);

}  // namespace mgx
