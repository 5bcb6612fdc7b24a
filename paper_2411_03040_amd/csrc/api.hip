// C ABI of the library: context, device memory, model validation and the
// iteration driver.  All arithmetic of the method runs in the kernels of
// trace.hip, formal_solve.hip, stateq.hip and ng.hip; this file only moves
// data, checks arguments and sequences launches on the context's stream.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgx.h"
#include "mgx_internal.h"

extern "C" hipError_t mgx_internal_scan(int64_t *counts, int64_t *offsets, int64_t n,
                                        void **tmp, size_t *tmp_bytes, hipStream_t s);

using namespace mgx;

namespace {

struct Err {
    mgx_status st;
    std::string msg;
};

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess)                                                             \
            throw Err{e_ == hipErrorOutOfMemory ? MGX_ENOMEM : MGX_EHIP,                  \
                      std::string(#x) + ": " + hipGetErrorString(e_)};                    \
    } while (0)

#define REQUIRE(cond, code, text)                                                         \
    do {                                                                                  \
        if (!(cond)) throw Err{code, text};                                               \
    } while (0)

// Owning device allocation.
struct DMem {
    void *p = nullptr;
    size_t bytes = 0;
    DMem() = default;
    DMem(const DMem &) = delete;
    DMem &operator=(const DMem &) = delete;
    ~DMem() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t b)
    {
        if (b <= bytes && p) return;
        release();
        if (b == 0) b = 16;
        HIPCHK(hipMalloc(&p, b));
        bytes = b;
    }
    template <typename T>
    T *as() const
    {
        return (T *)p;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) HIPCHK(hipSetDevice(dev));
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

thread_local std::string g_create_error;

template <typename T>
bool all_finite(const T *a, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite((double)a[i])) return false;
    return true;
}

}  // namespace

struct mgx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mgx_options opt{};
    std::string err;

    // model
    bool loaded = false, traced = false, have_pops = false, have_rad = false;
    int dim = 3, N = 0, R = 0, nlev = 0, nlines = 0, ncoll_tr = 0, nbins = 0, npairs = 0;
    double mass = 0, xmax = 5, Tcmb = 2.72548, L_unit = 1;
    int64_t n_records = 0;

    DMem pos, vel, nbs_off, nbs, bdy, T, vturb2, nspec, ncoll, ray_dir, ray_w, antipode;
    DMem E, g, up, lo, A, nu, cu, cl, K0;
    DMem b2, b, bf, ibf, bd, ibd, xf, W;
    DMem Bul, Blu, hnu4pi, chiscale, Iref, acmb;
    DMem pair_r, pair_a, pair_w;
    DMem pops, pops_new, J, L, S64, chiT, ST;
    DMem counters;
    // trace
    DMem counts, offsets, scan_tmp_owner;
    void *scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
    DMem r_idx, r_semi, r_Z, r_dv, r_dx, r_ibb, rec;
    // Ng
    bool ng_active = false, ng_have_prev = false;
    int ng_cap = 0, ng_nh = 0;
    std::vector<DMem *> ng_y, ng_r;
    std::vector<DMem *> ng_pool;
    DMem ng_G, ng_coef, ng_status, ng_partial, ng_pred, ng_prev, ng_bits;
    // images
    DMem rg_proj, rg_pix, rg_off, rg_walk, rg_img;
    // diagnostics
    mgx_counters host_cnt{};
    hipEvent_t ev_fs0 = nullptr, ev_fs1 = nullptr;
    bool fs_pending = false;

    ~mgx_ctx()
    {
        for (DMem *m : ng_pool) delete m;
        if (scan_tmp) (void)hipFree(scan_tmp);
        if (ev_fs0) (void)hipEventDestroy(ev_fs0);
        if (ev_fs1) (void)hipEventDestroy(ev_fs1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    int64_t npop() const { return (int64_t)N * nlev; }
    int64_t nrad() const { return (int64_t)N * nlines; }
    bool fp32() const { return opt.precision == MGX_FP32; }

    void sync()
    {
        HIPCHK(hipStreamSynchronize(stream));
        collect_timing();
    }

    // Duration of the last formal-solution kernel, once its events completed.
    void collect_timing()
    {
        if (!fs_pending) return;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev_fs0, ev_fs1));
        fs_pending = false;
        host_cnt.fs_launches++;
        host_cnt.fs_ms_total += ms;
        host_cnt.fs_ms_last = ms;
    }

    Counters read_counters()
    {
        Counters c;
        HIPCHK(hipMemcpyAsync(&c, counters.p, sizeof(Counters), hipMemcpyDeviceToHost, stream));
        sync();
        return c;
    }
};

#define API_BEGIN(ctx)                                                                    \
    if (!(ctx)) return MGX_EINVAL;                                                        \
    try {                                                                                 \
        DeviceGuard dg_((ctx)->device);                                                   \
        (ctx)->err.clear();

#define API_END(ctx)                                                                      \
    }                                                                                     \
    catch (const Err &e)                                                                  \
    {                                                                                     \
        (ctx)->err = e.msg;                                                               \
        return e.st;                                                                      \
    }                                                                                     \
    catch (const std::bad_alloc &)                                                        \
    {                                                                                     \
        (ctx)->err = "host allocation failed";                                            \
        return MGX_ENOMEM;                                                                \
    }                                                                                     \
    catch (...)                                                                           \
    {                                                                                     \
        (ctx)->err = "unexpected internal error";                                         \
        return MGX_EHIP;                                                                  \
    }                                                                                     \
    return MGX_OK;

template <typename T>
static void upload(mgx_ctx *c, DMem &d, const T *src, size_t n)
{
    d.ensure(sizeof(T) * n);
    if (n) HIPCHK(hipMemcpyAsync(d.p, src, sizeof(T) * n, hipMemcpyHostToDevice, c->stream));
}

// ---------------------------------------------------------------------------

extern "C" void mgx_default_options(mgx_options *opt)
{
    if (!opt) return;
    opt->precision = MGX_FP32;
    opt->branch_threshold = 0.35;
    opt->tau_floor = 1e-15;
    opt->chi_min = 1e-30;
    opt->pop_floor = 1e-12;
}

extern "C" mgx_status mgx_create(mgx_ctx **out, int device, void *stream,
                                 const mgx_options *opt)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return MGX_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_create_error = "no such HIP device";
        return MGX_EINVAL;
    }
    mgx_options o;
    mgx_default_options(&o);
    if (opt) o = *opt;
    if ((o.precision != MGX_FP32 && o.precision != MGX_FP64) || !(o.branch_threshold >= 0) ||
        !(o.tau_floor > 0) || !(o.chi_min > 0) || !(o.pop_floor > 0)) {
        g_create_error = "invalid options";
        return MGX_EINVAL;
    }
    mgx_ctx *c = new (std::nothrow) mgx_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return MGX_ENOMEM;
    }
    c->device = device;
    c->opt = o;
    try {
        DeviceGuard dg(device);
        if (stream) {
            c->stream = (hipStream_t)stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPCHK(hipEventCreate(&c->ev_fs0));
        HIPCHK(hipEventCreate(&c->ev_fs1));
        c->counters.ensure(sizeof(Counters));
        HIPCHK(hipMemsetAsync(c->counters.p, 0, sizeof(Counters), c->stream));
        c->sync();
    } catch (const Err &e) {
        g_create_error = e.msg;
        delete c;
        return e.st;
    }
    *out = c;
    return MGX_OK;
}

extern "C" void mgx_destroy(mgx_ctx *ctx)
{
    if (!ctx) return;
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        delete ctx;
        if (prev >= 0) (void)hipSetDevice(prev);
    }
}

extern "C" const char *mgx_last_error(const mgx_ctx *ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

// ---------------------------------------------------------------------------
// Model
// ---------------------------------------------------------------------------

static void validate_model(const mgx_model *m)
{
    REQUIRE(m, MGX_EINVAL, "model is NULL");
    REQUIRE(m->dim == 1 || m->dim == 3, MGX_EINVAL, "dim must be 1 or 3");
    const int N = m->npoints;
    REQUIRE(N >= 1, MGX_EINVAL, "npoints must be >= 1");
    REQUIRE(m->pos && m->vel && m->nbs_off && m->bdy && m->T && m->vturb2 && m->nspec &&
                m->ncoll && m->ray_dir && m->ray_w && m->antipode && m->E && m->g && m->up &&
                m->lo && m->A && m->nu,
            MGX_EINVAL, "required model array is NULL");
    REQUIRE(m->nbs_off[0] == 0, MGX_EINVAL, "nbs_off[0] must be 0");
    for (int i = 0; i < N; i++)
        REQUIRE(m->nbs_off[i + 1] >= m->nbs_off[i], MGX_EINVAL, "nbs_off not monotone");
    const int64_t E = m->nbs_off[N];
    REQUIRE(E == 0 || m->nbs, MGX_EINVAL, "nbs is NULL");
    for (int64_t q = 0; q < E; q++)
        REQUIRE(m->nbs[q] >= 0 && m->nbs[q] < N, MGX_EINVAL, "neighbour index out of range");
    REQUIRE(all_finite(m->pos, 3 * (size_t)N) && all_finite(m->vel, 3 * (size_t)N) &&
                all_finite(m->T, N) && all_finite(m->vturb2, N) && all_finite(m->nspec, N) &&
                all_finite(m->ncoll, N),
            MGX_ENONFINITE, "non-finite per-point input");
    for (int i = 0; i < N; i++) {
        REQUIRE(m->T[i] > 0 && m->vturb2[i] >= 0 && m->nspec[i] >= 0 && m->ncoll[i] >= 0,
                MGX_EINVAL, "T must be > 0 and vturb2, nspec, ncoll >= 0");
    }
    if (m->dim == 1) {
        for (int i = 0; i + 1 < N; i++)
            REQUIRE(m->pos[i + 1] > m->pos[i], MGX_EINVAL, "shell radii must increase");
        REQUIRE(m->pos[0] > 0, MGX_EINVAL, "shell radii must be > 0");
        REQUIRE(m->bdy[0] && m->bdy[N - 1], MGX_EINVAL, "first and last shells are boundaries");
    }
    const int R = m->nrays;
    REQUIRE(R >= 2 && R % 2 == 0, MGX_EINVAL, "nrays must be even and >= 2");
    REQUIRE(all_finite(m->ray_dir, 3 * (size_t)R) && all_finite(m->ray_w, R), MGX_ENONFINITE,
            "non-finite ray input");
    for (int r = 0; r < R; r++) {
        const int a = m->antipode[r];
        REQUIRE(a >= 0 && a < R && a != r && m->antipode[a] == r, MGX_EINVAL,
                "antipode table is not an involution");
        REQUIRE(m->ray_w[r] == m->ray_w[a] && m->ray_w[r] >= 0, MGX_EINVAL,
                "antipodal rays need equal non-negative weights");
        if (m->dim == 1) {
            REQUIRE(m->ray_dir[3 * a] == -m->ray_dir[3 * r] && fabs(m->ray_dir[3 * r]) <= 1.0,
                    MGX_EINVAL, "1D rays: mu of an antipode must be -mu");
        } else {
            for (int k = 0; k < 3; k++)
                REQUIRE(m->ray_dir[3 * a + k] == -m->ray_dir[3 * r + k], MGX_EINVAL,
                        "antipode direction must be the exact negative");
        }
    }
    REQUIRE(m->nlev >= 2 && m->nlev <= kMaxLevels, MGX_EINVAL, "nlev must be in 2..64");
    REQUIRE(m->nlines >= 1, MGX_EINVAL, "nlines must be >= 1");
    REQUIRE(m->mass > 0 && std::isfinite(m->mass), MGX_EINVAL, "mass must be > 0");
    REQUIRE(all_finite(m->E, m->nlev) && all_finite(m->g, m->nlev) &&
                all_finite(m->A, m->nlines) && all_finite(m->nu, m->nlines),
            MGX_ENONFINITE, "non-finite level or line data");
    for (int i = 0; i < m->nlev; i++) REQUIRE(m->g[i] > 0, MGX_EINVAL, "g must be > 0");
    std::vector<char> seen((size_t)m->nlev * m->nlev, 0);
    for (int l = 0; l < m->nlines; l++) {
        const int u = m->up[l], lw = m->lo[l];
        REQUIRE(u >= 0 && u < m->nlev && lw >= 0 && lw < m->nlev && u != lw, MGX_EINVAL,
                "line level index out of range");
        REQUIRE(m->nu[l] > 0 && m->A[l] >= 0, MGX_EINVAL, "line nu must be > 0, A >= 0");
        char &s = seen[(size_t)u * m->nlev + lw];
        REQUIRE(!s, MGX_EINVAL, "duplicate radiative transition");
        s = 1;
    }
    REQUIRE(m->ncoll_tr >= 0, MGX_EINVAL, "ncoll_tr must be >= 0");
    if (m->ncoll_tr) {
        REQUIRE(m->cu && m->cl && m->K0, MGX_EINVAL, "collision arrays are NULL");
        REQUIRE(all_finite(m->K0, m->ncoll_tr), MGX_ENONFINITE, "non-finite K0");
    }
    std::fill(seen.begin(), seen.end(), 0);
    for (int t = 0; t < m->ncoll_tr; t++) {
        const int u = m->cu[t], lw = m->cl[t];
        REQUIRE(u >= 0 && u < m->nlev && lw >= 0 && lw < m->nlev && u != lw, MGX_EINVAL,
                "collision level index out of range");
        REQUIRE(m->K0[t] >= 0, MGX_EINVAL, "K0 must be >= 0");
        char &s = seen[(size_t)u * m->nlev + lw];
        REQUIRE(!s, MGX_EINVAL, "duplicate collisional transition");
        s = 1;
    }
    REQUIRE(m->nbins >= 1 && m->nbins <= kMaxBins, MGX_EINVAL, "nbins must be in 1..1024");
    REQUIRE(m->xmax >= 0 && std::isfinite(m->xmax), MGX_EINVAL, "xmax must be >= 0");
    REQUIRE(m->Tcmb > 0 && std::isfinite(m->Tcmb), MGX_EINVAL, "Tcmb must be > 0");
}

extern "C" mgx_status mgx_load_model(mgx_ctx *ctx, const mgx_model *m)
{
    API_BEGIN(ctx)
    validate_model(m);
    ctx->loaded = ctx->traced = ctx->have_pops = ctx->have_rad = false;
    ctx->ng_active = false;
    const int N = m->npoints, R = m->nrays;
    ctx->dim = m->dim;
    ctx->N = N;
    ctx->R = R;
    ctx->nlev = m->nlev;
    ctx->nlines = m->nlines;
    ctx->ncoll_tr = m->ncoll_tr;
    ctx->nbins = m->nbins;
    ctx->mass = m->mass;
    ctx->xmax = m->xmax;
    ctx->Tcmb = m->Tcmb;
    // Length unit of the scaled optical-depth arithmetic: bounding-box
    // diagonal over N^(1/3) (about one point spacing).
    double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < N; i++) {
            lo3[k] = std::min(lo3[k], m->pos[(size_t)k * N + i]);
            hi3[k] = std::max(hi3[k], m->pos[(size_t)k * N + i]);
        }
    double diag = sqrt((hi3[0] - lo3[0]) * (hi3[0] - lo3[0]) + (hi3[1] - lo3[1]) * (hi3[1] - lo3[1]) +
                       (hi3[2] - lo3[2]) * (hi3[2] - lo3[2]));
    ctx->L_unit = diag > 0 ? diag / cbrt((double)N) : 1.0;

    upload(ctx, ctx->pos, m->pos, 3 * (size_t)N);
    upload(ctx, ctx->vel, m->vel, 3 * (size_t)N);
    upload(ctx, ctx->nbs_off, m->nbs_off, (size_t)N + 1);
    upload(ctx, ctx->nbs, m->nbs, (size_t)m->nbs_off[N]);
    upload(ctx, ctx->bdy, m->bdy, (size_t)N);
    upload(ctx, ctx->T, m->T, (size_t)N);
    upload(ctx, ctx->vturb2, m->vturb2, (size_t)N);
    upload(ctx, ctx->nspec, m->nspec, (size_t)N);
    upload(ctx, ctx->ncoll, m->ncoll, (size_t)N);
    upload(ctx, ctx->ray_dir, m->ray_dir, 3 * (size_t)R);
    upload(ctx, ctx->ray_w, m->ray_w, (size_t)R);
    upload(ctx, ctx->antipode, m->antipode, (size_t)R);
    upload(ctx, ctx->E, m->E, (size_t)m->nlev);
    upload(ctx, ctx->g, m->g, (size_t)m->nlev);
    upload(ctx, ctx->up, m->up, (size_t)m->nlines);
    upload(ctx, ctx->lo, m->lo, (size_t)m->nlines);
    upload(ctx, ctx->A, m->A, (size_t)m->nlines);
    upload(ctx, ctx->nu, m->nu, (size_t)m->nlines);
    upload(ctx, ctx->cu, m->cu, (size_t)m->ncoll_tr);
    upload(ctx, ctx->cl, m->cl, (size_t)m->ncoll_tr);
    upload(ctx, ctx->K0, m->K0, (size_t)m->ncoll_tr);

    // ray pairs: (r, antipode r) with r < antipode
    std::vector<int32_t> pr, pa;
    std::vector<double> pw;
    for (int r = 0; r < R; r++)
        if (r < m->antipode[r]) {
            pr.push_back(r);
            pa.push_back(m->antipode[r]);
            pw.push_back(2.0 * m->ray_w[r]);
        }
    ctx->npairs = (int)pr.size();
    upload(ctx, ctx->pair_r, pr.data(), pr.size());
    upload(ctx, ctx->pair_a, pa.data(), pa.size());
    upload(ctx, ctx->pair_w, pw.data(), pw.size());

    ctx->b2.ensure(sizeof(double) * N);
    ctx->b.ensure(sizeof(double) * N);
    ctx->bf.ensure(sizeof(float) * N);
    ctx->ibf.ensure(sizeof(float) * N);
    ctx->bd.ensure(sizeof(double) * N);
    ctx->ibd.ensure(sizeof(double) * N);
    HIPCHK(launch_point_widths(N, ctx->T.as<double>(), ctx->vturb2.as<double>(), m->mass,
                               ctx->b2.as<double>(), ctx->b.as<double>(), ctx->bf.as<float>(),
                               ctx->ibf.as<float>(), ctx->bd.as<double>(), ctx->ibd.as<double>(),
                               ctx->stream));
    ctx->xf.ensure(sizeof(double) * m->nbins);
    ctx->W.ensure(sizeof(double) * m->nbins);
    HIPCHK(launch_bin_table(m->nbins, m->xmax, ctx->xf.as<double>(), ctx->W.as<double>(),
                            ctx->stream));
    const int nl = m->nlines;
    for (DMem *d : {&ctx->Bul, &ctx->Blu, &ctx->hnu4pi, &ctx->chiscale, &ctx->Iref, &ctx->acmb})
        d->ensure(sizeof(double) * nl);
    HIPCHK(launch_line_table(nl, m->nlev, ctx->A.as<double>(), ctx->nu.as<double>(),
                             ctx->g.as<double>(), ctx->up.as<int32_t>(), ctx->lo.as<int32_t>(),
                             ctx->L_unit, m->Tcmb, ctx->Bul.as<double>(), ctx->Blu.as<double>(),
                             ctx->hnu4pi.as<double>(), ctx->chiscale.as<double>(),
                             ctx->Iref.as<double>(), ctx->acmb.as<double>(), ctx->stream));
    const size_t tsz = ctx->fp32() ? sizeof(float) : sizeof(double);
    ctx->pops.ensure(sizeof(double) * ctx->npop());
    ctx->pops_new.ensure(sizeof(double) * ctx->npop());
    ctx->J.ensure(sizeof(double) * ctx->nrad());
    ctx->L.ensure(sizeof(double) * ctx->nrad());
    ctx->S64.ensure(sizeof(double) * ctx->nrad());
    ctx->chiT.ensure(tsz * ctx->nrad());
    ctx->ST.ensure(tsz * ctx->nrad());
    ctx->sync();
    ctx->loaded = true;
    ctx->host_cnt = mgx_counters{};
    API_END(ctx)
}

// ---------------------------------------------------------------------------
// Trace
// ---------------------------------------------------------------------------

extern "C" mgx_status mgx_trace_rays(mgx_ctx *ctx, int64_t *total_records_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->loaded, MGX_ESTATE, "mgx_trace_rays before mgx_load_model");
    const int64_t NW = (int64_t)ctx->N * ctx->R;
    ctx->counts.ensure(sizeof(int64_t) * (NW + 1));
    ctx->offsets.ensure(sizeof(int64_t) * (NW + 1));
    HIPCHK(hipMemsetAsync(ctx->counts.p, 0, sizeof(int64_t) * (NW + 1), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->counters.p, 0, sizeof(Counters), ctx->stream));
    TraceArgs a{};
    a.dim = ctx->dim;
    a.N = ctx->N;
    a.R = ctx->R;
    const double *pos = ctx->pos.as<double>(), *vel = ctx->vel.as<double>();
    a.x = pos;
    a.y = pos + ctx->N;
    a.z = pos + 2 * (size_t)ctx->N;
    a.vx = vel;
    a.vy = vel + ctx->N;
    a.vz = vel + 2 * (size_t)ctx->N;
    a.nbs_off = ctx->nbs_off.as<int32_t>();
    a.nbs = ctx->nbs.as<int32_t>();
    a.bdy = ctx->bdy.as<uint8_t>();
    a.ray_dir = ctx->ray_dir.as<double>();
    a.b2 = ctx->b2.as<double>();
    a.thr = ctx->opt.branch_threshold;
    a.counts = ctx->counts.as<int64_t>();
    a.cnt = ctx->counters.as<Counters>();
    HIPCHK(launch_trace(a, false, ctx->stream));
    HIPCHK(mgx_internal_scan(ctx->counts.as<int64_t>(), ctx->offsets.as<int64_t>(), NW + 1,
                             &ctx->scan_tmp, &ctx->scan_tmp_bytes, ctx->stream));
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, ctx->offsets.as<int64_t>() + NW, sizeof(int64_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    ctx->n_records = total;
    const size_t n = (size_t)(total > 0 ? total : 1);
    ctx->r_idx.ensure(sizeof(int32_t) * n);
    ctx->r_semi.ensure(n);
    ctx->r_Z.ensure(sizeof(double) * n);
    ctx->r_dv.ensure(sizeof(double) * n);
    ctx->r_dx.ensure(sizeof(double) * n);
    ctx->r_ibb.ensure(sizeof(double) * n);
    a.off = ctx->offsets.as<int64_t>();
    a.r_idx = ctx->r_idx.as<int32_t>();
    a.r_semi = ctx->r_semi.as<uint8_t>();
    a.r_Z = ctx->r_Z.as<double>();
    a.r_dv = ctx->r_dv.as<double>();
    a.r_dx = ctx->r_dx.as<double>();
    a.r_ibb = ctx->r_ibb.as<double>();
    HIPCHK(launch_trace(a, true, ctx->stream));
    const bool f32 = ctx->fp32();
    ctx->rec.ensure((f32 ? sizeof(Rec<float>) : sizeof(Rec<double>)) * n);
    HIPCHK(launch_pack_trace(total, ctx->r_idx.as<int32_t>(), ctx->r_semi.as<uint8_t>(),
                             ctx->r_dx.as<double>(), ctx->r_dv.as<double>(),
                             ctx->r_ibb.as<double>(), 1.0 / ctx->L_unit, f32, ctx->rec.p,
                             ctx->stream));
    Counters c = ctx->read_counters();
    ctx->host_cnt.total_records = total;
    ctx->host_cnt.holes = (int64_t)c.holes;
    ctx->host_cnt.semi_segments = (int64_t)c.semi;
    ctx->traced = true;
    if (total_records_out) *total_records_out = total;
    API_END(ctx)
}

extern "C" mgx_status mgx_get_trace_offsets(mgx_ctx *ctx, int64_t *offsets)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "no trace");
    REQUIRE(offsets, MGX_EINVAL, "offsets is NULL");
    const int64_t NW = (int64_t)ctx->N * ctx->R;
    HIPCHK(hipMemcpyAsync(offsets, ctx->offsets.p, sizeof(int64_t) * (NW + 1), hipMemcpyDefault,
                          ctx->stream));
    ctx->sync();
    API_END(ctx)
}

static void copy_records(mgx_ctx *ctx, int64_t first, int64_t count, int32_t *idx, double *Z,
                         double *dv, uint8_t *semi)
{
    if (count <= 0) return;
    if (idx)
        HIPCHK(hipMemcpyAsync(idx, ctx->r_idx.as<int32_t>() + first, sizeof(int32_t) * count,
                              hipMemcpyDefault, ctx->stream));
    if (Z)
        HIPCHK(hipMemcpyAsync(Z, ctx->r_Z.as<double>() + first, sizeof(double) * count,
                              hipMemcpyDefault, ctx->stream));
    if (dv)
        HIPCHK(hipMemcpyAsync(dv, ctx->r_dv.as<double>() + first, sizeof(double) * count,
                              hipMemcpyDefault, ctx->stream));
    if (semi)
        HIPCHK(hipMemcpyAsync(semi, ctx->r_semi.as<uint8_t>() + first, count, hipMemcpyDefault,
                              ctx->stream));
}

extern "C" mgx_status mgx_get_trace_records(mgx_ctx *ctx, int64_t first, int64_t count,
                                            int32_t *idx, double *Z, double *dv, uint8_t *semi)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "no trace");
    REQUIRE(first >= 0 && count >= 0 && first + count <= ctx->n_records, MGX_EINVAL,
            "record range out of bounds");
    copy_records(ctx, first, count, idx, Z, dv, semi);
    ctx->sync();
    API_END(ctx)
}

extern "C" mgx_status mgx_get_trace(mgx_ctx *ctx, int32_t origin, int32_t ray, int32_t cap,
                                    int32_t *idx, double *Z, double *dv, uint8_t *semi,
                                    int32_t *len_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "no trace");
    REQUIRE(origin >= 0 && origin < ctx->N && ray >= 0 && ray < ctx->R && cap >= 0, MGX_EINVAL,
            "origin/ray out of range");
    int64_t ab[2];
    const int64_t w = (int64_t)origin * ctx->R + ray;
    HIPCHK(hipMemcpyAsync(ab, ctx->offsets.as<int64_t>() + w, 2 * sizeof(int64_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    const int64_t len = ab[1] - ab[0];
    copy_records(ctx, ab[0], std::min<int64_t>(len, cap), idx, Z, dv, semi);
    ctx->sync();
    if (len_out) *len_out = (int32_t)len;
    API_END(ctx)
}

// ---------------------------------------------------------------------------
// Populations and radiation field
// ---------------------------------------------------------------------------

extern "C" mgx_status mgx_set_populations(mgx_ctx *ctx, const double *pops)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->loaded, MGX_ESTATE, "no model");
    REQUIRE(pops, MGX_EINVAL, "pops is NULL");
    HIPCHK(hipMemcpyAsync(ctx->pops.p, pops, sizeof(double) * ctx->npop(), hipMemcpyDefault,
                          ctx->stream));
    ctx->sync();
    ctx->have_pops = true;
    ctx->have_rad = false;
    API_END(ctx)
}

extern "C" mgx_status mgx_get_populations(mgx_ctx *ctx, double *pops)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->have_pops, MGX_ESTATE, "no populations");
    REQUIRE(pops, MGX_EINVAL, "pops is NULL");
    HIPCHK(hipMemcpyAsync(pops, ctx->pops.p, sizeof(double) * ctx->npop(), hipMemcpyDefault,
                          ctx->stream));
    ctx->sync();
    API_END(ctx)
}

extern "C" mgx_status mgx_set_lte_populations(mgx_ctx *ctx)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->loaded, MGX_ESTATE, "no model");
    HIPCHK(launch_lte(ctx->N, ctx->nlev, ctx->T.as<double>(), ctx->E.as<double>(),
                      ctx->g.as<double>(), ctx->pops.as<double>(), ctx->stream));
    ctx->sync();
    ctx->have_pops = true;
    ctx->have_rad = false;
    API_END(ctx)
}

static void run_line_coeffs(mgx_ctx *ctx)
{
    LineArgs la{};
    la.N = ctx->N;
    la.nlev = ctx->nlev;
    la.nlines = ctx->nlines;
    la.pops = ctx->pops.as<double>();
    la.nspec = ctx->nspec.as<double>();
    la.b = ctx->b.as<double>();
    la.up = ctx->up.as<int32_t>();
    la.lo = ctx->lo.as<int32_t>();
    la.A = ctx->A.as<double>();
    la.Bul = ctx->Bul.as<double>();
    la.Blu = ctx->Blu.as<double>();
    la.hnu4pi = ctx->hnu4pi.as<double>();
    la.chiscale = ctx->chiscale.as<double>();
    la.Iref = ctx->Iref.as<double>();
    la.chi_min = ctx->opt.chi_min;
    la.S64 = ctx->S64.as<double>();
    la.chiT = ctx->chiT.p;
    la.ST = ctx->ST.p;
    la.fp32 = ctx->fp32() ? 1 : 0;
    la.cnt = ctx->counters.as<Counters>();
    HIPCHK(launch_reset_counters(ctx->counters.as<Counters>(), ctx->stream));
    HIPCHK(launch_line_coeffs(la, ctx->stream));
}

// Launch shape of one model's formal solution: lines per chunk (balanced)
// and threads per workgroup (a multiple of 64 covering nlc * nbins).
template <typename T>
static FSArgs<T> fs_args(mgx_ctx *ctx)
{
    FSArgs<T> a{};
    a.N = ctx->N;
    a.R = ctx->R;
    a.npairs = ctx->npairs;
    a.nlines = ctx->nlines;
    a.nbins = ctx->nbins;
    const int max_threads = (sizeof(T) == 8 && ctx->nbins <= 512) ? 512 : kMaxBins;
    int nlc = std::max(1, max_threads / ctx->nbins);
    if (nlc > ctx->nlines) nlc = ctx->nlines;
    // balance the line chunks so the last one is not nearly empty
    const int nchunks = (ctx->nlines + nlc - 1) / nlc;
    nlc = (ctx->nlines + nchunks - 1) / nchunks;
    a.nlc = nlc;
    a.nthreads = ((nlc * ctx->nbins + 63) / 64) * 64;
    a.off = ctx->offsets.as<int64_t>();
    a.rec = (const Rec<T> *)ctx->rec.p;
    a.pair_r = ctx->pair_r.as<int32_t>();
    a.pair_a = ctx->pair_a.as<int32_t>();
    a.pair_w = ctx->pair_w.as<double>();
    a.chi = (const T *)ctx->chiT.p;
    a.S = (const T *)ctx->ST.p;
    if (sizeof(T) == 4) {
        a.bpt = (const T *)ctx->bf.p;
        a.ibpt = (const T *)ctx->ibf.p;
    } else {
        a.bpt = (const T *)ctx->bd.p;
        a.ibpt = (const T *)ctx->ibd.p;
    }
    a.b64 = ctx->b.as<double>();
    a.xf = ctx->xf.as<double>();
    a.W = ctx->W.as<double>();
    a.acmb = ctx->acmb.as<double>();
    a.Iref = ctx->Iref.as<double>();
    a.tau_floor = ctx->opt.tau_floor;
    a.J = ctx->J.as<double>();
    a.L = ctx->L.as<double>();
    return a;
}

template <typename T>
static void run_formal_solve_t(mgx_ctx *ctx)
{
    FSArgs<T> a = fs_args<T>(ctx);
    if (ctx->fs_pending) ctx->sync();  // previous launch's events must be read first
    HIPCHK(hipEventRecord(ctx->ev_fs0, ctx->stream));
    HIPCHK(launch_formal_solve<T>(a, ctx->stream));
    HIPCHK(hipEventRecord(ctx->ev_fs1, ctx->stream));
    ctx->fs_pending = true;
}

static void run_formal_solve(mgx_ctx *ctx)
{
    run_line_coeffs(ctx);
    if (ctx->fp32())
        run_formal_solve_t<float>(ctx);
    else
        run_formal_solve_t<double>(ctx);
}

extern "C" mgx_status mgx_formal_solve(mgx_ctx *ctx, double *Jbar, double *Lstar)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "mgx_formal_solve before mgx_trace_rays");
    REQUIRE(ctx->have_pops, MGX_ESTATE, "mgx_formal_solve without populations");
    run_formal_solve(ctx);
    if (Jbar)
        HIPCHK(hipMemcpyAsync(Jbar, ctx->J.p, sizeof(double) * ctx->nrad(), hipMemcpyDefault,
                              ctx->stream));
    if (Lstar)
        HIPCHK(hipMemcpyAsync(Lstar, ctx->L.p, sizeof(double) * ctx->nrad(), hipMemcpyDefault,
                              ctx->stream));
    Counters c = ctx->read_counters();
    ctx->host_cnt.masing = (int64_t)c.masing;
    ctx->have_rad = true;
    API_END(ctx)
}

extern "C" mgx_status mgx_set_radiation(mgx_ctx *ctx, const double *Jbar, const double *Lstar)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->have_pops, MGX_ESTATE, "mgx_set_radiation without populations");
    REQUIRE(Jbar && Lstar, MGX_EINVAL, "Jbar / Lstar is NULL");
    run_line_coeffs(ctx);  // source function of the current populations
    HIPCHK(hipMemcpyAsync(ctx->J.p, Jbar, sizeof(double) * ctx->nrad(), hipMemcpyDefault,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->L.p, Lstar, sizeof(double) * ctx->nrad(), hipMemcpyDefault,
                          ctx->stream));
    ctx->sync();
    ctx->have_rad = true;
    API_END(ctx)
}

// ---------------------------------------------------------------------------
// Statistical equilibrium and Ng
// ---------------------------------------------------------------------------

static DMem *ng_buffer(mgx_ctx *ctx)
{
    DMem *m = new DMem();
    ctx->ng_pool.push_back(m);
    m->ensure(sizeof(double) * ctx->npop());
    return m;
}

static void ng_append(mgx_ctx *ctx)
{
    if (ctx->ng_nh == ctx->ng_cap) {  // window full: drop the oldest iterate
        DMem *y0 = ctx->ng_y.front();
        ctx->ng_y.erase(ctx->ng_y.begin());
        ctx->ng_y.push_back(y0);
        DMem *r0 = ctx->ng_r.front();
        ctx->ng_r.erase(ctx->ng_r.begin());
        ctx->ng_r.push_back(r0);
        HIPCHK(launch_ng_shift(ctx->ng_nh - 1, ctx->ng_G.as<double>(), ctx->stream));
        ctx->ng_nh--;
    }
    const int nh = ctx->ng_nh;
    PtrTable rt{};
    for (int a = 0; a < nh - 1; a++) rt.p[a] = ctx->ng_r[a]->as<double>();
    HIPCHK(launch_ng_append(ctx->npop(), nh, ctx->pops.as<double>(),
                            ctx->ng_y[nh - 1]->as<double>(), ctx->ng_y[nh]->as<double>(),
                            ctx->ng_r[nh - 1]->as<double>(), rt, ctx->ng_partial.as<double>(),
                            ctx->ng_G.as<double>(), ctx->stream));
    ctx->ng_nh = nh + 1;
}

static void ng_restart(mgx_ctx *ctx)
{
    HIPCHK(launch_copy(ctx->npop(), ctx->pops.as<double>(), ctx->ng_y[0]->as<double>(),
                       ctx->stream));
    ctx->ng_nh = 1;
    ctx->ng_have_prev = false;
}

static StateqArgs stateq_args(mgx_ctx *ctx)
{
    StateqArgs s{};
    s.N = ctx->N;
    s.nlev = ctx->nlev;
    s.nlines = ctx->nlines;
    s.ncoll_tr = ctx->ncoll_tr;
    const size_t per_wave = sizeof(double) * ctx->nlev * (ctx->nlev + 1);
    s.wpb = (int)std::max<size_t>(1, std::min<size_t>(4, (48 * 1024) / per_wave));
    s.J = ctx->J.as<double>();
    s.L = ctx->L.as<double>();
    s.S64 = ctx->S64.as<double>();
    s.T = ctx->T.as<double>();
    s.ncoll = ctx->ncoll.as<double>();
    s.E = ctx->E.as<double>();
    s.g = ctx->g.as<double>();
    s.up = ctx->up.as<int32_t>();
    s.lo = ctx->lo.as<int32_t>();
    s.cu = ctx->cu.as<int32_t>();
    s.cl = ctx->cl.as<int32_t>();
    s.A = ctx->A.as<double>();
    s.Bul = ctx->Bul.as<double>();
    s.Blu = ctx->Blu.as<double>();
    s.K0 = ctx->K0.as<double>();
    s.pops_old = ctx->pops.as<double>();
    s.pops_new = ctx->pops_new.as<double>();
    s.pop_floor = ctx->opt.pop_floor;
    s.cnt = ctx->counters.as<Counters>();
    s.active = nullptr;
    s.model = 0;
    return s;
}

static mgx_status update_populations(mgx_ctx *ctx, double *change_out)
{
    StateqArgs s = stateq_args(ctx);
    HIPCHK(launch_reset_counters(ctx->counters.as<Counters>(), ctx->stream));
    HIPCHK(launch_stateq(s, ctx->stream));
    std::swap(ctx->pops.p, ctx->pops_new.p);
    std::swap(ctx->pops.bytes, ctx->pops_new.bytes);
    if (ctx->ng_active) ng_append(ctx);
    Counters c = ctx->read_counters();
    double change;
    memcpy(&change, &c.change_bits, sizeof(double));
    ctx->host_cnt.singular = (int64_t)c.singular;
    ctx->host_cnt.last_change = change;
    ctx->have_rad = false;
    if (change_out) *change_out = change;
    if (c.singular) {
        ctx->err = "singular statistical-equilibrium system at " + std::to_string(c.singular) +
                   " point(s)";
        return MGX_ESINGULAR;
    }
    if (c.nonfinite || !std::isfinite(change)) {
        ctx->err = "non-finite populations";
        return MGX_ENONFINITE;
    }
    return MGX_OK;
}

extern "C" mgx_status mgx_update_populations(mgx_ctx *ctx, double *max_rel_change_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->have_rad, MGX_ESTATE, "mgx_update_populations without a radiation field");
    mgx_status st = update_populations(ctx, max_rel_change_out);
    if (st != MGX_OK) return st;
    API_END(ctx)
}

static void ng_reset(mgx_ctx *ctx, int capacity)
{
    REQUIRE(capacity >= 2 && capacity <= kNgMaxHist, MGX_EINVAL, "Ng capacity must be 2..32");
    REQUIRE(ctx->have_pops, MGX_ESTATE, "Ng reset without populations");
    while ((int)ctx->ng_y.size() < capacity) ctx->ng_y.push_back(ng_buffer(ctx));
    while ((int)ctx->ng_r.size() < capacity) ctx->ng_r.push_back(ng_buffer(ctx));
    ctx->ng_G.ensure(sizeof(double) * kNgMaxHist * kNgMaxHist);
    ctx->ng_coef.ensure(sizeof(double) * kNgMaxHist);
    ctx->ng_status.ensure(sizeof(int) * 4);
    ctx->ng_partial.ensure(sizeof(double) * 1024 * kNgMaxHist);
    ctx->ng_pred.ensure(sizeof(double) * ctx->npop());
    ctx->ng_prev.ensure(sizeof(double) * ctx->npop());
    ctx->ng_bits.ensure(sizeof(unsigned long long) * 2);
    ctx->ng_cap = capacity;
    ctx->ng_active = true;
    ng_restart(ctx);
}

extern "C" mgx_status mgx_ng_reset(mgx_ctx *ctx, int capacity)
{
    API_BEGIN(ctx)
    ng_reset(ctx, capacity);
    ctx->sync();
    API_END(ctx)
}

// Forms the prediction into ng_prev (when accepted).  Returns 1 accepted.
static int ng_predict(mgx_ctx *ctx, double *pred_change)
{
    const int K = ctx->ng_nh - 1;
    *pred_change = INFINITY;
    if (K < 1) return 0;
    PtrTable yt{};
    for (int k = 0; k < K; k++) yt.p[k] = ctx->ng_y[k + 1]->as<double>();
    HIPCHK(hipMemsetAsync(ctx->ng_status.p, 0, sizeof(int) * 4, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->ng_bits.p, 0, sizeof(unsigned long long) * 2, ctx->stream));
    int *st = ctx->ng_status.as<int>();
    HIPCHK(launch_ng_predict(ctx->npop(), K, ctx->ng_G.as<double>(), yt,
                             ctx->ng_coef.as<double>(), st, ctx->ng_pred.as<double>(), st + 1,
                             ctx->stream));
    if (ctx->ng_have_prev)
        HIPCHK(launch_rel_change(ctx->npop(), ctx->ng_pred.as<double>(), ctx->ng_prev.as<double>(),
                                 ctx->opt.pop_floor, ctx->ng_bits.as<unsigned long long>(),
                                 ctx->stream));
    int hs[2];
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(hs, st, sizeof(int) * 2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(&bits, ctx->ng_bits.p, sizeof(bits), hipMemcpyDeviceToHost,
                          ctx->stream));
    ctx->sync();
    const bool ok = hs[0] == 0 && hs[1] == 0;
    if (ok) {
        if (ctx->ng_have_prev) memcpy(pred_change, &bits, sizeof(double));
        std::swap(ctx->ng_pred.p, ctx->ng_prev.p);
        std::swap(ctx->ng_pred.bytes, ctx->ng_prev.bytes);
        ctx->ng_have_prev = true;
    }
    return ok ? 1 : 0;
}

static void ng_apply(mgx_ctx *ctx, bool accepted)
{
    if (accepted) {
        HIPCHK(launch_copy(ctx->npop(), ctx->ng_prev.as<double>(), ctx->pops.as<double>(),
                           ctx->stream));
        ctx->host_cnt.ng_applied++;
    } else {
        ctx->host_cnt.ng_rejected++;
    }
    ng_restart(ctx);
}

extern "C" mgx_status mgx_ng_accelerate(mgx_ctx *ctx, int apply, int *status_out,
                                        double *pred_change_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->ng_active, MGX_ESTATE, "mgx_ng_accelerate without mgx_ng_reset");
    double pc = INFINITY;
    const int ok = ng_predict(ctx, &pc);
    if (apply) ng_apply(ctx, ok != 0);
    ctx->sync();
    if (status_out) *status_out = ok;
    if (pred_change_out) *pred_change_out = pc;
    API_END(ctx)
}

extern "C" mgx_status mgx_iterate(mgx_ctx *ctx, double tol, int max_iter, int ng_mode,
                                  int ng_param, int *iters_out, double *final_change_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "mgx_iterate before mgx_trace_rays");
    REQUIRE(ctx->have_pops, MGX_ESTATE, "mgx_iterate without populations");
    REQUIRE(max_iter >= 1 && tol >= 0, MGX_EINVAL, "max_iter >= 1 and tol >= 0 required");
    REQUIRE(ng_mode == MGX_NG_NONE || ng_mode == MGX_NG_CLASSICAL || ng_mode == MGX_NG_ADAPTIVE,
            MGX_EINVAL, "unknown ng_mode");
    ctx->ng_active = false;
    if (ng_mode == MGX_NG_CLASSICAL) {
        REQUIRE(ng_param >= 1 && ng_param + 1 <= kNgMaxHist, MGX_EINVAL,
                "classical Ng order must be 1..31");
        ng_reset(ctx, ng_param + 1);
    } else if (ng_mode == MGX_NG_ADAPTIVE) {
        REQUIRE(ng_param >= 3 && ng_param <= kNgMaxHist, MGX_EINVAL,
                "adaptive Ng N_max must be 3..32");
        ng_reset(ctx, ng_param);
    }
    ctx->host_cnt.ng_applied = ctx->host_cnt.ng_rejected = 0;
    double change = INFINITY;
    int it = 0;
    mgx_status result = MGX_ENOCONV;
    for (it = 1; it <= max_iter; it++) {
        run_formal_solve(ctx);
        ctx->have_rad = true;
        const mgx_status st = update_populations(ctx, &change);
        if (st != MGX_OK) {
            result = st;
            break;
        }
        if (change <= tol) {
            result = MGX_OK;
            break;
        }
        if (ng_mode == MGX_NG_CLASSICAL) {
            if (ctx->ng_nh == ng_param + 1) {
                double pc;
                ng_apply(ctx, ng_predict(ctx, &pc) != 0);
            }
        } else if (ng_mode == MGX_NG_ADAPTIVE) {
            bool use = false;
            if (ctx->ng_nh >= 3) {
                double pc;
                const int ok = ng_predict(ctx, &pc);
                use = ok && (pc < change || ctx->ng_nh >= ng_param);
            }
            if (use) {
                ng_apply(ctx, true);
            } else if (ctx->ng_nh >= ng_param) {
                ng_apply(ctx, false);
            }
        }
    }
    if (it > max_iter) it = max_iter;
    ctx->ng_active = false;
    ctx->host_cnt.iterations = it;
    ctx->host_cnt.last_change = change;
    if (iters_out) *iters_out = it;
    if (final_change_out) *final_change_out = change;
    ctx->sync();
    if (result == MGX_ENOCONV)
        ctx->err = "no convergence within max_iter (last change " + std::to_string(change) + ")";
    if (result != MGX_OK) return result;
    API_END(ctx)
}

extern "C" mgx_status mgx_get_counters(mgx_ctx *ctx, mgx_counters *out)
{
    API_BEGIN(ctx)
    REQUIRE(out, MGX_EINVAL, "out is NULL");
    ctx->sync();
    *out = ctx->host_cnt;
    API_END(ctx)
}

extern "C" mgx_status mgx_reset_timers(mgx_ctx *ctx)
{
    API_BEGIN(ctx)
    ctx->sync();
    ctx->host_cnt.fs_launches = 0;
    ctx->host_cnt.fs_ms_total = 0.0;
    ctx->host_cnt.fs_ms_last = 0.0;
    API_END(ctx)
}

// Image basis: d = dir / |dir|, e1 = unit(a x d) with a = z (x when
// |d_z| > 0.9), e2 = d x e1; plain double arithmetic, no contraction.
static void render_basis(const double dir[3], double d[3], double e1[3], double e2[3])
{
#pragma clang fp contract(off)
    const double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    d[0] = dir[0] / n;
    d[1] = dir[1] / n;
    d[2] = dir[2] / n;
    double a[3] = {0.0, 0.0, 1.0};
    if (fabs(d[2]) > 0.9) {
        a[0] = 1.0;
        a[2] = 0.0;
    }
    const double c[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2],
                         a[0] * d[1] - a[1] * d[0]};
    const double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    e1[0] = c[0] / cn;
    e1[1] = c[1] / cn;
    e1[2] = c[2] / cn;
    e2[0] = d[1] * e1[2] - d[2] * e1[1];
    e2[1] = d[2] * e1[0] - d[0] * e1[2];
    e2[2] = d[0] * e1[1] - d[1] * e1[0];
}

extern "C" mgx_status mgx_render_image(mgx_ctx *ctx, const double dir[3], int npx, int npy,
                                       double f_min, double f_max, int nfreq, float *img)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->loaded && ctx->have_pops, MGX_ESTATE, "mgx_render_image needs a model and populations");
    REQUIRE(ctx->dim == 3, MGX_EINVAL, "mgx_render_image supports point clouds (dim 3)");
    REQUIRE(dir && img, MGX_EINVAL, "dir / img is NULL");
    REQUIRE(std::isfinite(dir[0]) && std::isfinite(dir[1]) && std::isfinite(dir[2]) &&
                (dir[0] != 0.0 || dir[1] != 0.0 || dir[2] != 0.0),
            MGX_EINVAL, "dir must be finite and non-zero");
    REQUIRE(npx >= 1 && npy >= 1 && (int64_t)npx * npy <= (1 << 26), MGX_EINVAL,
            "pixel counts out of range");
    REQUIRE(nfreq >= 1 && nfreq <= 1024, MGX_EINVAL, "nfreq must be 1..1024");
    REQUIRE(f_min > 0 && f_max >= f_min && std::isfinite(f_max), MGX_EINVAL,
            "need 0 < f_min <= f_max");
    run_line_coeffs(ctx);
    const int N = ctx->N;
    const int64_t npix = (int64_t)npx * npy;
    RenderGeom g{};
    g.N = N;
    g.npx = npx;
    g.npy = npy;
    render_basis(dir, g.d, g.e1, g.e2);
    g.h = ctx->L_unit;
    const double *pos = ctx->pos.as<double>(), *vel = ctx->vel.as<double>();
    g.x = pos;
    g.y = pos + N;
    g.z = pos + 2 * (size_t)N;
    g.vx = vel;
    g.vy = vel + N;
    g.vz = vel + 2 * (size_t)N;
    g.nbs_off = ctx->nbs_off.as<int32_t>();
    g.nbs = ctx->nbs.as<int32_t>();
    g.bdy = ctx->bdy.as<uint8_t>();
    ctx->rg_proj.ensure(sizeof(double) * 4 * (size_t)N + sizeof(double) * 4);
    g.u = ctx->rg_proj.as<double>();
    g.v = g.u + N;
    g.Z = g.v + N;
    g.w = g.Z + N;
    g.ext = g.w + N;
    ctx->rg_pix.ensure((sizeof(unsigned long long) + sizeof(int32_t)) * npix + 16);
    g.key = ctx->rg_pix.as<unsigned long long>();
    g.entry = (int32_t *)(g.key + npix);
    ctx->rg_off.ensure(sizeof(int64_t) * 2 * (npix + 1));
    g.counts = ctx->rg_off.as<int64_t>();
    int64_t *off = g.counts + (npix + 1);
    HIPCHK(hipMemsetAsync(g.counts, 0, sizeof(int64_t) * (npix + 1), ctx->stream));
    HIPCHK(launch_render_geometry(g, ctx->stream));
    HIPCHK(launch_render_walk(g, false, ctx->stream));
    HIPCHK(mgx_internal_scan(g.counts, off, npix + 1, &ctx->scan_tmp, &ctx->scan_tmp_bytes,
                             ctx->stream));
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, off + npix, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    ctx->rg_walk.ensure(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    g.off = off;
    g.walk = ctx->rg_walk.as<int32_t>();
    HIPCHK(launch_render_walk(g, true, ctx->stream));
    ctx->rg_img.ensure(sizeof(float) * (size_t)npix * nfreq);
    const double I_img = 2.0 * kH * pow(0.5 * (f_min + f_max), 3) / (kC * kC);
    auto fill_args = [&](auto &ra) {
        ra.npx = npx;
        ra.npy = npy;
        ra.nfreq = nfreq;
        ra.nlines = ctx->nlines;
        ra.off = off;
        ra.walk = g.walk;
        ra.Z = g.Z;
        ra.w = g.w;
        ra.b = ctx->bd.as<double>();
        ra.ib = ctx->ibd.as<double>();
        ra.nu_line = ctx->nu.as<double>();
        ra.Iref = ctx->Iref.as<double>();
        ra.inv_L = 1.0 / ctx->L_unit;
        ra.f_min = f_min;
        ra.f_max = f_max;
        ra.Tcmb = ctx->Tcmb;
        ra.I_img = I_img;
        ra.thr = ctx->opt.branch_threshold;
        ra.b2 = ctx->b2.as<double>();
        ra.img = ctx->rg_img.as<float>();
    };
    if (ctx->fp32()) {
        RenderArgs<float> ra{};
        fill_args(ra);
        ra.chi = (const float *)ctx->chiT.p;
        ra.S = (const float *)ctx->ST.p;
        HIPCHK(launch_render_integrate<float>(ra, ctx->stream));
    } else {
        RenderArgs<double> ra{};
        fill_args(ra);
        ra.chi = (const double *)ctx->chiT.p;
        ra.S = (const double *)ctx->ST.p;
        HIPCHK(launch_render_integrate<double>(ra, ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(img, ctx->rg_img.p, sizeof(float) * (size_t)npix * nfreq,
                          hipMemcpyDefault, ctx->stream));
    ctx->sync();
    API_END(ctx)
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

struct mgx_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mgx_options opt{};
    std::string err;
    std::vector<mgx_ctx *> m;
    bool prepared = false, tuned = false;
    // device tables
    DMem descs, active, changes, cnt_ptrs, counts, tune_count;
    // work items per class: every item in longest-first order, and the items
    // of the models still iterating (same order; *counts[k] of them)
    DMem items_all[MGX_BATCH_CLASSES], items[MGX_BATCH_CLASSES];
    DMem sample[MGX_BATCH_CLASSES];  // strided sample of the items, for tuning
    int class_nsample[MGX_BATCH_CLASSES] = {};
    void *select_tmp = nullptr;
    size_t select_tmp_bytes = 0;
    int nclass = 0;
    // lane class k: workgroups of 64 (k + 1) threads
    int class_threads[MGX_BATCH_CLASSES] = {};
    int class_nitems[MGX_BATCH_CLASSES] = {};
    int class_nlc_max[MGX_BATCH_CLASSES] = {};
    int class_ch[MGX_BATCH_CLASSES] = {};
    int64_t work_items = 0;
    std::vector<int> host_active;
    // one iteration as three captured graphs: line coefficients, formal
    // solution (timed with events between the launches), populations
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    mgx_batch_stats st{};

    ~mgx_batch()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        for (int i = 0; i < 3; i++) {
            if (gexec[i]) (void)hipGraphExecDestroy(gexec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
        }
        for (mgx_ctx *c : m) delete c;
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (select_tmp) (void)hipFree(select_tmp);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    bool fp32() const { return opt.precision == MGX_FP32; }
    void sync() { HIPCHK(hipStreamSynchronize(stream)); }
};

#define BATCH_BEGIN(b)                                                                    \
    if (!(b)) return MGX_EINVAL;                                                          \
    try {                                                                                 \
        DeviceGuard dg_((b)->device);                                                     \
        (b)->err.clear();

#define BATCH_END(b)                                                                      \
    }                                                                                     \
    catch (const Err &e)                                                                  \
    {                                                                                     \
        (b)->err = e.msg;                                                                 \
        return e.st;                                                                      \
    }                                                                                     \
    catch (const std::bad_alloc &)                                                        \
    {                                                                                     \
        (b)->err = "host allocation failed";                                              \
        return MGX_ENOMEM;                                                                \
    }                                                                                     \
    catch (...)                                                                           \
    {                                                                                     \
        (b)->err = "unexpected internal error";                                           \
        return MGX_EHIP;                                                                  \
    }                                                                                     \
    return MGX_OK;

static void check_sub(mgx_batch *b, mgx_ctx *c, mgx_status st)
{
    if (st != MGX_OK) throw Err{st, c->err};
    (void)b;
}

extern "C" mgx_status mgx_batch_create(mgx_batch **out, int device, void *stream,
                                       const mgx_options *opt)
{
    g_create_error.clear();
    if (!out) return MGX_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_create_error = "no such HIP device";
        return MGX_EINVAL;
    }
    mgx_options o;
    mgx_default_options(&o);
    if (opt) o = *opt;
    mgx_batch *b = new (std::nothrow) mgx_batch();
    if (!b) return MGX_ENOMEM;
    b->device = device;
    b->opt = o;
    try {
        DeviceGuard dg(device);
        if (stream) {
            b->stream = (hipStream_t)stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        HIPCHK(hipEventCreate(&b->ev0));
        HIPCHK(hipEventCreate(&b->ev1));
    } catch (const Err &e) {
        g_create_error = e.msg;
        delete b;
        return e.st;
    }
    *out = b;
    return MGX_OK;
}

extern "C" void mgx_batch_destroy(mgx_batch *b)
{
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    delete b;
    if (prev >= 0) (void)hipSetDevice(prev);
}

extern "C" const char *mgx_batch_last_error(const mgx_batch *b)
{
    if (!b) return g_create_error.c_str();
    return b->err.c_str();
}

extern "C" mgx_status mgx_batch_add_model(mgx_batch *b, const mgx_model *model, int *id_out)
{
    BATCH_BEGIN(b)
    REQUIRE(!b->prepared, MGX_ESTATE, "mgx_batch_add_model after mgx_batch_prepare");
    mgx_ctx *c = nullptr;
    const mgx_status st = mgx_create(&c, b->device, b->stream, &b->opt);
    if (st != MGX_OK) throw Err{st, g_create_error};
    const mgx_status ls = mgx_load_model(c, model);
    if (ls != MGX_OK) {
        Err e{ls, c->err};
        delete c;
        throw e;
    }
    b->m.push_back(c);
    if (id_out) *id_out = (int)b->m.size() - 1;
    BATCH_END(b)
}

template <typename T>
static void batch_build_tables(mgx_batch *b)
{
    const int M = (int)b->m.size();
    std::vector<FSArgs<T>> d(M);
    std::vector<std::vector<std::pair<int64_t, int4>>> cls(MGX_BATCH_CLASSES);
    DMem cost;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        b->class_threads[k] = 64 * (k + 1);
        b->class_nlc_max[k] = 0;
        b->class_ch[k] = 64;
    }
    for (int i = 0; i < M; i++) {
        mgx_ctx *c = b->m[i];
        d[i] = fs_args<T>(c);
        // a model's workgroup size is a multiple of 64 up to 1024
        const int k = d[i].nthreads / 64 - 1;
        b->class_nlc_max[k] = std::max(b->class_nlc_max[k], d[i].nlc);
        cost.ensure(sizeof(int64_t) * c->N);
        HIPCHK(launch_origin_cost(c->N, c->R, c->offsets.as<int64_t>(), cost.as<int64_t>(),
                                  b->stream));
        std::vector<int64_t> hc(c->N);
        HIPCHK(hipMemcpyAsync(hc.data(), cost.p, sizeof(int64_t) * c->N, hipMemcpyDeviceToHost,
                              b->stream));
        b->sync();
        const int nchunks = (c->nlines + d[i].nlc - 1) / d[i].nlc;
        const int64_t lanes = (int64_t)d[i].nlc * c->nbins;
        for (int o = 0; o < c->N; o++)
            for (int ch = 0; ch < nchunks; ch++)
                cls[k].push_back({(hc[o] + c->npairs) * lanes, make_int4(i, o, ch, 0)});
    }
    upload(b->m[0], b->descs, d.data(), d.size());
    b->st.updates_per_iteration = b->st.lane_records = b->st.lane_semi = 0;
    b->st.lane_origin_pairs = 0;
    for (mgx_ctx *c : b->m) {
        const int64_t lanes = (int64_t)c->nlines * c->nbins;
        b->st.updates_per_iteration += (int64_t)c->N * c->R * lanes;
        b->st.lane_records += lanes * c->host_cnt.total_records;
        b->st.lane_semi += lanes * c->host_cnt.semi_segments;
        b->st.lane_origin_pairs += lanes * c->N * c->npairs;
    }
    b->work_items = 0;
    b->nclass = 0;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        auto &v = cls[k];
        std::stable_sort(v.begin(), v.end(),
                         [](const std::pair<int64_t, int4> &x, const std::pair<int64_t, int4> &y) {
                             return x.first > y.first;
                         });
        std::vector<int4> it(v.size());
        for (size_t j = 0; j < v.size(); j++) it[j] = v[j].second;
        b->class_nitems[k] = (int)it.size();
        b->work_items += (int64_t)it.size();
        if (!it.empty()) b->nclass++;
        upload(b->m[0], b->items_all[k], it.data(), it.size());
        b->items[k].ensure(sizeof(int4) * std::max<size_t>(1, it.size()));
        const size_t stride = it.size() >= 32768 ? 8 : 1;
        std::vector<int4> smp;
        for (size_t j = 0; j < it.size(); j += stride) smp.push_back(it[j]);
        b->class_nsample[k] = (int)smp.size();
        upload(b->m[0], b->sample[k], smp.data(), smp.size());
    }
    b->counts.ensure(sizeof(int) * MGX_BATCH_CLASSES);
    b->tune_count.ensure(sizeof(int));
    b->sync();
}

extern "C" mgx_status mgx_batch_prepare(mgx_batch *b)
{
    BATCH_BEGIN(b)
    REQUIRE(!b->m.empty(), MGX_ESTATE, "mgx_batch_prepare on an empty batch");
    REQUIRE(!b->prepared, MGX_ESTATE, "batch already prepared");
    const int M = (int)b->m.size();
    for (mgx_ctx *c : b->m) {
        check_sub(b, c, mgx_trace_rays(c, nullptr));
        // iterations read only the packed records: drop the raw trace
        c->r_idx.release();
        c->r_semi.release();
        c->r_Z.release();
        c->r_dv.release();
        c->r_dx.release();
        c->r_ibb.release();
        c->counts.release();
    }
    if (b->fp32())
        batch_build_tables<float>(b);
    else
        batch_build_tables<double>(b);
    std::vector<Counters *> cp(M);
    for (int i = 0; i < M; i++) cp[i] = b->m[i]->counters.as<Counters>();
    upload(b->m[0], b->cnt_ptrs, cp.data(), cp.size());
    b->host_active.assign(M, 1);
    upload(b->m[0], b->active, b->host_active.data(), (size_t)M);
    b->changes.ensure(sizeof(double) * 2 * M);
    b->sync();
    b->prepared = true;
    BATCH_END(b)
}

extern "C" mgx_status mgx_batch_set_lte_populations(mgx_batch *b)
{
    BATCH_BEGIN(b)
    for (mgx_ctx *c : b->m) check_sub(b, c, mgx_set_lte_populations(c));
    BATCH_END(b)
}

extern "C" mgx_status mgx_batch_set_populations(mgx_batch *b, int id, const double *pops)
{
    BATCH_BEGIN(b)
    REQUIRE(id >= 0 && id < (int)b->m.size(), MGX_EINVAL, "model id out of range");
    check_sub(b, b->m[id], mgx_set_populations(b->m[id], pops));
    BATCH_END(b)
}

extern "C" mgx_status mgx_batch_get_populations(mgx_batch *b, int id, double *pops)
{
    BATCH_BEGIN(b)
    REQUIRE(id >= 0 && id < (int)b->m.size(), MGX_EINVAL, "model id out of range");
    check_sub(b, b->m[id], mgx_get_populations(b->m[id], pops));
    BATCH_END(b)
}

// All items of every class in play again (start of an iterate call).
static void batch_restore_items(mgx_batch *b)
{
    for (int k = 0; k < MGX_BATCH_CLASSES; k++)
        if (b->class_nitems[k])
            HIPCHK(hipMemcpyAsync(b->items[k].p, b->items_all[k].p,
                                  sizeof(int4) * b->class_nitems[k], hipMemcpyDeviceToDevice,
                                  b->stream));
    HIPCHK(hipMemcpyAsync(b->counts.p, b->class_nitems, sizeof(int) * MGX_BATCH_CLASSES,
                          hipMemcpyHostToDevice, b->stream));
    b->sync();
}

// Keep only the items of models still iterating (after the mask changed).
static void batch_compact_items(mgx_batch *b)
{
    for (int k = 0; k < MGX_BATCH_CLASSES; k++)
        if (b->class_nitems[k])
            HIPCHK(launch_compact_items(b->items_all[k].as<int4>(), b->class_nitems[k],
                                        b->items[k].as<int4>(), b->counts.as<int>() + k,
                                        b->active.as<int>(), &b->select_tmp,
                                        &b->select_tmp_bytes, b->stream));
}

template <typename T>
static void batch_launch_class(mgx_batch *b, int k, const int4 *items, const int *count,
                               int blocks, int ch)
{
    const size_t lds = formal_solve_lds<T>(ch, b->class_nlc_max[k], b->class_threads[k]);
    HIPCHK(launch_formal_solve_batch<T>((const FSArgs<T> *)b->descs.p, items, count, blocks,
                                        b->active.as<int>(), ch, b->class_threads[k], lds,
                                        b->stream));
}

// Schedule tuning: per lane class, time each LDS chunk size (records staged
// per half-ray) on a strided sample of the class's items and keep the
// fastest.
template <typename T>
static void batch_tune(mgx_batch *b)
{
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        const int n = b->class_nitems[k];
        if (n == 0) continue;
        const int nlc = b->class_nlc_max[k], nth = b->class_threads[k];
        // the largest chunk that fits 60 KB (at least 8, as the single-model
        // launch does) and every smaller candidate
        int chmax = 64;
        while (formal_solve_lds<T>(chmax, nlc, nth) > 60 * 1024 && chmax > 8) chmax /= 2;
        REQUIRE(formal_solve_lds<T>(chmax, nlc, nth) <= 160 * 1024, MGX_EINVAL,
                "line chunk does not fit the LDS");
        const int ns = b->class_nsample[k];
        HIPCHK(hipMemcpyAsync(b->tune_count.p, &ns, sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
        float best = INFINITY;
        for (int ch : {8, 16, 32, 64}) {
            if (ch > chmax || (ch == 8 && chmax > 8)) continue;
            HIPCHK(hipEventRecord(b->ev0, b->stream));
            batch_launch_class<T>(b, k, b->sample[k].as<int4>(), b->tune_count.as<int>(), ns, ch);
            HIPCHK(hipEventRecord(b->ev1, b->stream));
            b->sync();
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            if (ms < best) {
                best = ms;
                b->class_ch[k] = ch;
            }
        }
    }
}

// One Lambda-iteration of every model, captured once as three HIP graphs.
static void batch_capture_part(mgx_batch *b, int part, const std::function<void()> &body)
{
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    try {
        body();
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    HIPCHK(hipStreamEndCapture(b->stream, &b->graph[part]));
    HIPCHK(hipGraphInstantiate(&b->gexec[part], b->graph[part], nullptr, nullptr, 0));
}

template <typename T>
static void batch_capture(mgx_batch *b)
{
    const int M = (int)b->m.size();
    batch_capture_part(b, 0, [&]() {
        for (mgx_ctx *c : b->m) run_line_coeffs(c);
    });
    batch_capture_part(b, 1, [&]() {
        for (int k = 0; k < MGX_BATCH_CLASSES; k++)
            if (b->class_nitems[k])
                batch_launch_class<T>(b, k, b->items[k].as<int4>(), b->counts.as<int>() + k,
                                      b->class_nitems[k], b->class_ch[k]);
    });
    batch_capture_part(b, 2, [&]() {
        for (int i = 0; i < M; i++) {
            mgx_ctx *c = b->m[i];
            StateqArgs s = stateq_args(c);
            s.active = b->active.as<int>();
            s.model = i;
            HIPCHK(launch_reset_counters(c->counters.as<Counters>(), b->stream));
            HIPCHK(launch_stateq(s, b->stream));
            HIPCHK(launch_copy_if_active(c->npop(), c->pops_new.as<double>(), c->pops.as<double>(),
                                         b->active.as<int>(), i, b->stream));
        }
        HIPCHK(launch_gather_changes(M, b->cnt_ptrs.as<Counters *>(), b->changes.as<double>(),
                                     b->stream));
    });
}

extern "C" mgx_status mgx_batch_iterate(mgx_batch *b, double tol, int max_iter, int ng_order,
                                        int *iters, double *changes, int *converged_out)
{
    BATCH_BEGIN(b)
    REQUIRE(b->prepared, MGX_ESTATE, "mgx_batch_iterate before mgx_batch_prepare");
    REQUIRE(max_iter >= 1 && tol >= 0, MGX_EINVAL, "max_iter >= 1 and tol >= 0 required");
    REQUIRE(ng_order >= 0 && ng_order + 1 <= kNgMaxHist, MGX_EINVAL, "Ng order must be 0..31");
    const int M = (int)b->m.size();
    for (mgx_ctx *c : b->m) REQUIRE(c->have_pops, MGX_ESTATE, "batch model without populations");
    auto wall = []() {
        struct timespec ts;
        clock_gettime(CLOCK_MONOTONIC, &ts);
        return ts.tv_sec + 1e-9 * ts.tv_nsec;
    };
    batch_restore_items(b);
    if (!b->tuned) {
        const double t0 = wall();
        for (mgx_ctx *c : b->m) run_line_coeffs(c);
        if (b->fp32())
            batch_tune<float>(b);
        else
            batch_tune<double>(b);
        b->st.tune_seconds = wall() - t0;
        if (b->fp32())
            batch_capture<float>(b);
        else
            batch_capture<double>(b);
        b->tuned = true;
    }
    const double t0 = wall();
    b->st.fs_launches = 0;
    b->st.fs_ms_total = b->st.fs_ms_last = 0.0;
    for (mgx_ctx *c : b->m) {
        c->ng_active = false;
        if (ng_order > 0) ng_reset(c, ng_order + 1);
    }
    b->host_active.assign(M, 1);
    HIPCHK(hipMemcpyAsync(b->active.p, b->host_active.data(), sizeof(int) * M,
                          hipMemcpyHostToDevice, b->stream));
    std::vector<double> ch(M, INFINITY);
    std::vector<int> its(M, 0);
    int n_active = M, it = 0;
    mgx_status result = MGX_OK;
    for (it = 1; it <= max_iter && n_active > 0; it++) {
        HIPCHK(hipGraphLaunch(b->gexec[0], b->stream));
        HIPCHK(hipEventRecord(b->ev0, b->stream));
        HIPCHK(hipGraphLaunch(b->gexec[1], b->stream));
        HIPCHK(hipEventRecord(b->ev1, b->stream));
        HIPCHK(hipGraphLaunch(b->gexec[2], b->stream));
        std::vector<double> hc(2 * M);
        HIPCHK(hipMemcpyAsync(hc.data(), b->changes.p, sizeof(double) * 2 * M,
                              hipMemcpyDeviceToHost, b->stream));
        b->sync();
        float fs_ms = 0.f;
        HIPCHK(hipEventElapsedTime(&fs_ms, b->ev0, b->ev1));
        b->st.fs_ms_last = fs_ms;
        b->st.fs_ms_total += fs_ms;
        b->st.fs_launches++;
        bool mask_changed = false;
        for (int i = 0; i < M; i++) {
            if (!b->host_active[i]) continue;
            its[i] = it;
            ch[i] = hc[i];
            const bool failed = hc[M + i] != 0.0 || !std::isfinite(hc[i]);
            if (failed && result == MGX_OK) {
                const bool sing = hc[M + i] == 1.0;
                result = sing ? MGX_ESINGULAR : MGX_ENONFINITE;
                b->err = std::string(sing ? "singular statistical equilibrium"
                                          : "non-finite populations") +
                         " in model " + std::to_string(i);
            }
            if (hc[i] <= tol || failed) {
                b->host_active[i] = 0;
                mask_changed = true;
                n_active--;
                continue;
            }
            if (ng_order > 0) {
                mgx_ctx *c = b->m[i];
                ng_append(c);
                if (c->ng_nh == ng_order + 1) {
                    double pc;
                    ng_apply(c, ng_predict(c, &pc) != 0);
                }
            }
        }
        if (mask_changed) {
            HIPCHK(hipMemcpyAsync(b->active.p, b->host_active.data(), sizeof(int) * M,
                                  hipMemcpyHostToDevice, b->stream));
            if (n_active > 0) batch_compact_items(b);
        }
    }
    b->sync();
    for (mgx_ctx *c : b->m) c->ng_active = false;
    b->st.iterate_seconds = wall() - t0;
    b->st.iterations = it - 1;
    b->st.active = n_active;
    if (iters)
        for (int i = 0; i < M; i++) iters[i] = its[i];
    if (changes)
        for (int i = 0; i < M; i++) changes[i] = ch[i];
    if (converged_out) *converged_out = M - n_active;
    if (result == MGX_OK && n_active > 0) {
        result = MGX_ENOCONV;
        b->err = std::to_string(n_active) + " model(s) did not converge within max_iter";
    }
    if (result != MGX_OK) return result;
    BATCH_END(b)
}

extern "C" mgx_status mgx_batch_get_stats(mgx_batch *b, mgx_batch_stats *out)
{
    BATCH_BEGIN(b)
    REQUIRE(out, MGX_EINVAL, "out is NULL");
    b->st.models = (int)b->m.size();
    b->st.lane_classes = b->nclass;
    b->st.work_items = b->work_items;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        b->st.class_items[k] = b->class_nitems[k];
        b->st.class_threads[k] = b->class_nitems[k] ? b->class_threads[k] : 0;
        b->st.class_chunk[k] = b->class_nitems[k] ? b->class_ch[k] : 0;
    }
    *out = b->st;
    BATCH_END(b)
}
