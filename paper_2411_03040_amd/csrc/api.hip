// C ABI of the library: context, device memory, model validation and the
// iteration driver.  All arithmetic of the method runs in the kernels of
// trace.hip, formal_solve.hip, stateq.hip, ng.hip and render.hip; this file
// only moves data, checks arguments and sequences launches on the context's
// stream.

#include <algorithm>
#include <new>
#include <utility>

#include "host.h"

thread_local std::string mgxh::g_create_error;

// ---------------------------------------------------------------------------

extern "C" void mgx_default_options(mgx_options *opt)
{
    if (!opt) return;
    opt->precision = MGX_FP32;
    opt->branch_threshold = 0.35;
    opt->tau_floor = 1e-15;
    opt->chi_min = 1e-30;
    opt->pop_floor = 1e-12;
    opt->trace_slot_min_bytes = int64_t(4) << 30;
}

// The semi-analytic form needs segments with a shift of at least
// MGX_MIN_BRANCH_THRESHOLD widths (its divided difference and the
// opposite-sign erf difference lose precision as the shift goes to 0).
bool mgxh::options_valid(const mgx_options &o)
{
    return (o.precision == MGX_FP32 || o.precision == MGX_FP64) &&
           o.branch_threshold >= MGX_MIN_BRANCH_THRESHOLD && std::isfinite(o.branch_threshold) &&
           o.tau_floor > 0 && o.chi_min > 0 && o.pop_floor > 0;
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
    mgx_options o;
    mgx_default_options(&o);
    if (opt) o = *opt;
    if (!options_valid(o)) {
        g_create_error = "invalid options";
        return MGX_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_create_error = "no such HIP device";
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

    // Origins in Morton order of their positions -- kept only where the
    // formal solution uses it: when the line table (chi' and S' in the solve
    // precision) outgrows one XCD's 4 MB L2.
    ctx->order.release();
    const size_t table = (size_t)N * m->nlines * 2 * (ctx->fp32() ? sizeof(float) : sizeof(double));
    if (table > ((size_t)4 << 20)) {
        const std::vector<int32_t> ord = morton_order(m->pos, N);
        upload(ctx, ctx->order, ord.data(), ord.size());
        ctx->sync();
    }
    upload(ctx, ctx->pos, m->pos, 3 * (size_t)N);
    {
        std::vector<double> p4(4 * (size_t)N);
        for (int i = 0; i < N; i++) {
            p4[4 * (size_t)i + 0] = m->pos[i];
            p4[4 * (size_t)i + 1] = m->pos[(size_t)N + i];
            p4[4 * (size_t)i + 2] = m->pos[2 * (size_t)N + i];
            p4[4 * (size_t)i + 3] = 0.0;
        }
        upload(ctx, ctx->pos4, p4.data(), p4.size());
        ctx->sync();  // the host copy goes out of scope
    }
    upload(ctx, ctx->vel, m->vel, 3 * (size_t)N);
    upload(ctx, ctx->nbs_off, m->nbs_off, (size_t)N + 1);
    upload(ctx, ctx->nbs, m->nbs, (size_t)m->nbs_off[N]);
    upload(ctx, ctx->bdy, m->bdy, (size_t)N);
    upload(ctx, ctx->T, m->T, (size_t)N);
    upload(ctx, ctx->vturb2, m->vturb2, (size_t)N);
    // one Doppler width everywhere (bit-identical T and v_turb^2): every
    // segment's averaged width is then the same number, which the formal
    // solution exploits
    ctx->one_width = true;
    for (int i = 1; i < N && ctx->one_width; i++)
        ctx->one_width = m->T[i] == m->T[0] && m->vturb2[i] == m->vturb2[0];
    // bounds for the images' line culling
    ctx->vmax = ctx->bmax = 0.0;
    for (int i = 0; i < N; i++) {
        const double vx = m->vel[i], vy = m->vel[(size_t)N + i], vz = m->vel[2 * (size_t)N + i];
        ctx->vmax = std::max(ctx->vmax, std::sqrt(vx * vx + vy * vy + vz * vz));
        ctx->bmax = std::max(ctx->bmax, std::sqrt(2.0 * kKB * m->T[i] / m->mass + m->vturb2[i]));
    }
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
    ctx->nu_host.assign(m->nu, m->nu + m->nlines);
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
    ctx->vel4.ensure(sizeof(double) * 4 * (size_t)N);
    HIPCHK(launch_pack_vel4(N, ctx->vel.as<double>(), ctx->b2.as<double>(),
                            (double4 *)ctx->vel4.p, ctx->stream));
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
    // line-table rows longer than half a 128-byte cache line start on a line
    // of their own (a gather of a point's row then touches as few lines as
    // it can); shorter rows stay packed
    {
        const int row = ctx->nlines * (int)tsz;
        ctx->ldl = row > 64 ? (int)(((row + 127) / 128) * 128 / tsz) : ctx->nlines;
    }
    ctx->chiT.ensure(tsz * (size_t)ctx->N * ctx->ldl);
    ctx->ST.ensure(tsz * (size_t)ctx->N * ctx->ldl);
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
    a.p4 = (const double4 *)ctx->pos4.p;
    a.v4 = (const double4 *)ctx->vel4.p;
    a.nbs_off = ctx->nbs_off.as<int32_t>();
    a.nbs = ctx->nbs.as<int32_t>();
    a.bdy = ctx->bdy.as<uint8_t>();
    a.ray_dir = ctx->ray_dir.as<double>();
    a.b2 = ctx->b2.as<double>();
    a.thr = ctx->opt.branch_threshold;
    a.counts = ctx->counts.as<int64_t>();
    a.cnt = ctx->counters.as<Counters>();
    // Large 3D models: the searching pass also keeps each walk's points in a
    // slot of the expected walk length (a temporary of at least
    // trace_slot_min_bytes, at most 16 GiB and a quarter of the free memory);
    // if no walk outgrew its slot, the records are then written from the
    // slots without a second search.  Otherwise (small models, whose second
    // search costs less than the temporary's allocation; 1D; no room) the
    // search runs again to write them.
    DMem slots, longest_d;
    const int64_t cap = (int64_t)(4.0 * cbrt((double)ctx->N) + 16.0);
    const size_t slot_bytes = sizeof(int32_t) * (size_t)NW * (size_t)cap;
    bool use_slots = false;
    if (ctx->dim == 3) {
        size_t free_b = 0, total_b = 0;
        const int64_t min_b = ctx->opt.trace_slot_min_bytes;
        if (min_b >= 0 && slot_bytes >= (size_t)min_b &&
            hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
            slot_bytes <= std::min(size_t(16) << 30, free_b / 4)) {
            if (hipMalloc(&slots.p, slot_bytes) == hipSuccess) {
                slots.bytes = slot_bytes;
                use_slots = true;
            } else {
                slots.p = nullptr;
                (void)hipGetLastError();  // no room after all: two passes
            }
        }
    }
    if (use_slots) {
        longest_d.ensure(sizeof(unsigned long long));
        HIPCHK(hipMemsetAsync(longest_d.p, 0, sizeof(unsigned long long), ctx->stream));
        a.slot = slots.as<int32_t>();
        a.cap = cap;
        a.maxn = longest_d.as<unsigned long long>();
        HIPCHK(launch_trace(a, TraceMode::slots, ctx->stream));
    } else {
        HIPCHK(launch_trace(a, TraceMode::count, ctx->stream));
    }
    HIPCHK(mgx_internal_scan(ctx->counts.as<int64_t>(), ctx->offsets.as<int64_t>(), NW + 1,
                             &ctx->scan_tmp, &ctx->scan_tmp_bytes, ctx->stream));
    int64_t total = 0;
    unsigned long long longest = 0;
    HIPCHK(hipMemcpyAsync(&total, ctx->offsets.as<int64_t>() + NW, sizeof(int64_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    if (use_slots)
        HIPCHK(hipMemcpyAsync(&longest, longest_d.p, sizeof(longest), hipMemcpyDeviceToHost,
                              ctx->stream));
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
    if (use_slots && (int64_t)longest <= cap)
        HIPCHK(launch_trace_emit(a, ctx->stream));
    else
        HIPCHK(launch_trace(a, TraceMode::fill, ctx->stream));
    const bool f32 = ctx->fp32();
    ctx->rec.ensure((f32 ? sizeof(Rec<float>) : sizeof(Rec<double>)) * n);
    HIPCHK(launch_pack_trace(total, ctx->r_idx.as<int32_t>(), ctx->r_semi.as<uint8_t>(),
                             f32 ? ctx->bf.p : ctx->bd.p, f32 ? ctx->ibf.p : ctx->ibd.p,
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

void mgxh::line_coeffs_into(mgx_ctx *ctx, const double *pops, void *chiT, void *ST, int ldt,
                            double *S64, Counters *cnt, hipStream_t s, double S_unit)
{
    LineArgs la{};
    la.N = ctx->N;
    la.nlev = ctx->nlev;
    la.nlines = ctx->nlines;
    la.pops = pops;
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
    la.S_unit = S_unit;
    la.S64 = S64;
    la.chiT = chiT;
    la.ST = ST;
    la.ldt = ldt;
    la.fp32 = ctx->fp32() ? 1 : 0;
    la.cnt = cnt;
    HIPCHK(launch_reset_counters(cnt, s));
    HIPCHK(launch_line_coeffs(la, s));
}

std::vector<int32_t> mgxh::morton_order(const double *pos, int N)
{
    double lo3[3], hi3[3];
    for (int k = 0; k < 3; k++) {
        lo3[k] = INFINITY;
        hi3[k] = -INFINITY;
        for (int i = 0; i < N; i++) {
            lo3[k] = std::min(lo3[k], pos[(size_t)k * N + i]);
            hi3[k] = std::max(hi3[k], pos[(size_t)k * N + i]);
        }
    }
    auto spread = [](uint32_t v) {
        uint64_t x = v & 0x3ff;
        x = (x | (x << 16)) & 0x030000ffull;
        x = (x | (x << 8)) & 0x0300f00full;
        x = (x | (x << 4)) & 0x030c30c3ull;
        x = (x | (x << 2)) & 0x09249249ull;
        return x;
    };
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)N);
    for (int i = 0; i < N; i++) {
        uint64_t code = 0;
        for (int k = 0; k < 3; k++) {
            const double w = hi3[k] - lo3[k];
            const double f = w > 0 ? (pos[(size_t)k * N + i] - lo3[k]) / w : 0.0;
            const uint32_t c = (uint32_t)std::min(1023.0, std::max(0.0, f * 1024.0));
            code |= spread(c) << k;
        }
        key[i] = {code, i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> ord((size_t)N);
    for (int i = 0; i < N; i++) ord[i] = key[i].second;
    return ord;
}

void mgxh::run_line_coeffs(mgx_ctx *ctx)
{
    line_coeffs_into(ctx, ctx->pops.as<double>(), ctx->chiT.p, ctx->ST.p, ctx->ldl,
                     ctx->S64.as<double>(),
                     ctx->counters.as<Counters>(), ctx->stream);
}

// Launch shape of a formal solution: lines per chunk (balanced) and threads
// per workgroup (a multiple of 64 covering nlc * nbins, at most 1024: as many
// lines as fit, so the per-(record, bin) staging is shared by all of them;
// in FP64, 19 lines in one workgroup instead of two of 10 took the clumpy
// cloud from 433 to 358 ms, the lower occupancy included).  The line chunk is
// also capped so that the LDS staging of one record per half stays within
// 64 KiB: with one bin per line a workgroup would otherwise stage up to 1024
// lines per record.  *lds_out: the LDS of the record chunk the launch picks.
void mgxh::fs_shape(size_t tsize, int nlines, int nbins, int *nlc_out, int *nthreads_out,
                    size_t *lds_out)
{
    const int max_threads = kMaxBins;
    auto threads = [nbins](int nlc) { return ((nlc * nbins + 63) / 64) * 64; };
    auto lds_at = [tsize, nbins, &threads](int ch, int nlc) {
        return tsize == 8 ? formal_solve_lds<double>(ch, nlc, nbins, threads(nlc))
                          : formal_solve_lds<float>(ch, nlc, nbins, threads(nlc));
    };
    auto lds = [&lds_at](int nlc) { return lds_at(1, nlc); };
    int nlc = std::max(1, max_threads / nbins);
    if (nlc > nlines) nlc = nlines;
    while (nlc > 1 && lds(nlc) > 64 * 1024) nlc--;
    // balance the line chunks so the last one is not nearly empty
    const int nchunks = (nlines + nlc - 1) / nlc;
    nlc = (nlines + nchunks - 1) / nchunks;
    *nlc_out = nlc;
    *nthreads_out = threads(nlc);
    const int ch = tsize == 8 ? formal_solve_chunk<double>(nlc, nbins, threads(nlc))
                              : formal_solve_chunk<float>(nlc, nbins, threads(nlc));
    *lds_out = lds_at(ch, nlc);
}

extern "C" mgx_status mgx_formal_solve_shape(int precision, int nlines, int nbins,
                                             int *lines_per_chunk, int *threads,
                                             int64_t *lds_bytes)
{
    if ((precision != MGX_FP32 && precision != MGX_FP64) || nlines < 1 || nbins < 1 ||
        nbins > kMaxBins)
        return MGX_EINVAL;
    int nlc, nth;
    size_t lds;
    fs_shape(precision == MGX_FP64 ? 8 : 4, nlines, nbins, &nlc, &nth, &lds);
    if (lines_per_chunk) *lines_per_chunk = nlc;
    if (threads) *threads = nth;
    if (lds_bytes) *lds_bytes = (int64_t)lds;
    return MGX_OK;
}

template <typename T>
FSArgs<T> mgxh::fs_args(mgx_ctx *ctx)
{
    FSArgs<T> a{};
    a.N = ctx->N;
    a.R = ctx->R;
    a.npairs = ctx->npairs;
    a.nlines = ctx->nlines;
    a.nbins = ctx->nbins;
    size_t lds;
    fs_shape(sizeof(T), ctx->nlines, ctx->nbins, &a.nlc, &a.nthreads, &lds);
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
    a.order = ctx->order.as<int32_t>();  // null where the table fits the L2
    a.one_width = ctx->one_width ? 1 : 0;
    a.ldl = ctx->ldl;
    return a;
}
template FSArgs<float> mgxh::fs_args<float>(mgx_ctx *);
template FSArgs<double> mgxh::fs_args<double>(mgx_ctx *);

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

void mgxh::ng_append(mgx_ctx *ctx)
{
    if (ctx->ng_nh == 0) {  // emptied history: the iterate becomes y_1, no residual yet
        HIPCHK(launch_copy(ctx->npop(), ctx->pops.as<double>(), ctx->ng_y[0]->as<double>(),
                           ctx->stream));
        ctx->ng_nh = 1;
        return;
    }
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

StateqArgs mgxh::stateq_args(mgx_ctx *ctx)
{
    StateqArgs s{};
    s.N = ctx->N;
    s.nlev = ctx->nlev;
    s.nlines = ctx->nlines;
    s.ncoll_tr = ctx->ncoll_tr;
    s.group = stateq_group(ctx->nlev);
    const size_t per_wave =
        sizeof(double) * ctx->nlev * (ctx->nlev + 1) * (size_t)(64 / s.group);
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
    HIPCHK(launch_reset_counters(ctx->counters.as<Counters>(), ctx->stream, false));
    HIPCHK(launch_stateq(s, ctx->stream));
    std::swap(ctx->pops.p, ctx->pops_new.p);
    std::swap(ctx->pops.bytes, ctx->pops_new.bytes);
    if (ctx->ng_active) ng_append(ctx);
    Counters c = ctx->read_counters();
    double change;
    memcpy(&change, &c.change_bits, sizeof(double));
    ctx->host_cnt.singular = (int64_t)c.singular;
    ctx->host_cnt.masing = (int64_t)c.masing;
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

void mgxh::ng_reset(mgx_ctx *ctx, int capacity)
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

// Forms the prediction from all stored iterates into ng_prev (when valid).
// Returns 1 if valid (Gram matrix regular, no negative entry).
int mgxh::ng_predict(mgx_ctx *ctx, double *pred_change)
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

// Use the last valid prediction (or keep the plain iterate) and restart the
// history: from the populations, or, with `fresh` after a used prediction,
// empty, so that only regular iterates computed after it are stored.
void mgxh::ng_apply(mgx_ctx *ctx, bool accepted, bool fresh)
{
    if (accepted) {
        HIPCHK(launch_copy(ctx->npop(), ctx->ng_prev.as<double>(), ctx->pops.as<double>(),
                           ctx->stream));
        ctx->host_cnt.ng_applied++;
    } else {
        ctx->host_cnt.ng_rejected++;
    }
    if (accepted && fresh) {
        ctx->ng_nh = 0;
        ctx->ng_have_prev = false;
    } else {
        ng_restart(ctx);
    }
}

// One decision of the classical or adaptive schedule after a regular
// iterate has been appended; `change` is the relative change between the
// last two iterates.  Returns 1 if a prediction replaced the populations.
int mgxh::ng_schedule_step(mgx_ctx *ctx, int mode, int param, double change)
{
    const bool fresh = (mode & MGX_NG_FRESH) != 0;
    if ((mode & MGX_NG_MODE_MASK) == MGX_NG_CLASSICAL) {
        if (ctx->ng_nh != param + 1) return 0;
        double pc;
        const bool ok = ng_predict(ctx, &pc) != 0;
        ng_apply(ctx, ok, fresh);
        return ok ? 1 : 0;
    }
    bool use = false;
    if (ctx->ng_nh >= 3) {
        double pc;
        const int ok = ng_predict(ctx, &pc);
        use = ok && (pc < change || ctx->ng_nh >= param);
    }
    if (use)
        ng_apply(ctx, true, fresh);
    else if (ctx->ng_nh >= param)
        ng_apply(ctx, false, fresh);
    return use ? 1 : 0;
}

static void check_ng_mode(int ng_mode, int ng_param, bool allow_none)
{
    REQUIRE((ng_mode & ~(MGX_NG_MODE_MASK | MGX_NG_FRESH)) == 0, MGX_EINVAL, "unknown ng_mode");
    const int m = ng_mode & MGX_NG_MODE_MASK;
    REQUIRE(m == MGX_NG_CLASSICAL || m == MGX_NG_ADAPTIVE || (allow_none && m == MGX_NG_NONE),
            MGX_EINVAL, "unknown ng_mode");
    if (m == MGX_NG_CLASSICAL)
        REQUIRE(ng_param >= 1 && ng_param + 1 <= kNgMaxHist, MGX_EINVAL,
                "classical Ng order must be 1..31");
    if (m == MGX_NG_ADAPTIVE)
        REQUIRE(ng_param >= 3 && ng_param <= kNgMaxHist, MGX_EINVAL,
                "adaptive Ng N_max must be 3..32");
}

extern "C" mgx_status mgx_ng_push(mgx_ctx *ctx)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->ng_active, MGX_ESTATE, "mgx_ng_push without mgx_ng_reset");
    ng_append(ctx);
    ctx->sync();
    API_END(ctx)
}

extern "C" mgx_status mgx_ng_predict(mgx_ctx *ctx, int apply, int *status_out,
                                     double *pred_change_out, double *coef_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->ng_active, MGX_ESTATE, "mgx_ng_predict without mgx_ng_reset");
    REQUIRE(ctx->ng_nh >= 2, MGX_ESTATE, "mgx_ng_predict needs two stored iterates");
    const int K = ctx->ng_nh - 1;
    double pc = INFINITY;
    const int ok = ng_predict(ctx, &pc);
    if (ok && coef_out)
        HIPCHK(hipMemcpyAsync(coef_out, ctx->ng_coef.p, sizeof(double) * K, hipMemcpyDefault,
                              ctx->stream));
    if (apply) ng_apply(ctx, ok != 0, false);
    ctx->sync();
    if (status_out) *status_out = ok;
    if (pred_change_out) *pred_change_out = pc;
    API_END(ctx)
}

extern "C" mgx_status mgx_ng_accelerate(mgx_ctx *ctx, int mode, int order_or_nmax,
                                        int *applied_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->ng_active, MGX_ESTATE, "mgx_ng_accelerate without mgx_ng_reset");
    check_ng_mode(mode, order_or_nmax, false);
    const int need = (mode & MGX_NG_MODE_MASK) == MGX_NG_CLASSICAL ? order_or_nmax + 1
                                                                   : order_or_nmax;
    REQUIRE(need <= ctx->ng_cap, MGX_EINVAL, "Ng history capacity below what the mode needs");
    const int applied = ng_schedule_step(ctx, mode, order_or_nmax, ctx->host_cnt.last_change);
    ctx->sync();
    if (applied_out) *applied_out = applied;
    API_END(ctx)
}

extern "C" mgx_status mgx_iterate(mgx_ctx *ctx, double tol, int max_iter, int ng_mode,
                                  int ng_param, int *iters_out, double *final_change_out)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->traced, MGX_ESTATE, "mgx_iterate before mgx_trace_rays");
    REQUIRE(ctx->have_pops, MGX_ESTATE, "mgx_iterate without populations");
    REQUIRE(max_iter >= 1 && tol >= 0, MGX_EINVAL, "max_iter >= 1 and tol >= 0 required");
    check_ng_mode(ng_mode, ng_param, true);
    const int mode = ng_mode & MGX_NG_MODE_MASK;
    ctx->ng_active = false;
    if (mode == MGX_NG_CLASSICAL)
        ng_reset(ctx, ng_param + 1);
    else if (mode == MGX_NG_ADAPTIVE)
        ng_reset(ctx, ng_param);
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
        if (mode != MGX_NG_NONE) ng_schedule_step(ctx, ng_mode, ng_param, change);
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

void mgxh::check_render_args(const double dir[3], int npx, int npy, double f_min, double f_max,
                             int nfreq)
{
    REQUIRE(dir, MGX_EINVAL, "dir is NULL");
    REQUIRE(std::isfinite(dir[0]) && std::isfinite(dir[1]) && std::isfinite(dir[2]) &&
                (dir[0] != 0.0 || dir[1] != 0.0 || dir[2] != 0.0),
            MGX_EINVAL, "dir must be finite and non-zero");
    REQUIRE(npx >= 1 && npy >= 1 && (int64_t)npx * npy <= (1 << 26), MGX_EINVAL,
            "pixel counts out of range");
    REQUIRE(nfreq >= 1 && nfreq <= 1024, MGX_EINVAL, "nfreq must be 1..1024");
    REQUIRE(f_min > 0 && f_max >= f_min && std::isfinite(f_max), MGX_EINVAL,
            "need 0 < f_min <= f_max");
}

void mgxh::render_image(mgx_ctx *ctx, RenderBufs &rb, const double *pops, hipStream_t s,
                        const double dir[3], int npx, int npy, double f_min, double f_max,
                        int nfreq, float *img)
{
    const int N = ctx->N;
    const size_t tsz = ctx->fp32() ? sizeof(float) : sizeof(double);
    rb.chiT.ensure(tsz * ctx->nrad());
    rb.ST.ensure(tsz * ctx->nrad());
    rb.S64.ensure(sizeof(double) * ctx->nrad());
    rb.cnt.ensure(sizeof(Counters));
    // intensities in units of I_img = 2 h f_mid^3 / c^2 (source functions too)
    const double I_img = 2.0 * kH * pow(0.5 * (f_min + f_max), 3) / (kC * kC);
    line_coeffs_into(ctx, pops, rb.chiT.p, rb.ST.p, ctx->nlines, rb.S64.as<double>(),
                     rb.cnt.as<Counters>(), s, I_img);
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
    rb.proj.ensure(sizeof(double) * 4 * (size_t)N + sizeof(double) * 4);
    g.u = rb.proj.as<double>();
    g.v = g.u + N;
    g.Z = g.v + N;
    g.w = g.Z + N;
    g.ext = g.w + N;
    rb.pix.ensure((sizeof(unsigned long long) + sizeof(int32_t)) * npix + 16);
    g.key = rb.pix.as<unsigned long long>();
    g.entry = (int32_t *)(g.key + npix);
    rb.off.ensure(sizeof(int64_t) * 2 * (npix + 1));
    g.counts = rb.off.as<int64_t>();
    int64_t *off = g.counts + (npix + 1);
    HIPCHK(hipMemsetAsync(g.counts, 0, sizeof(int64_t) * (npix + 1), s));
    HIPCHK(launch_render_geometry(g, s));
    // One pass into fixed slots of cap points (the expected walk length) when
    // they fit 256 MiB.  A walk longer than its slot sends the image through
    // the exact two-pass route (lengths, offsets, walks), whose lengths the
    // first pass has already written.
    const int64_t cap = render_walk_cap(N);
    bool csr = (size_t)npix * (size_t)cap * sizeof(int32_t) > (size_t(256) << 20);
    if (!csr) {
        rb.walk.ensure(sizeof(int32_t) * (size_t)npix * (size_t)cap);
        rb.maxn.ensure(sizeof(unsigned long long));
        g.cap = cap;
        g.maxn = rb.maxn.as<unsigned long long>();
        g.walk = rb.walk.as<int32_t>();
        HIPCHK(hipMemsetAsync(g.maxn, 0, sizeof(unsigned long long), s));
        HIPCHK(launch_render_walk(g, WalkMode::capped, s));
        unsigned long long longest = 0;
        HIPCHK(hipMemcpyAsync(&longest, g.maxn, sizeof(longest), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        csr = (int64_t)longest > cap;
    } else {
        HIPCHK(launch_render_walk(g, WalkMode::count, s));
    }
    if (csr) {
        HIPCHK(mgx_internal_scan(g.counts, off, npix + 1, &rb.scan_tmp, &rb.scan_tmp_bytes, s));
        int64_t total = 0;
        HIPCHK(hipMemcpyAsync(&total, off + npix, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        rb.walk.ensure(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
        g.off = off;
        g.walk = rb.walk.as<int32_t>();
        HIPCHK(launch_render_walk(g, WalkMode::fill, s));
    }
    rb.img.ensure(sizeof(float) * (size_t)npix * nfreq);
    // Lines whose profile can reach the band.  At a point moving with w
    // (|w| <= vmax) and width b (<= bmax) the offset of frequency nu from line
    // l is |x| = (c - w) |nu - c nu_l / (c - w)| / (nu_l b), so a line whose
    // shifted centres c nu_l / (c +- vmax) all lie further than
    // X nu_l bmax / (c - vmax) from the band has |x| > X everywhere: beyond
    // X = 10.5 (FP32) or 27.5 (FP64) its Gaussian and erfc are exactly zero
    // in the working precision, so its terms are skipped without changing a
    // bit (1 % margin for the rounding of the offsets).
    {
        const double X = ctx->fp32() ? 10.5 : 27.5, vm = ctx->vmax;
        rb.act_host.clear();
        for (int l = 0; l < ctx->nlines; l++) {
            const double nl = ctx->nu_host[l];
            bool seen = true;
            if (vm < 0.5 * kC) {
                const double lo = kC * nl / (kC + vm), hi = kC * nl / (kC - vm);
                const double d = 1.01 * X * nl * ctx->bmax / (kC - vm);
                seen = f_max >= lo - d && f_min <= hi + d;
            }
            if (seen) rb.act_host.push_back(l);
        }
        rb.act.ensure(sizeof(int32_t) * std::max<size_t>(1, rb.act_host.size()));
        if (!rb.act_host.empty())
            HIPCHK(hipMemcpyAsync(rb.act.p, rb.act_host.data(),
                                  sizeof(int32_t) * rb.act_host.size(), hipMemcpyHostToDevice, s));
    }
    auto fill_args = [&](auto &ra) {
        ra.npx = npx;
        ra.npy = npy;
        ra.nfreq = nfreq;
        ra.nlines = ctx->nlines;
        ra.off = csr ? off : nullptr;
        ra.cnt = g.counts;
        ra.cap = cap;
        ra.walk = g.walk;
        ra.Z = g.Z;
        ra.w = g.w;
        ra.b = ctx->bd.as<double>();
        ra.ib = ctx->ibd.as<double>();
        ra.nu_line = ctx->nu.as<double>();
        ra.act = rb.act.as<int32_t>();
        ra.nact = (int)rb.act_host.size();
        ra.inv_L = 1.0 / ctx->L_unit;
        ra.f_min = f_min;
        ra.f_max = f_max;
        ra.Tcmb = ctx->Tcmb;
        ra.I_img = I_img;
        ra.thr = ctx->opt.branch_threshold;
        ra.b2 = ctx->b2.as<double>();
        ra.img = rb.img.as<float>();
    };
    if (ctx->fp32()) {
        RenderArgs<float> ra{};
        fill_args(ra);
        ra.chi = (const float *)rb.chiT.p;
        ra.S = (const float *)rb.ST.p;
        HIPCHK(launch_render_integrate<float>(ra, s));
    } else {
        RenderArgs<double> ra{};
        fill_args(ra);
        ra.chi = (const double *)rb.chiT.p;
        ra.S = (const double *)rb.ST.p;
        HIPCHK(launch_render_integrate<double>(ra, s));
    }
    HIPCHK(hipMemcpyAsync(img, rb.img.p, sizeof(float) * (size_t)npix * nfreq, hipMemcpyDefault,
                          s));
    HIPCHK(hipStreamSynchronize(s));
}

extern "C" mgx_status mgx_render_image(mgx_ctx *ctx, const double dir[3], int npx, int npy,
                                       double f_min, double f_max, int nfreq, float *img)
{
    API_BEGIN(ctx)
    REQUIRE(ctx->loaded && ctx->have_pops, MGX_ESTATE, "mgx_render_image needs a model and populations");
    REQUIRE(ctx->dim == 3, MGX_EINVAL, "mgx_render_image supports point clouds (dim 3)");
    REQUIRE(img, MGX_EINVAL, "img is NULL");
    check_render_args(dir, npx, npy, f_min, f_max, nfreq);
    ctx->sync();
    render_image(ctx, ctx->rb, ctx->pops.as<double>(), ctx->stream, dir, npx, npy, f_min, f_max,
                 nfreq, img);
    API_END(ctx)
}

size_t mgxh::ctx_bytes(const mgx_ctx *c)
{
    const DMem *all[] = {&c->pos, &c->vel, &c->nbs_off, &c->nbs, &c->bdy, &c->T, &c->vturb2,
                         &c->nspec, &c->ncoll, &c->ray_dir, &c->ray_w, &c->antipode, &c->E,
                         &c->g, &c->up, &c->lo, &c->A, &c->nu, &c->cu, &c->cl, &c->K0, &c->b2,
                         &c->b, &c->bf, &c->ibf, &c->bd, &c->ibd, &c->xf, &c->W, &c->Bul,
                         &c->Blu, &c->hnu4pi, &c->chiscale, &c->Iref, &c->acmb, &c->pair_r,
                         &c->pair_a, &c->pair_w, &c->pops, &c->pops_new, &c->J, &c->L, &c->S64,
                         &c->chiT, &c->ST, &c->counters, &c->order, &c->counts, &c->offsets, &c->r_idx,
                         &c->r_semi, &c->r_Z, &c->r_dv, &c->r_dx, &c->r_ibb, &c->rec, &c->ng_G,
                         &c->ng_coef, &c->ng_status, &c->ng_partial, &c->ng_pred, &c->ng_prev,
                         &c->ng_bits};
    size_t n = c->scan_tmp_bytes + c->rb.bytes();
    for (const DMem *m : all) n += m->bytes;
    for (const DMem *m : c->ng_pool) n += m->bytes;
    return n;
}

