// Batches: many independent models iterated together on one GPU (the C ABI's
// mgx_batch_* calls).  Every Lambda-iteration replays three captured graphs
// (line coefficients of every model; one formal-solution launch per lane
// class; statistical equilibrium of every model); converged models are masked
// and their work items compacted away, classical Ng runs per model between
// replays.

#include <algorithm>
#include <new>
#include <utility>

#include "host.h"

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
    API_BEGIN(b)
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
    API_END(b)
}

template <typename T>
static void batch_build_tables(mgx_batch *b)
{
    const int M = (int)b->m.size();
    std::vector<FSArgs<T>> d(M);
    std::vector<std::vector<std::pair<int64_t, int4>>> cls(MGX_BATCH_CLASSES);
    std::vector<std::vector<int32_t>> rank(M);  // origin -> its Morton rank
    DMem cost;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        b->class_threads[k] = 64 * (k + 1);
        b->class_nlc_max[k] = 0;
        b->class_nb_max[k] = 0;
        b->class_ch[k] = 64;
    }
    for (int i = 0; i < M; i++) {
        mgx_ctx *c = b->m[i];
        d[i] = fs_args<T>(c);
        // a model's workgroup size is a multiple of 64 up to 1024
        const int k = d[i].nthreads / 64 - 1;
        b->class_nlc_max[k] = std::max(b->class_nlc_max[k], d[i].nlc);
        b->class_nb_max[k] = std::max(b->class_nb_max[k], d[i].nbins);
        cost.ensure(sizeof(int64_t) * c->N);
        HIPCHK(launch_origin_cost(c->N, c->R, c->offsets.as<int64_t>(), cost.as<int64_t>(),
                                  b->stream));
        std::vector<int64_t> hc(c->N);
        HIPCHK(hipMemcpyAsync(hc.data(), cost.p, sizeof(int64_t) * c->N, hipMemcpyDeviceToHost,
                              b->stream));
        std::vector<double> pos(3 * (size_t)c->N);
        HIPCHK(hipMemcpyAsync(pos.data(), c->pos.p, sizeof(double) * pos.size(),
                              hipMemcpyDeviceToHost, b->stream));
        b->sync();
        const std::vector<int32_t> ord = morton_order(pos.data(), c->N);
        rank[i].resize(c->N);
        for (int j = 0; j < c->N; j++) rank[i][ord[j]] = j;
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
        // the alternative order: by model, origin in Morton order, line chunk
        // (workgroups dealt to one XCD then gather neighbouring points)
        std::vector<int4> loc = it;
        std::stable_sort(loc.begin(), loc.end(), [&rank](const int4 &x, const int4 &y) {
            if (x.x != y.x) return x.x < y.x;
            const int rx = rank[x.x][x.y], ry = rank[y.x][y.y];
            if (rx != ry) return rx < ry;
            return x.z < y.z;
        });
        b->items_alt[k].release();
        if (!loc.empty()) upload(b->m[0], b->items_alt[k], loc.data(), loc.size());
        b->class_order[k] = 0;
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

void mgxh::batch_prepare(mgx_batch *b)
{
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
    std::vector<int> ones(M, 1);
    upload(b->m[0], b->all_active, ones.data(), (size_t)M);
    b->host_active.assign(M, 0);
    upload(b->m[0], b->active, b->host_active.data(), (size_t)M);
    b->runs.assign(M, BatchRun{});
    b->changes.ensure(sizeof(double) * 2 * M);
    b->sync();
    b->prepared = true;
}

extern "C" mgx_status mgx_batch_prepare(mgx_batch *b)
{
    API_BEGIN(b)
    batch_prepare(b);
    API_END(b)
}

extern "C" mgx_status mgx_batch_set_lte_populations(mgx_batch *b)
{
    API_BEGIN(b)
    for (mgx_ctx *c : b->m) check_sub(b, c, mgx_set_lte_populations(c));
    API_END(b)
}

extern "C" mgx_status mgx_batch_set_populations(mgx_batch *b, int id, const double *pops)
{
    API_BEGIN(b)
    REQUIRE(id >= 0 && id < (int)b->m.size(), MGX_EINVAL, "model id out of range");
    check_sub(b, b->m[id], mgx_set_populations(b->m[id], pops));
    API_END(b)
}

extern "C" mgx_status mgx_batch_get_populations(mgx_batch *b, int id, double *pops)
{
    API_BEGIN(b)
    REQUIRE(id >= 0 && id < (int)b->m.size(), MGX_EINVAL, "model id out of range");
    check_sub(b, b->m[id], mgx_get_populations(b->m[id], pops));
    API_END(b)
}

// Upload the host mask and keep only the work items of active models (same
// order; *counts[k] of them per class).
void mgxh::batch_push_mask(mgx_batch *b)
{
    const int M = (int)b->m.size();
    HIPCHK(hipMemcpyAsync(b->active.p, b->host_active.data(), sizeof(int) * M,
                          hipMemcpyHostToDevice, b->stream));
    for (int k = 0; k < MGX_BATCH_CLASSES; k++)
        if (b->class_nitems[k])
            HIPCHK(launch_compact_items(b->items_all[k].as<int4>(), b->class_nitems[k],
                                        b->items[k].as<int4>(), b->counts.as<int>() + k,
                                        b->active.as<int>(), &b->select_tmp,
                                        &b->select_tmp_bytes, b->stream));
    b->sync();
}

template <typename T>
static void batch_launch_class(mgx_batch *b, int k, const int4 *items, const int *count,
                               int blocks, const int *active, int ch)
{
    const size_t lds = formal_solve_lds<T>(ch, b->class_nlc_max[k], b->class_nb_max[k],
                                           b->class_threads[k]);
    HIPCHK(launch_formal_solve_batch<T>((const FSArgs<T> *)b->descs.p, items, count, blocks,
                                        active, ch, b->class_threads[k], lds, b->stream));
}

// Schedule tuning, per lane class: the LDS chunk (records staged per
// half-ray), timed on a strided sample of the class's items, then the item
// order, timed on full launches at that chunk; the fastest of each is kept.
template <typename T>
static void batch_tune(mgx_batch *b)
{
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        const int n = b->class_nitems[k];
        if (n == 0) continue;
        const int nlc = b->class_nlc_max[k], nth = b->class_threads[k];
        const int nbm = b->class_nb_max[k];
        // the largest chunk the LDS budget allows (as the single-model
        // launch picks it), half and a quarter of it
        const int chmax = formal_solve_chunk<T>(nlc, nbm, nth);
        REQUIRE(formal_solve_lds<T>(chmax, nlc, nbm, nth) <= 160 * 1024, MGX_EINVAL,
                "line chunk does not fit the LDS");
        const int ns = b->class_nsample[k];
        HIPCHK(hipMemcpyAsync(b->tune_count.p, &ns, sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
        float best = INFINITY;
        b->class_ch[k] = chmax;
        int tried = 0;
        for (int ch : {chmax, (chmax + 1) / 2, (chmax + 3) / 4}) {
            if (ch == tried) continue;
            tried = ch;
            HIPCHK(hipEventRecord(b->ev0, b->stream));
            batch_launch_class<T>(b, k, b->sample[k].as<int4>(), b->tune_count.as<int>(), ns,
                                  b->all_active.as<int>(), ch);
            HIPCHK(hipEventRecord(b->ev1, b->stream));
            b->sync();
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            if (ms < best) {
                best = ms;
                b->class_ch[k] = ch;
            }
        }
        // item order: one full launch of the class in each order at the
        // chosen chunk; keep the faster
        HIPCHK(hipMemcpyAsync(b->tune_count.p, &n, sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
        float t[2] = {INFINITY, INFINITY};
        for (int ord = 0; ord < 2; ord++) {
            const int4 *items = (ord ? b->items_alt[k] : b->items_all[k]).as<int4>();
            HIPCHK(hipEventRecord(b->ev0, b->stream));
            batch_launch_class<T>(b, k, items, b->tune_count.as<int>(), n,
                                  b->all_active.as<int>(), b->class_ch[k]);
            HIPCHK(hipEventRecord(b->ev1, b->stream));
            b->sync();
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            t[ord] = ms;
        }
        b->class_order[k] = t[1] < t[0] ? 1 : 0;
        if (b->class_order[k]) b->items_all[k].swap(b->items_alt[k]);
        b->items_alt[k].release();
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
                                      b->class_nitems[k], b->active.as<int>(), b->class_ch[k]);
    });
    batch_capture_part(b, 2, [&]() {
        for (int i = 0; i < M; i++) {
            mgx_ctx *c = b->m[i];
            StateqArgs s = stateq_args(c);
            s.active = b->active.as<int>();
            s.model = i;
            HIPCHK(launch_reset_counters(c->counters.as<Counters>(), b->stream, false));
            HIPCHK(launch_stateq(s, b->stream));
            HIPCHK(launch_copy_if_active(c->npop(), c->pops_new.as<double>(), c->pops.as<double>(),
                                         b->active.as<int>(), i, b->stream));
        }
        HIPCHK(launch_gather_changes(M, b->cnt_ptrs.as<Counters *>(), b->changes.as<double>(),
                                     b->stream));
    });
}

static double wall_seconds()
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

void mgxh::batch_begin(mgx_batch *b)
{
    REQUIRE(b->prepared, MGX_ESTATE, "batch not prepared");
    if (b->tuned) return;
    const double t0 = wall_seconds();
    for (mgx_ctx *c : b->m) run_line_coeffs(c);
    if (b->fp32())
        batch_tune<float>(b);
    else
        batch_tune<double>(b);
    b->st.tune_seconds = wall_seconds() - t0;
    if (b->fp32())
        batch_capture<float>(b);
    else
        batch_capture<double>(b);
    b->tuned = true;
}

void mgxh::batch_activate(mgx_batch *b, int i, double tol, int max_iter, int ng_order)
{
    mgx_ctx *c = b->m[i];
    REQUIRE(c->have_pops, MGX_ESTATE, "batch model without populations");
    BatchRun &r = b->runs[i];
    r = BatchRun{};
    r.active = true;
    r.tol = tol;
    r.max_iter = max_iter;
    r.ng_order = ng_order;
    c->ng_active = false;
    if (ng_order > 0) ng_reset(c, ng_order + 1);
    b->host_active[i] = 1;
}

void mgxh::batch_replay(mgx_batch *b, std::vector<double> &hc)
{
    const int M = (int)b->m.size();
    HIPCHK(hipGraphLaunch(b->gexec[0], b->stream));
    HIPCHK(hipEventRecord(b->ev0, b->stream));
    HIPCHK(hipGraphLaunch(b->gexec[1], b->stream));
    HIPCHK(hipEventRecord(b->ev1, b->stream));
    HIPCHK(hipGraphLaunch(b->gexec[2], b->stream));
    hc.resize(2 * (size_t)M);
    HIPCHK(hipMemcpyAsync(hc.data(), b->changes.p, sizeof(double) * 2 * M,
                          hipMemcpyDeviceToHost, b->stream));
    b->sync();
    float fs_ms = 0.f;
    HIPCHK(hipEventElapsedTime(&fs_ms, b->ev0, b->ev1));
    b->st.fs_ms_last = fs_ms;
    b->st.fs_ms_total += fs_ms;
    b->st.fs_launches++;
}

void mgxh::batch_step(mgx_batch *b, std::vector<int> &finished)
{
    const int M = (int)b->m.size();
    std::vector<double> hc;
    batch_replay(b, hc);
    bool mask_changed = false;
    for (int i = 0; i < M; i++) {
        BatchRun &r = b->runs[i];
        if (!r.active) continue;
        r.iters++;
        r.change = hc[i];
        const bool failed = hc[M + i] != 0.0 || !std::isfinite(hc[i]);
        bool done = true;
        if (failed)
            r.status = hc[M + i] == 1.0 ? MGX_ESINGULAR : MGX_ENONFINITE;
        else if (hc[i] <= r.tol)
            r.status = MGX_OK;
        else if (r.iters >= r.max_iter)
            r.status = MGX_ENOCONV;
        else
            done = false;
        if (done) {
            r.active = false;
            b->m[i]->ng_active = false;
            b->host_active[i] = 0;
            mask_changed = true;
            finished.push_back(i);
            continue;
        }
        if (r.ng_order > 0) {
            mgx_ctx *c = b->m[i];
            ng_append(c);
            if (c->ng_nh == r.ng_order + 1) {
                double pc;
                ng_apply(c, ng_predict(c, &pc) != 0);
            }
        }
    }
    if (mask_changed) batch_push_mask(b);
}

extern "C" mgx_status mgx_batch_iterate(mgx_batch *b, double tol, int max_iter, int ng_order,
                                        int *iters, double *changes, int *converged_out)
{
    API_BEGIN(b)
    REQUIRE(b->prepared, MGX_ESTATE, "mgx_batch_iterate before mgx_batch_prepare");
    REQUIRE(max_iter >= 1 && tol >= 0, MGX_EINVAL, "max_iter >= 1 and tol >= 0 required");
    REQUIRE(ng_order >= 0 && ng_order + 1 <= kNgMaxHist, MGX_EINVAL, "Ng order must be 0..31");
    const int M = (int)b->m.size();
    for (mgx_ctx *c : b->m) REQUIRE(c->have_pops, MGX_ESTATE, "batch model without populations");
    batch_begin(b);
    const double t0 = wall_seconds();
    b->st.fs_launches = 0;
    b->st.fs_ms_total = b->st.fs_ms_last = 0.0;
    for (int i = 0; i < M; i++) batch_activate(b, i, tol, max_iter, ng_order);
    batch_push_mask(b);
    int replays = 0;
    std::vector<int> finished;
    b->st.last_converged_seconds = 0.0;
    while (std::any_of(b->runs.begin(), b->runs.end(), [](const BatchRun &r) { return r.active; })) {
        finished.clear();
        batch_step(b, finished);
        replays++;
        for (int i : finished)
            if (b->runs[i].status == MGX_OK) b->st.last_converged_seconds = wall_seconds() - t0;
    }
    b->st.iterate_seconds = wall_seconds() - t0;
    b->st.iterations = replays;
    int nconv = 0;
    mgx_status result = MGX_OK;
    for (int i = 0; i < M; i++) {
        const BatchRun &r = b->runs[i];
        if (iters) iters[i] = r.iters;
        if (changes) changes[i] = r.change;
        if (r.status == MGX_OK) {
            nconv++;
        } else if (result == MGX_OK || (result == MGX_ENOCONV && r.status != MGX_ENOCONV)) {
            result = r.status;
            b->err = std::string(r.status == MGX_ESINGULAR    ? "singular statistical equilibrium"
                                 : r.status == MGX_ENONFINITE ? "non-finite populations"
                                                              : "no convergence within max_iter") +
                     " in model " + std::to_string(i);
        }
    }
    b->st.active = 0;
    if (converged_out) *converged_out = nconv;
    if (result == MGX_ENOCONV)
        b->err = std::to_string(M - nconv) + " model(s) did not converge within max_iter";
    if (result != MGX_OK) return result;
    API_END(b)
}

extern "C" mgx_status mgx_batch_get_stats(mgx_batch *b, mgx_batch_stats *out)
{
    API_BEGIN(b)
    REQUIRE(out, MGX_EINVAL, "out is NULL");
    b->st.models = (int)b->m.size();
    b->st.lane_classes = b->nclass;
    b->st.work_items = b->work_items;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++) {
        b->st.class_items[k] = b->class_nitems[k];
        b->st.class_threads[k] = b->class_nitems[k] ? b->class_threads[k] : 0;
        b->st.class_chunk[k] = b->class_nitems[k] ? b->class_ch[k] : 0;
        b->st.class_order[k] = b->class_nitems[k] ? b->class_order[k] : 0;
    }
    *out = b->st;
    API_END(b)
}


size_t mgxh::batch_bytes(const mgx_batch *b)
{
    size_t n = b->descs.bytes + b->active.bytes + b->all_active.bytes + b->changes.bytes +
               b->cnt_ptrs.bytes + b->counts.bytes + b->tune_count.bytes + b->select_tmp_bytes;
    for (int k = 0; k < MGX_BATCH_CLASSES; k++)
        n += b->items_all[k].bytes + b->items[k].bytes + b->sample[k].bytes;
    for (const mgx_ctx *c : b->m) n += ctx_bytes(c);
    return n;
}
