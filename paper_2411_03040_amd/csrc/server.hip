// Server: a resident set of models answering converge and render requests
// (the C ABI's mgx_server_* calls).
//
// One iteration worker drives a batch over all resident models: every
// converge request in flight is one active model of the batch, so a single
// replay advances all of them (continuous batching at iteration
// granularity); requests join when they arrive and leave when their model
// converges.  Render workers, each with its own stream and buffers, image
// the published populations of a model concurrently with the iterations.
// Published populations change only when a converge request succeeds, under
// a per-model lock that renders hold while they read them.

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <shared_mutex>
#include <thread>

#include "host.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t id = 0;
    int kind = MGX_REQ_CONVERGE;
    int model = 0;
    // converge
    double tol = 0.0;
    int max_iter = 0, ng_order = 0;
    // render
    double dir[3] = {0.0, 0.0, 1.0};
    int npx = 0, npy = 0, nfreq = 0;
    double f_min = 0.0, f_max = 0.0;
    float *img = nullptr;
    size_t footprint = 0;
    // outcome
    int status = MGX_EPENDING;
    double t_submit = 0.0, t_start = -1.0, t_done = -1.0;
    int iters = 0;
    double change = NAN;
    std::string msg;
};

struct RenderSlot {
    hipStream_t stream = nullptr;
    RenderBufs rb;
    size_t reserved = 0;  // footprint admitted for the running request
    size_t held = 0;      // bytes the slot's buffers hold when idle
    bool busy = false;
};

}  // namespace

struct mgx_server {
    int device = 0;
    mgx_options opt{};
    std::string err;
    mgx_batch *b = nullptr;
    Clock::time_point t0 = Clock::now();
    uint64_t budget = 0;
    int nslots = 1;
    bool started = false, stopping = false;

    std::vector<std::unique_ptr<DMem>> published;
    std::vector<std::unique_ptr<std::shared_mutex>> pub_mu;
    std::vector<int64_t> updates_per_iter;  // N x rays x lines x bins per model
    size_t resident = 0, render_peak = 0;

    std::mutex mu;
    std::condition_variable cv_iter, cv_render, cv_done;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_id = 1;
    std::vector<std::deque<Request *>> conv_pending;  // per model, arrival order
    std::vector<Request *> conv_running;              // per model
    std::deque<Request *> render_queue;
    std::vector<std::unique_ptr<RenderSlot>> slots;
    std::thread iter_thread;
    std::vector<std::thread> render_threads;

    int64_t submitted = 0, completed = 0, failed = 0, replays = 0, updates = 0;
    double iter_busy = 0.0, render_busy = 0.0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void stop();
    ~mgx_server();
};

namespace {

// Finish a request (caller holds s->mu).
void complete(mgx_server *s, Request *r, int status, const std::string &msg)
{
    r->status = status;
    r->msg = msg;
    r->t_done = s->now();
    s->completed++;
    if (status != MGX_OK) s->failed++;
    s->cv_done.notify_all();
}

// Device bytes one image needs beyond the resident model: line tables of the
// populations, projected geometry, pixel entries and walk offsets, the walks
// (estimated at 4 N^(1/3) + 16 points per pixel) and the image.
size_t render_footprint(const mgx_ctx *c, int npx, int npy, int nfreq)
{
    const size_t npix = (size_t)npx * npy;
    const size_t tsz = c->fp32() ? sizeof(float) : sizeof(double);
    const size_t walk = (size_t)render_walk_cap(c->N);
    return (size_t)c->nrad() * (2 * tsz + sizeof(double)) + 32 * (size_t)c->N + 12 * npix +
           16 * (npix + 1) + 4 * npix * walk + 4 * npix * (size_t)nfreq + (1 << 16);
}

// Bytes in use by render slots if `head` were admitted to slot j.
size_t render_use(const mgx_server *s, int j, size_t head)
{
    size_t n = 0;
    for (int k = 0; k < (int)s->slots.size(); k++) {
        const RenderSlot &sl = *s->slots[k];
        const size_t want = (k == j) ? head : (sl.busy ? sl.reserved : 0);
        n += std::max(sl.held, want);
    }
    return n;
}

void publish(mgx_server *s, int i)
{
    mgx_ctx *c = s->b->m[i];
    std::unique_lock<std::shared_mutex> wl(*s->pub_mu[i]);
    HIPCHK(hipMemcpyAsync(s->published[i]->p, c->pops.p, sizeof(double) * c->npop(),
                          hipMemcpyDeviceToDevice, s->b->stream));
    s->b->sync();
}

void iterate_worker(mgx_server *s)
{
    (void)hipSetDevice(s->device);
    mgx_batch *b = s->b;
    const int M = (int)b->m.size();
    std::vector<int> finished;
    for (;;) {
        std::vector<Request *> starting;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_iter.wait(lk, [&] {
                if (s->stopping) return true;
                for (int i = 0; i < M; i++)
                    if (s->conv_running[i] || !s->conv_pending[i].empty()) return true;
                return false;
            });
            if (s->stopping) return;
            for (int i = 0; i < M; i++)
                if (!s->conv_running[i] && !s->conv_pending[i].empty()) {
                    Request *r = s->conv_pending[i].front();
                    s->conv_pending[i].pop_front();
                    s->conv_running[i] = r;
                    r->t_start = s->now();
                    starting.push_back(r);
                }
        }
        try {
            for (Request *r : starting) {
                mgx_ctx *c = b->m[r->model];
                const mgx_status st = mgx_set_lte_populations(c);
                if (st != MGX_OK) throw Err{st, c->err};
                batch_activate(b, r->model, r->tol, r->max_iter, r->ng_order);
            }
            if (!starting.empty()) batch_push_mask(b);
            int64_t upd = 0;
            for (int i = 0; i < M; i++)
                if (b->runs[i].active) upd += s->updates_per_iter[i];
            const double t = s->now();
            finished.clear();
            batch_step(b, finished);
            for (int i : finished)
                if (b->runs[i].status == MGX_OK) publish(s, i);
            std::lock_guard<std::mutex> lk(s->mu);
            s->iter_busy += s->now() - t;
            s->replays++;
            s->updates += upd;
            for (int i : finished) {
                Request *r = s->conv_running[i];
                const BatchRun &run = b->runs[i];
                r->iters = run.iters;
                r->change = run.change;
                complete(s, r, run.status,
                         run.status == MGX_OK ? std::string() : std::string("converge failed"));
                s->conv_running[i] = nullptr;
            }
        } catch (...) {
            // a device, runtime or host failure ends every converge request in
            // flight (no exception may leave the worker thread)
            mgx_status st = MGX_EHIP;
            std::string msg = "unexpected internal error";
            try {
                throw;
            } catch (const Err &e) {
                st = e.st;
                msg = e.msg;
            } catch (const std::bad_alloc &) {
                st = MGX_ENOMEM;
                msg = "host allocation failed";
            } catch (...) {
            }
            std::lock_guard<std::mutex> lk(s->mu);
            for (int i = 0; i < M; i++) {
                if (b->runs[i].active) {
                    b->runs[i].active = false;
                    b->host_active[i] = 0;
                }
                if (s->conv_running[i]) {
                    complete(s, s->conv_running[i], st, msg);
                    s->conv_running[i] = nullptr;
                }
            }
            try {
                batch_push_mask(b);
            } catch (...) {
            }
        }
    }
}

void render_worker(mgx_server *s, int j)
{
    (void)hipSetDevice(s->device);
    RenderSlot &sl = *s->slots[j];
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stopping) return;
                if (!s->render_queue.empty()) {
                    Request *h = s->render_queue.front();
                    const size_t avail = s->budget > s->resident ? s->budget - s->resident : 0;
                    if (render_use(s, j, h->footprint) <= avail) {
                        r = h;
                        s->render_queue.pop_front();
                        break;
                    }
                    // the head fits nowhere even with every render buffer
                    // freed: it can never run
                    if (h->footprint > avail) {
                        s->render_queue.pop_front();
                        complete(s, h, MGX_ENOMEM, "render does not fit the HBM budget");
                        continue;
                    }
                    // cached buffers of idle slots stand in the way: free
                    // them all (no render reads them) and look again
                    bool freed = false;
                    for (auto &o : s->slots)
                        if (!o->busy && o->held > 0) {
                            o->rb.release();
                            o->held = 0;
                            freed = true;
                        }
                    if (freed) continue;
                }
                s->cv_render.wait(lk);
            }
            sl.busy = true;
            sl.reserved = r->footprint;
            s->render_peak = std::max(s->render_peak, render_use(s, -1, 0));
            r->t_start = s->now();
        }
        int status = MGX_OK;
        std::string msg;
        const double t = s->now();
        try {
            std::shared_lock<std::shared_mutex> rl(*s->pub_mu[r->model]);
            render_image(s->b->m[r->model], sl.rb, s->published[r->model]->as<double>(), sl.stream,
                         r->dir, r->npx, r->npy, r->f_min, r->f_max, r->nfreq, r->img);
        } catch (const Err &e) {
            status = e.st;
            msg = e.msg;
        } catch (const std::bad_alloc &) {
            status = MGX_ENOMEM;
            msg = "host allocation failed";
        } catch (...) {
            status = MGX_EHIP;
            msg = "unexpected internal error";
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->render_busy += s->now() - t;
        sl.busy = false;
        sl.reserved = 0;
        sl.held = sl.rb.bytes();
        complete(s, r, status, msg);
        s->cv_render.notify_all();
    }
}

}  // namespace

void mgx_server::stop()
{
    {
        std::lock_guard<std::mutex> lk(mu);
        stopping = true;
    }
    cv_iter.notify_all();
    cv_render.notify_all();
    if (iter_thread.joinable()) iter_thread.join();
    for (std::thread &t : render_threads)
        if (t.joinable()) t.join();
    render_threads.clear();
    std::lock_guard<std::mutex> lk(mu);
    for (auto &kv : reqs)
        if (kv.second->status == MGX_EPENDING) complete(this, kv.second.get(), MGX_ESTATE, "server stopped");
}

mgx_server::~mgx_server()
{
    stop();
    for (auto &sl : slots)
        if (sl->stream) {
            (void)hipStreamSynchronize(sl->stream);
            (void)hipStreamDestroy(sl->stream);
        }
    slots.clear();
    published.clear();
    if (b) mgx_batch_destroy(b);
}

extern "C" mgx_status mgx_server_create(mgx_server **out, int device, const mgx_options *opt,
                                        uint64_t hbm_budget, int render_slots)
{
    g_create_error.clear();
    if (!out) return MGX_EINVAL;
    *out = nullptr;
    if (render_slots < 1 || render_slots > 8) {
        g_create_error = "render_slots must be 1..8";
        return MGX_EINVAL;
    }
    mgx_options o;
    mgx_default_options(&o);
    if (opt) o = *opt;
    mgx_batch *b = nullptr;
    const mgx_status st = mgx_batch_create(&b, device, nullptr, &o);
    if (st != MGX_OK) return st;  // message already in g_create_error
    mgx_server *s = new (std::nothrow) mgx_server();
    if (!s) {
        mgx_batch_destroy(b);
        return MGX_ENOMEM;
    }
    s->device = device;
    s->opt = o;
    s->b = b;
    s->nslots = render_slots;
    s->budget = hbm_budget;
    if (s->budget == 0) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        size_t fr = 0, tot = 0;
        if (hipSetDevice(device) == hipSuccess && hipMemGetInfo(&fr, &tot) == hipSuccess)
            s->budget = tot;
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    *out = s;
    return MGX_OK;
}

extern "C" void mgx_server_destroy(mgx_server *s)
{
    if (!s) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    delete s;
    if (prev >= 0) (void)hipSetDevice(prev);
}

extern "C" const char *mgx_server_last_error(const mgx_server *s)
{
    if (!s) return g_create_error.c_str();
    return s->err.c_str();
}

extern "C" mgx_status mgx_server_add_model(mgx_server *s, const mgx_model *m, int *id_out)
{
    API_BEGIN(s)
    REQUIRE(!s->started, MGX_ESTATE, "mgx_server_add_model after mgx_server_start");
    const mgx_status st = mgx_batch_add_model(s->b, m, id_out);
    if (st != MGX_OK) throw Err{st, s->b->err};
    API_END(s)
}

extern "C" mgx_status mgx_server_start(mgx_server *s)
{
    API_BEGIN(s)
    REQUIRE(!s->started, MGX_ESTATE, "server already started");
    REQUIRE(!s->b->m.empty(), MGX_ESTATE, "server without models");
    mgx_batch *b = s->b;
    const int M = (int)b->m.size();
    batch_prepare(b);
    for (int i = 0; i < M; i++) {
        mgx_ctx *c = b->m[i];
        const mgx_status st = mgx_set_lte_populations(c);
        if (st != MGX_OK) throw Err{st, c->err};
        s->published.emplace_back(new DMem());
        s->published[i]->ensure(sizeof(double) * c->npop());
        HIPCHK(hipMemcpyAsync(s->published[i]->p, c->pops.p, sizeof(double) * c->npop(),
                              hipMemcpyDeviceToDevice, b->stream));
        s->pub_mu.emplace_back(new std::shared_mutex());
        s->updates_per_iter.push_back((int64_t)c->N * c->R * c->nlines * c->nbins);
        // Ng history for the default order (4) up front, so it counts as
        // resident; a request of higher order grows it when it starts
        ng_reset(c, 5);
        c->ng_active = false;
    }
    b->sync();
    batch_begin(b);
    s->resident = batch_bytes(b);
    for (auto &p : s->published) s->resident += p->bytes;
    REQUIRE(s->resident <= s->budget, MGX_ENOMEM,
            "resident models need " + std::to_string(s->resident) + " bytes, budget " +
                std::to_string(s->budget));
    for (int j = 0; j < s->nslots; j++) {
        s->slots.emplace_back(new RenderSlot());
        HIPCHK(hipStreamCreateWithFlags(&s->slots[j]->stream, hipStreamNonBlocking));
    }
    s->conv_pending.assign(M, {});
    s->conv_running.assign(M, nullptr);
    s->started = true;
    s->iter_thread = std::thread(iterate_worker, s);
    for (int j = 0; j < s->nslots; j++) s->render_threads.emplace_back(render_worker, s, j);
    API_END(s)
}

extern "C" double mgx_server_clock(const mgx_server *s)
{
    return s ? s->now() : 0.0;
}

extern "C" mgx_status mgx_server_submit_converge(mgx_server *s, int model, double tol,
                                                 int max_iter, int ng_order, int64_t *id_out)
{
    API_BEGIN(s)
    REQUIRE(s->started, MGX_ESTATE, "server not started");
    REQUIRE(model >= 0 && model < (int)s->b->m.size(), MGX_EINVAL, "model id out of range");
    REQUIRE(max_iter >= 1 && tol >= 0, MGX_EINVAL, "max_iter >= 1 and tol >= 0 required");
    REQUIRE(ng_order >= 0 && ng_order + 1 <= kNgMaxHist, MGX_EINVAL, "Ng order must be 0..31");
    std::unique_ptr<Request> r(new Request());
    r->kind = MGX_REQ_CONVERGE;
    r->model = model;
    r->tol = tol;
    r->max_iter = max_iter;
    r->ng_order = ng_order;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        REQUIRE(!s->stopping, MGX_ESTATE, "server stopped");
        r->id = s->next_id++;
        r->t_submit = s->now();
        if (id_out) *id_out = r->id;
        s->conv_pending[model].push_back(r.get());
        s->reqs[r->id] = std::move(r);
        s->submitted++;
    }
    s->cv_iter.notify_one();
    API_END(s)
}

extern "C" mgx_status mgx_server_submit_render(mgx_server *s, int model, const double dir[3],
                                               int npx, int npy, double f_min, double f_max,
                                               int nfreq, float *img, int64_t *id_out)
{
    API_BEGIN(s)
    REQUIRE(s->started, MGX_ESTATE, "server not started");
    REQUIRE(model >= 0 && model < (int)s->b->m.size(), MGX_EINVAL, "model id out of range");
    REQUIRE(s->b->m[model]->dim == 3, MGX_EINVAL, "images need a point cloud (dim 3)");
    REQUIRE(img, MGX_EINVAL, "img is NULL");
    check_render_args(dir, npx, npy, f_min, f_max, nfreq);
    std::unique_ptr<Request> r(new Request());
    r->kind = MGX_REQ_RENDER;
    r->model = model;
    for (int k = 0; k < 3; k++) r->dir[k] = dir[k];
    r->npx = npx;
    r->npy = npy;
    r->nfreq = nfreq;
    r->f_min = f_min;
    r->f_max = f_max;
    r->img = img;
    r->footprint = render_footprint(s->b->m[model], npx, npy, nfreq);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        REQUIRE(!s->stopping, MGX_ESTATE, "server stopped");
        r->id = s->next_id++;
        r->t_submit = s->now();
        if (id_out) *id_out = r->id;
        s->render_queue.push_back(r.get());
        s->reqs[r->id] = std::move(r);
        s->submitted++;
    }
    s->cv_render.notify_all();
    API_END(s)
}

extern "C" mgx_status mgx_server_wait(mgx_server *s, int64_t id, double timeout_s,
                                      mgx_request_info *info)
{
    if (!s) return MGX_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) {
        s->err = "unknown request id";
        return MGX_EINVAL;
    }
    Request *r = it->second.get();
    auto done = [&] { return r->status != MGX_EPENDING; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, done);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    if (info) {
        info->id = r->id;
        info->kind = r->kind;
        info->model = r->model;
        info->status = r->status;
        info->t_submit = r->t_submit;
        info->t_start = r->t_start;
        info->t_done = r->t_done;
        info->iterations = r->iters;
        info->change = r->change;
    }
    if (r->status != MGX_OK && r->status != MGX_EPENDING) s->err = r->msg;
    return (mgx_status)r->status;
}

extern "C" mgx_status mgx_server_get_populations(mgx_server *s, int model, double *pops)
{
    API_BEGIN(s)
    REQUIRE(s->started, MGX_ESTATE, "server not started");
    REQUIRE(model >= 0 && model < (int)s->b->m.size(), MGX_EINVAL, "model id out of range");
    REQUIRE(pops, MGX_EINVAL, "pops is NULL");
    const mgx_ctx *c = s->b->m[model];
    std::shared_lock<std::shared_mutex> rl(*s->pub_mu[model]);
    HIPCHK(hipMemcpy(pops, s->published[model]->p, sizeof(double) * c->npop(), hipMemcpyDefault));
    API_END(s)
}

extern "C" mgx_status mgx_server_get_stats(mgx_server *s, mgx_server_stats *out)
{
    API_BEGIN(s)
    REQUIRE(out, MGX_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    mgx_server_stats st{};
    st.models = (int)s->b->m.size();
    st.render_slots = s->nslots;
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.failed = s->failed;
    st.replays = s->replays;
    st.updates = s->updates;
    st.iterate_busy_s = s->iter_busy;
    st.render_busy_s = s->render_busy;
    st.hbm_budget = s->budget;
    st.hbm_resident = s->resident;
    st.hbm_render_peak = s->render_peak;
    *out = st;
    API_END(s)
}
