// Host-side internals shared by the library's C ABI sources (context,
// batches, server): error handling, device allocations, the context and
// batch objects, and the helpers one source calls in another.
#pragma once

#include <math.h>
#include <string.h>

#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgx.h"
#include "mgx_internal.h"

extern "C" hipError_t mgx_internal_scan(int64_t *counts, int64_t *offsets, int64_t n,
                                        void **tmp, size_t *tmp_bytes, hipStream_t s);

namespace mgxh {

using namespace mgx;


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
    void swap(DMem &o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
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

// message of the last failed create call on this thread
extern thread_local std::string g_create_error;

template <typename T>
inline bool all_finite(const T *a, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite((double)a[i])) return false;
    return true;
}


}  // namespace mgxh

using namespace mgxh;

// Buffers of one synthetic-image call: projected geometry, pixel entry
// points, walks, the image, and line coefficients of the populations the
// image is made from (own copies, so an image never races an iteration).
struct RenderBufs {
    DMem proj, pix, off, walk, img;
    DMem chiT, ST, S64, cnt, act, maxn;
    std::vector<int32_t> act_host;  // lines that can be seen in the image's band
    void *scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
    RenderBufs() = default;
    RenderBufs(const RenderBufs &) = delete;
    RenderBufs &operator=(const RenderBufs &) = delete;
    ~RenderBufs() { release(); }
    void release()
    {
        for (DMem *m : {&proj, &pix, &off, &walk, &img, &chiT, &ST, &S64, &cnt, &act, &maxn})
            m->release();
        if (scan_tmp) (void)hipFree(scan_tmp);
        scan_tmp = nullptr;
        scan_tmp_bytes = 0;
    }
    size_t bytes() const
    {
        return proj.bytes + pix.bytes + off.bytes + walk.bytes + img.bytes + chiT.bytes +
               ST.bytes + S64.bytes + cnt.bytes + act.bytes + maxn.bytes + scan_tmp_bytes;
    }
};

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
    bool one_width = false;  // T and v_turb^2 the same at every point
    int ldl = 0;             // row stride of the solve's line table (chiT, ST)
    double vmax = 0, bmax = 0;  // largest |v| and Doppler width b over the points
    std::vector<double> nu_host;  // line centres
    int64_t n_records = 0;

    DMem pos, vel, nbs_off, nbs, bdy, T, vturb2, nspec, ncoll, ray_dir, ray_w, antipode;
    DMem pos4;  // positions as {x, y, z, 0} for the neighbour gathers of the walk
    DMem vel4;  // {vx, vy, vz, b^2} per point, one load per walk step
    DMem E, g, up, lo, A, nu, cu, cl, K0;
    DMem b2, b, bf, ibf, bd, ibd, xf, W;
    DMem Bul, Blu, hnu4pi, chiscale, Iref, acmb;
    DMem pair_r, pair_a, pair_w;
    DMem pops, pops_new, J, L, S64, chiT, ST;
    DMem counters;
    DMem order;  // origins in Morton order of their positions
    // trace
    DMem counts, offsets;
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
    RenderBufs rb;
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


// Entry-point bracket for any library object with `device` and `err`:
// selects the device, turns exceptions into status codes and messages.
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

namespace mgxh {

template <typename T>
inline void upload(mgx_ctx *c, DMem &d, const T *src, size_t n)
{
    d.ensure(sizeof(T) * n);
    if (n) HIPCHK(hipMemcpyAsync(d.p, src, sizeof(T) * n, hipMemcpyHostToDevice, c->stream));
}

// context internals used by the batch and server sources
void run_line_coeffs(mgx_ctx *ctx);
// (S_unit > 0: the solve-precision source function is S / S_unit, else S / Iref)
// (ldt: row stride of chiT and ST)
void line_coeffs_into(mgx_ctx *ctx, const double *pops, void *chiT, void *ST, int ldt,
                      double *S64, Counters *cnt, hipStream_t s, double S_unit = 0.0);
bool options_valid(const mgx_options &o);
void fs_shape(size_t tsize, int nlines, int nbins, int *nlc_out, int *nthreads_out,
              size_t *lds_out);
template <typename T>
FSArgs<T> fs_args(mgx_ctx *ctx);
StateqArgs stateq_args(mgx_ctx *ctx);
void ng_reset(mgx_ctx *ctx, int capacity);
void ng_append(mgx_ctx *ctx);
int ng_predict(mgx_ctx *ctx, double *pred_change);
void ng_apply(mgx_ctx *ctx, bool accepted, bool fresh = false);
int ng_schedule_step(mgx_ctx *ctx, int mode, int param, double change);
// expected points per pixel walk (4 N^(1/3) + 16): the slot size of the
// one-pass walk and the server's footprint estimate
inline int64_t render_walk_cap(int N) { return (int64_t)(4.0 * cbrt((double)N) + 16.0); }
void check_render_args(const double dir[3], int npx, int npy, double f_min, double f_max,
                       int nfreq);
// Synthetic image of populations `pops` of the model in ctx, on stream s,
// with the buffers of rb; img is host or device memory.
void render_image(mgx_ctx *ctx, RenderBufs &rb, const double *pops, hipStream_t s,
                  const double dir[3], int npx, int npy, double f_min, double f_max, int nfreq,
                  float *img);
// device bytes held by a context
size_t ctx_bytes(const mgx_ctx *ctx);
// points 0..N-1 in Morton (Z-curve) order of their positions ([3][N]), 10
// bits per axis over the bounding box, ties by index
std::vector<int32_t> morton_order(const double *pos, int N);

}  // namespace mgxh

// Progress of one model of a batch through its current iteration run.
struct BatchRun {
    bool active = false;
    int iters = 0, max_iter = 0, ng_order = 0;
    double tol = 0.0, change = INFINITY;
    mgx_status status = MGX_OK;
};

struct mgx_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mgx_options opt{};
    std::string err;
    std::vector<mgx_ctx *> m;
    bool prepared = false, tuned = false;
    // device tables
    DMem descs, active, all_active, changes, cnt_ptrs, counts, tune_count;
    // work items per class: every item in the tuned order (longest first, or
    // by model and Morton origin), and the items of the models still
    // iterating (same order; *counts[k] of them)
    DMem items_all[MGX_BATCH_CLASSES], items[MGX_BATCH_CLASSES];
    // the same items by model, origin in Morton order and line chunk (the
    // tuner keeps the faster order in items_all; freed after tuning)
    DMem items_alt[MGX_BATCH_CLASSES];
    DMem sample[MGX_BATCH_CLASSES];  // strided sample of the items, for tuning
    int class_nsample[MGX_BATCH_CLASSES] = {};
    void *select_tmp = nullptr;
    size_t select_tmp_bytes = 0;
    int nclass = 0;
    // lane class k: workgroups of 64 (k + 1) threads
    int class_threads[MGX_BATCH_CLASSES] = {};
    int class_nitems[MGX_BATCH_CLASSES] = {};
    int class_nlc_max[MGX_BATCH_CLASSES] = {};
    int class_nb_max[MGX_BATCH_CLASSES] = {};
    int class_ch[MGX_BATCH_CLASSES] = {};
    int class_order[MGX_BATCH_CLASSES] = {};  // 0 longest first, 1 by model and origin
    int64_t work_items = 0;
    std::vector<int> host_active;
    std::vector<BatchRun> runs;
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

namespace mgxh {

// batch internals used by the server source
void batch_prepare(mgx_batch *b);  // trace every model, build the work tables
void batch_begin(mgx_batch *b);    // tune the schedule and capture the graphs (once)
// start iterating model i (its populations are the start), with its own
// tolerance, iteration limit and Ng order; takes effect at batch_push_mask
void batch_activate(mgx_batch *b, int i, double tol, int max_iter, int ng_order);
void batch_push_mask(mgx_batch *b);  // upload the mask, compact the work items
// one iteration of every active model (synchronised): per-model changes
// [M] and failure flags [M] into `changes`
void batch_replay(mgx_batch *b, std::vector<double> &changes);
// batch_replay plus per-model bookkeeping: convergence, limits, failures and
// Ng; models that stopped are appended to `finished` (and masked)
void batch_step(mgx_batch *b, std::vector<int> &finished);
size_t batch_bytes(const mgx_batch *b);

}  // namespace mgxh
