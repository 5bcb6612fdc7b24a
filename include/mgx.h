/*
 * mgx.h -- C ABI of the MI355X (gfx950) line radiative transfer library.
 *
 * The library computes the hot path of non-LTE line radiative transfer on
 * a point cloud (arXiv:2411.03040, "Magritte"): for every point, every ray
 * direction and every frequency bin of every line it traces the ray through
 * the cloud, gathers the Doppler-shifted Gaussian line opacity and source
 * function along it (semi-analytic optical depth where the velocity
 * gradient is large), solves the second-order Feautrier equation on each
 * ray pair, averages the result into the mean intensity J-bar and the
 * approximate Lambda-operator diagonal, solves statistical equilibrium per
 * point and iterates, with Ng acceleration.
 *
 * Conventions for every entry point:
 *  - Status: every function returns mgx_status; no C++ exception crosses the
 *    ABI.  On failure mgx_last_error() returns a message, valid until the
 *    next call on the same context.
 *  - Pointers: "host or device" pointers may be either (unified addressing
 *    decides the copy direction).  Functions that hand results back
 *    synchronise the context's stream before returning.  Host input arrays
 *    are read during the call and never retained.
 *  - Ownership: all device state (model, traces, populations, radiation
 *    field, Ng history) is allocated by the context on its device and freed
 *    by mgx_destroy.
 *  - Call order: load_model -> trace_rays -> (set populations) ->
 *    formal_solve / update_populations / iterate.  Out-of-order calls
 *    return MGX_ESTATE.
 *  - Streams: all device work is enqueued on the stream given to
 *    mgx_create (NULL: the context creates its own).
 *  - Threading: one context must not be used from two threads at once.
 *  - Layouts: per-point arrays are [N]; per-point-per-line arrays [N][nlines]
 *    (line index fastest); populations [N][nlev] as fractions of the line
 *    species density (rows sum to 1).
 *  - Units: SI (m, m/s, K, kg, J, Hz, m^-3, m^3 s^-1, W m^-2 Hz^-1 sr^-1).
 */
#ifndef MGX_H
#define MGX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgx_ctx mgx_ctx;

typedef enum {
    MGX_OK = 0,
    MGX_EINVAL = -1,      /* invalid argument or model                      */
    MGX_ESTATE = -2,      /* call out of order                              */
    MGX_ENOMEM = -3,      /* device allocation failed                       */
    MGX_EHIP = -4,        /* HIP runtime error                              */
    MGX_ENOCONV = -5,     /* iteration did not converge within max_iter     */
    MGX_ESINGULAR = -6,   /* singular statistical-equilibrium system        */
    MGX_ENONFINITE = -7,  /* non-finite input or result                     */
    MGX_EPENDING = -8     /* server request not finished (wait timed out)   */
} mgx_status;

enum { MGX_FP64 = 0, MGX_FP32 = 1 };
enum { MGX_NG_NONE = 0, MGX_NG_CLASSICAL = 1, MGX_NG_ADAPTIVE = 2 };
/* Mask of the schedule in an ng_mode value, and a flag or'ed into it: after
   a used prediction the history is emptied and holds only the regular
   iterates computed after it (the footnote of the adaptive-Ng paragraph);
   without the flag the prediction itself is the first stored iterate. */
enum { MGX_NG_MODE_MASK = 0x0f, MGX_NG_FRESH = 0x10 };

typedef struct {
    /* Precision of the opacity gather, optical depths and Feautrier sweeps.
       MGX_FP64: all in double.  MGX_FP32: float with double accumulation of
       J-bar; statistical equilibrium and Ng always run in double. */
    int precision;
    /* Trapezoidal optical depth while the Doppler shift across a segment is
       below this many line widths, else the semi-analytic form (Section
       "Semi-analytical approximation for line optical depths"; 0.35).  At
       least MGX_MIN_BRANCH_THRESHOLD. */
    double branch_threshold;
    double tau_floor;     /* added to every segment optical depth (1e-15)    */
    double chi_min;       /* masing clamp on chi^ij [m^-1 Hz] (1e-30)         */
    double pop_floor;     /* floor of the relative-change denominator (1e-12) */
    /* 3D traces search each walk once and keep its points in a temporary of
       4 N^(1/3) + 16 points per walk when that temporary is at least this
       many bytes (and fits 16 GiB and a quarter of the free memory); smaller
       models search twice (lengths, then records).  Results are identical
       either way.  Default 4 GiB; 0: whenever it fits; < 0: never. */
    int64_t trace_slot_min_bytes;
} mgx_options;

/* Smallest accepted branch_threshold: the semi-analytic optical depth
   divides by the shift across the segment and, for arguments of opposite
   sign, forms 2 - erfc(|a|) - erfc(|b|), both of which lose precision as the
   shift goes to zero. */
#define MGX_MIN_BRANCH_THRESHOLD 0.1

/* Fills the defaults listed above (precision MGX_FP32). */
void mgx_default_options(mgx_options *opt);

/* Model description (Section "Application / programmer interface": points,
   velocities, neighbour lists, boundary, temperature, turbulence, species,
   rays, CMB boundary condition, line data).  All host arrays. */
typedef struct {
    int dim;                  /* 3: point cloud; 1: spherically symmetric shells
                                 (pos[0][k] = radius, strictly increasing,
                                 vel[0][k] = radial velocity, ray_dir[r][0] = mu,
                                 shells 0 and N-1 are the boundaries)        */
    int npoints;              /* N >= 1                                        */
    const double *pos;        /* [3][N] positions [m]                          */
    const double *vel;        /* [3][N] velocities [m/s]                       */
    const int32_t *nbs_off;   /* [N+1] CSR offsets into nbs                    */
    const int32_t *nbs;       /* [nbs_off[N]] neighbour indices; order matters:
                                 ties in the walk go to the earlier entry      */
    const uint8_t *bdy;       /* [N] 1 = boundary point                        */
    const double *T;          /* [N] gas temperature [K]                       */
    const double *vturb2;     /* [N] squared turbulent velocity [m^2/s^2]      */
    const double *nspec;      /* [N] line-species number density [m^-3]        */
    const double *ncoll;      /* [N] collision-partner density [m^-3]          */
    int nrays;                /* R, even                                       */
    const double *ray_dir;    /* [R][3] unit directions                        */
    const double *ray_w;      /* [R] weights (sum 1, equal for antipodes)      */
    const int32_t *antipode;  /* [R] index of the opposite direction           */
    double mass;              /* line species mass [kg]                        */
    int nlev;                 /* 2..64 levels                                  */
    const double *E;          /* [nlev] level energies [J]                     */
    const double *g;          /* [nlev] statistical weights                    */
    int nlines;               /* >= 1 radiative transitions                    */
    const int32_t *up, *lo;   /* [nlines] upper / lower level                  */
    const double *A;          /* [nlines] Einstein A [1/s]                     */
    const double *nu;         /* [nlines] line centre [Hz]                     */
    int ncoll_tr;             /* collisional transitions                       */
    const int32_t *cu, *cl;   /* [ncoll_tr] upper / lower level (unique pairs) */
    const double *K0;         /* [ncoll_tr] de-excitation coefficient at 100 K;
                                 K(T) = K0 sqrt(T / 100 K) [m^3/s]             */
    int nbins;                /* frequency bins per line (1..1024)             */
    double xmax;              /* bins span +-xmax local line widths            */
    double Tcmb;              /* boundary radiation temperature [K]            */
} mgx_model;

typedef struct {
    int64_t total_records;    /* trace records (sum over origins and rays)     */
    int64_t holes;            /* walks that ended on a non-boundary point      */
    int64_t semi_segments;    /* segments that use the semi-analytic form      */
    int64_t masing;           /* chi^ij clamps in the last line-coefficient pass */
    int64_t singular;         /* points with a singular stat-eq system (last pass) */
    int iterations;           /* Lambda-iterations done by mgx_iterate          */
    int ng_applied;           /* Ng predictions used                            */
    int ng_rejected;          /* Ng predictions rejected                        */
    double last_change;       /* last max relative population change            */
    int64_t fs_launches;      /* formal-solution kernel launches timed          */
    double fs_ms_total;       /* their summed duration (HIP events on the
                                 context's stream) [ms]                         */
    double fs_ms_last;        /* duration of the last one [ms]                  */
} mgx_counters;

/* Zero the timing fields of the counters. */
mgx_status mgx_reset_timers(mgx_ctx *ctx);

/* Create a context on HIP device `device`; `stream` is a hipStream_t (or
   NULL for a private stream).  opt may be NULL (defaults).  Options are
   checked before any HIP call.
   Errors: MGX_EINVAL (bad options, then bad device), MGX_EHIP. */
mgx_status mgx_create(mgx_ctx **out, int device, void *stream, const mgx_options *opt);

/* Frees all device memory of the context.  NULL is ignored. */
void mgx_destroy(mgx_ctx *ctx);

/* Last error message of the context (or of a failed mgx_create when ctx is
   NULL). */
const char *mgx_last_error(const mgx_ctx *ctx);

/* Copy a model to the device and precompute the per-point Doppler widths,
   line-centred bin offsets x_f = -xmax + 2 xmax f / (nbins - 1), the bin
   weights W_f = exp(-x_f^2) / sum exp(-x^2) (line width equation; Gaussian
   profile equation).  Replaces any previously loaded model and resets all
   derived state.  Errors: MGX_EINVAL (inconsistent sizes, indices out of
   range, rays without antipodes, nlev > 64, duplicate collisional pairs),
   MGX_ENONFINITE (non-finite inputs), MGX_ENOMEM. */
mgx_status mgx_load_model(mgx_ctx *ctx, const mgx_model *m);

/* Ray tracing (Section "Magritte design": the ray-tracing algorithm of the
   geometric data structures, which the paper defers to its earlier papers;
   the walk implemented is: from the current point step to the listed
   neighbour that lies further along the ray and is closest to the ray line,
   ties to the earlier list entry, until a boundary point is reached; for
   dim 1 the shell crossings in path order).  Every (origin, ray) is traced
   once and the records stay on the device (geometry is static).  Each
   record holds the point index, the projected distance Z from the origin,
   the projected velocity difference dv = n.(v - v_origin) and whether the
   segment ending at the record uses the semi-analytic optical depth
   (shift >= branch_threshold widths; Section "Semi-analytical approximation
   for line optical depths").  total_records_out may be NULL.
   Errors: MGX_ESTATE (no model), MGX_ENOMEM. */
mgx_status mgx_trace_rays(mgx_ctx *ctx, int64_t *total_records_out);

/* Host copy of the trace of one (origin, ray): up to cap records into idx /
   Z / dv (host or device; any may be NULL), length in *len_out. */
mgx_status mgx_get_trace(mgx_ctx *ctx, int32_t origin, int32_t ray, int32_t cap,
                         int32_t *idx, double *Z, double *dv, uint8_t *semi,
                         int32_t *len_out);

/* Record offsets of all traces: offsets[N * R + 1] (int64, host or device),
   trace of (o, r) = records offsets[o R + r] .. offsets[o R + r + 1] - 1. */
mgx_status mgx_get_trace_offsets(mgx_ctx *ctx, int64_t *offsets);

/* Bulk copy of records [first, first + count) (any output may be NULL). */
mgx_status mgx_get_trace_records(mgx_ctx *ctx, int64_t first, int64_t count, int32_t *idx,
                                 double *Z, double *dv, uint8_t *semi);

/* Level populations [N][nlev] (host or device).  set: rows must be finite,
   >= 0; they are used as given.  Errors: MGX_ESTATE before load_model. */
mgx_status mgx_set_populations(mgx_ctx *ctx, const double *pops);
mgx_status mgx_get_populations(mgx_ctx *ctx, double *pops);

/* LTE populations f_i ~ g_i exp(-E_i / k T), normalised per point
   (compute_LTE_level_populations of the radiative transfer listing in
   Section "Application / programmer interface": the initial guess of the
   non-LTE iteration).  Errors: MGX_ESTATE (no model). */
mgx_status mgx_set_lte_populations(mgx_ctx *ctx);

/* One formal solution from the current populations (the radiation-field
   half of the non-LTE iteration that compute_level_populations_sparse
   runs; opacity factorisation chi = chi^ij phi^ij(nu), Gaussian profile,
   line width and Doppler shift equations, trapezoidal-rule and
   semi-analytic optical depths of Section "Semi-analytical approximation
   for line optical depths"; the second-order Feautrier solve is the
   textbook one the paper refers to): line coefficients
   chi^ij = (h nu / 4 pi)(n_l B_lu - n_u B_ul), S = eta^ij / chi^ij, then for
   every origin, ray pair, line and bin the optical depths (trapezoidal or
   semi-analytic) and the Feautrier solve, reduced to
     Jbar  = sum_pairs 2 w_r sum_f W_f u_origin
     Lstar = sum_pairs 2 w_r sum_f W_f (T^-1)_origin,origin.
   Results stay on the device; if Jbar / Lstar are non-NULL they also
   receive copies ([N][nlines] double, host or device).
   Errors: MGX_ESTATE (no trace or populations), MGX_EHIP. */
mgx_status mgx_formal_solve(mgx_ctx *ctx, double *Jbar, double *Lstar);

/* Launch shape the formal solution uses for a model with `nlines` lines of
   `nbins` bins in `precision`: lines per workgroup (line chunk), threads per
   workgroup, and LDS bytes per workgroup at the record chunk the launch
   picks (the largest chunk that lets the workgroups the registers allow
   share a CU's 160 KiB).  A host-only query (no device needed).
   Errors: MGX_EINVAL. */
mgx_status mgx_formal_solve_shape(int precision, int nlines, int nbins, int *lines_per_chunk,
                                  int *threads, int64_t *lds_bytes);

/* Replace the device radiation field ([N][nlines] double each, host or
   device), e.g. to run statistical equilibrium on given inputs. */
mgx_status mgx_set_radiation(mgx_ctx *ctx, const double *Jbar, const double *Lstar);

/* Statistical equilibrium at every point from the current radiation field
   (the state-of-the-medium half of the iteration that
   compute_level_populations_sparse runs; the Lambda operator of the Ng
   appendix comprises this solve and the formal solution) with the
   accelerated Lambda-iteration rates (J_eff = Jbar - Lstar S_old,
   R_ul = A (1 - Lstar) + B_ul J_eff + C_ul, R_lu = B_lu J_eff + C_lu, row 0
   replaced by sum f = 1), in double.  Replaces the populations; the max over
   points and levels of |new - old| / max(new, pop_floor) goes to
   *max_rel_change_out (may be NULL).  If Ng history is active the new
   iterate is appended to it.  Errors: MGX_ESINGULAR (populations of the
   affected points are left unchanged), MGX_ENONFINITE. */
mgx_status mgx_update_populations(mgx_ctx *ctx, double *max_rel_change_out);

/* Ng acceleration (Section "Adaptive Ng-acceleration" and its appendix).
   mgx_ng_reset starts a history of at most `capacity` (2..32) iterates with
   the current populations as its first entry; each mgx_update_populations
   then appends the new iterate, as does mgx_ng_push (for iterates set with
   mgx_set_populations).  A full history drops its oldest iterate.
   Errors: MGX_EINVAL (capacity), MGX_ESTATE (no populations / no history). */
mgx_status mgx_ng_reset(mgx_ctx *ctx, int capacity);
mgx_status mgx_ng_push(mgx_ctx *ctx);

/* One decision of the Ng schedule, made after each regular iterate (the
   paper's non-LTE call takes only the Ng switch; the schedules are those of
   Section "Adaptive Ng-acceleration"):
     mode MGX_NG_CLASSICAL, order_or_nmax = N_steps: once N_steps iterates
       follow the start of the history, the prediction from all N_steps + 1
       stored iterates replaces the populations;
     mode MGX_NG_ADAPTIVE, order_or_nmax = N_max: with N >= 3 stored, the
       prediction P_N from all of them replaces the populations if
       rel(P_N, P_{N-1}) < rel(y_N, y_{N-1}) (running predictions converge
       faster than the iterates; rel is the last mgx_update_populations
       change), or if N = N_max;
   or'ed with MGX_NG_FRESH for the footnote's restart.  After a used
   prediction, or when the history is full, the history restarts.  An
   invalid prediction (see mgx_ng_predict) keeps the plain iterate.
   *applied_out (may be NULL): 1 if a prediction replaced the populations.
   Errors: MGX_ESTATE (no mgx_ng_reset), MGX_EINVAL (mode, or a parameter
   needing more history than the capacity). */
mgx_status mgx_ng_accelerate(mgx_ctx *ctx, int mode, int order_or_nmax, int *applied_out);

/* The prediction itself (appendix "Derivation of Ng-acceleration") from the
   N >= 2 stored iterates y_1..y_N: residuals r_k = y_{k+1} - y_k,
   G = R R^T, c = G^-1 1 / 1^T G^-1 1, n* = sum c_k y_{k+1}.  Invalid if G is
   numerically singular (a pivot below 1e-14 of its largest diagonal entry)
   or n* has a negative entry.  With `apply`, a valid prediction replaces
   the populations and the history restarts from the populations either
   way.  *status_out: 1 valid, 0 invalid.  *pred_change_out: relative change
   between this prediction and the previous valid one since the last
   restart (+inf if none).  coef_out (host or device, N - 1 doubles, may be
   NULL) receives c when valid.  Any output may be NULL.
   Errors: MGX_ESTATE (fewer than two stored iterates). */
mgx_status mgx_ng_predict(mgx_ctx *ctx, int apply, int *status_out, double *pred_change_out,
                          double *coef_out);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the
   prediction of mgx_ng_predict from nhist (2..32) iterates the caller keeps
   on device `device`, without a context and without allocating.
   iterates: host array of nhist device pointers, oldest first, each to n
   doubles.  prediction (n doubles), coef (nhist - 1 doubles) and status (one
   int) are device memory the caller owns: coef and prediction are written
   when the Gram matrix is regular, *status = 1 if the prediction is valid
   (regular Gram matrix, no negative entry), else 0.  All work is enqueued on
   `stream` (a hipStream_t; NULL: the default stream) and nothing is
   synchronised: the results are ready when the stream reaches them.  The
   Gram rows' partial sums, the Gram matrix and the flags live in a fixed
   area of about 265 KiB compiled into the library, one per GPU, held until
   the process ends; every call on a GPU shares it, so calls that overlap on
   one GPU (other streams, other threads) race and must be serialised by the
   caller.  Errors (message from mgx_last_error(NULL)): MGX_EINVAL (nhist
   outside 2..32, n < 1, NULL pointers, no such device), MGX_EHIP. */
mgx_status mgx_ng_predict_noalloc(int device, void *stream, const double *const *iterates,
                                  int nhist, int64_t n, double *prediction, double *coef,
                                  int *status);

/* The non-LTE solver: compute_level_populations_sparse(Ng_acc, N_iter_max)
   of the radiative transfer listing (Section "Application / programmer
   interface"), with the Ng switch widened to a schedule.  Lambda-iteration
   from the current populations until the max relative change is <= tol (at
   most max_iter iterations): line coefficients -> formal solution ->
   statistical equilibrium, then one mgx_ng_accelerate decision with
   ng_mode MGX_NG_NONE, MGX_NG_CLASSICAL (ng_param = N_steps iterates
   combined, history of ng_param + 1) or MGX_NG_ADAPTIVE (N_max = ng_param),
   optionally or'ed with MGX_NG_FRESH.  Counters report the predictions used
   and rejected.  Errors: MGX_EINVAL (mode or parameter), MGX_ENOCONV
   (populations hold the last iterate), MGX_ESINGULAR, MGX_ENONFINITE. */
mgx_status mgx_iterate(mgx_ctx *ctx, double tol, int max_iter, int ng_mode, int ng_param,
                       int *iters_out, double *final_change_out);

/* Diagnostics of the last calls. */
mgx_status mgx_get_counters(mgx_ctx *ctx, mgx_counters *out);

/* Synthetic channel maps (Listing of the radiative transfer script:
   spectral discretisation f_min..f_max with nfreq bins, image along a ray
   direction with npx x npy pixels).  Pixel rays run parallel to dir through
   the cloud's projected extent; the intensity of each pixel and frequency
   is integrated along the ray from the far side with the CMB behind it.
   img is [npy][npx][nfreq] float (host or device).  dim 3 only. */
mgx_status mgx_render_image(mgx_ctx *ctx, const double dir[3], int npx, int npy,
                            double f_min, double f_max, int nfreq, float *img);

/* ------------------------------------------------------------------------
 * Batches: many independent models (grids of medium-sized models, the
 * use the paper's limitations section names) solved together on one GPU.
 * Each model keeps its own state; every Lambda-iteration of the batch is a
 * replay of captured HIP graphs: line coefficients of every model, one
 * formal-solution launch per lane class (models grouped by workgroup size;
 * one workgroup per work item (model, origin, line chunk), items ordered
 * longest first), statistical equilibrium of every model.  Converged models
 * are masked on the device and their work items compacted away; classical Ng
 * runs per model between replays.  Per-model results equal those of a lone
 * context with the same options, bit for bit.
 * ---------------------------------------------------------------------- */
typedef struct mgx_batch mgx_batch;

/* Lane classes: class k holds the models whose workgroup (lines of one chunk
   x bins, rounded up to whole waves) has 64 (k + 1) threads. */
#define MGX_BATCH_CLASSES 16

typedef struct {
    int models;               /* models in the batch                            */
    int active;               /* models not yet converged                       */
    int iterations;           /* graph replays in the last mgx_batch_iterate    */
    int lane_classes;         /* formal-solution launches per iteration         */
    int64_t work_items;       /* (model, origin, line chunk) items              */
    int class_items[MGX_BATCH_CLASSES];    /* work items per lane class (0: unused) */
    int class_threads[MGX_BATCH_CLASSES];  /* workgroup size of each used class     */
    int class_chunk[MGX_BATCH_CLASSES];    /* tuned LDS records per half            */
    int class_order[MGX_BATCH_CLASSES];    /* tuned item order: 0 longest first,
                                              1 by model, Morton origin, chunk      */
    double tune_seconds;      /* time spent tuning the schedule                  */
    double iterate_seconds;   /* wall time of the last mgx_batch_iterate        */
    double last_converged_seconds;  /* ... until its last converged model stopped */
    /* work of one iteration over all models (lanes = lines x bins of a model) */
    int64_t updates_per_iteration;  /* sum of N x rays x lanes                  */
    int64_t lane_records;           /* sum of lanes x trace records             */
    int64_t lane_semi;              /* sum of lanes x semi-analytic segments    */
    int64_t lane_origin_pairs;      /* sum of lanes x N x ray pairs             */
    /* formal-solution launches of the last mgx_batch_iterate, timed with
       events around them on the batch stream */
    int64_t fs_launches;
    double fs_ms_total;
    double fs_ms_last;
} mgx_batch_stats;

/* Create an empty batch on `device` with options for all models.  `stream`
   must be a created (capturable) stream; NULL makes the batch create and own
   a non-blocking one.  Sub-models share it. */
mgx_status mgx_batch_create(mgx_batch **out, int device, void *stream, const mgx_options *opt);
void mgx_batch_destroy(mgx_batch *b);
const char *mgx_batch_last_error(const mgx_batch *b);

/* Copy a model into the batch (same validation as mgx_load_model); its
   index in the batch goes to *id_out.  Not after mgx_batch_prepare. */
mgx_status mgx_batch_add_model(mgx_batch *b, const mgx_model *m, int *id_out);

/* Trace every model and build the work tables.  Errors: MGX_ESTATE (empty
   batch), MGX_ENOMEM. */
mgx_status mgx_batch_prepare(mgx_batch *b);

/* LTE populations for every model / populations of one model (host or
   device pointers, [N][nlev]). */
mgx_status mgx_batch_set_lte_populations(mgx_batch *b);
mgx_status mgx_batch_set_populations(mgx_batch *b, int id, const double *pops);
mgx_status mgx_batch_get_populations(mgx_batch *b, int id, double *pops);

/* Lambda-iterate every model until its max relative change is <= tol (each
   model stops on its own), at most max_iter replays, classical Ng of order
   ng_order per model (0: none).  The first call tunes the schedule and
   captures the iteration graph.  iters[M], changes[M] (host, may be NULL)
   receive per-model iteration counts and last changes; *converged_out the
   number of converged models.  Errors: MGX_ENOCONV if any model did not
   converge, MGX_ESINGULAR / MGX_ENONFINITE as for mgx_iterate. */
mgx_status mgx_batch_iterate(mgx_batch *b, double tol, int max_iter, int ng_order, int *iters,
                             double *changes, int *converged_out);

mgx_status mgx_batch_get_stats(mgx_batch *b, mgx_batch_stats *out);

/* ------------------------------------------------------------------------
 * Server: a resident set of models answering a stream of requests.  The two
 * request kinds are the two steps of the paper's workflow (section
 * "Application / programmer interface"): determine the state of the medium
 * (level populations), then create synthetic observations of it.  Requests:
 *  - converge: restart a model from LTE and Lambda-iterate it (tolerance,
 *    iteration limit, Ng order of the request); on success its populations
 *    are published.  All converge requests in flight share every iteration
 *    (one batch replay advances all of them: continuous batching); requests
 *    for one model run one after another in arrival order.
 *  - render: a synthetic image (as mgx_render_image) of a model's published
 *    populations (LTE until its first converge completes).  Renders run on
 *    their own streams, concurrently with the iterations.
 * Admission: the resident models (geometry, traces, iteration state,
 * published populations) must fit the HBM budget at mgx_server_start
 * (MGX_ENOMEM otherwise); a render is admitted to a render slot only while
 * its estimated device footprint fits what the budget leaves, else it
 * waits; one that can never fit fails with MGX_ENOMEM.
 * Threads: one iteration worker and `render_slots` render workers inside
 * the library; the entry points may be called from any thread.  Results
 * per request are identical (bit for bit) to the same request run alone.
 * ---------------------------------------------------------------------- */
typedef struct mgx_server mgx_server;

enum { MGX_REQ_CONVERGE = 0, MGX_REQ_RENDER = 1 };

typedef struct {
    int64_t id;
    int kind;             /* MGX_REQ_CONVERGE or MGX_REQ_RENDER             */
    int model;
    int status;           /* mgx_status of the request (MGX_EPENDING: not done) */
    double t_submit;      /* seconds on the server clock (mgx_server_clock)  */
    double t_start;       /* admitted / started (-1 if not yet)             */
    double t_done;        /* finished (-1 if not yet)                       */
    int iterations;       /* converge: iterations run                       */
    double change;        /* converge: last max relative change             */
} mgx_request_info;

typedef struct {
    int models;
    int render_slots;
    int64_t submitted, completed, failed;
    int64_t replays;          /* batch iterations run                       */
    int64_t updates;          /* formal-solution point x ray x bin updates  */
    double iterate_busy_s;    /* wall time the iteration worker was busy    */
    double render_busy_s;     /* summed wall time of renders                */
    uint64_t hbm_budget;      /* bytes                                      */
    uint64_t hbm_resident;    /* bytes held by the resident models          */
    uint64_t hbm_render_peak; /* peak bytes admitted to render slots        */
} mgx_server_stats;

/* Create a server on `device`: options for every model, HBM budget in bytes
   (0: the device's total memory), render slots 1..8. */
mgx_status mgx_server_create(mgx_server **out, int device, const mgx_options *opt,
                             uint64_t hbm_budget, int render_slots);
/* Stop the workers (requests not finished end with MGX_ESTATE) and free.
   No other call on `s` may be in progress or follow: a thread blocked in
   mgx_server_wait must have returned first. */
void mgx_server_destroy(mgx_server *s);
const char *mgx_server_last_error(const mgx_server *s);

/* Copy a model into the resident set (before mgx_server_start). */
mgx_status mgx_server_add_model(mgx_server *s, const mgx_model *m, int *id_out);
/* Trace and tabulate every model, publish LTE populations, tune and capture
   the iteration, check the budget and start the workers. */
mgx_status mgx_server_start(mgx_server *s);
/* Seconds since mgx_server_create (the clock of mgx_request_info). */
double mgx_server_clock(const mgx_server *s);

/* Queue a converge request; *id_out receives its id. */
mgx_status mgx_server_submit_converge(mgx_server *s, int model, double tol, int max_iter,
                                      int ng_order, int64_t *id_out);
/* Queue a render request; img ([npy][npx][nfreq] float, host or device)
   must stay valid until the request is finished. */
mgx_status mgx_server_submit_render(mgx_server *s, int model, const double dir[3], int npx,
                                    int npy, double f_min, double f_max, int nfreq, float *img,
                                    int64_t *id_out);
/* Wait up to timeout_s seconds (< 0: no limit) for a request; fills *info
   (may be NULL).  Returns the request's status, MGX_EPENDING on timeout,
   MGX_EINVAL for an unknown id. */
mgx_status mgx_server_wait(mgx_server *s, int64_t id, double timeout_s, mgx_request_info *info);
/* Published populations of a model ([N][nlev], host or device). */
mgx_status mgx_server_get_populations(mgx_server *s, int model, double *pops);
mgx_status mgx_server_get_stats(mgx_server *s, mgx_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* MGX_H */
