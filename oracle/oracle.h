/*
 * oracle.h -- plain, slow FP64 CPU definition of the line radiative transfer
 * hot path (ray trace, line opacity, optical depth, Feautrier formal
 * solution, mean intensity, statistical equilibrium, Ng acceleration).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library; the two read the same
 * seeded inputs and nothing else.
 *
 * All arrays are host arrays owned by the caller.  Units are SI.
 */
#ifndef MGX_ORACLE_H
#define MGX_ORACLE_H
#include <stdint.h>

typedef struct {
    int dim;                 /* 1: spherical shells, 3: point cloud          */
    int npoints;
    const double *pos;       /* [3][N]; dim 1: pos[0][k] = shell radius       */
    const double *vel;       /* [3][N]; dim 1: vel[0][k] = radial velocity    */
    const int32_t *nbs_off;  /* [N+1]                                         */
    const int32_t *nbs;      /* [nbs_off[N]]                                  */
    const uint8_t *bdy;      /* [N]                                           */
    const double *T, *vturb2, *nspec, *ncoll;   /* [N]                        */
    int nrays;
    const double *ray_dir;   /* [R][3]                                        */
    const double *ray_w;     /* [R]                                           */
    const int32_t *antipode; /* [R]                                           */
    double mass;             /* line species mass [kg]                       */
    int nlev;
    const double *E, *g;     /* [nlev]                                        */
    int nlines;
    const int32_t *up, *lo;  /* [nlines]                                      */
    const double *A, *nu;    /* [nlines]                                      */
    int ncoll_tr;
    const int32_t *cu, *cl;  /* [ncoll_tr]                                    */
    const double *K0;        /* [ncoll_tr], coefficient at 100 K              */
    int nbins;
    double xmax;
    double Tcmb;
    double branch_threshold; /* trapezoid below this Doppler shift in widths */
    double tau_floor;        /* added to every segment optical depth         */
    double chi_min;          /* masing clamp on the line opacity factor      */
    double pop_floor;        /* floor of the relative-change denominator     */
} orc_model;

/* ray trace: returns the number of records (writes at most cap) */
int orc_trace(const orc_model *m, int origin, int ray, int cap, int32_t *idx,
              double *Z, double *dv, int *hole);

/* segment branch rule: 1 if the semi-analytic optical depth is used */
int orc_use_semi_analytic(const orc_model *m, int p0, double dv0, int p1, double dv1);

/* line opacity factor chi^ij, emissivity factor eta^ij and source function */
int orc_line_coeffs(const orc_model *m, const double *pops, double *chi_ij,
                    double *eta_ij, double *S);

/* optical depth of one segment, both forms */
double orc_dtau_trapezoid(double dx, double chi0, double chi1);
double orc_dtau_semi_analytic(double dx, double chi_ij0, double chi_ij1, double d0,
                              double d1, double dnu_bar);
double orc_erf_difference(double a, double b);

/* second-order Feautrier system on a grid of M+1 points */
void orc_feautrier(int M, const double *dtau, const double *S, double I0, double IM,
                   int o, double *u_o, double *lstar_oo, double *u_all);

double orc_planck(double nu, double T);

/* mean intensity and Lambda* diagonal for one origin, all lines */
void orc_solve_origin(const orc_model *m, const double *chi_ij, const double *S,
                      int origin, double *Jbar, double *Lstar);
void orc_solve_origins(const orc_model *m, const double *chi_ij, const double *S,
                       int count, const int32_t *origins, double *Jbar, double *Lstar);

/* statistical equilibrium */
void orc_lte(const orc_model *m, double *pops);
int orc_stateq_point(const orc_model *m, int p, const double *Jbar, const double *Lstar,
                     const double *S, double *pops_out);
int orc_stateq(const orc_model *m, const double *Jbar, const double *Lstar,
               const double *S, double *pops_out);
double orc_rel_change(const orc_model *m, const double *a, const double *b, int64_t n);

/* Ng extrapolation from nhist iterates (oldest first) of length n */
int orc_ng(int nhist, int64_t n, const double *hist, double *out, double *coeffs);

/* Ng schedule flag: after a used prediction the history holds only the
   regular iterates computed after it */
#define ORC_NG_FRESH 0x10

/* one application of a fixed-point map: out = step(in); nonzero aborts */
typedef int (*orc_map_fn)(void *ud, const double *in, double *out);

/* fixed-point iteration of `step` on x[n] with ng_mode 0 none, 1 classical
   order ng_param, 2 adaptive with N_max = ng_param (| ORC_NG_FRESH);
   events[max_iter] (may be NULL) logs the Ng decision of each iteration;
   returns 0 on convergence, -5 without, -6 if step failed */
int orc_iterate_map(orc_map_fn step, void *ud, int64_t n, double pop_floor, double *x,
                    double tol, int max_iter, int ng_mode, int ng_param, int *iters_out,
                    double *change_out, double *change_hist, int8_t *events);

/* full Lambda-iteration of a model on that schedule */
int orc_iterate(const orc_model *m, double *pops, double tol, int max_iter, int ng_mode,
                int ng_param, int *iters_out, double *change_out, double *change_hist);
int orc_iterate_ev(const orc_model *m, double *pops, double tol, int max_iter, int ng_mode,
                   int ng_param, int *iters_out, double *change_out, double *change_hist,
                   int8_t *events);

/* Synthetic image (channel maps) along direction dir: npx x npy pixels over
   the projected extent of the cloud, nfreq observer-frame frequencies
   f_min..f_max.  Computes one pixel: intensity I[nfreq] and the walk (point
   indices, at most cap; *nwalk its full length, 0 if the pixel misses the
   cloud). */
void orc_render_pixel(const orc_model *m, const double *chi_ij, const double *S,
                      const double dir[3], int npx, int npy, double f_min, double f_max,
                      int nfreq, int ix, int iy, double *I, int32_t *walk, int cap,
                      int *nwalk);

int orc_num_threads(void);
void orc_set_num_threads(int n);

#endif
