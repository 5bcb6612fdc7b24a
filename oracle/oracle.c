/*
 * oracle.c -- plain FP64 CPU definition of the line radiative transfer hot
 * path.  TEST INFRASTRUCTURE ONLY: called by the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg; never by the product library.
 *
 * Written for readability against the paper (arXiv:2411.03040) and the
 * textbook definitions it relies on.  No blocking, fusion or reordering.
 * Compiled with -ffp-contract=off so that every multiply and add rounds on
 * its own (ray-trace decisions are compared bit for bit).
 *
 * Sources followed, by function:
 *   orc_trace            neighbour-walk ray tracer on the point cloud (the
 *                        paper's ray-tracing design; the walk rule is the
 *                        reading stated at the function)
 *   orc_line_coeffs      line opacity chi = chi^ij phi^ij(nu) (Section
 *                        "Semi-analytical approximation for line optical
 *                        depths", opacity factorisation), textbook chi^ij,
 *                        eta^ij from Einstein coefficients
 *   profile              Gaussian line profile and line width equations
 *   orc_dtau_trapezoid   trapezoidal-rule optical depth equation
 *   orc_dtau_semi_...    semi-analytic optical depth equation
 *   orc_use_semi_...     the 0.35 line-width switch between the two forms
 *   orc_feautrier        second-order Feautrier equation (Feautrier 1964,
 *                        boundary rows after Auer 1967) solved by Gaussian
 *                        elimination tracking the pivot excess (Rybicki &
 *                        Hummer 1991, Appendix A)
 *   orc_solve_origin     direction- and line-profile-averaged mean
 *                        intensity J-bar and approximate-operator diagonal
 *   orc_stateq_point     statistical equilibrium with the accelerated
 *                        Lambda-iteration rates (Rybicki & Hummer 1991)
 *   orc_ng               Ng prediction c = (R R^T)^-1 1 / 1^T (R R^T)^-1 1
 *                        (Section "Adaptive Ng-acceleration" and Appendix A)
 *   orc_iterate_map      the classical and adaptive Ng schedules around any
 *                        fixed-point map (Section "Adaptive Ng-acceleration",
 *                        including its footnote's reading as an option)
 *   orc_iterate          Lambda-iteration of a model on that schedule
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 exact SI values */
static const double H_PLANCK = 6.62607015e-34;
static const double K_BOLTZ = 1.380649e-23;
static const double C_LIGHT = 299792458.0;
static const double PI = 3.14159265358979323846;

#define POS(m, c, i) ((m)->pos[(int64_t)(c) * (m)->npoints + (i)])
#define VEL(m, c, i) ((m)->vel[(int64_t)(c) * (m)->npoints + (i)])

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later parallel loops (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Line width (line width equation):  delta nu = (nu / c) sqrt(2 k T / m +
 * v_turb^2).  b^2 = 2 k T / m + v_turb^2 is the squared Doppler speed.
 * ---------------------------------------------------------------------- */
static double doppler_b2(const orc_model *m, int p)
{
    return ((2.0 * K_BOLTZ) * m->T[p]) / m->mass + m->vturb2[p];
}

/* ------------------------------------------------------------------------
 * Ray trace.
 *
 * Point cloud (dim 3), reading of the neighbour walk: from the current
 * point c (initially the origin o) step to the listed neighbour j of c that
 * lies further along the ray (Z_j > Z_c, Z = (x - x_o).n) and is closest to
 * the ray line (smallest squared distance |(x_j - x_o) - Z_j n|^2); ties go
 * to the earliest entry of c's neighbour list.  The walk ends after stepping
 * onto a boundary point, or when no neighbour lies further along (a "hole"
 * if the current point is not a boundary point).
 *
 * Spherical shells (dim 1): the ray with direction cosine mu from shell o
 * has impact parameter b^2 = r_o^2 - s_o^2 (s_o = r_o mu) and crosses every
 * shell with r_k^2 > b^2 at path coordinate s = +-sqrt(r_k^2 - b^2); the
 * crossings beyond s_o are visited in order.  Shell 0 (inner) and shell N-1
 * (outer) are boundaries and end the ray.
 *
 * Each record is (point index, Z = projected distance from the origin,
 * dv = n.(v_point - v_origin)).
 * ---------------------------------------------------------------------- */
int orc_trace(const orc_model *m, int o, int r, int cap, int32_t *idx, double *Z,
              double *dv, int *hole)
{
    int n = 0;
    *hole = 0;
    if (m->dim == 1) {
        const double mu = m->ray_dir[3 * r + 0];
        const double ro = POS(m, 0, o);
        const double so = ro * mu;
        double b2 = ro * ro - so * so;
        if (b2 < 0.0) b2 = 0.0;
        const int N = m->npoints;
        if (mu >= 0.0) {
            for (int k = o + 1; k < N; k++) {
                double s = sqrt(POS(m, 0, k) * POS(m, 0, k) - b2);
                if (n < cap) {
                    idx[n] = k;
                    Z[n] = s - so;
                    dv[n] = VEL(m, 0, k) * (s / POS(m, 0, k)) - VEL(m, 0, o) * mu;
                }
                n++;
                if (m->bdy[k]) return n;
            }
            return n;
        }
        if (o == 0) return 0;  /* heading into the inner boundary */
        int k = o - 1;
        while (k >= 0 && POS(m, 0, k) * POS(m, 0, k) > b2) {
            double s = -sqrt(POS(m, 0, k) * POS(m, 0, k) - b2);
            if (n < cap) {
                idx[n] = k;
                Z[n] = s - so;
                dv[n] = VEL(m, 0, k) * (s / POS(m, 0, k)) - VEL(m, 0, o) * mu;
            }
            n++;
            if (m->bdy[k]) return n;
            k--;
        }
        for (int kk = k + 1; kk < N; kk++) {
            double s = sqrt(POS(m, 0, kk) * POS(m, 0, kk) - b2);
            if (n < cap) {
                idx[n] = kk;
                Z[n] = s - so;
                dv[n] = VEL(m, 0, kk) * (s / POS(m, 0, kk)) - VEL(m, 0, o) * mu;
            }
            n++;
            if (m->bdy[kk]) return n;
        }
        return n;
    }

    const double nx = m->ray_dir[3 * r + 0];
    const double ny = m->ray_dir[3 * r + 1];
    const double nz = m->ray_dir[3 * r + 2];
    const double xo = POS(m, 0, o), yo = POS(m, 1, o), zo = POS(m, 2, o);
    const double vxo = VEL(m, 0, o), vyo = VEL(m, 1, o), vzo = VEL(m, 2, o);
    int c = o;
    double Zc = 0.0;
    for (;;) {
        int best = -1;
        double best_d2 = INFINITY, best_Z = 0.0;
        for (int q = m->nbs_off[c]; q < m->nbs_off[c + 1]; q++) {
            const int j = m->nbs[q];
            const double ddx = POS(m, 0, j) - xo;
            const double ddy = POS(m, 1, j) - yo;
            const double ddz = POS(m, 2, j) - zo;
            const double Zj = ddx * nx + ddy * ny + ddz * nz;
            if (!(Zj > Zc)) continue;
            const double ex = ddx - Zj * nx;
            const double ey = ddy - Zj * ny;
            const double ez = ddz - Zj * nz;
            const double d2 = ex * ex + ey * ey + ez * ez;
            if (d2 < best_d2) {
                best = j;
                best_d2 = d2;
                best_Z = Zj;
            }
        }
        if (best < 0) {
            if (!m->bdy[c]) *hole = 1;
            return n;
        }
        if (n < cap) {
            idx[n] = best;
            Z[n] = best_Z;
            dv[n] = (VEL(m, 0, best) - vxo) * nx + (VEL(m, 1, best) - vyo) * ny +
                    (VEL(m, 2, best) - vzo) * nz;
        }
        n++;
        c = best;
        Zc = best_Z;
        if (m->bdy[c]) return n;
    }
}

/* ------------------------------------------------------------------------
 * Branch rule: the trapezoidal rule is used while the Doppler shift across
 * the segment is below the threshold (0.35) in line widths, else the
 * semi-analytic form.  The shift in widths is |dv1 - dv0| / b-bar with the
 * averaged width b-bar^2 = (b0^2 + b1^2) / 2 (the average of temperature and
 * turbulence, as the semi-analytic form uses); the factor nu / nu_line
 * (1 +- 1e-5) is dropped so the rule is the same for every bin.  Compared in
 * squares; equality selects the semi-analytic form.
 * ---------------------------------------------------------------------- */
int orc_use_semi_analytic(const orc_model *m, int p0, double dv0, int p1, double dv1)
{
    const double d = dv1 - dv0;
    const double thr = m->branch_threshold;
    const double bbar2 = (doppler_b2(m, p0) + doppler_b2(m, p1)) * 0.5;
    return d * d >= (thr * thr) * bbar2;
}

/* ------------------------------------------------------------------------
 * Line coefficients from populations (fractions of nspec):
 *   B_ul = A c^2 / (2 h nu^3),  B_lu = (g_u / g_l) B_ul
 *   chi^ij = (h nu / 4 pi) (n_l B_lu - n_u B_ul),  eta^ij = (h nu / 4 pi) n_u A
 *   S = eta^ij / chi^ij
 * Layout [N][nlines].  chi^ij at or below chi_min (masing) is clamped.
 * Returns the number of clamped entries.
 * ---------------------------------------------------------------------- */
int orc_line_coeffs(const orc_model *m, const double *pops, double *chi_ij,
                    double *eta_ij, double *S)
{
    int masing = 0;
    for (int p = 0; p < m->npoints; p++) {
        for (int l = 0; l < m->nlines; l++) {
            const int u = m->up[l], lw = m->lo[l];
            const double nu = m->nu[l];
            const double Bul = m->A[l] * C_LIGHT * C_LIGHT / (2.0 * H_PLANCK * nu * nu * nu);
            const double Blu = m->g[u] / m->g[lw] * Bul;
            const double nu_up = m->nspec[p] * pops[(int64_t)p * m->nlev + u];
            const double n_lo = m->nspec[p] * pops[(int64_t)p * m->nlev + lw];
            const double hnu4pi = H_PLANCK * nu / (4.0 * PI);
            double chi = hnu4pi * (n_lo * Blu - nu_up * Bul);
            const double eta = hnu4pi * nu_up * m->A[l];
            if (chi <= m->chi_min) {
                chi = m->chi_min;
                masing++;
            }
            chi_ij[(int64_t)p * m->nlines + l] = chi;
            if (eta_ij) eta_ij[(int64_t)p * m->nlines + l] = eta;
            S[(int64_t)p * m->nlines + l] = eta / chi;
        }
    }
    return masing;
}

/* Gaussian line profile phi(nu') = exp(-((nu' - nu_l)/dnu)^2) / (dnu sqrt(pi))
 * evaluated at the comoving frequency nu' = nu (1 + dv / c) of a photon that
 * has frequency nu = nu_l (1 + x_f b_o / c) in the origin's frame.  The
 * offset (nu' - nu_l) / dnu is formed in velocity units,
 * (x_f b_o + dv + x_f b_o dv / c) / b, which is the same quantity without
 * the cancellation of nu' - nu_l (nu / dnu ~ 1e6). */
static double profile_offset(double xf_bo, double dv, double b)
{
    return (xf_bo + dv + xf_bo * dv / C_LIGHT) / b;
}

double orc_planck(double nu, double T)
{
    return 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT) /
           expm1(H_PLANCK * nu / (K_BOLTZ * T));
}

/* Trapezoidal rule:  dtau = dx (chi_0 + chi_1) / 2 */
double orc_dtau_trapezoid(double dx, double chi0, double chi1)
{
    return dx * (chi0 + chi1) / 2.0;
}

/* erf(b) - erf(a), written with erfc when both arguments share a sign so the
 * difference of two numbers near +-1 does not cancel. */
double orc_erf_difference(double a, double b)
{
    if (a >= 0.0 && b >= 0.0) return erfc(a) - erfc(b);
    if (a <= 0.0 && b <= 0.0) return erfc(-b) - erfc(-a);
    return erf(b) - erf(a);
}

/* Semi-analytic optical depth: chi^ij averaged over the segment, Gaussian
 * integrated exactly along the linear frequency path between the comoving
 * frequencies at the two ends, with the averaged width dnu_bar:
 *   dtau = dx (chi0 + chi1)/2 * (erf(x1) - erf(x0)) / (2 (nu1 - nu0)),
 *   x_k = (nu_k - nu_line) / dnu_bar.
 * This is the paper's semi-analytic equation written with both end
 * frequencies (the sign convention of the shift then drops out).  The ends
 * are passed as offsets d_k = nu_k - nu_line. */
double orc_dtau_semi_analytic(double dx, double chi_ij0, double chi_ij1, double d0,
                              double d1, double dnu_bar)
{
    const double x0 = d0 / dnu_bar;
    const double x1 = d1 / dnu_bar;
    return dx * (chi_ij0 + chi_ij1) / 2.0 * orc_erf_difference(x0, x1) / (2.0 * (d1 - d0));
}

/* ------------------------------------------------------------------------
 * Second-order Feautrier system on grid points j = 0..M with segment optical
 * depths dtau[j] between j and j+1, u = (I+ + I-)/2:
 *   interior:  -A_j u_{j-1} + (1 + A_j + C_j) u_j - C_j u_{j+1} = S_j,
 *              A_j = 1/(dtau_{j-1/2} dtau_j), C_j = 1/(dtau_{j+1/2} dtau_j),
 *              dtau_j = (dtau_{j-1/2} + dtau_{j+1/2}) / 2
 *   j = 0:     (1 + 2/dt + 2/dt^2) u_0 - (2/dt^2) u_1 = S_0 + (2/dt) I_0
 *   j = M:     symmetric with I_M,
 * from the second-order Taylor boundary condition with the incoming
 * intensity I_0 (I_M).  Writing the diagonal as H_j + A_j + C_j (H = 1 in the
 * interior, 1 + 2/dt at the ends), Gaussian elimination keeps the pivot
 * excess E_j = P_j - C_j = H_j + A_j E_{j-1} / P_{j-1} (positive, no
 * cancellation; Rybicki & Hummer 1991 App. A) and back-substitutes.
 * u_o = (T^-1 R)_o and lstar_oo = (T^-1)_oo (the solution for R = e_o).
 * ---------------------------------------------------------------------- */
static void tridiag_solve(int M, const double *Aj, const double *Hj, const double *Cj,
                          const double *R, double *u, double *E, double *P, double *Zt)
{
    for (int j = 0; j <= M; j++) {
        if (j == 0) {
            E[j] = Hj[j];
            P[j] = E[j] + Cj[j];
            Zt[j] = R[j] / P[j];
        } else {
            E[j] = Hj[j] + Aj[j] * (E[j - 1] / P[j - 1]);
            P[j] = E[j] + Cj[j];
            Zt[j] = (R[j] + Aj[j] * Zt[j - 1]) / P[j];
        }
    }
    u[M] = Zt[M];
    for (int j = M - 1; j >= 0; j--) u[j] = (Cj[j] / P[j]) * u[j + 1] + Zt[j];
}

void orc_feautrier(int M, const double *dtau, const double *S, double I0, double IM, int o,
                   double *u_o, double *lstar_oo, double *u_all)
{
    if (M == 0) {
        *u_o = (I0 + IM) / 2.0;
        *lstar_oo = 0.0;
        if (u_all) u_all[0] = *u_o;
        return;
    }
    double *buf = (double *)malloc(sizeof(double) * 9 * (M + 1));
    double *Aj = buf, *Hj = buf + (M + 1), *Cj = buf + 2 * (M + 1), *R = buf + 3 * (M + 1);
    double *u = buf + 4 * (M + 1), *E = buf + 5 * (M + 1), *P = buf + 6 * (M + 1);
    double *Zt = buf + 7 * (M + 1), *e = buf + 8 * (M + 1);
    for (int j = 0; j <= M; j++) {
        if (j == 0) {
            const double dt = dtau[0];
            Aj[j] = 0.0;
            Cj[j] = 2.0 / (dt * dt);
            Hj[j] = 1.0 + 2.0 / dt;
            R[j] = S[0] + 2.0 / dt * I0;
        } else if (j == M) {
            const double dt = dtau[M - 1];
            Aj[j] = 2.0 / (dt * dt);
            Cj[j] = 0.0;
            Hj[j] = 1.0 + 2.0 / dt;
            R[j] = S[M] + 2.0 / dt * IM;
        } else {
            const double dtj = (dtau[j - 1] + dtau[j]) / 2.0;
            Aj[j] = 1.0 / (dtau[j - 1] * dtj);
            Cj[j] = 1.0 / (dtau[j] * dtj);
            Hj[j] = 1.0;
            R[j] = S[j];
        }
    }
    tridiag_solve(M, Aj, Hj, Cj, R, u, E, P, Zt);
    *u_o = u[o];
    if (u_all) memcpy(u_all, u, sizeof(double) * (M + 1));
    for (int j = 0; j <= M; j++) e[j] = (j == o) ? 1.0 : 0.0;
    tridiag_solve(M, Aj, Hj, Cj, e, u, E, P, Zt);
    *lstar_oo = u[o];
    free(buf);
}

/* ------------------------------------------------------------------------
 * One origin: for every ray pair (r, antipode r) build the pair grid
 * (the antipodal half reversed, the origin, the ray half), and for every line
 * and bin form the optical depths and solve the Feautrier system.  The bin
 * offsets are x_f = -xmax + 2 xmax f / (nbins - 1) line widths around the
 * line centre in the origin's frame; the comoving frequency at a grid point
 * of a photon that reaches the origin at nu is nu (1 + dv / c) with dv
 * projected on that half's own outward direction.
 *   Jbar  = sum_pairs 2 w_r sum_f W_f u_o,  W_f = exp(-x_f^2) / sum exp(-x^2)
 *   Lstar = sum_pairs 2 w_r sum_f W_f (T^-1)_oo
 * Incoming intensity at both ends: CMB Planck function at the end point's
 * comoving frequency.
 * ---------------------------------------------------------------------- */
void orc_solve_origin(const orc_model *m, const double *chi_ij, const double *S, int o,
                      double *Jbar, double *Lstar)
{
    const int N = m->npoints, nl = m->nlines, nb = m->nbins;
    const int cap = 2 * N + 2; /* a spherical ray crosses each shell at most twice */
    int32_t *ia = (int32_t *)malloc(sizeof(int32_t) * 2 * cap);
    int32_t *ib = ia + cap;
    double *dbl = (double *)malloc(sizeof(double) * 4 * cap);
    double *Za = dbl, *dva = dbl + cap, *Zb = dbl + 2 * cap, *dvb = dbl + 3 * cap;
    const int gcap = 2 * cap + 1;
    int32_t *gp = (int32_t *)malloc(sizeof(int32_t) * gcap);
    double *g = (double *)malloc(sizeof(double) * 6 * gcap);
    double *gZ = g, *gdv = g + gcap, *dtau = g + 2 * gcap, *Sg = g + 3 * gcap;
    double *chig = g + 4 * gcap, *nug = g + 5 * gcap;
    double *W = (double *)malloc(sizeof(double) * nb);
    double *xf = (double *)malloc(sizeof(double) * nb);

    double wsum = 0.0;
    for (int f = 0; f < nb; f++) {
        xf[f] = (nb == 1) ? 0.0 : -m->xmax + 2.0 * m->xmax * f / (nb - 1);
        W[f] = exp(-xf[f] * xf[f]);
        wsum += W[f];
    }
    for (int f = 0; f < nb; f++) W[f] /= wsum;
    for (int l = 0; l < nl; l++) Jbar[l] = Lstar[l] = 0.0;

    const double bo = sqrt(doppler_b2(m, o));
    for (int r = 0; r < m->nrays; r++) {
        const int ra = m->antipode[r];
        if (!(r < ra)) continue;
        int hole;
        const int nplus = orc_trace(m, o, r, cap, ia, Za, dva, &hole);
        const int nminus = orc_trace(m, o, ra, cap, ib, Zb, dvb, &hole);
        const int M = nplus + nminus;
        const int og = nminus;
        for (int k = 0; k < nminus; k++) {
            gp[nminus - 1 - k] = ib[k];
            gZ[nminus - 1 - k] = -Zb[k];
            gdv[nminus - 1 - k] = dvb[k];
        }
        gp[og] = o;
        gZ[og] = 0.0;
        gdv[og] = 0.0;
        for (int k = 0; k < nplus; k++) {
            gp[og + 1 + k] = ia[k];
            gZ[og + 1 + k] = Za[k];
            gdv[og + 1 + k] = dva[k];
        }
        const double wpair = 2.0 * m->ray_w[r];
        for (int l = 0; l < nl; l++) {
            const double nul = m->nu[l];
            for (int f = 0; f < nb; f++) {
                const double xf_bo = xf[f] * bo;
                const double nu = nul * (1.0 + xf_bo / C_LIGHT);
                for (int j = 0; j <= M; j++) {
                    const int p = gp[j];
                    const double b = sqrt(doppler_b2(m, p));
                    const double dnu = nul * b / C_LIGHT;
                    const double x = profile_offset(xf_bo, gdv[j], b);
                    const double phi = exp(-x * x) / (dnu * sqrt(PI));
                    chig[j] = chi_ij[(int64_t)p * nl + l] * phi;
                    Sg[j] = S[(int64_t)p * nl + l];
                    nug[j] = nu * (1.0 + gdv[j] / C_LIGHT);
                }
                for (int j = 0; j < M; j++) {
                    const int p0 = gp[j], p1 = gp[j + 1];
                    const double dx = gZ[j + 1] - gZ[j];
                    double dt;
                    if (orc_use_semi_analytic(m, p0, gdv[j], p1, gdv[j + 1])) {
                        const double bbar =
                            sqrt((doppler_b2(m, p0) + doppler_b2(m, p1)) * 0.5);
                        const double dnu_bar = nul * bbar / C_LIGHT;
                        /* end offsets (nu_k - nu_line) in frequency units, formed
                           from the velocity-unit offsets to avoid cancellation */
                        const double o0 = profile_offset(xf_bo, gdv[j], bbar) * dnu_bar;
                        const double o1 = profile_offset(xf_bo, gdv[j + 1], bbar) * dnu_bar;
                        dt = orc_dtau_semi_analytic(dx, chi_ij[(int64_t)p0 * nl + l],
                                                    chi_ij[(int64_t)p1 * nl + l], o0, o1,
                                                    dnu_bar);
                    } else {
                        dt = orc_dtau_trapezoid(dx, chig[j], chig[j + 1]);
                    }
                    dt += m->tau_floor;  /* keeps every segment depth positive */
                    dtau[j] = dt;
                }
                const double I0 = orc_planck(nug[0], m->Tcmb);
                const double IM = orc_planck(nug[M], m->Tcmb);
                double u_o, lst;
                orc_feautrier(M, dtau, Sg, I0, IM, og, &u_o, &lst, NULL);
                Jbar[l] += wpair * W[f] * u_o;
                Lstar[l] += wpair * W[f] * lst;
            }
        }
    }
    free(ia);
    free(dbl);
    free(gp);
    free(g);
    free(W);
    free(xf);
}

void orc_solve_origins(const orc_model *m, const double *chi_ij, const double *S, int count,
                       const int32_t *origins, double *Jbar, double *Lstar)
{
    const int nl = m->nlines;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < count; i++) {
        const int o = origins ? origins[i] : i;
        orc_solve_origin(m, chi_ij, S, o, Jbar + (int64_t)i * nl, Lstar + (int64_t)i * nl);
    }
}

/* ------------------------------------------------------------------------
 * Statistical equilibrium.
 * LTE (initial guess): f_i proportional to g_i exp(-E_i / k T).
 * ---------------------------------------------------------------------- */
void orc_lte(const orc_model *m, double *pops)
{
    for (int p = 0; p < m->npoints; p++) {
        double z = 0.0;
        for (int i = 0; i < m->nlev; i++) {
            pops[(int64_t)p * m->nlev + i] = m->g[i] * exp(-m->E[i] / (K_BOLTZ * m->T[p]));
            z += pops[(int64_t)p * m->nlev + i];
        }
        for (int i = 0; i < m->nlev; i++) pops[(int64_t)p * m->nlev + i] /= z;
    }
}

/* Rates with the approximate operator (accelerated Lambda-iteration):
 *   Jeff = Jbar - Lstar S_old
 *   R_ul = A (1 - Lstar) + B_ul Jeff + C_ul,   R_lu = B_lu Jeff + C_lu
 *   C_ul = n_coll K0 sqrt(T / 100 K),  C_lu = C_ul (g_u/g_l) exp(-(E_u-E_l)/kT)
 * Rate matrix M n = 0 with M_ij = R_{j->i}, M_ii = -sum_j R_{i->j}; row 0 is
 * replaced by sum_i f_i = 1; Gaussian elimination with partial pivoting. */
int orc_stateq_point(const orc_model *m, int p, const double *Jbar, const double *Lstar,
                     const double *S, double *out)
{
    const int L = m->nlev;
    double *M = (double *)calloc((size_t)L * (L + 1), sizeof(double));
#define MM(i, j) M[(i) * (L + 1) + (j)]
    for (int l = 0; l < m->nlines; l++) {
        const int u = m->up[l], lw = m->lo[l];
        const double nu = m->nu[l];
        const double Bul = m->A[l] * C_LIGHT * C_LIGHT / (2.0 * H_PLANCK * nu * nu * nu);
        const double Blu = m->g[u] / m->g[lw] * Bul;
        const double Jeff = Jbar[l] - Lstar[l] * S[l];
        const double Rul = m->A[l] * (1.0 - Lstar[l]) + Bul * Jeff;
        const double Rlu = Blu * Jeff;
        MM(lw, u) += Rul;
        MM(u, u) -= Rul;
        MM(u, lw) += Rlu;
        MM(lw, lw) -= Rlu;
    }
    const double T = m->T[p];
    for (int t = 0; t < m->ncoll_tr; t++) {
        const int u = m->cu[t], lw = m->cl[t];
        const double Cul = m->ncoll[p] * m->K0[t] * sqrt(T / 100.0);
        const double Clu = Cul * (m->g[u] / m->g[lw]) * exp(-(m->E[u] - m->E[lw]) / (K_BOLTZ * T));
        MM(lw, u) += Cul;
        MM(u, u) -= Cul;
        MM(u, lw) += Clu;
        MM(lw, lw) -= Clu;
    }
    for (int j = 0; j < L; j++) MM(0, j) = 1.0;
    for (int i = 0; i < L; i++) MM(i, L) = (i == 0) ? 1.0 : 0.0;
    int status = 0;
    for (int k = 0; k < L; k++) {
        int piv = k;
        for (int i = k + 1; i < L; i++)
            if (fabs(MM(i, k)) > fabs(MM(piv, k))) piv = i;
        if (!(fabs(MM(piv, k)) >= 1e-300)) {
            status = -6;
            break;
        }
        if (piv != k)
            for (int j = 0; j <= L; j++) {
                double t = MM(k, j);
                MM(k, j) = MM(piv, j);
                MM(piv, j) = t;
            }
        for (int i = k + 1; i < L; i++) {
            const double f = MM(i, k) / MM(k, k);
            for (int j = k; j <= L; j++) MM(i, j) -= f * MM(k, j);
        }
    }
    if (status == 0) {
        for (int i = L - 1; i >= 0; i--) {
            double s = MM(i, L);
            for (int j = i + 1; j < L; j++) s -= MM(i, j) * out[j];
            out[i] = s / MM(i, i);
        }
    }
#undef MM
    free(M);
    return status;
}

int orc_stateq(const orc_model *m, const double *Jbar, const double *Lstar, const double *S,
               double *pops_out)
{
    int status = 0;
    const int nl = m->nlines, L = m->nlev;
    for (int p = 0; p < m->npoints; p++) {
        int s = orc_stateq_point(m, p, Jbar + (int64_t)p * nl, Lstar + (int64_t)p * nl,
                                 S + (int64_t)p * nl, pops_out + (int64_t)p * L);
        if (s) status = s;
    }
    return status;
}

/* max_i |a_i - b_i| / max(a_i, floor) */
double orc_rel_change(const orc_model *m, const double *a, const double *b, int64_t n)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double den = a[i] > m->pop_floor ? a[i] : m->pop_floor;
        double d = fabs(a[i] - b[i]) / den;
        if (d > mx) mx = d;
    }
    return mx;
}

/* ------------------------------------------------------------------------
 * Ng prediction from N stored iterates y_1..y_N (oldest first).
 * Residuals r_k = y_{k+1} - y_k (k = 1..N-1), Gram G = R R^T,
 *   c = G^-1 1 / (1^T G^-1 1),   n* = sum_k c_k y_{k+1}.
 * The paper's indices reference one iterate too many (r_1 would need an
 * iterate after the newest); here each residual pairs an iterate with its
 * Lambda-image and the prediction combines the images (Ng 1974; Olson,
 * Auer & Buchler 1986).  sum c = 1 keeps sum f = 1.
 * Returns -1 if G is numerically singular (a pivot below 1e-14 max G_kk),
 * -2 if any predicted component is negative; out is then untouched.
 * ---------------------------------------------------------------------- */
int orc_ng(int nhist, int64_t n, const double *hist, double *out, double *coeffs)
{
    const int K = nhist - 1;
    if (K < 1) return -1;
    double *G = (double *)calloc((size_t)K * (K + 1), sizeof(double));
#define GG(i, j) G[(i) * (K + 1) + (j)]
    for (int a = 0; a < K; a++)
        for (int b = 0; b < K; b++) {
            double s = 0.0;
            for (int64_t i = 0; i < n; i++) {
                const double ra = hist[(int64_t)(a + 1) * n + i] - hist[(int64_t)a * n + i];
                const double rb = hist[(int64_t)(b + 1) * n + i] - hist[(int64_t)b * n + i];
                s += ra * rb;
            }
            GG(a, b) = s;
        }
    double gmax = 0.0;
    for (int a = 0; a < K; a++)
        if (GG(a, a) > gmax) gmax = GG(a, a);
    for (int a = 0; a < K; a++) GG(a, K) = 1.0;
    int status = 0;
    for (int k = 0; k < K && status == 0; k++) {
        int piv = k;
        for (int i = k + 1; i < K; i++)
            if (fabs(GG(i, k)) > fabs(GG(piv, k))) piv = i;
        if (!(fabs(GG(piv, k)) > 1e-14 * gmax)) {
            status = -1;
            break;
        }
        if (piv != k)
            for (int j = 0; j <= K; j++) {
                double t = GG(k, j);
                GG(k, j) = GG(piv, j);
                GG(piv, j) = t;
            }
        for (int i = k + 1; i < K; i++) {
            const double f = GG(i, k) / GG(k, k);
            for (int j = k; j <= K; j++) GG(i, j) -= f * GG(k, j);
        }
    }
    double *c = (double *)malloc(sizeof(double) * K);
    if (status == 0) {
        double csum = 0.0;
        for (int i = K - 1; i >= 0; i--) {
            double s = GG(i, K);
            for (int j = i + 1; j < K; j++) s -= GG(i, j) * c[j];
            c[i] = s / GG(i, i);
        }
        for (int i = 0; i < K; i++) csum += c[i];
        for (int i = 0; i < K; i++) c[i] /= csum;
        for (int64_t i = 0; i < n && status == 0; i++) {
            double s = 0.0;
            for (int k = 0; k < K; k++) s += c[k] * hist[(int64_t)(k + 1) * n + i];
            if (s < 0.0) status = -2;
        }
        if (status == 0) {
            for (int64_t i = 0; i < n; i++) {
                double s = 0.0;
                for (int k = 0; k < K; k++) s += c[k] * hist[(int64_t)(k + 1) * n + i];
                out[i] = s;
            }
            if (coeffs)
                for (int k = 0; k < K; k++) coeffs[k] = c[k];
        }
    }
#undef GG
    free(c);
    free(G);
    return status;
}

/* ------------------------------------------------------------------------
 * Fixed-point iteration x <- step(x) with Ng acceleration (Section
 * "Adaptive Ng-acceleration").  The schedule is independent of what the map
 * computes; orc_iterate drives it with one Lambda-iteration of the model.
 * Stops when the relative change max |new - old| / max(new, floor) is <= tol.
 *   ng_mode 1 (classical): once ng_param plain iterates have been stored
 *     after the start of the history, replace the iterate by the Ng
 *     prediction from the ng_param + 1 stored iterates.
 *   ng_mode 2 (adaptive): after each iterate with at least 3 stored, form the
 *     prediction P_N from all N stored iterates; use it if the relative
 *     change between the last two running predictions is below that between
 *     the last two iterates, or if N = N_max (= ng_param).
 *   A rejected prediction (singular Gram matrix, negative component) keeps
 *   the plain iterate.  Whenever a prediction is used, or the store is full,
 *   the history restarts:
 *     default: from the current populations (the prediction, if one was
 *       used, becomes y_1 of the new history);
 *     ORC_NG_FRESH (or'ed into ng_mode): after a used prediction the history
 *       is emptied and only the regular iterates computed after it are
 *       stored (the footnote of the adaptive-Ng paragraph); a full store
 *       without a used prediction restarts from the last regular iterate.
 * events[it - 1] (may be NULL): 0 no prediction formed, 1 formed and not
 * used, 2 used, 3 formed but invalid (singular or negative).
 * ---------------------------------------------------------------------- */
int orc_iterate_map(orc_map_fn step, void *ud, int64_t n, double pop_floor, double *x,
                    double tol, int max_iter, int ng_mode, int ng_param, int *iters_out,
                    double *change_out, double *change_hist, int8_t *events)
{
    const int fresh = (ng_mode & ORC_NG_FRESH) != 0;
    const int mode = ng_mode & 0xf;
    double *nw = (double *)malloc(sizeof(double) * (size_t)n);
    const int hcap = (mode == 0) ? 1 : (mode == 1 ? ng_param + 1 : ng_param);
    double *hist = (double *)malloc(sizeof(double) * (size_t)n * (hcap > 0 ? hcap : 1));
    double *pred = (double *)malloc(sizeof(double) * (size_t)n);
    double *prev_pred = (double *)malloc(sizeof(double) * (size_t)n);
    orc_model fl;  /* only pop_floor is read by orc_rel_change */
    memset(&fl, 0, sizeof(fl));
    fl.pop_floor = pop_floor;
    int have_prev = 0;
    int nh = 1;
    memcpy(hist, x, sizeof(double) * n);
    int status = -5, it = 0;
    double change = INFINITY;
    for (it = 1; it <= max_iter; it++) {
        if (events) events[it - 1] = 0;
        if (step(ud, x, nw) != 0) {
            status = -6;
            break;
        }
        change = orc_rel_change(&fl, nw, x, n);
        if (change_hist) change_hist[it - 1] = change;
        memcpy(x, nw, sizeof(double) * n);
        if (change <= tol) {
            status = 0;
            break;
        }
        if (mode == 0) continue;
        memcpy(hist + (int64_t)nh * n, nw, sizeof(double) * n);
        nh++;
        int use = 0, full = 0;
        if (mode == 1) {
            if (nh == ng_param + 1) {
                full = 1;
                if (orc_ng(nh, n, hist, pred, NULL) == 0) {
                    use = 1;
                    if (events) events[it - 1] = 2;
                } else if (events) {
                    events[it - 1] = 3;
                }
            }
        } else {
            full = (nh >= ng_param);
            if (nh >= 3) {
                const int ok = (orc_ng(nh, n, hist, pred, NULL) == 0);
                if (ok) {
                    if (have_prev &&
                        orc_rel_change(&fl, pred, prev_pred, n) <
                            orc_rel_change(&fl, hist + (int64_t)(nh - 1) * n,
                                           hist + (int64_t)(nh - 2) * n, n))
                        use = 1;
                    if (full) use = 1;
                    memcpy(prev_pred, pred, sizeof(double) * n);
                    have_prev = 1;
                }
                if (events) events[it - 1] = ok ? (use ? 2 : 1) : 3;
            }
        }
        if (use) memcpy(x, pred, sizeof(double) * n);
        if (use || full) {
            have_prev = 0;
            if (use && fresh) {
                nh = 0;
            } else {
                memcpy(hist, x, sizeof(double) * n);
                nh = 1;
            }
        }
    }
    if (it > max_iter) it = max_iter;
    *iters_out = it;
    *change_out = change;
    free(nw);
    free(hist);
    free(pred);
    free(prev_pred);
    return status;
}

/* One Lambda-iteration of a model: line coefficients -> formal solution at
 * every origin -> statistical equilibrium. */
typedef struct {
    const orc_model *m;
    double *chi, *S, *J, *Ls;
} lambda_ctx;

static int lambda_step(void *ud, const double *pops, double *out)
{
    lambda_ctx *c = (lambda_ctx *)ud;
    orc_line_coeffs(c->m, pops, c->chi, NULL, c->S);
    orc_solve_origins(c->m, c->chi, c->S, c->m->npoints, NULL, c->J, c->Ls);
    return orc_stateq(c->m, c->J, c->Ls, c->S, out);
}

int orc_iterate(const orc_model *m, double *pops, double tol, int max_iter, int ng_mode,
                int ng_param, int *iters_out, double *change_out, double *change_hist)
{
    return orc_iterate_ev(m, pops, tol, max_iter, ng_mode, ng_param, iters_out, change_out,
                          change_hist, NULL);
}

int orc_iterate_ev(const orc_model *m, double *pops, double tol, int max_iter, int ng_mode,
                   int ng_param, int *iters_out, double *change_out, double *change_hist,
                   int8_t *events)
{
    const size_t nl = (size_t)m->npoints * m->nlines;
    lambda_ctx c;
    c.m = m;
    c.chi = (double *)malloc(sizeof(double) * nl);
    c.S = (double *)malloc(sizeof(double) * nl);
    c.J = (double *)malloc(sizeof(double) * nl);
    c.Ls = (double *)malloc(sizeof(double) * nl);
    const int st = orc_iterate_map(lambda_step, &c, (int64_t)m->npoints * m->nlev, m->pop_floor,
                                   pops, tol, max_iter, ng_mode, ng_param, iters_out,
                                   change_out, change_hist, events);
    free(c.chi);
    free(c.S);
    free(c.J);
    free(c.Ls);
    return st;
}

/* ------------------------------------------------------------------------
 * Synthetic images (the API's image call: a direction, a pixel count per
 * axis, and an observer-frame frequency range).  The paper names the call
 * but not the algorithm; the reading implemented here:
 *  - orthographic view along the unit direction d; image axes
 *    e1 = unit(z x d) (unit(x x d) when |d_z| > 0.9), e2 = d x e1;
 *  - pixels tile the bounding rectangle of the projected points
 *    (u = x.e1, v = x.e2), pixel centres at the cell centres;
 *  - a pixel ray enters at the boundary point of smallest Z = x.d among those
 *    within R of the pixel line (R = max(pixel width, pixel height, h), h =
 *    bounding-box diagonal / N^(1/3)); ties to the lower index; none: the
 *    pixel sees the CMB alone;
 *  - it walks forward by the neighbour rule measured from the pixel line
 *    (next Z larger, smallest squared distance to the line, ties to the earlier
 *    list entry) until no neighbour lies further along;
 *  - along the walk, with w = d.v and the comoving frequency nu (1 - w / c),
 *    every line adds its opacity and emissivity; segment optical depths use
 *    the trapezoidal or semi-analytic form by the same switch as the solver
 *    (on |w1 - w0|); the intensity, started at the CMB at the entry point,
 *    is propagated with a source function linear in optical depth:
 *      I1 = I0 e^-dt + S0 ((1 - e^-dt)/dt - e^-dt) + S1 (1 - (1 - e^-dt)/dt),
 *    exact for linear S (series for dt < 1e-4).
 * ---------------------------------------------------------------------- */
static void render_basis(const double dir[3], double d[3], double e1[3], double e2[3])
{
    const double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    d[0] = dir[0] / n;
    d[1] = dir[1] / n;
    d[2] = dir[2] / n;
    double a[3] = {0.0, 0.0, 1.0};
    if (fabs(d[2]) > 0.9) {
        a[0] = 1.0;
        a[2] = 0.0;
    }
    double c[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
    const double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    e1[0] = c[0] / cn;
    e1[1] = c[1] / cn;
    e1[2] = c[2] / cn;
    e2[0] = d[1] * e1[2] - d[2] * e1[1];
    e2[1] = d[2] * e1[0] - d[0] * e1[2];
    e2[2] = d[0] * e1[1] - d[1] * e1[0];
}

static double proj(const orc_model *m, int j, const double e[3])
{
    return POS(m, 0, j) * e[0] + POS(m, 1, j) * e[1] + POS(m, 2, j) * e[2];
}

/* intensity contributions of a linear source over a segment of depth dt */
static void linear_source_weights(double dt, double *att, double *w0, double *w1)
{
    if (dt < 1e-4) {
        *att = exp(-dt);
        *w0 = dt / 2.0 - dt * dt / 3.0 + dt * dt * dt / 8.0;
        *w1 = dt / 2.0 - dt * dt / 6.0 + dt * dt * dt / 24.0;
        return;
    }
    const double e = exp(-dt);
    const double a = (1.0 - e) / dt;
    *att = e;
    *w0 = a - e;
    *w1 = 1.0 - a;
}

void orc_render_pixel(const orc_model *m, const double *chi_ij, const double *S,
                      const double dir[3], int npx, int npy, double f_min, double f_max,
                      int nfreq, int ix, int iy, double *I, int32_t *walk, int cap, int *nwalk)
{
    const int N = m->npoints, nl = m->nlines;
    double d[3], e1[3], e2[3];
    render_basis(dir, d, e1, e2);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = 0; j < N; j++) {
        const double u = proj(m, j, e1), v = proj(m, j, e2);
        if (u < umin) umin = u;
        if (u > umax) umax = u;
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
        for (int k = 0; k < 3; k++) {
            if (POS(m, k, j) < lo[k]) lo[k] = POS(m, k, j);
            if (POS(m, k, j) > hi[k]) hi[k] = POS(m, k, j);
        }
    }
    const double du = (umax - umin) / npx, dv = (vmax - vmin) / npy;
    const double diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                             (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double h = diag / cbrt((double)N);
    double R = du > dv ? du : dv;
    if (h > R) R = h;
    const double R2 = R * R;
    const double uc = umin + (ix + 0.5) * du, vc = vmin + (iy + 0.5) * dv;

    /* entry point */
    int entry = -1;
    double entryZ = INFINITY;
    for (int j = 0; j < N; j++) {
        if (!m->bdy[j]) continue;
        const double a = proj(m, j, e1) - uc, b = proj(m, j, e2) - vc;
        const double r2 = a * a + b * b;
        if (!(r2 <= R2)) continue;
        const double Z = proj(m, j, d);
        if (Z < entryZ) {
            entryZ = Z;
            entry = j;
        }
    }
    for (int f = 0; f < nfreq; f++) {
        const double nu = (nfreq == 1) ? f_min : f_min + (f_max - f_min) * f / (nfreq - 1);
        I[f] = orc_planck(nu, m->Tcmb);
    }
    *nwalk = 0;
    if (entry < 0) return;

    /* walk */
    int n = 0, c = entry;
    double Zc = entryZ;
    int32_t *pts = (int32_t *)malloc(sizeof(int32_t) * (N + 1));
    pts[n++] = entry;
    for (;;) {
        int best = -1;
        double bd = INFINITY, bZ = 0.0;
        for (int q = m->nbs_off[c]; q < m->nbs_off[c + 1]; q++) {
            const int j = m->nbs[q];
            const double Zj = proj(m, j, d);
            if (!(Zj > Zc)) continue;
            const double a = proj(m, j, e1) - uc, b = proj(m, j, e2) - vc;
            const double r2 = a * a + b * b;
            if (r2 < bd) {
                bd = r2;
                best = j;
                bZ = Zj;
            }
        }
        if (best < 0) break;
        pts[n++] = best;
        c = best;
        Zc = bZ;
    }
    *nwalk = n;
    for (int k = 0; k < n && k < cap; k++) walk[k] = pts[k];

    /* integration */
    for (int f = 0; f < nfreq; f++) {
        const double nu = (nfreq == 1) ? f_min : f_min + (f_max - f_min) * f / (nfreq - 1);
        double S0 = 0.0, Icur = 0.0;
        for (int k = 0; k < n; k++) {
            const int p = pts[k];
            const double w = VEL(m, 0, p) * d[0] + VEL(m, 1, p) * d[1] + VEL(m, 2, p) * d[2];
            const double b = sqrt(doppler_b2(m, p));
            /* source function S = eta / chi over all lines.  S is
               the profile-weighted mean of the line source functions; the
               weights are taken relative to the nearest line, exp(-(x_l^2 -
               x_min^2)), so S keeps its value where every profile underflows
               (large Doppler offsets) instead of becoming 0/0. */
            double dt = 0.0, x2min = INFINITY;
            for (int l = 0; l < nl; l++) {
                const double nul = m->nu[l];
                /* offset of the comoving frequency nu (1 - w/c) from the line,
                   in widths, in velocity units */
                const double x = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w) / b;
                if (x * x < x2min) x2min = x * x;
            }
            double sw = 0.0, sws = 0.0;
            for (int l = 0; l < nl; l++) {
                const double nul = m->nu[l];
                const double x = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w) / b;
                const double dnu = nul * b / C_LIGHT;
                const double wt = chi_ij[(int64_t)p * nl + l] * exp(-(x * x - x2min)) / dnu;
                sw += wt;
                sws += wt * S[(int64_t)p * nl + l];
            }
            const double S1 = sw > 0.0 ? sws / sw : 0.0;
            if (k == 0) {
                Icur = orc_planck(nu * (1.0 - w / C_LIGHT), m->Tcmb);
            } else {
                const int p0 = pts[k - 1];
                const double w0 = VEL(m, 0, p0) * d[0] + VEL(m, 1, p0) * d[1] + VEL(m, 2, p0) * d[2];
                const double dx = proj(m, p, d) - proj(m, p0, d);
                const int semi = orc_use_semi_analytic(m, p0, w0, p, w);
                for (int l = 0; l < nl; l++) {
                    const double nul = m->nu[l];
                    if (semi) {
                        const double bbar = sqrt((doppler_b2(m, p0) + doppler_b2(m, p)) * 0.5);
                        const double dnb = nul * bbar / C_LIGHT;
                        const double o0 = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w0) / bbar * dnb;
                        const double o1 = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w) / bbar * dnb;
                        dt += orc_dtau_semi_analytic(dx, chi_ij[(int64_t)p0 * nl + l],
                                                     chi_ij[(int64_t)p * nl + l], o0, o1, dnb);
                    } else {
                        const double b0 = sqrt(doppler_b2(m, p0));
                        const double x0 = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w0) / b0;
                        const double x1 = (C_LIGHT * (nu - nul) / nul - (nu / nul) * w) / b;
                        const double c0 = chi_ij[(int64_t)p0 * nl + l] * exp(-x0 * x0) /
                                          (nul * b0 / C_LIGHT * sqrt(PI));
                        const double c1 = chi_ij[(int64_t)p * nl + l] * exp(-x1 * x1) /
                                          (nul * b / C_LIGHT * sqrt(PI));
                        dt += orc_dtau_trapezoid(dx, c0, c1);
                    }
                }
                double att, wa, wb;
                linear_source_weights(dt, &att, &wa, &wb);
                Icur = Icur * att + S0 * wa + S1 * wb;
            }
            S0 = S1;
        }
        I[f] = Icur;
    }
    free(pts);
}
