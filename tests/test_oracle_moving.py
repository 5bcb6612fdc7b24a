"""Pin of the oracle's formal solution in a moving medium.

A lattice column traced along the coordinate axes only: every ray pair is a
straight line of lattice points, so the pair grid, the Doppler shifts, the
optical depths, the boundary intensities and the Feautrier system can all be
written down independently of the oracle and solved at 60 digits.

* Hubble-flow column (uniform temperature, v_x linear in x, every segment
  along x shifted by more than 0.35 widths): the optical depth of each
  segment is the integral of the Gaussian profile along the linear
  comoving-frequency path (Doppler shift equation, Gaussian profile and
  line width equations), computed here by adaptive quadrature, so the
  semi-analytic optical depth of the paper must reproduce it exactly.
* Temperature-gradient column (T linear in x, v_x cubic in x): the local
  widths differ from the averaged width, and the segments next to the
  origin are trapezoidal while those further out are semi-analytic; the
  optical depths follow the trapezoidal-rule and semi-analytic equations.

In both, the comoving frequency at a grid point is derived from the photon's
own direction of travel (towards the origin), the boundary intensity is the
CMB at the end point's comoving frequency, and the second-order Feautrier
system (Auer 1967 boundary rows) is solved densely.  Each test also shows
that the bar would catch the two plausible assembly mistakes: the -n half's
Doppler shift not mirrored, and the CMB taken at the origin-frame frequency.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_2411_03040_amd import synth

DPS = 60


def _mp_consts():
    return (mpmath.mpf("6.62607015e-34"), mpmath.mpf("1.380649e-23"),
            mpmath.mpf(299792458))


def _planck_mp(nu, T):
    h, kb, c = _mp_consts()
    return 2 * h * nu ** 3 / c ** 2 / mpmath.expm1(h * nu / (kb * T))


def _feautrier_dense(dtau, S, I0, IM, o):
    """Second-order Feautrier system, dense LU at working precision."""
    M = len(dtau)
    T = mpmath.zeros(M + 1, M + 1)
    R = mpmath.matrix(list(S))
    for j in range(M + 1):
        if j == 0:
            d = dtau[0]
            T[0, 0] = 1 + 2 / d + 2 / d ** 2
            T[0, 1] = -2 / d ** 2
            R[0] += 2 / d * I0
        elif j == M:
            d = dtau[M - 1]
            T[M, M] = 1 + 2 / d + 2 / d ** 2
            T[M, M - 1] = -2 / d ** 2
            R[M] += 2 / d * IM
        else:
            dj = (dtau[j - 1] + dtau[j]) / 2
            T[j, j - 1] = -1 / (dtau[j - 1] * dj)
            T[j, j + 1] = -1 / (dtau[j] * dj)
            T[j, j] = 1 - T[j, j - 1] - T[j, j + 1]
    u = mpmath.lu_solve(T, R)
    e = mpmath.matrix([1 if j == o else 0 for j in range(M + 1)])
    x = mpmath.lu_solve(T, e)
    return u[o], x[o]


def _column_model(n, T_of_i, vx_of_i, nspec, nbins=7, nlev=3):
    """n^3 lattice, axis rays, rotor species; T and v_x depend on the x index."""
    m = synth.cubic_lattice(n=n, nbins=nbins)
    sp = synth.rotor_species(nlev, np.random.default_rng(5))
    for k, v in sp.items():
        setattr(m, k, v)
    ix = np.rint(m.pos[0] / 1e12).astype(int)
    m.T = np.array([T_of_i(i) for i in ix], np.float64)
    m.vel = np.zeros((3, m.npoints))
    m.vel[0] = [vx_of_i(i) for i in ix]
    m.nspec[:] = nspec
    ax = np.eye(3)
    return synth.with_rays(m, np.concatenate([ax, -ax]))


def _lattice_index(n, c):
    return (c[0] * n + c[1]) * n + c[2]


def _reference(m, n, oc, *, quad_linear, mirror=True, cmb_comoving=True):
    """J-bar and Lambda-bar* at lattice point oc, at DPS digits.

    quad_linear: optical depth of every semi-analytic segment by quadrature of
    the Gaussian along the (linear) comoving-frequency path instead of the
    paper's closed form (valid when the velocity is linear along the segment
    and the width uniform)."""
    mpmath.mp.dps = DPS
    h, kb, c = _mp_consts()
    mass = mpmath.mpf(m.mass)
    N = m.npoints
    b = [mpmath.sqrt(2 * kb * mpmath.mpf(m.T[p]) / mass + mpmath.mpf(m.vturb2[p]))
         for p in range(N)]
    # LTE populations and line coefficients (textbook definitions)
    L, nl = m.nlev, m.nlines
    chi = [[None] * nl for _ in range(N)]
    Sl = [[None] * nl for _ in range(N)]
    for p in range(N):
        w = [mpmath.mpf(m.g[i]) * mpmath.exp(-mpmath.mpf(m.E[i]) / (kb * mpmath.mpf(m.T[p])))
             for i in range(L)]
        z = sum(w)
        f = [x / z for x in w]
        n_sp = mpmath.mpf(m.nspec[p])
        for l in range(nl):
            u, lo = int(m.up[l]), int(m.lo[l])
            nu = mpmath.mpf(m.nu[l])
            A = mpmath.mpf(m.A[l])
            Bul = A * c ** 2 / (2 * h * nu ** 3)
            Blu = mpmath.mpf(m.g[u]) / mpmath.mpf(m.g[lo]) * Bul
            k = h * nu / (4 * mpmath.pi)
            chi[p][l] = k * n_sp * (f[lo] * Blu - f[u] * Bul)
            Sl[p][l] = k * n_sp * f[u] * A / chi[p][l]
    nb = m.nbins
    xf = [(-m.xmax + 2 * mpmath.mpf(m.xmax) * f / (nb - 1)) for f in range(nb)]
    Wf = [mpmath.exp(-x * x) for x in xf]
    ws = sum(Wf)
    Wf = [x / ws for x in Wf]
    o = _lattice_index(n, oc)
    vo = [mpmath.mpf(m.vel[k][o]) for k in range(3)]
    Jb = [mpmath.mpf(0)] * nl
    Lb = [mpmath.mpf(0)] * nl
    thr = mpmath.mpf("0.35")
    for axis in range(3):
        nvec = [0, 0, 0]
        nvec[axis] = 1
        # points of the +n half and of the -n half, from the origin outwards
        # (the walk stops on the first face point)
        halves = []
        for sgn in (1, -1):
            pts = []
            k = oc[axis] + sgn
            while 0 <= k <= n - 1:
                cc = list(oc)
                cc[axis] = k
                pts.append(_lattice_index(n, cc))
                if k in (0, n - 1):
                    break
                k += sgn
            halves.append(pts)
        plus, minus = halves
        grid = list(reversed(minus)) + [o] + plus
        # photon direction of travel at each grid point: towards the origin
        dirn = [+1] * len(minus) + [0] + [-1] * len(plus)
        og = len(minus)
        M = len(grid) - 1
        # ray-pair weight: 2 w_r with w_r = 1/6
        wpair = mpmath.mpf(2) / 6
        for l in range(nl):
            nul = mpmath.mpf(m.nu[l])
            for f in range(nb):
                nu = nul * (1 + xf[f] * b[o] / c)
                nup = []
                for j, p in enumerate(grid):
                    dv = mpmath.mpf(m.vel[axis][p]) - vo[axis]
                    s = dirn[j] if mirror else (-1 if j != og else 0)
                    # comoving frequency: nu (1 - n_photon . (v_p - v_o) / c)
                    nup.append(nu * (1 - s * dv / c))
                x = [(nup[j] - nul) / (nul * b[p] / c) for j, p in enumerate(grid)]
                dtau = []
                for j in range(M):
                    p0, p1 = grid[j], grid[j + 1]
                    dx = mpmath.mpf(1e12)
                    bbar = mpmath.sqrt((b[p0] ** 2 + b[p1] ** 2) / 2)
                    shift = abs(mpmath.mpf(m.vel[axis][p1]) - mpmath.mpf(m.vel[axis][p0])) / bbar
                    assert abs(shift - thr) > mpmath.mpf("0.01")  # well clear of the switch
                    if shift >= thr:
                        dnub = nul * bbar / c
                        xb0 = (nup[j] - nul) / dnub
                        xb1 = (nup[j + 1] - nul) / dnub
                        chibar = (chi[p0][l] + chi[p1][l]) / 2
                        if quad_linear:
                            g = lambda t: mpmath.exp(-(xb0 + (xb1 - xb0) * t) ** 2)
                            dt = chibar / (dnub * mpmath.sqrt(mpmath.pi)) * dx * \
                                mpmath.quad(g, [0, 1])
                        else:
                            dt = dx * chibar * (mpmath.erf(xb1) - mpmath.erf(xb0)) / \
                                (2 * dnub * (xb1 - xb0))
                    else:
                        phi0 = mpmath.exp(-x[j] ** 2) / (nul * b[p0] / c * mpmath.sqrt(mpmath.pi))
                        phi1 = mpmath.exp(-x[j + 1] ** 2) / (nul * b[p1] / c *
                                                             mpmath.sqrt(mpmath.pi))
                        dt = dx * (chi[p0][l] * phi0 + chi[p1][l] * phi1) / 2
                    # optical-depth floor, added (far-wing lanes of the shifted halves)
                    dtau.append(dt + mpmath.mpf("1e-15"))
                Tc = mpmath.mpf(m.Tcmb)
                if cmb_comoving:
                    I0, IM = _planck_mp(nup[0], Tc), _planck_mp(nup[M], Tc)
                else:
                    I0 = IM = _planck_mp(nu, Tc)
                S = [Sl[p][l] for p in grid]
                uo, lo_ = _feautrier_dense(dtau, S, I0, IM, og)
                Jb[l] += wpair * Wf[f] * uo
                Lb[l] += wpair * Wf[f] * lo_
    return np.array([float(v) for v in Jb]), np.array([float(v) for v in Lb])


def _oracle_at(m, n, oc):
    o = oracle.Oracle(m)
    pops = o.lte()
    J, L = o.solve_origins(pops, np.array([_lattice_index(n, oc)], np.int32))
    return J[0], L[0], o


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def test_hubble_flow_column_against_quadrature():
    n = 9
    oc = (3, 4, 4)          # off-centre: halves of 3 and 5 points along x
    sp = synth.rotor_species(3, np.random.default_rng(5))
    b = math.sqrt(2 * 1.380649e-23 * 40.0 / sp["mass"] + 150.0 ** 2)
    g = 1.3 * b             # 1.3 widths per lattice segment along x
    m = _column_model(n, lambda i: 40.0, lambda i: g * (i - 4), nspec=6e7)
    J, L, orc = _oracle_at(m, n, oc)
    # every x segment is semi-analytic, every y/z segment static (trapezoid)
    idx, _, dv, _ = orc.trace(_lattice_index(n, oc), 0)
    assert list(idx) == [_lattice_index(n, (i, 4, 4)) for i in range(4, 9)]
    Jr, Lr = _reference(m, n, oc, quad_linear=True)
    assert _rel(J, Jr) < 1e-12, (J, Jr)
    assert _rel(L, Lr) < 1e-12, (L, Lr)
    # the line is optically thick at line centre along x, so the shifts matter
    Js, Ls = _reference(m, n, oc, quad_linear=True, mirror=False)
    assert _rel(J, Js) > 1e-6 and _rel(L, Ls) > 1e-4
    Jc, _ = _reference(m, n, oc, quad_linear=True, cmb_comoving=False)
    assert _rel(J, Jc) > 1e-9


def test_temperature_gradient_column_mixed_branches():
    n = 9
    oc = (3, 4, 4)
    sp = synth.rotor_species(3, np.random.default_rng(5))
    b = math.sqrt(2 * 1.380649e-23 * 60.0 / sp["mass"] + 150.0 ** 2)
    v1 = 0.15 * b            # cubic: shifts 0.15, 1.05, 2.85, ... widths
    m = _column_model(n, lambda i: 40.0 + 6.0 * i, lambda i: v1 * (i - 3) ** 3, nspec=6e7)
    J, L, orc = _oracle_at(m, n, oc)
    o = _lattice_index(n, oc)
    semi = []
    for r in (0, 3):         # +x and -x
        idx, Z, dv, _ = orc.trace(o, r)
        prev_p, prev_dv = o, 0.0
        for p, d in zip(idx, dv):
            semi.append(orc.use_semi_analytic(prev_p, prev_dv, int(p), d))
            prev_p, prev_dv = int(p), d
    assert any(semi) and not all(semi)
    Jr, Lr = _reference(m, n, oc, quad_linear=False)
    assert _rel(J, Jr) < 1e-12, (J, Jr)
    assert _rel(L, Lr) < 1e-12, (L, Lr)
    Js, Ls = _reference(m, n, oc, quad_linear=False, mirror=False)
    assert _rel(J, Js) > 1e-9 and _rel(L, Ls) > 1e-6
