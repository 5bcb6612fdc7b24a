"""Seeded synthetic model generators.

This module builds the *inputs* of the line radiative transfer problem: point
clouds, neighbour lists, ray sets, thermodynamic fields and synthetic line
data.  It holds none of the radiative-transfer arithmetic (no profiles, no
optical depths, no Feautrier, no statistical equilibrium) and imports neither
the oracle nor the HIP library, so both sides can read identical inputs.

Model inputs follow the Magritte model description (Section "Application /
programmer interface": positions and velocities of shape (npoints, 3), a
linearised neighbour list with per-point counts, boundary indices, gas
temperature, squared turbulent velocity, species abundances, uniform rays,
CMB boundary condition, line data).  The paper's LAMDA files and datasets are
not used; every workload here is synthetic and seeded.

Units are SI throughout (m, m/s, K, kg, J, m^-3, m^3 s^-1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Physical constants used only to *generate* inputs (CODATA 2018, exact SI).
_H = 6.62607015e-34
_KB = 1.380649e-23
_C = 299792458.0
_AMU = 1.66053906660e-27
_EPS0 = 8.8541878128e-12
_DEBYE = 3.33564095198152e-30  # C m
T_CMB = 2.72548


@dataclasses.dataclass
class Model:
    """Host-side model description (structure-of-arrays, float64 / int32)."""

    dim: int                      # 1 = spherically symmetric shells, 3 = point cloud
    pos: np.ndarray               # (3, N) float64; dim 1: pos[0] = shell radius
    vel: np.ndarray               # (3, N) float64; dim 1: vel[0] = radial velocity
    nbs_off: np.ndarray           # (N+1,) int32 CSR offsets
    nbs: np.ndarray               # (E,)   int32 neighbour indices (order significant)
    bdy: np.ndarray               # (N,)   uint8 boundary flag
    T: np.ndarray                 # (N,)   gas temperature [K]
    vturb2: np.ndarray            # (N,)   squared turbulent velocity [m^2 s^-2]
    nspec: np.ndarray             # (N,)   line-species number density [m^-3]
    ncoll: np.ndarray             # (N,)   collision-partner number density [m^-3]
    ray_dir: np.ndarray           # (R, 3) unit vectors; dim 1: ray_dir[:,0] = mu
    ray_w: np.ndarray             # (R,)   weights, sum 1
    antipode: np.ndarray          # (R,)   int32 index of -n
    mass: float                   # line species mass [kg]
    E: np.ndarray                 # (nlev,) level energies [J]
    g: np.ndarray                 # (nlev,) statistical weights
    up: np.ndarray                # (nlines,) int32 upper level
    lo: np.ndarray                # (nlines,) int32 lower level
    A: np.ndarray                 # (nlines,) Einstein A [s^-1]
    nu: np.ndarray                # (nlines,) line centre [Hz]
    cu: np.ndarray                # (ncoll_tr,) int32 collisional upper level
    cl: np.ndarray                # (ncoll_tr,) int32 collisional lower level
    K0: np.ndarray                # (ncoll_tr,) de-excitation coefficient at 100 K [m^3 s^-1]
    nbins: int = 31               # frequency bins per line
    xmax: float = 5.0             # bins span +-xmax line widths
    Tcmb: float = T_CMB
    name: str = "model"

    @property
    def npoints(self) -> int:
        return int(self.pos.shape[1])

    @property
    def nrays(self) -> int:
        return int(self.ray_dir.shape[0])

    @property
    def nlev(self) -> int:
        return int(self.E.shape[0])

    @property
    def nlines(self) -> int:
        return int(self.A.shape[0])

    def copy(self) -> "Model":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        return Model(**kw)

    def validate(self) -> None:
        N = self.npoints
        assert self.pos.shape == (3, N) and self.vel.shape == (3, N)
        assert self.nbs_off.shape == (N + 1,) and self.nbs_off[0] == 0
        assert self.nbs_off[-1] == self.nbs.shape[0]
        assert self.bdy.shape == (N,)
        for a in (self.T, self.vturb2, self.nspec, self.ncoll):
            assert a.shape == (N,) and np.all(np.isfinite(a))
        R = self.nrays
        assert self.ray_w.shape == (R,) and self.antipode.shape == (R,)
        assert np.all(self.antipode[self.antipode] == np.arange(R))
        assert np.all(self.ray_dir[self.antipode] == -self.ray_dir)

    def arrays(self) -> dict:
        """Contiguous typed arrays, ready to hand to a C ABI."""
        f8 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i4 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        return dict(
            pos=f8(self.pos), vel=f8(self.vel), nbs_off=i4(self.nbs_off), nbs=i4(self.nbs),
            bdy=np.ascontiguousarray(self.bdy, dtype=np.uint8), T=f8(self.T),
            vturb2=f8(self.vturb2), nspec=f8(self.nspec), ncoll=f8(self.ncoll),
            ray_dir=f8(self.ray_dir), ray_w=f8(self.ray_w), antipode=i4(self.antipode),
            E=f8(self.E), g=f8(self.g), up=i4(self.up), lo=i4(self.lo), A=f8(self.A),
            nu=f8(self.nu), cu=i4(self.cu), cl=i4(self.cl), K0=f8(self.K0))


# --------------------------------------------------------------------------
# Ray sets
# --------------------------------------------------------------------------

def healpix_directions(nside: int) -> np.ndarray:
    """HEALPix ring-scheme pixel centres (Gorski et al. 2005), (12 nside^2, 3).

    Antipodal pixels are made exact negatives of each other so that ray pairs
    are unambiguous.
    """
    dirs = []
    n = nside
    for i in range(1, 4 * n):
        if i < n:                       # north polar cap
            z = 1.0 - i * i / (3.0 * n * n)
            phis = [math.pi / (2 * i) * (j - 0.5) for j in range(1, 4 * i + 1)]
        elif i <= 3 * n:                # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * n)
            s = (i - n + 1) % 2
            phis = [math.pi / (2 * n) * (j - s / 2.0) for j in range(1, 4 * n + 1)]
        else:                           # south polar cap
            ii = 4 * n - i
            z = -1.0 + ii * ii / (3.0 * n * n)
            phis = [math.pi / (2 * ii) * (j - 0.5) for j in range(1, 4 * ii + 1)]
        st = math.sqrt(max(0.0, 1.0 - z * z))
        for p in phis:
            dirs.append((st * math.cos(p), st * math.sin(p), z))
    d = np.array(dirs, dtype=np.float64)
    assert d.shape[0] == 12 * n * n
    return _make_exact_antipodes(d)


def _make_exact_antipodes(d: np.ndarray) -> np.ndarray:
    R = d.shape[0]
    d = d.copy()
    done = np.zeros(R, dtype=bool)
    for r in range(R):
        if done[r]:
            continue
        dist = np.linalg.norm(d + d[r], axis=1)
        dist[r] = np.inf
        dist[done] = np.inf
        a = int(np.argmin(dist))
        assert dist[a] < 1e-9, "ray set has no antipode"
        d[a] = -d[r]
        done[r] = done[a] = True
    return d


def antipodes(d: np.ndarray) -> np.ndarray:
    R = d.shape[0]
    out = np.empty(R, dtype=np.int32)
    for r in range(R):
        m = np.where(np.all(d == -d[r], axis=1))[0]
        assert m.size == 1
        out[r] = m[0]
    return out


def rays_3d(nside: int):
    d = healpix_directions(nside)
    R = d.shape[0]
    return d, np.full(R, 1.0 / R), antipodes(d)


def rays_1d(nmu: int):
    """Gauss-Legendre direction cosines on [-1, 1] for spherical symmetry."""
    assert nmu % 2 == 0
    mu, w = np.polynomial.legendre.leggauss(nmu)
    half = nmu // 2
    pos_mu = mu[half:]
    pos_w = w[half:]
    mus = np.concatenate([-pos_mu[::-1], pos_mu])
    ws = np.concatenate([pos_w[::-1], pos_w]) / 2.0
    d = np.zeros((nmu, 3))
    d[:, 0] = mus
    d[:, 1] = np.sqrt(1.0 - mus * mus)
    d[half:, 1] = d[:half, 1][::-1]
    # make (mu, s, 0) and (-mu, -s, 0) exact antipodes
    d[:half] = -d[half:][::-1]
    return d, ws, antipodes(d)


# --------------------------------------------------------------------------
# Geometry helpers
# --------------------------------------------------------------------------

def knn_lists(pos: np.ndarray, k: int):
    """Directed k-nearest-neighbour lists, sorted by (distance, index)."""
    from scipy.spatial import cKDTree
    P = pos.T
    N = P.shape[0]
    tree = cKDTree(P)
    dist, idx = tree.query(P, k=k + 1)
    self_hit = idx == np.arange(N)[:, None]
    # drop the point itself (or the farthest candidate if it was not returned)
    drop = np.where(self_hit.any(axis=1), self_hit.argmax(axis=1), k)
    keep = np.ones_like(self_hit)
    keep[np.arange(N), drop] = False
    idx = idx[keep].reshape(N, k)
    dist = dist[keep].reshape(N, k)
    order = np.lexsort((idx, dist), axis=1)
    nbs = np.take_along_axis(idx, order, axis=1).astype(np.int32)
    off = np.arange(0, N * k + 1, k, dtype=np.int32)
    return off, nbs.reshape(-1)


def _uniform_in_shell(rng, n, r0, r1):
    u = rng.random(n)
    r = (r0 ** 3 + u * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return (v * r[:, None]).T.copy()


def _mode_field(rng, nmodes, kmin, kmax):
    """Unit-variance Gaussian random field from seeded Fourier modes."""
    kdir = rng.normal(size=(nmodes, 3))
    kdir /= np.linalg.norm(kdir, axis=1)[:, None]
    kmag = rng.uniform(kmin, kmax, size=nmodes)
    kv = kdir * kmag[:, None]
    ph = rng.uniform(0, 2 * np.pi, size=nmodes)

    def f(pos):
        arg = kv @ pos + ph[:, None]
        return math.sqrt(2.0 / nmodes) * np.cos(arg).sum(axis=0)
    return f


# --------------------------------------------------------------------------
# Synthetic line data
# --------------------------------------------------------------------------

def two_level_species(nu0=100e9, A=1e-5, gu=3.0, gl=1.0, K=1e-16, mass_amu=28.0):
    return dict(
        mass=mass_amu * _AMU, E=np.array([0.0, _H * nu0]), g=np.array([gl, gu]),
        up=np.array([1], np.int32), lo=np.array([0], np.int32), A=np.array([A]),
        nu=np.array([nu0]), cu=np.array([1], np.int32), cl=np.array([0], np.int32),
        K0=np.array([K]))


def rotor_species(nlev, rng, B=57.6e9, dipole_debye=0.11, K_base=3e-17, mass_amu=28.0):
    """Synthetic linear rotor: E_J = h B J(J+1), g = 2J+1, lines J -> J-1.

    Einstein A from the rigid-rotor dipole formula.  Collisional
    de-excitation coefficients for every u > l fall off with the level jump,
    K_ul = K_base * exp(-(u - l - 1)) * 10^U(-0.2, 0.2) (seeded scatter), at
    100 K; the rate law scales them with sqrt(T / 100 K).  (Rates that do not
    fall off with the jump pump the lowest, nearly thermal line into
    inversion in warm gas.)
    """
    J = np.arange(nlev, dtype=np.float64)
    E = _H * B * J * (J + 1)
    g = 2 * J + 1
    Ju = np.arange(1, nlev)
    nu = 2.0 * B * Ju
    mu = dipole_debye * _DEBYE
    A = 16 * math.pi ** 3 * nu ** 3 * mu ** 2 / (3 * _EPS0 * _H * _C ** 3) * Ju / (2 * Ju + 1)
    cu, cl, K0 = [], [], []
    for u in range(1, nlev):
        for l in range(u):
            cu.append(u)
            cl.append(l)
            K0.append(K_base * math.exp(-(u - l - 1)) * 10 ** rng.uniform(-0.2, 0.2))
    return dict(mass=mass_amu * _AMU, E=E, g=g, up=Ju.astype(np.int32),
                lo=(Ju - 1).astype(np.int32), A=A, nu=nu,
                cu=np.array(cu, np.int32), cl=np.array(cl, np.int32), K0=np.array(K0))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

CM3 = 1e-6        # cm^3 -> m^3
PER_CM3 = 1e6     # cm^-3 -> m^-3


def spherical_shells(variant: str = "a", npoints: int = 64, nmu: int = 12, nbins: int = 31,
                     length_unit: float = 1e14) -> Model:
    """1D spherically symmetric two-level cloud (shells log-spaced r in [1, 10]).

    n_coll = 1e6 r^-2 cm^-3, T = 100 K, v = 0, v_turb = 150 m/s, two-level
    species (100 GHz, A = 1e-5 s^-1, g_u = 3, g_l = 1, K = 1e-10 cm^3 s^-1).
    Species abundance X: variant "a" 1e-8 (moderate optical depth), "b" 1e-6
    (optically thick), "thin" 1e-12.
    """
    X = {"a": 1e-8, "b": 1e-6, "thin": 1e-12}[variant]
    i = np.arange(npoints)
    r = 10.0 ** (i / (npoints - 1))
    pos = np.zeros((3, npoints))
    pos[0] = r * length_unit
    vel = np.zeros((3, npoints))
    nb_lists = []
    for k in range(npoints):
        nb_lists.append([j for j in (k - 1, k + 1) if 0 <= j < npoints])
    off = np.zeros(npoints + 1, np.int32)
    off[1:] = np.cumsum([len(x) for x in nb_lists])
    nbs = np.array([j for x in nb_lists for j in x], np.int32)
    bdy = np.zeros(npoints, np.uint8)
    bdy[0] = bdy[-1] = 1
    ncoll = 1e6 * r ** -2 * PER_CM3
    sp = two_level_species(K=1e-10 * CM3)
    d, w, ap = rays_1d(nmu)
    return Model(dim=1, pos=pos, vel=vel, nbs_off=off, nbs=nbs, bdy=bdy,
                 T=np.full(npoints, 100.0), vturb2=np.full(npoints, 150.0 ** 2),
                 nspec=X * ncoll, ncoll=ncoll, ray_dir=d, ray_w=w, antipode=ap,
                 nbins=nbins, name=f"shells_{variant}", **sp)


def outflow_3d(npoints: int = 50_000, seed: int = 2, k: int = 16, nside: int = 2,
               nlev: int = 10, nbins: int = 31, length_unit: float = 1e12) -> Model:
    """3D spherical outflow in the shell r in [1, 20] (length unit 1e14 cm).

    v(r) = 15 km/s (1 - 1/r)^0.5 radial (floor 0.1 km/s), n_coll = n0 r^-2
    (v_inf / v) with n0 = 1e8 cm^-3, T = 2000 r^-0.7 K, abundance 1e-4,
    v_turb = 150 m/s, 10-level rotor, 48 HEALPix rays, 31 bins per line.
    Rotor collision rates as in rotor_species (seeded).
    """
    rng = np.random.default_rng(seed)
    r0, r1 = 1.0, 20.0
    p = _uniform_in_shell(rng, npoints, r0, r1)
    r = np.linalg.norm(p, axis=0)
    h = (4.0 / 3.0 * math.pi * (r1 ** 3 - r0 ** 3) / npoints) ** (1.0 / 3.0)
    bdy = ((r < r0 + h) | (r > r1 - h)).astype(np.uint8)
    off, nbs = knn_lists(p, k)
    vinf = 15e3
    v = np.maximum(vinf * np.sqrt(np.clip(1.0 - 1.0 / r, 0.0, None)), 100.0)
    vel = p / r * v
    ncoll = 1e8 * PER_CM3 * r ** -2 * (vinf / v)
    T = 2000.0 * r ** -0.7
    sp = rotor_species(nlev, rng)
    d, w, ap = rays_3d(nside)
    return Model(dim=3, pos=p * length_unit, vel=vel, nbs_off=off, nbs=nbs, bdy=bdy,
                 T=T, vturb2=np.full(npoints, 150.0 ** 2), nspec=1e-4 * ncoll,
                 ncoll=ncoll, ray_dir=d, ray_w=w, antipode=ap, nbins=nbins,
                 name=f"outflow_{npoints}", **sp)


def clumpy_cloud(npoints: int = 200_000, seed: int = 3, k: int = 16, nside: int = 2,
                 nlev: int = 20, nbins: int = 39, max_shift_widths: float = 20.0,
                 radius: float = 3e15) -> Model:
    """Clumpy sphere with a large velocity gradient.

    Log-normal density (sigma = 1) from a 64-mode Gaussian field, rotation
    about z plus turbulence of equal RMS, scaled so the largest projected
    velocity difference over any neighbour edge is `max_shift_widths` local
    line widths.  T = 100 K, n0 = 1e4 cm^-3, abundance 1e-6, 20-level rotor.
    """
    rng = np.random.default_rng(seed)
    p = _uniform_in_shell(rng, npoints, 0.0, 1.0)
    r = np.linalg.norm(p, axis=0)
    h = (4.0 / 3.0 * math.pi / npoints) ** (1.0 / 3.0)
    bdy = (r > 1.0 - h).astype(np.uint8)
    off, nbs = knn_lists(p, k)
    sigma = 1.0
    G = _mode_field(rng, 64, 2 * math.pi, 8 * math.pi)(p)
    ncoll = 1e4 * PER_CM3 * np.exp(sigma * G - sigma ** 2 / 2)
    rot = np.stack([-p[1], p[0], np.zeros(npoints)])
    turb = np.stack([_mode_field(rng, 64, 2 * math.pi, 8 * math.pi)(p) for _ in range(3)])
    rot *= np.sqrt(np.mean(turb ** 2)) / np.sqrt(np.mean(rot ** 2))
    vel = rot + turb
    T = np.full(npoints, 100.0)
    sp = rotor_species(nlev, rng)
    b = math.sqrt(2 * _KB * 100.0 / sp["mass"] + 150.0 ** 2)
    src = np.repeat(np.arange(npoints), np.diff(off))
    e = p[:, nbs] - p[:, src]
    e /= np.linalg.norm(e, axis=0)
    shift = np.abs(np.sum(e * (vel[:, nbs] - vel[:, src]), axis=0)).max()
    vel *= max_shift_widths * b / shift
    d, w, ap = rays_3d(nside)
    return Model(dim=3, pos=p * radius, vel=vel, nbs_off=off, nbs=nbs, bdy=bdy,
                 T=T, vturb2=np.full(npoints, 150.0 ** 2), nspec=1e-6 * ncoll,
                 ncoll=ncoll, ray_dir=d, ray_w=w, antipode=ap, nbins=nbins,
                 name=f"clumpy_{npoints}", **sp)


def tiny_cloud(npoints: int = 24, seed: int = 0, k: Optional[int] = None, nside: int = 1,
               nlev: int = 3, nbins: int = 11, vmax: float = 2e3, tau_scale: float = 1.0,
               radius: float = 1e13, rotor_B: float = 57.6e9) -> Model:
    """Small random cloud for brute-force checks (complete or kNN lists)."""
    rng = np.random.default_rng(seed)
    p = _uniform_in_shell(rng, npoints, 0.0, 1.0)
    r = np.linalg.norm(p, axis=0)
    bdy = (r > 0.75).astype(np.uint8)
    if k is None or k >= npoints - 1:
        off = np.arange(0, npoints * (npoints - 1) + 1, npoints - 1, dtype=np.int32)
        nbs = np.array([j for i in range(npoints) for j in range(npoints) if j != i], np.int32)
    else:
        off, nbs = knn_lists(p, k)
    vel = rng.uniform(-vmax, vmax, size=(3, npoints))
    T = rng.uniform(30.0, 300.0, size=npoints)
    ncoll = 10 ** rng.uniform(8, 11, size=npoints)
    if nlev == 2:
        sp = two_level_species(K=1e-10 * CM3)
    else:
        sp = rotor_species(nlev, rng, B=rotor_B)
    d, w, ap = rays_3d(nside)
    return Model(dim=3, pos=p * radius, vel=vel, nbs_off=off, nbs=nbs, bdy=bdy,
                 T=T, vturb2=np.full(npoints, 150.0 ** 2),
                 nspec=tau_scale * 1e-4 * ncoll, ncoll=ncoll, ray_dir=d, ray_w=w,
                 antipode=ap, nbins=nbins, name=f"tiny_{npoints}_{seed}", **sp)


def cubic_lattice(n: int = 4, spacing: float = 1e12, nside: int = 1, nlev: int = 2,
                  nbins: int = 7) -> Model:
    """n^3 cubic lattice with 26-neighbour lists; faces are boundary points."""
    g = np.arange(n)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).astype(np.float64)
    N = P.shape[1]
    index = {tuple(P[:, i].astype(int)): i for i in range(N)}
    lists = []
    for i in range(N):
        c = P[:, i].astype(int)
        li = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    q = (c[0] + dx, c[1] + dy, c[2] + dz)
                    if q in index:
                        li.append(index[q])
        lists.append(li)
    off = np.zeros(N + 1, np.int32)
    off[1:] = np.cumsum([len(x) for x in lists])
    nbs = np.array([j for x in lists for j in x], np.int32)
    bdy = np.any((P == 0) | (P == n - 1), axis=0).astype(np.uint8)
    sp = two_level_species(K=1e-10 * CM3)
    d, w, ap = rays_3d(nside)
    return Model(dim=3, pos=P * spacing, vel=np.zeros((3, N)), nbs_off=off, nbs=nbs,
                 bdy=bdy, T=np.full(N, 50.0), vturb2=np.full(N, 150.0 ** 2),
                 nspec=np.full(N, 1e-2), ncoll=np.full(N, 1e9), ray_dir=d, ray_w=w,
                 antipode=ap, nbins=nbins, name=f"lattice_{n}", **sp)


def with_rays(m: Model, dirs: np.ndarray) -> Model:
    """Replace the ray set by explicit directions (must contain antipodes)."""
    m = m.copy()
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    m.ray_dir = d
    m.ray_w = np.full(d.shape[0], 1.0 / d.shape[0])
    m.antipode = antipodes(d)
    return m


def config(i: int, **kw) -> Model:
    """The named workloads: 0 spherical shells, 1 3D outflow, 2 clumpy cloud."""
    if i == 0:
        return spherical_shells(**kw)
    if i == 1:
        return outflow_3d(**kw)
    if i == 2:
        return clumpy_cloud(**kw)
    raise ValueError(i)


def batch_spec(count: int = 256, seed: int = 4):
    """Seeded recipe of a grid of independent models of uneven size: point
    counts log-uniform in [1e3, 1e5], 2-20 rotor levels, 12 or 48 rays, 31
    bins; each an outflow (as outflow_3d) with its own seed.  Returns a list
    of keyword dicts for outflow_3d."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        out.append(dict(npoints=int(round(10 ** rng.uniform(3.0, 5.0))),
                        nlev=int(rng.integers(2, 21)),
                        nside=1 if rng.random() < 0.5 else 2,
                        nbins=31, seed=10_000 + i))
    return out


def batch_models(count: int = 256, seed: int = 4, subset=None):
    """The models of batch_spec (all, or the listed indices)."""
    spec = batch_spec(count, seed)
    idx = range(count) if subset is None else subset
    return [outflow_3d(**spec[i]) for i in idx]


def serve_spec(count: int = 8, seed: int = 7):
    """Seeded recipe of the resident models of the serving workload: outflows
    (as outflow_3d) with point counts log-uniform in [1e4, 1e6], 5-20 levels,
    12 rays, 31 bins.  Returns keyword dicts for outflow_3d."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        out.append(dict(npoints=int(round(10 ** rng.uniform(4.0, 6.0))),
                        nlev=int(rng.integers(5, 21)), nside=1, nbins=31, seed=20_000 + i))
    return out


def origin_sample(N: int, count: int, seed: int = 12345) -> np.ndarray:
    """Seeded sorted sample of origin points (for sampled parity / timing)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(count, N), replace=False)).astype(np.int32)


def random_rotation(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
