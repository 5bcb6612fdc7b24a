"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Bars: ray traces bit-exact (indices, projected distances, velocity
differences, branch bits); J-bar, Lambda-bar* and populations to 1e-10
relative in the FP64 path (populations with a floor of 1e-12 in the
denominator); the FP32-bulk path to 1e-5 relative on J-bar / Lambda-bar* and
1e-4 on converged populations.  Full-size workloads (3D outflow, 50k points;
clumpy cloud, 200k points) are checked on seeded samples of origins the
oracle computes one by one, in the same launch configuration the benchmark
times.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2411_03040_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mgx():
    import torch
    assert torch.cuda.is_available(), "GPU test on a host without a GPU"
    from paper_2411_03040_amd import mgx as m
    m.lib()
    return m


def make_ctx(mgx, model, precision):
    c = mgx.Context(precision=precision)
    c.load_model(model)
    c.trace_rays()
    return c


def rel(a, b, floor=1e-300):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))) if a.size else 0.0


def bits_equal(a, b):
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


# ---------------------------------------------------------------------------
# Traces: bit-exact
# ---------------------------------------------------------------------------

def check_traces(ctx, model, pairs):
    orc = oracle.Oracle(model)
    off = ctx.get_trace_offsets()
    total = int(off[-1])
    idx, Z, dv, semi = ctx.get_trace_records(0, total)
    R = model.nrays
    nsemi = 0
    for (o, r) in pairs:
        w = o * R + r
        a, b = int(off[w]), int(off[w + 1])
        oi, oZ, odv, _ = orc.trace(o, r)
        assert np.array_equal(idx[a:b], oi), (o, r)
        assert bits_equal(Z[a:b], oZ), (o, r)
        assert bits_equal(dv[a:b], odv), (o, r)
        for k in range(b - a):
            p0, dv0 = (o, 0.0) if k == 0 else (int(oi[k - 1]), float(odv[k - 1]))
            exp = orc.use_semi_analytic(p0, dv0, int(oi[k]), float(odv[k]))
            assert bool(semi[a + k]) == exp, (o, r, k)
            nsemi += exp
    return nsemi


def all_pairs(model):
    return [(o, r) for o in range(model.npoints) for r in range(model.nrays)]


def test_trace_tiny_complete_lists(mgx):
    m = synth.tiny_cloud(npoints=40, seed=21, nside=2, vmax=3e3)
    say("trace tiny complete", m.npoints)
    ctx = make_ctx(mgx, m, mgx.FP64)
    n = check_traces(ctx, m, all_pairs(m))
    assert n > 0


def test_trace_knn_cloud(mgx):
    m = synth.tiny_cloud(npoints=600, seed=22, k=12, nside=2, vmax=5e3)
    say("trace knn cloud", m.npoints)
    ctx = make_ctx(mgx, m, mgx.FP32)
    check_traces(ctx, m, all_pairs(m))


def test_trace_lattice_ties(mgx):
    m = synth.cubic_lattice(n=6)
    say("trace lattice", m.npoints)
    ctx = make_ctx(mgx, m, mgx.FP32)
    check_traces(ctx, m, all_pairs(m))


def slot_ctx(mgx, model, precision, min_bytes):
    c = mgx.Context(precision=precision, trace_slot_min_bytes=min_bytes)
    c.load_model(model)
    c.trace_rays()
    return c


def test_trace_walks_longer_than_slots(mgx):
    """Walks longer than the searching pass's slots (4 N^(1/3) + 16 points)
    send the trace through the second search; records still bit-exact, and
    the semi-analytic count matches the oracle's."""
    m = _chain(300)
    ctx = slot_ctx(mgx, m, mgx.FP64, 0)
    off = ctx.get_trace_offsets()
    assert int(np.max(np.diff(off))) > 4 * m.npoints ** (1 / 3) + 16
    n = check_traces(ctx, m, all_pairs(m))
    assert ctx.counters()["semi_segments"] == n


@pytest.mark.parametrize("min_bytes", [0, -1])
def test_trace_slot_and_two_pass_records(mgx, min_bytes):
    """The same small cloud traced from slots (one search) and with two
    searches: records equal the oracle's bit for bit either way, with the
    same semi-analytic and hole counts."""
    m = synth.tiny_cloud(npoints=300, seed=57, k=6, nside=2, vmax=5e3)
    ctx = slot_ctx(mgx, m, mgx.FP32, min_bytes)
    n = check_traces(ctx, m, all_pairs(m))
    c = ctx.counters()
    assert c["semi_segments"] == n > 0
    orc = oracle.Oracle(m)
    holes = sum(orc.trace(o, r)[3] for o, r in all_pairs(m))
    assert c["holes"] == holes > 0


@pytest.mark.parametrize("variant", ["a", "b"])
def test_trace_spherical_shells(mgx, variant):
    m = synth.spherical_shells(variant)
    m.vel[0] = np.linspace(0, 3e3, m.npoints)   # radial velocity exercises dv
    say("trace shells", variant)
    ctx = make_ctx(mgx, m, mgx.FP64)
    check_traces(ctx, m, all_pairs(m))


@pytest.fixture(scope="module")
def outflow():
    return synth.config(1)


@pytest.fixture(scope="module")
def clumpy():
    return synth.config(2)


def test_trace_outflow_full_sampled(mgx, outflow):
    m = outflow
    say("trace outflow 50k sampled")
    ctx = make_ctx(mgx, m, mgx.FP32)
    rng = np.random.default_rng(31)
    pairs = [(int(o), int(r)) for o, r in zip(rng.integers(0, m.npoints, 3000),
                                              rng.integers(0, m.nrays, 3000))]
    nsemi = check_traces(ctx, m, pairs)
    assert nsemi > 0
    c = ctx.counters()
    assert c["total_records"] > 0


def test_trace_clumpy_full_sampled(mgx, clumpy):
    m = clumpy
    say("trace clumpy 200k sampled")
    ctx = make_ctx(mgx, m, mgx.FP32)
    rng = np.random.default_rng(32)
    pairs = [(int(o), int(r)) for o, r in zip(rng.integers(0, m.npoints, 1500),
                                              rng.integers(0, m.nrays, 1500))]
    nsemi = check_traces(ctx, m, pairs)
    assert nsemi > 0


# ---------------------------------------------------------------------------
# Formal solution: J-bar and Lambda-bar*
# ---------------------------------------------------------------------------

def fs_compare(mgx, model, precision, origins=None, pops=None, tolJ=None, tolL=None):
    orc = oracle.Oracle(model)
    if pops is None:
        pops = orc.lte()
    ctx = make_ctx(mgx, model, precision)
    ctx.set_populations(pops)
    J, L = ctx.formal_solve()
    Jo, Lo = orc.solve_origins(pops, origins)
    sel = slice(None) if origins is None else np.asarray(origins)
    eJ = rel(J[sel], Jo)
    eL = rel(L[sel], Lo)
    eLa = float(np.max(np.abs(L[sel] - Lo)))
    say(f"  {model.name} prec={precision} J rel {eJ:.3e} L rel {eL:.3e} (abs {eLa:.3e}, "
        f"min L {float(np.min(Lo)):.2e})")
    if tolJ is not None:
        assert eJ < tolJ
    if tolL is not None:
        assert eL < tolL
    return ctx, J, L


@pytest.mark.parametrize("variant", ["a", "b"])
def test_formal_solve_shells_fp64(mgx, variant):
    m = synth.spherical_shells(variant)
    fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)


@pytest.mark.parametrize("variant", ["a", "b"])
def test_formal_solve_shells_fp32(mgx, variant):
    m = synth.spherical_shells(variant)
    fs_compare(mgx, m, mgx.FP32, tolJ=1e-5, tolL=1e-5)


@pytest.mark.parametrize("prec,tolJ,tolL", [(0, 1e-10, 1e-10), (1, 1e-5, 1e-5)])
def test_formal_solve_moving_cloud(mgx, prec, tolJ, tolL):
    """Velocities large enough that many segments take the semi-analytic form."""
    m = synth.tiny_cloud(npoints=300, seed=23, k=12, nside=2, nlev=4, nbins=15, vmax=6e3,
                         tau_scale=20.0)
    ctx, J, L = fs_compare(mgx, m, prec, tolJ=tolJ, tolL=tolL)
    assert ctx.counters()["semi_segments"] > 0


@pytest.mark.parametrize("tau_scale", [1e4, 1e7, 1e10])
@pytest.mark.parametrize("prec,tolJ,tolL", [(0, 1e-10, 1e-10), (1, 1e-5, 1e-5)])
def test_formal_solve_optically_thick(mgx, tau_scale, prec, tolJ, tolL):
    """Line optical depths far beyond the workloads' (Lambda* up to 0.9999):
    the elimination rows that share one reciprocal per pair carry the
    product of two denominators, which must stay finite and accurate."""
    m = synth.tiny_cloud(npoints=300, seed=41, k=12, nside=2, nlev=4, nbins=15, vmax=4e3,
                         tau_scale=tau_scale)
    ctx, J, L = fs_compare(mgx, m, prec, tolJ=tolJ, tolL=tolL)
    assert np.all(np.isfinite(J)) and np.all(np.isfinite(L))


@pytest.mark.parametrize("prec,tolJ,tolL", [(0, 1e-10, 1e-10), (1, 1e-5, 1e-5)])
def test_formal_solve_outflow_full_sampled(mgx, outflow, prec, tolJ, tolL):
    origins = synth.origin_sample(outflow.npoints, 48, seed=41)
    fs_compare(mgx, outflow, prec, origins=origins, tolJ=tolJ, tolL=tolL)


@pytest.mark.parametrize("prec,tolJ,tolL", [(0, 1e-10, 1e-10), (1, 1e-5, 1e-5)])
def test_formal_solve_clumpy_full_sampled(mgx, clumpy, prec, tolJ, tolL):
    origins = synth.origin_sample(clumpy.npoints, 64, seed=42)
    ctx, _, _ = fs_compare(mgx, clumpy, prec, origins=origins, tolJ=tolJ, tolL=tolL)
    assert ctx.counters()["semi_segments"] > 0


def test_formal_solve_many_line_chunks(mgx):
    """nlines x nbins above one workgroup: lines split over chunks (ragged)."""
    m = synth.tiny_cloud(npoints=60, seed=24, k=10, nside=1, nlev=21, nbins=63, vmax=2e3)
    assert m.nlines * m.nbins > 1024
    fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)
    fs_compare(mgx, m, mgx.FP32, tolJ=1e-5, tolL=1e-5)


def test_formal_solve_one_width_moving_cloud(mgx):
    """One Doppler width everywhere (uniform T and v_turb) with steep
    velocities: consecutive semi-analytic segments share erfc values."""
    m = synth.tiny_cloud(npoints=300, seed=31, k=12, nside=2, nlev=4, nbins=15, vmax=6e3)
    m.T[:] = 80.0
    ctx, _, _ = fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)
    c = ctx.counters()
    assert c["semi_segments"] > 0.5 * c["total_records"]
    fs_compare(mgx, m, mgx.FP32, tolJ=1e-5, tolL=1e-5)


def test_formal_solve_maximum_bins(mgx):
    """The largest bin count (1024): one line per 1024-lane workgroup, the
    widest launch of either precision; steep velocities, so semi-analytic
    segments are mixed in."""
    m = synth.tiny_cloud(npoints=40, seed=30, k=8, nside=1, nlev=3, nbins=1024, vmax=6e3)
    ctx, _, _ = fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)
    assert ctx.counters()["semi_segments"] > 0
    fs_compare(mgx, m, mgx.FP32, tolJ=1e-5, tolL=1e-5)
    m.nbins = 1025
    c = mgx.Context()
    with pytest.raises(mgx.MgxError) as e:
        c.load_model(m)
    assert e.value.status == mgx.MGX_EINVAL


def test_formal_solve_single_bin_and_boundary_only(mgx):
    m = synth.tiny_cloud(npoints=20, seed=25, nside=1, nlev=2, nbins=1)
    fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)
    m2 = synth.tiny_cloud(npoints=12, seed=26, nside=1, nlev=3, nbins=5)
    m2.bdy[:] = 1               # every walk ends after one step
    fs_compare(mgx, m2, mgx.FP64, tolJ=1e-10, tolL=1e-10)


def test_formal_solve_isolated_points_and_holes(mgx):
    """Points without neighbours (isolated: both halves empty) and walks that
    stop on interior points (holes)."""
    m = synth.tiny_cloud(npoints=50, seed=27, k=6, nside=2, nlev=3, nbins=9)
    off = m.nbs_off.copy()
    lists = [list(m.nbs[off[i]:off[i + 1]]) for i in range(m.npoints)]
    for i in (3, 17, 30):
        lists[i] = []
    m.nbs_off = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int32)
    m.nbs = np.array([j for x in lists for j in x], np.int32)
    ctx, J, L = fs_compare(mgx, m, mgx.FP64, tolJ=1e-10, tolL=1e-10)
    assert ctx.counters()["holes"] > 0
    fs_compare(mgx, m, mgx.FP32, tolJ=1e-5, tolL=1e-5)


def _first_points(m, n):
    """The model restricted to its first n points (neighbour lists cut to
    them)."""
    lists = [[j for j in m.nbs[m.nbs_off[i]:m.nbs_off[i + 1]] if j < n] for i in range(n)]
    c = m.copy()
    c.pos, c.vel = m.pos[:, :n].copy(), m.vel[:, :n].copy()
    c.nbs_off = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int32)
    c.nbs = np.array([j for x in lists for j in x], np.int32)
    for f in ("bdy", "T", "vturb2", "nspec", "ncoll"):
        setattr(c, f, getattr(m, f)[:n].copy())
    return c


@pytest.mark.parametrize("n", [1, 2, 3])
def test_formal_solve_smallest_models(mgx, n):
    """Degenerate clouds: a single point (both halves of every pair empty),
    two and three points; the Lambda-iteration runs on them too."""
    m = _first_points(synth.tiny_cloud(npoints=8, seed=32, nside=1, nlev=3, nbins=7), n)
    assert m.npoints == n
    for prec, tol in ((mgx.FP64, 1e-10), (mgx.FP32, 1e-5)):
        fs_compare(mgx, m, prec, tolJ=tol, tolL=tol)
    r = oracle.Oracle(m).iterate(tol=1e-12, max_iter=500)
    assert r["status"] == 0
    c = make_ctx(mgx, m, mgx.FP64)
    c.set_lte_populations()
    it, ch, ok = c.iterate(tol=1e-12, max_iter=500)
    assert ok and rel(c.get_populations(), r["pops"]) < 1e-10


def test_formal_solve_deterministic(mgx):
    m = synth.tiny_cloud(npoints=400, seed=28, k=12, nside=2, nlev=5)
    orc = oracle.Oracle(m)
    ctx = make_ctx(mgx, m, mgx.FP32)
    ctx.set_populations(orc.lte())
    J1, L1 = ctx.formal_solve()
    J2, L2 = ctx.formal_solve()
    assert bits_equal(J1, J2) and bits_equal(L1, L2)


# ---------------------------------------------------------------------------
# Statistical equilibrium
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nlev,rotor_B,cap", [
    (2, 57.6e9, True), (10, 57.6e9, True), (20, 57.6e9, True), (64, 2e9, True),
    (64, 57.6e9, True), (64, 57.6e9, False)])
def test_stateq_parity(mgx, nlev, rotor_B, cap):
    """cap: Lambda* drawn so that J_eff = J - Lambda* S stays positive, as a
    converged radiation field has it (2 GHz rotor: every one of 64 levels
    populated; 57.6 GHz: populations spanning ~190 decades).  Without the cap
    (64 levels, 57.6 GHz) J_eff and rates go negative and the system is
    ill-conditioned (the oracle's own populations reach -23.5); the bar is
    then 50 kappa eps with kappa the oracle's measured sensitivity."""
    m = synth.tiny_cloud(npoints=500, seed=29, k=8, nside=1, nlev=nlev, nbins=3,
                         rotor_B=rotor_B)
    orc = oracle.Oracle(m)
    pops = orc.lte()
    rng = np.random.default_rng(30)
    _, _, S, _ = orc.line_coeffs(pops)
    J = S * rng.uniform(0.2, 1.5, S.shape)
    L = rng.uniform(0.0, 0.95, S.shape) * (np.minimum(1.0, J / S) if cap else 1.0)
    ctx = make_ctx(mgx, m, mgx.FP64)
    ctx.set_populations(pops)
    ctx.set_radiation(J, L)
    change = ctx.update_populations()
    got = ctx.get_populations()
    st, exp = orc.stateq(J, L, S)
    assert st == 0
    # conditioning of the problem, measured on the oracle itself: output change
    # under a relative input perturbation of a few ulps
    d = 8 * 2.2e-16
    _, exp2 = orc.stateq(J * (1 + d), L, S)
    kappa = rel(exp2, exp, 1e-12) / d
    bar = max(1e-10, 50 * kappa * 2.2e-16)
    e = rel(got, exp, 1e-12)
    say(f"  stateq nlev={nlev} B={rotor_B:.3g} cap={cap} rel {e:.3e} kappa {kappa:.2e} "
        f"bar {bar:.1e}")
    assert e < bar
    assert np.all(np.abs(got.sum(1) - 1) < 1e-13)
    if cap:
        # the oracle's own conditioning never widens the bar on these inputs
        assert bar == 1e-10
        assert np.all(exp > 0)
        assert abs(change / orc.rel_change(exp, pops) - 1) < 1e-8


# ---------------------------------------------------------------------------
# Lambda-iteration to convergence
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["a", "b"])
def test_iterate_shells_fp64_no_ng(mgx, variant):
    m = synth.spherical_shells(variant)
    orc = oracle.Oracle(m)
    ref = orc.iterate(tol=1e-10, max_iter=1000)
    ctx = make_ctx(mgx, m, mgx.FP64)
    ctx.set_lte_populations()
    it, ch, ok = ctx.iterate(tol=1e-10, max_iter=1000)
    got = ctx.get_populations()
    e = rel(got, ref["pops"], 1e-12)
    say(f"  shells {variant} iters gpu {it} oracle {ref['iters']} rel {e:.3e}")
    assert ok and it == ref["iters"]
    assert e < 1e-10


@pytest.mark.parametrize("variant,mode,param", [
    ("a", 1, 4), ("b", 1, 4), ("a", 2, 8), ("b", 2, 8), ("b", 1 | 0x10, 4), ("a", 2 | 0x10, 8),
    ("b", 2 | 0x10, 16), ("b", 2, 3)])
def test_iterate_shells_fp64_ng(mgx, variant, mode, param):
    """Same schedule as the oracle, decision by decision: the iteration count
    and the number of predictions used agree, and so do the populations."""
    m = synth.spherical_shells(variant)
    orc = oracle.Oracle(m)
    ref = orc.iterate(tol=1e-10, max_iter=2000, ng_mode=mode, ng_param=param)
    assert ref["status"] == 0
    ctx = make_ctx(mgx, m, mgx.FP64)
    ctx.set_lte_populations()
    it, ch, ok = ctx.iterate(tol=1e-10, max_iter=2000, ng_mode=mode, ng_param=param)
    got = ctx.get_populations()
    e = rel(got, ref["pops"], 1e-12)
    c = ctx.counters()
    used = int(np.sum(ref["events"] == 2))
    say(f"  shells {variant} ng {mode}/{param} iters gpu {it} oracle {ref['iters']} "
        f"applied {c['ng_applied']} oracle {used} rel {e:.3e}")
    assert ok and it == ref["iters"]
    assert c["ng_applied"] == used > 0
    assert e < 1e-10


@pytest.mark.parametrize("variant,mode,param", [("a", 1, 4), ("b", 2, 8)])
def test_iterate_shells_fp64_ng_tight(mgx, variant, mode, param):
    """Down to 1e-13 both reach the same fixed point."""
    m = synth.spherical_shells(variant)
    orc = oracle.Oracle(m)
    ref = orc.iterate(tol=1e-13, max_iter=2000, ng_mode=mode, ng_param=param)
    assert ref["status"] == 0
    ctx = make_ctx(mgx, m, mgx.FP64)
    ctx.set_lte_populations()
    it, ch, ok = ctx.iterate(tol=1e-13, max_iter=2000, ng_mode=mode, ng_param=param)
    e = rel(ctx.get_populations(), ref["pops"], 1e-12)
    say(f"  shells {variant} ng {mode}/{param} tol 1e-13 iters gpu {it} oracle {ref['iters']} "
        f"rel {e:.3e}")
    assert ok and e < 1e-10


def ng_bars(hist, rng):
    """Bars for the Ng coefficients (relative to their largest magnitude) and
    the prediction (relative, floor 1e-12): 1e-12, widened only where the
    oracle's own output moves more than that under a relative perturbation
    of the history of a few ulps (the Gram solve amplifies summation-order
    differences by its conditioning): max(1e-12, 50 kappa eps)."""
    st, p, c = oracle.ng(hist)
    d = 8 * 2.2e-16
    kc = kp = 0.0
    for _ in range(4):
        st2, p2, c2 = oracle.ng(hist * (1 + d * rng.uniform(-1, 1, hist.shape)))
        assert st2 == st == 0
        kc = max(kc, float(np.max(np.abs(c2 - c)) / np.max(np.abs(c))) / d)
        kp = max(kp, rel(p2, p, 1e-12) / d)
    return max(1e-12, 50 * kc * 2.2e-16), max(1e-12, 50 * kp * 2.2e-16), kc, kp


def test_ng_prediction_matches_oracle(mgx):
    """The same history through mgx_ng_predict and the oracle's Ng: the
    coefficients and the prediction element by element.  Histories: the
    first 3, 4 and 6 Lambda-iterates of the thick shells from LTE (pushed
    with mgx_ng_push), and synthetic histories (a valid one, one with a
    negative predicted entry, one with collinear residuals)."""
    m = synth.spherical_shells("b")
    ctx = make_ctx(mgx, m, mgx.FP64)
    ctx.set_lte_populations()
    hist = [ctx.get_populations()]
    for _ in range(5):
        ctx.formal_solve(copy=False)
        ctx.update_populations()
        hist.append(ctx.get_populations())
    rng = np.random.default_rng(76)
    for n in (3, 4, 6):
        ctx.set_populations(hist[0])
        ctx.ng_reset(n)
        for h in hist[1:n]:
            ctx.set_populations(h)
            ctx.ng_push()
        H = np.array([h.ravel() for h in hist[:n]])
        st, pred, c = oracle.ng(H)
        assert st == 0
        bar_c, bar_p, kc, kp = ng_bars(H, rng)
        ok, _, cg = ctx.ng_predict(apply=False)
        assert ok
        ec = float(np.max(np.abs(cg[:n - 1] - c)) / np.max(np.abs(c)))
        ctx.ng_predict(apply=True)
        ep = rel(ctx.get_populations().ravel(), pred, 1e-12)
        say(f"  Ng {n} iterates: coefficients rel {ec:.2e} (bar {bar_c:.1e}, kappa {kc:.1e}), "
            f"prediction rel {ep:.2e} (bar {bar_p:.1e}, kappa {kp:.1e}), c = {c}")
        assert ec < bar_c and ep < bar_p
        if n == 3:
            assert bar_c <= 5e-12 and bar_p == 1e-12

    N, L = m.npoints, m.nlev
    rng = np.random.default_rng(77)
    base = rng.uniform(0.2, 1.0, (N, L))
    base /= base.sum(1, keepdims=True)
    lam = rng.uniform(0.3, 0.9, (N, L))
    cases = {"valid": [base * (1 + 0.2 * lam ** k * rng.uniform(-1, 1, (N, L)))
                       for k in range(4)],
             "collinear": [base + 0.05 * 0.5 ** k * (base - 1.0 / L) for k in range(4)]}
    # two entries with different convergence ratios (so the residuals are
    # not collinear); entry (0, 0) extrapolates below zero: c = (-0.459,
    # 1.459), prediction -0.459 * 0.1 + 1.459 * 0.03 < 0
    neg = []
    for a0, a1 in ((0.3, 0.5), (0.1, 0.6), (0.03, 0.62)):
        y = base.copy()
        y[0, 0], y[0, 1] = a0, a1
        neg.append(y)
    cases["negative"] = neg
    for name, hs in cases.items():
        ctx.set_populations(hs[0])
        ctx.ng_reset(8)
        for h in hs[1:]:
            ctx.set_populations(h)
            ctx.ng_push()
        st, pred, c = oracle.ng(np.array([h.ravel() for h in hs]))
        ok, _, cg = ctx.ng_predict(apply=False)
        say(f"  Ng history {name}: oracle status {st}, gpu valid {ok}")
        assert ok == (st == 0)
        assert st == {"valid": 0, "collinear": -1, "negative": -2}[name]
        if ok:
            k = len(hs) - 1
            bar_c, bar_p, _, _ = ng_bars(np.array([h.ravel() for h in hs]), rng)
            assert float(np.max(np.abs(cg[:k] - c)) / np.max(np.abs(c))) < bar_c
            ctx.ng_predict(apply=True)
            assert rel(ctx.get_populations().ravel(), pred, 1e-12) < bar_p


def test_ng_accelerate_schedule_call_equals_iterate(mgx):
    """mgx_ng_accelerate driven by hand after each update reproduces
    mgx_iterate's adaptive schedule (same iterations, predictions, bits)."""
    m = synth.spherical_shells("b")
    a = make_ctx(mgx, m, mgx.FP64)
    a.set_lte_populations()
    it, _, ok = a.iterate(tol=1e-10, max_iter=500, ng_mode=mgx.NG_ADAPTIVE | mgx.NG_FRESH,
                          ng_param=8)
    b = make_ctx(mgx, m, mgx.FP64)
    b.set_lte_populations()
    b.ng_reset(8)
    n, used = 0, 0
    while n < 500:
        n += 1
        b.formal_solve(copy=False)
        if b.update_populations() <= 1e-10:
            break
        used += b.ng_accelerate(mgx.NG_ADAPTIVE | mgx.NG_FRESH, 8)
    assert ok and n == it and used == a.counters()["ng_applied"]
    assert bits_equal(a.get_populations(), b.get_populations())


@pytest.mark.parametrize("variant", ["a", "b"])
def test_iterate_shells_fp32_bulk(mgx, variant):
    m = synth.spherical_shells(variant)
    orc = oracle.Oracle(m)
    ref = orc.iterate(tol=1e-12, max_iter=2000, ng_mode=1, ng_param=4)
    ctx = make_ctx(mgx, m, mgx.FP32)
    ctx.set_lte_populations()
    it, ch, ok = ctx.iterate(tol=1e-7, max_iter=2000, ng_mode=1, ng_param=4)
    got = ctx.get_populations()
    e = rel(got, ref["pops"], 1e-12)
    say(f"  shells {variant} fp32 iters {it} rel {e:.3e}")
    assert ok and e < 1e-4


def test_iterate_small_outflow_fp32_and_fp64(mgx):
    """A reduced outflow (same physics as the 50k-point workload) converged by
    the oracle, the FP64 path and the FP32-bulk path."""
    m = synth.outflow_3d(npoints=600, seed=5, nside=1, nlev=6, nbins=15)
    orc = oracle.Oracle(m)
    ref = orc.iterate(tol=1e-12, max_iter=400, ng_mode=1, ng_param=4)
    assert ref["status"] == 0
    for prec, tol, bar in ((0, 1e-12, 1e-10), (1, 1e-7, 1e-4)):
        ctx = make_ctx(mgx, m, prec)
        ctx.set_lte_populations()
        it, ch, ok = ctx.iterate(tol=tol, max_iter=400, ng_mode=1, ng_param=4)
        got = ctx.get_populations()
        e = rel(got, ref["pops"], 1e-12)
        say(f"  small outflow prec {prec} iters {it} (oracle {ref['iters']}) rel {e:.3e}")
        assert ok and e < bar


def test_masing_count_matches_oracle(mgx):
    """Populations inverted on purpose at a third of the points: the line
    coefficients clamp chi^ij there; the count equals the oracle's, and it
    is still reported after the statistical-equilibrium step that follows
    (and after a whole mgx_iterate)."""
    m = synth.tiny_cloud(npoints=300, seed=71, k=10, nside=1, nlev=3, nbins=5)
    orc = oracle.Oracle(m)
    pops = orc.lte()
    pops[::3, 0] *= 0.01            # J=0 depleted: n_1/g_1 > n_0/g_0 on the 1-0 line
    pops /= pops.sum(1, keepdims=True)
    _, _, _, n_orc = orc.line_coeffs(pops)
    assert n_orc > 50
    for prec in (mgx.FP64, mgx.FP32):
        ctx = make_ctx(mgx, m, prec)
        ctx.set_populations(pops)
        ctx.formal_solve()
        assert ctx.counters()["masing"] == n_orc
        ctx.update_populations()
        assert ctx.counters()["masing"] == n_orc
        ctx.set_populations(pops)
        ctx.iterate(tol=1e-6, max_iter=1, raise_on_noconv=False)
        assert ctx.counters()["masing"] == n_orc


def oracle_step_residual(model, pops, count=48, seed=98):
    """max relative change of the oracle's own Lambda-iteration step (formal
    solution + statistical equilibrium) from `pops`, at sampled points."""
    orc = oracle.Oracle(model)
    sub = synth.origin_sample(model.npoints, count, seed=seed)
    Jc, Lc = orc.solve_origins(pops, sub)
    _, _, Sc, _ = orc.line_coeffs(pops)
    res = 0.0
    for k, o in enumerate(sub):
        st, new = orc.stateq_point(int(o), Jc[k], Lc[k], Sc[o])
        assert st == 0
        res = max(res, rel(new, pops[o], 1e-12))
    return res


def test_converged_outflow_full_oracle_step(mgx, outflow):
    """The 50k-point outflow converged from LTE in the benchmark's form (Ng
    order 4): FP32-bulk to 1e-6 and FP64 to 1e-10.  At 48 sampled points the
    oracle's own Lambda-iteration step from those populations moves them by
    at most 1e-4 (FP32-bulk) and 1e-10 (FP64); the two forms agree to 1e-4."""
    got = {}
    for prec, tol, bar in ((mgx.FP32, 1e-6, 1e-4), (mgx.FP64, 1e-10, 1e-10)):
        ctx = make_ctx(mgx, outflow, prec)
        ctx.set_lte_populations()
        it, ch, ok = ctx.iterate(tol=tol, max_iter=200, ng_mode=mgx.NG_CLASSICAL, ng_param=4)
        assert ok
        pops = ctx.get_populations()
        r = oracle_step_residual(outflow, pops)
        say(f"  outflow converged prec {prec}: {it} iterations, oracle step {r:.3e}")
        assert r < bar
        got[prec] = pops
        del ctx
    assert rel(got[mgx.FP32], got[mgx.FP64], 1e-12) < 1e-4


def test_converged_clumpy_full_fp32_bulk_oracle_step(mgx, clumpy):
    """The 200k-point clumpy cloud converged in the FP32-bulk form (1e-6, Ng
    order 4); the oracle's step from those populations at 48 sampled points
    moves them by at most 1e-4."""
    ctx = make_ctx(mgx, clumpy, mgx.FP32)
    ctx.set_lte_populations()
    it, ch, ok = ctx.iterate(tol=1e-6, max_iter=300, ng_mode=mgx.NG_CLASSICAL, ng_param=4)
    assert ok
    pops = ctx.get_populations()
    r = oracle_step_residual(clumpy, pops)
    # the J=1-0 line is inverted (clamped) at about half the points
    n_mas = ctx.counters()["masing"]
    inv = int(np.sum(pops[:, 1] / clumpy.g[1] > pops[:, 0] / clumpy.g[0]))
    say(f"  clumpy converged FP32-bulk: {it} iterations, oracle step {r:.3e}, masing clamps "
        f"{n_mas}, inverted J=1-0 at {inv} points")
    assert r < 1e-4
    assert n_mas > 0.3 * clumpy.npoints and abs(n_mas - inv) < 0.01 * inv


# ---------------------------------------------------------------------------
# Error handling through the ABI
# ---------------------------------------------------------------------------

def test_error_paths(mgx):
    m = synth.tiny_cloud(npoints=10, seed=30)
    c = mgx.Context(precision=mgx.FP32)
    with pytest.raises(mgx.MgxError) as e:
        c.trace_rays()
    assert e.value.status == mgx.MGX_ESTATE
    bad = m.copy()
    bad.nbs = bad.nbs.copy()
    bad.nbs[0] = 10_000
    with pytest.raises(mgx.MgxError) as e:
        c.load_model(bad)
    assert e.value.status == mgx.MGX_EINVAL
    bad = m.copy()
    bad.T[3] = np.nan
    with pytest.raises(mgx.MgxError) as e:
        c.load_model(bad)
    assert e.value.status == mgx.MGX_ENONFINITE
    c.load_model(m)
    with pytest.raises(mgx.MgxError) as e:
        c.formal_solve()
    assert e.value.status == mgx.MGX_ESTATE
    c.trace_rays()
    with pytest.raises(mgx.MgxError) as e:
        c.formal_solve()      # no populations yet
    assert e.value.status == mgx.MGX_ESTATE
    with pytest.raises(mgx.MgxError) as e:
        c.update_populations()
    assert e.value.status == mgx.MGX_ESTATE
    c.set_lte_populations()
    c.formal_solve()
    c.update_populations()
    # singular statistical equilibrium: no radiative or collisional coupling
    s = m.copy()
    s.A[:] = 0.0
    s.ncoll[:] = 0.0
    c.load_model(s)
    c.trace_rays()
    c.set_lte_populations()
    c.formal_solve()
    with pytest.raises(mgx.MgxError) as e:
        c.update_populations()
    assert e.value.status == mgx.MGX_ESINGULAR
    c.close()


# ---------------------------------------------------------------------------
# Synthetic images
# ---------------------------------------------------------------------------

def render_compare(mgx, model, prec, direction, npx, npy, f_min, f_max, nfreq, pixels, tol,
                   pops=None):
    orc = oracle.Oracle(model)
    if pops is None:
        pops = orc.lte()
    ctx = mgx.Context(precision=prec)
    ctx.load_model(model)
    ctx.set_populations(pops)
    img = ctx.render_image(direction, npx, npy, f_min, f_max, nfreq)
    assert img.shape == (npy, npx, nfreq) and np.all(np.isfinite(img))
    Io, walks = orc.render_pixels(pops, direction, npx, npy, f_min, f_max, nfreq, pixels)
    got = np.array([img[iy, ix] for ix, iy in pixels])
    e = rel(got, Io)
    say(f"  render {model.name} prec={prec} rel {e:.3e}  walks {[len(w) for w in walks[:6]]}")
    assert e < tol
    return img, walks


# The image is float32 (the API's output type), so the FP64 path is checked
# to float resolution; the FP32 path to the bulk-precision bar.
@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_moving_cloud_all_pixels(mgx, prec, tol):
    m = synth.tiny_cloud(npoints=500, seed=50, k=12, nside=1, nlev=3, nbins=5, vmax=4e3,
                         tau_scale=20.0)
    nu0 = m.nu[0]
    pix = [(ix, iy) for ix in range(12) for iy in range(10)]
    img, walks = render_compare(mgx, m, prec, [0.2, -0.4, 0.9], 12, 10, nu0 * (1 - 2e-5),
                                nu0 * (1 + 2e-5), 21, pix, tol)
    assert max(len(w) for w in walks) > 5


@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_outflow_full_sampled(mgx, outflow, prec, tol):
    m = outflow
    nu0 = m.nu[1]
    rng = np.random.default_rng(51)
    pix = [(int(a), int(b)) for a, b in zip(rng.integers(0, 64, 24), rng.integers(0, 64, 24))]
    pix += [(0, 0), (63, 63)]           # corners: off the projected shell
    img, walks = render_compare(mgx, m, prec, [0.0, 0.6, 0.8], 64, 64, nu0 * (1 - 8e-5),
                                nu0 * (1 + 8e-5), 63, pix, tol)
    assert len(walks[-1]) == 0 and len(walks[-2]) == 0


@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_clumpy_full_sampled(mgx, clumpy, prec, tol):
    """Large velocity gradients: offsets of tens of widths, profiles underflow."""
    m = clumpy
    nu0 = m.nu[2]
    rng = np.random.default_rng(53)
    pix = [(int(a), int(b)) for a, b in zip(rng.integers(0, 48, 12), rng.integers(0, 48, 12))]
    render_compare(mgx, m, prec, [0.5, 0.5, 0.7071], 48, 48, nu0 * (1 - 6e-5),
                   nu0 * (1 + 6e-5), 31, pix, tol)


@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_frequency_slices(mgx, prec, tol):
    """More frequencies than one wave (three 64-lane slices per pixel, the
    last ragged) and a single frequency."""
    m = synth.tiny_cloud(npoints=300, seed=54, k=12, nside=1, nlev=3, nbins=5, vmax=4e3,
                         tau_scale=20.0)
    nu0 = m.nu[0]
    pix = [(ix, iy) for ix in range(7) for iy in range(5)]
    render_compare(mgx, m, prec, [0.3, 0.2, -0.9], 7, 5, nu0 * (1 - 2e-5), nu0 * (1 + 2e-5),
                   130, pix, tol)
    render_compare(mgx, m, prec, [0.3, 0.2, -0.9], 7, 5, nu0 * (1 + 3e-6), nu0 * (1 + 3e-6),
                   1, pix, tol)


@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_many_lines(mgx, prec, tol):
    """Every level pair of an 18-level rotor as a line (153 lines): more
    lines than the per-lane LDS table holds, so the line factors are formed
    per point.  The window is centred on 6B, where the 2-0 and 3-2 lines
    coincide and their opacities add."""
    m = synth.tiny_cloud(npoints=120, seed=55, k=10, nside=1, nlev=18, nbins=5, vmax=3e3,
                         tau_scale=5.0)
    u, l = np.array([(u, l) for u in range(1, 18) for l in range(u)], np.int32).T
    nu = (m.E[u] - m.E[l]) / 6.62607015e-34
    m.up, m.lo, m.nu = u, l, nu
    m.A = 1e-6 * (nu / 1e11) ** 3 / (u - l)
    assert m.nlines == 153 and 8 * m.nlines * 64 > 64 * 1024
    nu0 = nu[(u == 2) & (l == 0)][0]
    assert abs(nu[(u == 3) & (l == 2)][0] / nu0 - 1) < 1e-12
    pix = [(ix, iy) for ix in range(6) for iy in range(6)]
    img, _ = render_compare(mgx, m, prec, [0.6, -0.3, 0.74], 6, 6, nu0 * (1 - 3e-5),
                            nu0 * (1 + 3e-5), 70, pix, tol)
    # the lines are seen: the image is not the CMB everywhere
    assert np.ptp(img) > 1e-3 * np.max(np.abs(img))
    # a band between lines (all lie at even multiples of B): no line reaches
    # it, every profile underflows, the pixels see the CMB
    nu7 = 3.5 * nu0 / 3.0
    render_compare(mgx, m, prec, [0.6, -0.3, 0.74], 6, 6, nu7 * (1 - 3e-5), nu7 * (1 + 3e-5), 9,
                   pix, tol)


def _chain(n, seed=56):
    """n points along x (a little jitter across), neighbours i-1 and i+1,
    the two ends boundary points: viewed along x every pixel walk that enters
    runs the whole chain, far longer than the one-pass walk slots."""
    m = synth.tiny_cloud(npoints=n, seed=seed, k=2, nside=1, nlev=3, nbins=5, vmax=2e3,
                         tau_scale=20.0)
    rng = np.random.default_rng(seed)
    m.pos = np.stack([np.arange(n) * 1e11, rng.normal(0, 2e10, n), rng.normal(0, 2e10, n)])
    lists = [[j for j in (i - 1, i + 1) if 0 <= j < n] for i in range(n)]
    m.nbs_off = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int32)
    m.nbs = np.array([j for x in lists for j in x], np.int32)
    m.bdy = np.zeros(n, np.uint8)
    m.bdy[[0, n - 1]] = 1
    return m


@pytest.mark.parametrize("prec,tol", [(0, 2e-7), (1, 2e-5)])
def test_render_walks_longer_than_slots(mgx, prec, tol):
    """Walks longer than the one-pass slots (4 N^(1/3) + 16 points) take the
    exact two-pass route; the image still matches the oracle."""
    n = 300
    m = _chain(n)
    nu0 = m.nu[0]
    pix = [(ix, iy) for ix in range(3) for iy in range(3)]
    img, walks = render_compare(mgx, m, prec, [-1.0, 0.0, 0.0], 3, 3, nu0 * (1 - 2e-5),
                                nu0 * (1 + 2e-5), 9, pix, tol)
    assert max(len(w) for w in walks) > 4 * n ** (1 / 3) + 16


def test_render_steep_gradient_column(mgx):
    n = 9
    m = synth.cubic_lattice(n=n, nbins=5)
    m.nspec[:] = 3e5
    m.vel[0] = 40e3 / ((n - 1) * 1e12) * m.pos[0]
    nu0 = m.nu[0]
    pix = [(ix, iy) for ix in range(n) for iy in range(n)]
    for prec, tol in ((0, 2e-7), (1, 2e-5)):
        render_compare(mgx, m, prec, [1.0, 0.0, 0.0], n, n, nu0 * (1 - 1.2e-4), nu0, 13, pix, tol)


def test_render_errors(mgx):
    m = synth.spherical_shells("a")
    c = mgx.Context()
    c.load_model(m)
    c.set_lte_populations()
    with pytest.raises(mgx.MgxError) as e:
        c.render_image([0, 0, 1], 8, 8, 1e11, 1e11, 3)
    assert e.value.status == mgx.MGX_EINVAL
    m3 = synth.tiny_cloud(npoints=30, seed=52)
    c.load_model(m3)
    c.set_lte_populations()
    with pytest.raises(mgx.MgxError) as e:
        c.render_image([0, 0, 0], 8, 8, 1e11, 1e11, 3)
    assert e.value.status == mgx.MGX_EINVAL
    with pytest.raises(mgx.MgxError) as e:
        c.render_image([0, 0, 1], 8, 8, 1e11, 1e11, 2000)
    assert e.value.status == mgx.MGX_EINVAL
