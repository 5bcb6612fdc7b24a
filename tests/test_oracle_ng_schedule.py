"""Pins of the oracle's Ng schedules (Section "Adaptive Ng-acceleration").

The schedule is driven here by small affine maps x -> A x + b instead of a
radiative transfer model, so that each decision can be derived by hand or
checked against a second, independent implementation of the rule written in
this file from the paper's text (coefficients from the constrained
least-squares problem of the appendix, solved through its Lagrange system).

Event codes: 0 no prediction formed, 1 formed and not used, 2 used,
3 formed but invalid (singular Gram matrix or a negative component).
"""
import numpy as np
import pytest

import oracle

NONE, FORMED, USED, INVALID = 0, 1, 2, 3


def _diag_map(lams, xstar):
    lams = np.asarray(lams, float)
    xstar = np.asarray(xstar, float)
    return lambda x: lams * x + (1.0 - lams) * xstar


def _rel(a, b, floor=1e-12):
    return float(np.max(np.abs(a - b) / np.maximum(a, floor)))


def _ng_lagrange(hist):
    """Prediction from iterates y_1..y_N: minimise ||sum c_k r_k||^2 with
    sum c = 1 (appendix), via the bordered system [2G 1; 1^T 0][c; l] = [0; 1];
    combine the Lambda-images y_2..y_N.  None if G is numerically singular
    (the reading: a pivot of its partially pivoted LU factorisation below
    1e-14 of its largest diagonal entry) or the prediction has a negative
    component."""
    import scipy.linalg
    Y = np.asarray(hist)
    R = np.diff(Y, axis=0)
    K = R.shape[0]
    G = R @ R.T
    _, _, U = scipy.linalg.lu(G)
    if not np.all(np.abs(np.diag(U)) > 1e-14 * np.max(np.diag(G))):
        return None
    B = np.zeros((K + 1, K + 1))
    B[:K, :K] = 2 * G
    B[:K, K] = 1
    B[K, :K] = 1
    rhs = np.zeros(K + 1)
    rhs[K] = 1
    c = np.linalg.solve(B, rhs)[:K]
    p = c @ Y[1:]
    return None if np.any(p < 0) else p


def _schedule_ref(step, x0, tol, max_iter, mode, param, fresh):
    """The paper's rule, written out again: regular iterate, then (classical)
    a prediction every param stored iterates after the start of the history,
    or (adaptive) a prediction from all stored iterates after each one, used
    when the last two predictions differ less than the last two iterates or
    when the store holds N_max.  fresh: after a used prediction only later
    regular iterates are stored."""
    x = np.array(x0, float)
    hist = [x.copy()]
    prev = None
    events = []
    for it in range(1, max_iter + 1):
        y = step(x)
        ch = _rel(y, x)
        x = y
        if ch <= tol:
            events.append(NONE)
            return it, x, events
        hist.append(x.copy())
        ev, use, full, p = NONE, False, False, None
        if mode == 1:
            if len(hist) == param + 1:
                full = True
                p = _ng_lagrange(hist)
                use = p is not None
                ev = USED if use else INVALID
        elif mode == 2:
            full = len(hist) >= param
            if len(hist) >= 3:
                p = _ng_lagrange(hist)
                if p is None:
                    ev = INVALID
                else:
                    use = (prev is not None and _rel(p, prev) < _rel(hist[-1], hist[-2])) or full
                    prev = p
                    ev = USED if use else FORMED
        events.append(ev)
        if use:
            x = p.copy()
        if use or full:
            prev = None
            hist = [] if (use and fresh) else [x.copy()]
    return max_iter, x, events


def _run(step, x0, mode, param, fresh=False, tol=1e-13, max_iter=60):
    r = oracle.iterate_map(step, x0, tol, max_iter, mode | (oracle.NG_FRESH if fresh else 0),
                           param)
    return r


def test_classical_cadence_keep_and_fresh():
    """Classical order 4 on a 10-dimensional contraction (no prediction is
    exact, none singular): predictions at iterations 4, 8, 12, ... when the
    prediction starts the next history; at 4, 9, 14, ... when only later
    regular iterates are kept (five new ones are needed each time)."""
    rng = np.random.default_rng(1)
    lams = np.linspace(0.55, 0.97, 10)
    xs = rng.uniform(1, 2, 10)
    step = _diag_map(lams, xs)
    x0 = xs * (1 + 0.3 * rng.uniform(-1, 1, 10))
    r = _run(step, x0, 1, 4, max_iter=20, tol=0.0)
    used = [i + 1 for i, e in enumerate(r["events"]) if e == USED]
    assert used == [4, 8, 12, 16, 20]
    assert all(e in (NONE, USED) for e in r["events"])
    r = _run(step, x0, 1, 4, fresh=True, max_iter=20, tol=0.0)
    used = [i + 1 for i, e in enumerate(r["events"]) if e == USED]
    assert used == [4, 9, 14, 19]


def test_classical_order_one_is_the_plain_iteration():
    """One residual: c = (1), the prediction is the newest iterate itself, so
    every iteration 'uses' a prediction and the trajectory is the plain one."""
    step = _diag_map([0.5, 0.8, 0.9], [1.0, 2.0, 3.0])
    x0 = np.array([2.0, 1.0, 4.0])
    r = _run(step, x0, 1, 1, max_iter=25, tol=0.0)
    assert all(e == USED for e in r["events"])
    x = x0.copy()
    for _ in range(25):
        x = step(x)
    assert np.array_equal(r["x"], x)


def test_constant_map_converges_on_the_second_iteration():
    """x -> x*: the first iterate is the fixed point, the second changes
    nothing; no prediction is formed after one iterate in any mode."""
    xs = np.array([0.3, 0.5, 0.2])
    step = lambda x: xs.copy()
    for mode, param in ((0, 4), (1, 4), (2, 8)):
        r = _run(step, np.array([0.1, 0.1, 0.8]), mode, param)
        assert r["status"] == 0 and r["iters"] == 2
        assert list(r["events"]) == [NONE, NONE]


def test_adaptive_first_prediction_never_used_below_nmax():
    """The first prediction after a restart has no predecessor to compare
    with, so it is formed and not used unless the store is full (N_max)."""
    rng = np.random.default_rng(2)
    lams = np.linspace(0.6, 0.95, 8)
    xs = rng.uniform(1, 2, 8)
    step = _diag_map(lams, xs)
    x0 = xs * 1.2
    r = _run(step, x0, 2, 16, max_iter=3, tol=0.0)
    assert list(r["events"]) == [NONE, FORMED, r["events"][2]]
    assert r["events"][2] in (FORMED, USED)


def test_adaptive_nmax3_cadence_keep_and_fresh():
    """N_max = 3: the first prediction is formed with 3 iterates stored and
    is used because the store is full.  Keeping the prediction as y_1, the
    next comes two iterations later (2, 4, 6, ...); with only later regular
    iterates stored, three iterations later (2, 5, 8, ...)."""
    rng = np.random.default_rng(3)
    lams = np.linspace(0.6, 0.95, 6)
    xs = rng.uniform(1, 2, 6)
    step = _diag_map(lams, xs)
    x0 = xs * (1 + 0.2 * rng.uniform(-1, 1, 6))
    r = _run(step, x0, 2, 3, max_iter=12, tol=0.0)
    assert [i + 1 for i, e in enumerate(r["events"]) if e == USED] == [2, 4, 6, 8, 10, 12]
    r = _run(step, x0, 2, 3, fresh=True, max_iter=12, tol=0.0)
    assert [i + 1 for i, e in enumerate(r["events"]) if e == USED] == [2, 5, 8, 11]


def test_singular_history_is_rejected_and_plain_iterate_kept():
    """A map with one eigenvalue: every residual is a multiple of the first,
    the Gram matrix has rank one and each prediction from three or more
    iterates is rejected; the trajectory is then the plain iteration."""
    xs = np.array([1.0, 2.0, 3.0, 4.0])
    step = _diag_map([0.7] * 4, xs)
    x0 = xs + np.array([0.5, -0.3, 0.2, 0.1])
    r = _run(step, x0, 1, 3, max_iter=9, tol=0.0)
    assert [i + 1 for i, e in enumerate(r["events"]) if e != NONE] == [3, 6, 9]
    assert all(e in (NONE, INVALID) for e in r["events"])
    x = x0.copy()
    for _ in range(9):
        x = step(x)
    assert np.allclose(r["x"], x, rtol=1e-15, atol=0)


@pytest.mark.parametrize("mode,param,fresh", [
    (1, 2, False), (1, 3, False), (1, 4, False), (1, 4, True), (1, 6, True),
    (2, 4, False), (2, 8, False), (2, 16, False), (2, 8, True), (2, 32, True)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_schedule_matches_independent_rule(mode, param, fresh, seed):
    """Event by event and iterate by iterate against the rule written out in
    this file, on contractions with spread-out eigenvalues (dimension 12) and
    a mildly nonlinear map, until convergence to 1e-8 (closer to convergence
    the two routes to the coefficients round differently on the nearly
    collinear residuals, which can move the last iteration by one)."""
    rng = np.random.default_rng(100 + seed)
    d = 12
    lams = np.sort(rng.uniform(0.3, 0.97, d))
    xs = rng.uniform(0.5, 2.0, d)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    A = Q @ np.diag(lams) @ Q.T * 0.999
    b = xs - A @ xs
    if seed == 2:
        step = lambda x: A @ x + b + 0.01 * (x - xs) ** 2
    else:
        step = lambda x: A @ x + b
    x0 = xs * (1 + 0.1 * rng.uniform(-1, 1, d))
    r = _run(step, x0, mode, param, fresh=fresh, tol=1e-8, max_iter=400)
    it, x, ev = _schedule_ref(step, x0, 1e-8, 400, mode, param, fresh)
    assert r["status"] == 0
    assert r["iters"] == it
    assert list(r["events"]) == ev
    assert sum(e == USED for e in ev) >= 2
    assert np.allclose(r["x"], x, rtol=1e-7, atol=0)


def test_adaptive_rule_compares_the_right_pairs():
    """Sensitivity: on this map the decisions of the adaptive rule change if
    the running predictions are compared with the wrong pair of iterates (the
    first two of the history instead of the last two), or if the prediction
    is dropped from the restarted history; the oracle follows the rule as
    stated."""
    rng = np.random.default_rng(7)
    d = 12
    lams = np.sort(rng.uniform(0.3, 0.97, d))
    xs = rng.uniform(0.5, 2.0, d)
    step = _diag_map(lams, xs)
    x0 = xs * (1 + 0.1 * rng.uniform(-1, 1, d))
    r = _run(step, x0, 2, 16, tol=1e-8, max_iter=400)
    _, _, ev = _schedule_ref(step, x0, 1e-8, 400, 2, 16, False)
    assert list(r["events"]) == ev
    _, _, ev_fresh = _schedule_ref(step, x0, 1e-8, 400, 2, 16, True)
    assert ev_fresh != ev

    def wrong_pair(step, x0, tol, max_iter, param):
        x = np.array(x0, float)
        hist, prev, events = [x.copy()], None, []
        for it in range(1, max_iter + 1):
            y = step(x)
            ch = _rel(y, x)
            x = y
            if ch <= tol:
                events.append(NONE)
                return events
            hist.append(x.copy())
            ev, use, full = NONE, False, len(hist) >= param
            if len(hist) >= 3:
                p = _ng_lagrange(hist)
                use = (prev is not None and _rel(p, prev) < _rel(hist[1], hist[0])) or full
                prev = p
                ev = USED if use else FORMED
            events.append(ev)
            if use:
                x = p.copy()
            if use or full:
                prev, hist = None, [x.copy()]
        return events
    assert wrong_pair(step, x0, 1e-8, 400, 16) != ev
