"""Fits of the erfc used by the formal solution's semi-analytic segments.

The kernel evaluates, for x >= 0,

    erfc(x) ~= t * 2^(P(t) - x^2 log2 e),   t = 1 / (1 + p x),

the product form of Numerical Recipes (Press et al., 2nd ed., Sec. 6.2) with
P a polynomial fitted here in base 2: P(t) ~= log2(erfc(x) / t) + x^2 log2 e.
The fit minimises the maximum error of P on a dense grid of x in [0, xmax]
(Lawson's iteratively reweighted least squares, which converges to the
minimax solution of a linear fit); an error dP in P is a relative error of
dP ln 2 in erfc.  Reference values come from mpmath at 30 digits.

Run:  python -m paper_2411_03040_amd.fit_erfc [--degree 6] [--p 0.62]
prints the coefficients (highest degree first, the kernel's Horner order),
p / sqrt(log2 e) (the kernel takes x already scaled by sqrt(log2 e)) and the
maximum relative error of erfc in exact arithmetic.

FP64 (--fp64, defaults degree 20, p = 0.5): the same product form in base e,
erfc(x) ~= t exp(P(t) - x^2), fitted by least squares at 50 digits on
Chebyshev nodes in t for x in [0, 26.5] (beyond, erfc is subnormal in double
and the kernel's result flushes to zero past 27.5); the script also reports
the largest relative error of the double-precision evaluation (Horner with
multiply-adds, the same operation order as the kernel) against 50-digit
erfc, which the rounding of x^2 dominates near the top of the range.
"""
import argparse

import mpmath as mp
import numpy as np

LOG2E = 1.0 / np.log(2.0)


def fit(degree: int, p: float, xmax: float = 9.6, n: int = 4000, iters: int = 400):
    mp.mp.dps = 30
    x = np.linspace(0.0, xmax, n)
    log2_erfc = np.array([float(mp.log(mp.erfc(mp.mpf(float(v))), 2)) for v in x])
    t = 1.0 / (1.0 + p * x)
    target = log2_erfc - np.log2(t) + x * x * LOG2E
    V = np.vander(t, degree + 1, increasing=True)
    w = np.full(n, 1.0 / n)
    best_err, best = np.inf, None
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], target * sw, rcond=None)
        r = np.abs(V @ c - target)
        if r.max() < best_err:
            best_err, best = r.max(), c
        w = w * r
        w /= w.sum()
    return best, best_err * np.log(2.0)


def max_rel_error(c, p: float, xmax: float = 9.6, n: int = 20001) -> float:
    mp.mp.dps = 30
    worst = 0.0
    for v in np.linspace(0.0, xmax, n):
        t = 1.0 / (1.0 + p * v)
        approx = t * 2.0 ** (np.polyval(c[::-1], t) - v * v * LOG2E)
        worst = max(worst, abs(approx / float(mp.erfc(mp.mpf(float(v)))) - 1.0))
    return worst


def fit64(degree: int, p: float, xmax: float = 26.5):
    mp.mp.dps = 50
    tmin = 1 / (1 + mp.mpf(p) * xmax)
    n = 3 * degree + 60
    ts = [tmin + (1 - tmin) * (1 + mp.cos(mp.pi * (k + mp.mpf(0.5)) / n)) / 2 for k in range(n)]
    A = mp.matrix(n, degree + 1)
    b = mp.matrix(n, 1)
    for i, t in enumerate(ts):
        x = (1 / t - 1) / p
        b[i] = mp.log(mp.erfc(x) / t) + x * x
        v = mp.mpf(1)
        for j in range(degree + 1):
            A[i, j] = v
            v *= t
    c, _ = mp.qr_solve(A, b)
    return [float(c[j]) for j in range(degree + 1)]


def max_rel_error64(c, p: float, xmax: float = 26.4, n: int = 6000) -> float:
    """The kernel's double evaluation against 50-digit erfc (normal range)."""
    mp.mp.dps = 50

    def fma(a, b, cc):
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(cc))
    worst = 0.0
    for v in np.concatenate([np.linspace(0.0, 4.0, n // 2), np.linspace(4.0, xmax, n // 2)]):
        d = fma(float(v), p, 1.0)
        t = 1.0 / d
        P = c[-1]
        for a in c[-2::-1]:
            P = fma(P, t, a)
        arg = fma(-float(v), float(v), P)
        approx = t * float(mp.exp(mp.mpf(arg)))
        worst = max(worst, abs(approx / float(mp.erfc(mp.mpf(float(v)))) - 1.0))
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--p", type=float, default=None)
    ap.add_argument("--fp64", action="store_true")
    args = ap.parse_args()
    if args.fp64:
        deg = args.degree or 20
        p = args.p or 0.5
        c = fit64(deg, p)
        print("coefficients, highest degree first:", ", ".join(f"{v:.17g}" for v in c[::-1]))
        print(f"t = 1 / (1 + {p} x)")
        print(f"max relative error of the double evaluation on [0, 26.4]: "
              f"{max_rel_error64(c, p):.2e}")
        return
    args.degree = args.degree or 6
    args.p = args.p or 0.62
    c, err = fit(args.degree, args.p)
    print("coefficients, highest degree first:", ", ".join(f"{v:.8f}" for v in c[::-1]))
    print(f"t = 1 / (1 + xs * {args.p / np.sqrt(LOG2E):.8f}),  xs = x sqrt(log2 e)")
    print(f"max relative error of erfc on the fit grid: {err:.2e}; "
          f"on a finer grid with the coefficients rounded to 8 digits: "
          f"{max_rel_error(np.round(c, 8), args.p):.2e}")


if __name__ == "__main__":
    main()
