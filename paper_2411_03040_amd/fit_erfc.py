"""Fit of the FP32 erfc used by the formal solution's semi-analytic segments.

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--degree", type=int, default=6)
    ap.add_argument("--p", type=float, default=0.62)
    args = ap.parse_args()
    c, err = fit(args.degree, args.p)
    print("coefficients, highest degree first:", ", ".join(f"{v:.8f}" for v in c[::-1]))
    print(f"t = 1 / (1 + xs * {args.p / np.sqrt(LOG2E):.8f}),  xs = x sqrt(log2 e)")
    print(f"max relative error of erfc on the fit grid: {err:.2e}; "
          f"on a finer grid with the coefficients rounded to 8 digits: "
          f"{max_rel_error(np.round(c, 8), args.p):.2e}")


if __name__ == "__main__":
    main()
