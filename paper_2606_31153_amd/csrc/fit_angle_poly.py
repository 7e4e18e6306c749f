"""Fits the float polynomials of the fan-beam angle kernels in proj2d.hip.

    atan(z) = z P(z^2), |z| <= 0.5      (the pixel fan angle from its tangent)
    asin(s) = s Q(s^2), |s| <= 1/sqrt(5) (the same angle from its sine: the
                                          sine of an angle of tangent 0.5)

Each polynomial has degree 5 in the square and a leading coefficient of 1.
The method is Lawson's iteratively reweighted least squares on 3000 Chebyshev
nodes of the square's interval, which drives the weighted least-squares fit
towards the minimax fit of the relative error.  The coefficients are rounded
to float one at a time, lowest degree first, and the ones above are refitted
after each rounding.  The script prints the float coefficients and the largest
relative error of the rounded polynomial on a fine grid, in exact (double)
arithmetic.

Run from anywhere: python fit_angle_poly.py
"""
import numpy as np

NODES, ITERS, DEG = 3000, 1500, 5


def lawson(a: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    w = np.full(a.shape[0], 1.0 / a.shape[0])
    best_err, best = np.inf, None
    for _ in range(ITERS):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(a * sw[:, None], rhs * sw, rcond=None)
        e = np.abs(a @ c - rhs)
        if e.max() < best_err:
            best_err, best = e.max(), c.copy()
        w = w * e
        w /= w.sum()
    return best


def fit(fun, tmax: float) -> list:
    """Float coefficients c_0 = 1, c_1..c_DEG of fun(s) ~ s sum_j c_j s^(2j)."""
    k = np.arange(NODES)
    t = 0.5 * tmax * (1.0 - np.cos(np.pi * (k + 0.5) / NODES))
    s = np.sqrt(t)
    g = fun(s) / s
    # relative error: (1 + sum_j c_j t^j) / g - 1, linear in c_1..c_DEG
    cols = [t ** j / g for j in range(1, DEG + 1)]
    rhs0 = 1.0 - 1.0 / g
    fixed = []
    for j in range(DEG):
        rhs = rhs0 - sum(c * cols[i] for i, c in enumerate(fixed))
        c = lawson(np.stack(cols[j:], 1), rhs)
        fixed.append(float(np.float32(c[0])))
    return [1.0] + fixed


def max_rel_err(fun, coef, tmax: float, n: int = 400001) -> float:
    t = np.linspace(tmax / n, tmax, n)
    s = np.sqrt(t)
    return float(np.max(np.abs(s * np.polyval(np.asarray(coef)[::-1], t) / fun(s) - 1.0)))


def main():
    for name, fun, tmax in (("atan", np.arctan, 0.25), ("asin", np.arcsin, 0.2)):
        c = fit(fun, tmax)
        print("%s: max relative error %.2e; coefficients c_0..c_%d:" % (name, max_rel_err(fun, c, tmax), DEG))
        print("  " + ", ".join("%.8gf" % np.float32(x) for x in c))


if __name__ == "__main__":
    main()
