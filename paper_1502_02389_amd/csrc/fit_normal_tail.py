"""Coefficients of the normal-tail approximation used by the BlackScholes kernel.

The upper tail of the standard normal distribution is Q(z) = phi(z) R(z) for
z >= 0, with phi the density and R the Mills ratio, R(z) = sqrt(pi/2)
erfcx(z / sqrt 2).  The kernel evaluates R as a polynomial in t = 1/(1 + p z),
R(z) ~ sum_{k=1..7} c_k t^k (t -> 0 as z grows, where R ~ 1/z ~ t/p).  The
coefficients below are a least-squares fit weighted by phi(z), i.e. they
minimise the absolute error of Q, on z in [0, 12]; p is the best of a grid
scan.  Run this script to regenerate the constants (it prints the C++ lines
and the worst absolute error of Q on [0, 40]).
"""
import numpy as np
from scipy.special import erfcx

DEGREE = 7


def mills(z):
    return np.sqrt(np.pi / 2) * erfcx(z / np.sqrt(2))


def density(z):
    return np.exp(-z * z / 2) / np.sqrt(2 * np.pi)


def fit(p, degree=DEGREE):
    z = np.linspace(0.0, 12.0, 60000)
    t = 1 / (1 + p * z)
    a = np.stack([t ** k for k in range(1, degree + 1)], 1)
    w = density(z)
    c, *_ = np.linalg.lstsq(a * w[:, None], mills(z) * w, rcond=None)
    return c


def worst_abs_error(p, c):
    z = np.linspace(0.0, 40.0, 400001)
    t = 1 / (1 + p * z)
    r = sum(ck * t ** (k + 1) for k, ck in enumerate(c))
    return float(np.max(np.abs(density(z) * (r - mills(z)))))


def main():
    best = None
    for p in np.round(np.linspace(0.20, 0.45, 51), 3):
        c = fit(p)
        e = worst_abs_error(p, c)
        if best is None or e < best[0]:
            best = (e, p, c)
    e, p, c = best
    print(f"// worst |Q error| on [0, 40]: {e:.3e}")
    print(f"constexpr float TAIL_P = {float(p)!r}f;")
    print("constexpr float TAIL_C[7] = {" + ", ".join(f"{v:.9e}f" for v in c) + "};")


if __name__ == "__main__":
    main()
