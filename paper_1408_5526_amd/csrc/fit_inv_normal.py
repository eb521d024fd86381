"""Fits the FP32 inverse-normal polynomials used by the kernels.

Form (after Giles, "Approximating the erfinv function", GPU Computing Gems
2011): with x = 2u - 1 and w = -ln(1 - x^2) = -ln(4u(1-u)),
    Phi^{-1}(u) = x * P(w - 2.5)            for w < 5   (u in ~(0.0017, 0.9983))
    Phi^{-1}(u) = x * Q(sqrt(w) - 3)        for w >= 5  (down to u = 2^-64)
P and Q approximate f(w) = Phi^{-1}(u)/x = sqrt(2) erfinv(x)/x, a smooth
function of w.  Their coefficients are fitted here (not taken from any
publication): weighted least squares on Chebyshev nodes for relative error,
refined by Lawson iterations towards the minimax solution, against mpmath at
40 digits.  Run this file to regenerate the table pasted in rq_device.h;
it prints the coefficients and the float32 evaluation error.
"""
from __future__ import annotations

import mpmath
import numpy as np

mpmath.mp.dps = 40
W_SPLIT = 5.0
W_MAX = float(-mpmath.log(4 * mpmath.mpf(2) ** -64 * (1 - mpmath.mpf(2) ** -64)))


def f_exact(w):
    w = mpmath.mpf(w)
    x = mpmath.sqrt(-mpmath.expm1(-w))
    return mpmath.sqrt(2) * mpmath.erfinv(x) / x


def fit(tmap, wlo, whi, deg, n=600, iters=60):
    k = np.arange(n)
    # Chebyshev nodes in the fitted variable t
    tlo, thi = tmap(wlo), tmap(whi)
    t = 0.5 * (tlo + thi) + 0.5 * (thi - tlo) * np.cos(np.pi * (k + 0.5) / n)
    if tmap is _t_tail:
        w = (t + 3.0) ** 2
    else:
        w = t + 2.5
    y = np.array([float(f_exact(v)) for v in w])
    V = np.vander(t, deg + 1, increasing=True)
    wt = np.ones(n)
    c = None
    for _ in range(iters):            # Lawson: reweight towards equal-ripple
        A = V * (wt / y)[:, None]
        c, *_ = np.linalg.lstsq(A, wt, rcond=None)
        r = np.abs(V @ c - y) / y
        wt = wt * (r / r.max() + 1e-3)
        wt /= wt.sum() / n
    return c, t, y


def _t_central(w):
    return w - 2.5


def _t_tail(w):
    return np.sqrt(w) - 3.0


def horner_f32(c, t):
    t = np.float32(t)
    acc = np.float32(c[-1])
    for a in c[-2::-1]:
        acc = np.float32(acc * t + np.float32(a))
    return acc


def main():
    cP, tP, yP = fit(_t_central, 0.0, W_SPLIT, 9)
    cQ, tQ, yQ = fit(_t_tail, W_SPLIT, W_MAX, 12)
    for name, c, t, y in (("P", cP, tP, yP), ("Q", cQ, tQ, yQ)):
        e64 = np.max(np.abs(np.polyval(c[::-1], t) - y) / y)
        e32 = max(abs(float(horner_f32(c, tt)) - yy) / yy for tt, yy in zip(t, y))
        print(f"{name}: degree {len(c) - 1}, max rel err fp64 {e64:.2e}, float32 Horner {e32:.2e}")
        print("  coefficients, highest degree first:")
        for a in c[::-1]:
            print(f"    {float(np.float32(a))!r}f,")


if __name__ == "__main__":
    main()
