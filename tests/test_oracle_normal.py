"""Pins for the oracle's inverse normal CDF (AS241 / PPND16), CPU only.

Pinned against mpmath at 50 digits (an independent arbitrary-precision
erfinv), against Python's libm erfc through Phi(Phi^{-1}(u)) = u, and the
symmetry Phi^{-1}(1-u) = -Phi^{-1}(u)."""
import math

import mpmath
import numpy as np
import pytest

import oracle as O

mpmath.mp.dps = 50


def _ref(u: float) -> float:
    # Phi^{-1}(u) = -sqrt(2) erfcinv(2u) (exact identity), at 50 digits
    return float(-mpmath.sqrt(2) * mpmath.erfinv(1 - 2 * mpmath.mpf(u)))


def _ref_tail(u: float) -> float:
    # for tiny u use the inverse of the complementary error function
    f = lambda z: mpmath.ncdf(z) - mpmath.mpf(u)
    z0 = _ref(max(u, 1e-300)) if u > 1e-15 else -math.sqrt(-2 * math.log(u))
    return float(mpmath.findroot(f, z0))


U_CENTRAL = [0.5, 0.5 + 2 ** -40, 0.51, 0.6, 0.7, 0.8, 0.9, 0.92, 0.925, 0.075,
             0.3, 0.4, 0.499, 0.2, 0.1]
U_TAIL = [0.07, 0.05, 0.01, 1e-3, 1e-5, 1e-8, 1e-11, 1.4e-11, 1e-12, 1e-15,
          1e-18, 0.93, 0.99, 0.999999]


@pytest.mark.parametrize("u", U_CENTRAL + U_TAIL)
def test_ppnd16_matches_mpmath(u):
    got = float(O.ppnd16(np.array([u]))[0])
    want = _ref_tail(u) if u < 1e-10 else _ref(u)
    assert abs(got - want) <= 4e-16 * max(1.0, abs(want)) + (2e-16 if abs(want) < 1e-3 else 0)


def test_ppnd16_dense_vs_erfc_roundtrip():
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.random(20000), 10.0 ** rng.uniform(-19, -1, 5000)])
    z = O.ppnd16(u)
    # Phi(z) = erfc(-z/sqrt2)/2 with libm's erfc; relative error in u from
    # one FP64 rounding of z is ~ |z phi(z)/Phi(z)| eps
    back = np.array([0.5 * math.erfc(-v / math.sqrt(2)) for v in z])
    rel = np.abs(back - u) / u
    slack = (1 + np.abs(z) * (np.abs(z) + 1)) * 2e-15
    assert (rel <= slack).all()


def test_ppnd16_symmetry():
    rng = np.random.default_rng(1)
    u = rng.random(5000) * 0.5
    u = u[u > 0]
    # 1 - u is exact for u in [0.25, 0.5]; elsewhere compare through 1-(1-u)
    one_minus = 1.0 - u
    u_exact = 1.0 - one_minus
    z1 = O.ppnd16(u_exact)
    z2 = O.ppnd16(one_minus)
    assert np.allclose(z1, -z2, rtol=1e-15, atol=0)


def test_ppnd16_endpoint_clamp_and_monotone():
    z0 = float(O.ppnd16(np.array([0.0]))[0])
    assert math.isfinite(z0)
    assert abs(z0 - _ref_tail(2.0 ** -64)) < 1e-13
    u = np.linspace(1e-6, 1 - 1e-6, 200001)
    z = O.ppnd16(u)
    assert (np.diff(z) > 0).all()
    assert O.ppnd16(np.array([0.5]))[0] == 0.0
