"""The paper's own LIBOR case (Table 3 Treasury curve -> cubic spline ->
6-month bond prices -> initial forwards by eq. (BL); caplet with
(t, T, delta, K, sigma) = (0, 5, 0.5, 0.01, 0.04)): the input construction
pinned against scipy and the defining identities, and the oracle's plain
Euler and log-Euler prices against the Black formula."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.stats import norm

import oracle as O
import rqmc_inputs as I


def test_spline_is_scipys_natural_cubic_spline():
    xs, ys = I.TREASURY_2012_02_24
    t = np.linspace(xs[0], xs[-1], 2001)
    f = I.natural_cubic_spline(xs, ys)
    ref = CubicSpline(np.array(xs), np.array(ys), bc_type="natural")
    assert np.abs(f(t) - ref(t)).max() < 1e-12
    assert np.allclose(f(np.array(xs)), ys, rtol=0, atol=1e-14)
    assert abs(ref(xs[0], 2)) < 1e-12 and abs(ref(xs[-1], 2)) < 1e-12


def test_forwards_reproduce_the_bond_prices():
    m = I.lmm_treasury_caplet()
    grid = np.arange(m.n_fwd + 2) * m.delta
    B = I.treasury_bond_prices(grid)
    rebuilt = np.cumprod(np.concatenate([[1.0], 1.0 / (1.0 + m.delta * m.L0)]))
    assert np.allclose(rebuilt, B, rtol=1e-14, atol=0)
    assert (np.diff(B) < 0).all() and (m.L0 > 0).all()
    # the 6-month yield on the table's 6-month point: L_0(0) = 0.14% exactly
    assert abs(m.L0[0] - 0.0014) < 1e-15


def _black(m):
    n = m.n_fwd
    B = I.treasury_bond_prices(np.array([(n + 1) * m.delta]))[0]
    L, K, s, T = m.L0[n], m.strike[n - 1], m.sigma[n], n * m.delta
    d1 = (math.log(L / K) + 0.5 * s * s * T) / (s * math.sqrt(T))
    d2 = d1 - s * math.sqrt(T)
    return m.delta * B * (L * norm.cdf(d1) - K * norm.cdf(d2))


@pytest.mark.parametrize("flags", [0, O.LMM_EULER, O.LMM_EULER | O.MC_PHILOX])
def test_paper_caplet_prices_against_black(flags):
    m = I.lmm_treasury_caplet()
    th = O.price_caplets(m, 4096, 16, 6, flags=flags)[:, -1]
    se = th.std(ddof=1) / math.sqrt(len(th))
    # deep in the money (L = 2.39% vs K = 1%) at 4% vol: the discretisation
    # bias of a ten-step scheme is far below 1e-7 of the price
    assert abs(th.mean() - _black(m)) < 4 * se + 1e-9


def test_euler_and_log_euler_differ_only_by_discretisation():
    m = I.lmm_treasury_caplet()
    a = O.price_caplets(m, 1024, 2, 6)[:, -1]
    b = O.price_caplets(m, 1024, 2, 6, flags=O.LMM_EULER)[:, -1]
    assert not np.array_equal(a, b)
    # per path the schemes differ by O(sigma^2 delta (z^2 - 1)) per step, mean 0
    assert np.allclose(a, b, rtol=1e-3, atol=0)
