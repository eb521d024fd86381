"""Pins for the oracle's LIBOR market model pricer (CPU only).

  * sigma = 0: forwards stay at L(0); each caplet is worth
    delta (L_n(0) - K)^+ B_{n+1}(0) exactly, B_{n+1}(0) = prod_{j<=n} 1/(1+delta L_j(0)).
  * n_fwd = 1 and n_fwd = 2 (one factor): the discrete scheme's price is a
    1-D / 2-D Gaussian integral, done by adaptive quadrature -- exact for the
    scheme, so the RQMC estimate must sit within a few standard errors.
  * Black's caplet formula (caplet section) within 3 standard errors plus
    the time-discretisation bias of the scheme, the latter estimated by a
    common-random-number Richardson run (step delta vs delta/2).
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

import oracle as O
import rqmc_inputs as I


def black_caplets(model):
    """delta B(0,T_{n+1}) [L Phi(d1) - K Phi(d2)], d1,2 = (ln(L/K) +- s^2 T/2)/(s sqrt T),
    T = T_n = n delta the fixing date; NaN strikes give 0."""
    d = model.delta
    out = np.zeros(model.n_fwd)
    B = 1.0 / (1.0 + d * model.L0[0])
    for n in range(1, model.n_fwd + 1):
        B /= 1.0 + d * model.L0[n]
        K = model.strike[n - 1]
        if np.isnan(K):
            continue
        L, s, T = model.L0[n], model.sigma[n], n * d
        d1 = (math.log(L / K) + 0.5 * s * s * T) / (s * math.sqrt(T))
        d2 = d1 - s * math.sqrt(T)
        out[n - 1] = d * B * (L * norm.cdf(d1) - K * norm.cdf(d2))
    return out


def crn_bias(model, n_paths, seed):
    """b = 2 (V_delta - V_delta/2) with shared Brownian increments:
    the coarse normal of a period is (z_a + z_b)/sqrt(2) of its two halves."""
    rng = np.random.default_rng(seed)
    nf, d = model.n_fwd, model.n_factors
    zf = rng.standard_normal((n_paths, nf, 2, d))
    zc = (zf[:, :, 0, :] + zf[:, :, 1, :]) / math.sqrt(2.0)
    pf = O.lmm_paths(model, zf.reshape(n_paths, -1), n_sub=2)
    pc = O.lmm_paths(model, zc.reshape(n_paths, -1), n_sub=1)
    diff = 2.0 * (pc - pf)
    return diff.mean(axis=0), diff.std(axis=0, ddof=1) / math.sqrt(n_paths)


def test_zero_vol_closed_form():
    m = I.lmm_curve80(n_fwd=12, n_factors=3)
    m.sigma[:] = 0.0
    m.strike = m.L0[1:] + np.linspace(-0.004, 0.004, 12)   # ITM and OTM
    z = np.random.default_rng(3).standard_normal((5, m.s))
    pay = O.lmm_paths(m, z)
    want = np.zeros(13)
    B = 1.0 / (1.0 + m.delta * m.L0[0])
    for n in range(1, 13):
        B /= 1.0 + m.delta * m.L0[n]
        want[n - 1] = m.delta * max(m.L0[n] - m.strike[n - 1], 0.0) * B
    want[12] = want[:12].sum()
    for row in pay:
        assert np.allclose(row, want, rtol=2e-15, atol=1e-18)


def _one_forward_model(L0=0.05, L1=0.055, vol=0.3, K=0.05, delta=0.5):
    return I.LmmModel(n_fwd=1, n_factors=1, delta=delta, L0=np.array([L0, L1]),
                      sigma=np.array([0.0, vol]), loadings=np.ones((1, 1)),
                      strike=np.array([K]))


def test_one_forward_quadrature_exact_for_scheme():
    m = _one_forward_model()
    d, a, L0, L1, K = m.delta, m.sigma[1], m.L0[0], m.L0[1], m.strike[0]
    g = d * L1 / (1 + d * L1)

    def L1T(z):   # single step of the spot-measure log-Euler scheme
        return L1 * math.exp((g * a * a - 0.5 * a * a) * d + math.sqrt(d) * a * z)

    def pay(z):
        LT = L1T(z)
        return d * max(LT - K, 0.0) / ((1 + d * L0) * (1 + d * LT)) * norm.pdf(z)

    zk = (math.log(K / L1) - (g * a * a - 0.5 * a * a) * d) / (math.sqrt(d) * a)
    val = integrate.quad(pay, zk, 12, epsabs=1e-15, epsrel=1e-13)[0]
    # per-path check against the same closed expression
    zs = np.array([[-1.3], [0.0], [0.4], [2.1]])
    pp = O.lmm_paths(m, zs)
    for z, row in zip(zs[:, 0], pp):
        LT = L1T(z)
        assert row[0] == pytest.approx(d * max(LT - K, 0) / ((1 + d * L0) * (1 + d * LT)), rel=1e-14, abs=1e-19)
    th = O.price_caplets(m, 1 << 14, 32, seed=21)
    rq, sd, se = O.finalize(th)
    assert abs(rq[0] - val) <= 4 * se[0], (rq[0], val, se[0])
    assert se[0] / val < 1e-4          # the bound above is a tight one


def test_two_forward_quadrature_exact_for_scheme():
    d = 0.5
    L = np.array([0.03, 0.035, 0.04])
    sig = np.array([0.0, 0.25, 0.2])
    K = np.array([0.033, 0.041])
    m = I.LmmModel(n_fwd=2, n_factors=1, delta=d, L0=L, sigma=sig, loadings=np.ones((2, 1)), strike=K)
    a1, a2 = sig[1], sig[2]
    sd_ = math.sqrt(d)

    def step0(z0):
        g1 = d * L[1] / (1 + d * L[1])
        g2 = d * L[2] / (1 + d * L[2])
        mu1 = a1 * (g1 * a1)
        mu2 = a2 * (g1 * a1 + g2 * a2)
        L1 = L[1] * math.exp((mu1 - 0.5 * a1 * a1) * d + sd_ * a1 * z0)
        L2 = L[2] * math.exp((mu2 - 0.5 * a2 * a2) * d + sd_ * a2 * z0)
        return L1, L2

    def cap1(z0):
        L1, _ = step0(z0)
        return d * max(L1 - K[0], 0) / ((1 + d * L[0]) * (1 + d * L1)) * norm.pdf(z0)

    def cap2_inner(z1, z0):
        L1, L2 = step0(z0)
        g = d * L2 / (1 + d * L2)
        L2T = L2 * math.exp((g * a2 * a2 - 0.5 * a2 * a2) * d + sd_ * a2 * z1)
        num = (1 + d * L[0]) * (1 + d * L1) * (1 + d * L2T)
        return d * max(L2T - K[1], 0) / num * norm.pdf(z1) * norm.pdf(z0)

    def cap2_outer(z0):
        L1, L2 = step0(z0)
        g = d * L2 / (1 + d * L2)
        zk = (math.log(K[1] / L2) - (g * a2 * a2 - 0.5 * a2 * a2) * d) / (sd_ * a2)
        return integrate.quad(cap2_inner, zk, 12, args=(z0,), epsabs=1e-16, epsrel=1e-12)[0]

    zk1 = brentq_kink = None
    from scipy.optimize import brentq
    zk1 = brentq(lambda z: step0(z)[0] - K[0], -10, 10)
    v1 = integrate.quad(cap1, zk1, 12, epsabs=1e-16, epsrel=1e-12)[0]
    v2 = integrate.quad(cap2_outer, -12, 12, epsabs=1e-15, epsrel=1e-11, limit=200)[0]
    th = O.price_caplets(m, 1 << 14, 32, seed=5)
    rq, sd, se = O.finalize(th)
    assert abs(rq[0] - v1) <= 4 * se[0] + 1e-12
    assert abs(rq[1] - v2) <= 4 * se[1] + 1e-12
    assert abs(rq[2] - (v1 + v2)) <= 4 * se[2] + 1e-12


def test_black_cfg1_within_se_plus_bias():
    c = I.cfg1()
    blk = black_caplets(c.model)
    assert blk[-1] == pytest.approx(1.3698347565136066e-3, rel=1e-13)
    th = O.price_caplets(c.model, c.N, c.M, c.seed)
    rq, sd, se = O.finalize(th)
    b, se_b = crn_bias(c.model, 400_000, seed=11)
    dev = rq[-1] - blk[-1] - b[-1]
    assert abs(dev) <= 3 * math.sqrt(se[-1] ** 2 + se_b[-1] ** 2), (rq[-1], blk[-1], b[-1], se[-1], se_b[-1])
    assert rq[9] == rq[10]           # the only caplet is the book


def test_black_multifactor_within_se_plus_bias():
    m = I.small_lmm(n_fwd=6, n_factors=2)
    blk = black_caplets(m)
    th = O.price_caplets(m, 1 << 13, 32, seed=17)
    rq, sd, se = O.finalize(th)
    b, se_b = crn_bias(m, 200_000, seed=12)
    for n in range(6):
        dev = rq[n] - blk[n] - b[n]
        assert abs(dev) <= 3.5 * math.sqrt(se[n] ** 2 + se_b[n] ** 2), (n, rq[n], blk[n], b[n])
    dev = rq[6] - blk.sum() - b[6]
    assert abs(dev) <= 3.5 * math.sqrt(se[6] ** 2 + se_b[6] ** 2)


@pytest.mark.slow
def test_black_cfg3_book_within_se_plus_bias():
    m = I.lmm_curve80()
    blk = black_caplets(m)
    assert blk.sum() == pytest.approx(0.1264663, abs=1e-7)
    th = O.price_caplets(m, 1 << 10, 16, seed=3)
    rq, sd, se = O.finalize(th)
    b, se_b = crn_bias(m, 6000, seed=13)
    dev = rq[80] - blk.sum() - b[80]
    assert abs(dev) <= 3.5 * math.sqrt(se[80] ** 2 + se_b[80] ** 2), (rq[80], blk.sum(), b[80], se[80], se_b[80])


def test_bias_shrinks_with_substeps():
    # the scheme's bias against Black is O(h): halving the step halves it
    m = I.lmm_flat(8, 0.5, 0.06, 0.35, 0.06, caplets=[8])
    rng = np.random.default_rng(4)
    n = 200_000
    zf = rng.standard_normal((n, 8, 4, 1))
    z2 = (zf[:, :, 0::2, :] + zf[:, :, 1::2, :]) / math.sqrt(2)
    z1 = (z2[:, :, 0, :] + z2[:, :, 1, :]) / math.sqrt(2)
    v4 = O.lmm_paths(m, zf.reshape(n, -1), n_sub=4)[:, -1]
    v2 = O.lmm_paths(m, z2.reshape(n, -1), n_sub=2)[:, -1]
    v1 = O.lmm_paths(m, z1.reshape(n, -1), n_sub=1)[:, -1]
    d1 = (v1 - v2).mean()
    d2 = (v2 - v4).mean()
    assert abs(d1) > 5 * (v1 - v2).std() / math.sqrt(n)
    assert 1.5 < d1 / d2 < 2.7


def test_factor_rotation_is_distributional_invariant():
    # loadings B and B Q (Q orthogonal) give the same law of the path
    m = I.small_lmm(n_fwd=5, n_factors=2)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    m2 = m.copy()
    m2.loadings = m.loadings @ Q
    a = O.finalize(O.price_caplets(m, 1 << 13, 32, seed=1))
    b = O.finalize(O.price_caplets(m2, 1 << 13, 32, seed=2))
    assert abs(a[0][-1] - b[0][-1]) <= 4 * math.hypot(a[2][-1], b[2][-1])


def test_plain_euler_flag_is_first_order_consistent():
    # plain Euler and log-Euler driven by the same Brownian increments are two
    # discretisations of the same SDE; their pathwise gap is dominated by
    # Euler's missing Ito term (a^2/2)(dW^2 - h), i.e. strong order 1/2:
    # halving h shrinks the mean gap by about sqrt(2)
    m = I.small_lmm(n_fwd=4, n_factors=1)
    n = 4000
    z8 = np.random.default_rng(9).standard_normal((n, m.n_fwd, 8, 1))
    z4 = (z8[:, :, 0::2, :] + z8[:, :, 1::2, :]) / math.sqrt(2)
    gaps = []
    for zz, ns in ((z4, 4), (z8, 8)):
        ve = O.lmm_paths(m, zz.reshape(n, -1), n_sub=ns, euler=True)[:, -1]
        vl = O.lmm_paths(m, zz.reshape(n, -1), n_sub=ns, euler=False)[:, -1]
        gaps.append(np.abs(ve - vl).mean())
    assert gaps[1] > 0
    assert 1.2 < gaps[0] / gaps[1] < 1.7, gaps
