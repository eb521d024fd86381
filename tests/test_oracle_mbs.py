"""Pins for the oracle's MBS pricer and the estimators (CPU only).

  * sigma = 0: rates stay at i0, the pool is a level-pay mortgage discounted
    at its own rate, and prepayment returns the remaining balance at par, so
    PV = 1 exactly for any prepayment constants and any term.
  * c_k against the geometric-series closed form.
  * The recursive path against the paper's closed product forms
    (i_k = K0^k e^{xi_1+...+xi_k} i0, u_k and r_k as products), evaluated by
    an independent vectorised computation on the same normals.
  * The RQMC estimate against a pseudo-random Monte Carlo estimate.
  * theta / RQ / sd / SE against math.fsum and the statistics module;
    replication-offset splitting is bit-exact.
"""
import math
import statistics

import numpy as np
import pytest

import oracle as O
import rqmc_inputs as I


@pytest.mark.parametrize("months", [1, 12, 120, 360])
@pytest.mark.parametrize("K", [(0.01, -0.005, 10.0, 0.5), (0.0, 0.0, 0.0, 0.0), (0.05, 0.02, 3.0, -1.0)])
def test_zero_vol_pays_par(months, K):
    p = I.MbsParams(months, 0.007, 0.0, *K)
    z = np.random.default_rng(months).standard_normal((3, months))
    pv = O.mbs_paths(p, z)
    assert np.allclose(pv, 1.0, rtol=0, atol=5e-14)


def test_annuity_factor_closed_form():
    for months, i0 in [(360, 0.007), (120, 0.01), (1, 0.02)]:
        ck = O.mbs_annuity(months, i0)
        v = 1.0 / (1.0 + i0)
        for k in range(1, months + 1):
            want = (1.0 - v ** (months - k + 1)) / (1.0 - v)
            assert ck[k] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("months,sig", [(360, 0.02), (120, 0.03), (37, 0.2)])
def test_recursion_matches_closed_product_forms(months, sig):
    p = I.mbs_paper(months, sig)
    z = np.random.default_rng(7).standard_normal((64, months))
    pv = O.mbs_paths(p, z)
    # independent evaluation: i_k = K0^k exp(xi_1+..+xi_k) i0
    K0 = math.exp(-sig * sig / 2)
    k = np.arange(1, months + 1)
    xi = sig * z
    i_k = p.i0 * K0 ** k * np.exp(np.cumsum(xi, axis=1))                # i_1..i_K
    i_prev = np.concatenate([np.full((64, 1), p.i0), i_k[:, :-1]], axis=1)  # i_0..i_{K-1}
    u_k = np.cumprod(1.0 / (1.0 + i_prev), axis=1)                      # prod_{j=0}^{k-1}
    w_k = p.K1 + p.K2 * np.arctan(p.K3 * i_k + p.K4)
    r_k = np.concatenate([np.ones((64, 1)), np.cumprod(1.0 - w_k, axis=1)[:, :-1]], axis=1)
    v = 1.0 / (1.0 + p.i0)
    c_k = (1.0 - v ** (months - k + 1)) / (1.0 - v)
    c = p.i0 / (1.0 - (1.0 + p.i0) ** (-months))
    m_k = c * r_k * ((1.0 - w_k) + w_k * c_k)
    want = (u_k * m_k).sum(axis=1)
    assert np.allclose(pv, want, rtol=1e-12, atol=0)


def test_rqmc_agrees_with_pseudorandom_mc():
    c = I.cfg2()
    th = O.price_mbs(c.model, 1 << 12, 16, seed=2)
    rq, sd, se = O.finalize(th)
    rng = np.random.default_rng(123)
    n = 40000
    pv = O.mbs_paths(c.model, rng.standard_normal((n, 360)))
    mc, mc_se = pv.mean(), pv.std(ddof=1) / math.sqrt(n)
    assert abs(rq[0] - mc) <= 4 * math.hypot(se[0], mc_se)
    assert se[0] < mc_se          # RQMC beats MC at far fewer points


def test_theta_is_fsum_of_paths_and_finalize_stats():
    m = I.small_lmm(n_fwd=4, n_factors=2)
    N, M = 300, 5
    th, pp = O.price_caplets(m, N, M, seed=4, per_path=True)
    for r in range(M):
        for o in range(m.n_out):
            want = math.fsum(pp[r, :, o]) / N
            assert th[r, o] == pytest.approx(want, rel=1e-15, abs=1e-300)
    mean, sd, se = O.finalize(th)
    for o in range(m.n_out):
        col = list(th[:, o])
        assert mean[o] == pytest.approx(statistics.fmean(col), rel=1e-14)
        assert sd[o] == pytest.approx(statistics.stdev(col), rel=1e-12)
        assert se[o] == pytest.approx(statistics.stdev(col) / math.sqrt(M), rel=1e-12)


def test_single_replication_gives_nan_spread():
    th = O.price_mbs(I.mbs_paper(12), 64, 1, seed=1)
    mean, sd, se = O.finalize(th)
    assert math.isnan(sd[0]) and math.isnan(se[0]) and math.isfinite(mean[0])


def test_pricer_wires_points_to_normals_to_paths():
    # per-path output of the pricer == path function on Phi^{-1}(points),
    # dimension j = k*d + f time-major
    m = I.small_lmm(n_fwd=5, n_factors=2)
    N, M = 128, 3
    th, pp = O.price_caplets(m, N, M, seed=31, per_path=True)
    x, _ = O.sequence(m.s, N, M, seed=31)
    z = O.ppnd16(x.reshape(M * N, m.s))
    want = O.lmm_paths(m, z).reshape(M, N, m.n_out)
    assert np.array_equal(pp, want)
    p = I.mbs_paper(24)
    th, pp = O.price_mbs(p, N, M, seed=32, per_path=True)
    x, _ = O.sequence(24, N, M, seed=32)
    want = O.mbs_paths(p, O.ppnd16(x.reshape(M * N, 24))).reshape(M, N, 1)
    assert np.array_equal(pp, want)


def test_m_offset_split_bit_exact():
    m = I.small_lmm(n_fwd=3, n_factors=1)
    a = O.price_caplets(m, 256, 6, seed=9)
    b = np.concatenate([O.price_caplets(m, 256, 2, seed=9, m_offset=0),
                        O.price_caplets(m, 256, 4, seed=9, m_offset=2)])
    assert np.array_equal(a, b)


def test_rqmc_sd_decays_faster_than_mc():
    # the paper reports sd ~ N^-0.87 (CPU) / N^-0.86 (GPU) for caplets
    # against N^-0.5 for pseudo-random sequences; check the slope is well
    # below -0.5 on the 10-forward caplet.
    c = I.cfg1()
    sds = []
    Ns = [1 << 9, 1 << 11, 1 << 13]
    for N in Ns:
        th = O.price_caplets(c.model, N, 32, seed=1)
        sds.append(O.finalize(th)[1][-1])
    slope = np.polyfit(np.log(Ns), np.log(sds), 1)[0]
    assert slope < -0.6, slope
