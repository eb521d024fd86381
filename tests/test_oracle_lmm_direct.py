"""Per-path pins of the oracle's multi-forward LIBOR paths (CPU only).

The oracle's forward-step keeps a running sum v over the forwards it has
already visited in the step.  Here the same discretised SDE (caplet
section: spot measure, drift mu_n(t) = sum_{j=eta(t)}^{n} delta L_j a_n.a_j
/ (1 + delta L_j), log-Euler step of length delta from T_k with eta = k+1
and the drift taken from the values at T_k) is written a second way: the
drift of every forward as the paper's direct double sum over the step's
pre-step values, evaluated in 40-digit mpmath.  Fixed normals drive both;
each path's discounted payoffs must agree to FP64 rounding.  A variant that
takes the drift from already-updated forwards (the plausible slip: post-step
L_j for j < n) must NOT agree -- that is what makes the pin sharp.

The tiny-N check wires everything: the oracle's own points (pinned
elsewhere) mapped to normals by mpmath's erfinv, paths by the direct sum,
theta_N^m by math.fsum, against the oracle's theta.

The Black Greeks used by the GPU check are pinned here against central
differences of Black's price.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import rqmc_inputs as I
from black_caplet import black_book_greeks, black_caplets, crn_bias_greeks

mp.mp.dps = 40


def random_model(nf, d, seed):
    """Forwards 1%..8%, vols 5%..60% (one forward at 0.8%), random unit
    loading rows, strikes around the forwards (ITM and OTM) and one forward
    without a caplet."""
    rng = np.random.default_rng(seed)
    L0 = rng.uniform(0.01, 0.08, nf + 1)
    sigma = rng.uniform(0.05, 0.6, nf + 1)
    sigma[0] = 0.0
    sigma[1 + nf // 2] = 0.008
    b = rng.standard_normal((nf, d))
    b /= np.linalg.norm(b, axis=1)[:, None]
    K = L0[1:] * rng.uniform(0.7, 1.3, nf)
    K[nf - 2] = np.nan
    return I.LmmModel(n_fwd=nf, n_factors=d, delta=0.25 if seed % 2 else 0.5, L0=L0, sigma=sigma,
                      loadings=b, strike=K)


def direct_path(model, z, post_step=False):
    """Discounted caplet payoffs and book of one path, the drift as the
    direct sum over pre-step forwards (post_step=True: the slip)."""
    nf, d = model.n_fwd, model.n_factors
    dl = mp.mpf(model.delta)
    sqd = mp.sqrt(dl)
    a = [[mp.mpf(0)] * d] + [[mp.mpf(model.sigma[n]) * mp.mpf(model.loadings[n - 1][f]) for f in range(d)]
                             for n in range(1, nf + 1)]
    dot = lambda u, v: mp.fsum(x * y for x, y in zip(u, v))
    L = [mp.mpf(x) for x in model.L0]
    num = 1 + dl * L[0]
    pay = []
    for k in range(nf):
        Z = [mp.mpf(x) for x in z[k * d:(k + 1) * d]]
        pre = list(L)
        for n in range(k + 1, nf + 1):
            src = L if post_step else pre
            mu = mp.fsum(dl * src[j] * dot(a[n], a[j]) / (1 + dl * src[j]) for j in range(k + 1, n + 1))
            L[n] = pre[n] * mp.exp((mu - dot(a[n], a[n]) / 2) * dl + sqd * dot(a[n], Z))
        n = k + 1
        K = model.strike[n - 1]
        p = mp.mpf(0)
        if not math.isnan(K):
            p = dl * max(L[n] - mp.mpf(K), 0) / (num * (1 + dl * L[n]))
        pay.append(p)
        num *= 1 + dl * L[n]
    pay.append(mp.fsum(pay))
    return pay


SHAPES = [(3, 2, 1), (4, 3, 2), (5, 2, 3), (6, 3, 4), (6, 2, 5)]


@pytest.mark.parametrize("strikes", ["mixed", "zero"])
@pytest.mark.parametrize("nf,d,seed", SHAPES, ids=[f"nf{s[0]}d{s[1]}" for s in SHAPES])
def test_multiforward_paths_equal_direct_drift_sum(nf, d, seed, strikes):
    # zero strikes: every payoff is delta L_n(T_n) / numeraire, so every
    # forward's fixing value is compared on every path
    m = random_model(nf, d, seed)
    if strikes == "zero":
        m.strike = np.where(np.isnan(m.strike), np.nan, 0.0)
    rng = np.random.default_rng(100 + seed)
    z = rng.standard_normal((6, nf * d))
    z[0, :] = 3.5                       # a far-up and a far-down path
    z[1, :] = -3.5
    got = O.lmm_paths(m, z)
    scale = m.delta * np.nanmax(m.L0)   # size of an at-the-money payoff
    worst = 0.0
    for row, zz in zip(got, z):
        want = np.array([float(v) for v in direct_path(m, zz)])
        err = np.abs(row - want) / (np.abs(want) + scale)
        worst = max(worst, err.max())
    assert worst <= 1e-14, worst


@pytest.mark.parametrize("nf,d,seed", SHAPES[1:4], ids=[f"nf{s[0]}d{s[1]}" for s in SHAPES[1:4]])
def test_post_step_drift_slip_is_detected(nf, d, seed):
    # taking g_j from forwards already stepped changes the scheme by O(delta):
    # the pin above would see it on every path (zero strikes: no payoff is
    # cut off by its strike)
    m = random_model(nf, d, seed)
    m.strike = np.where(np.isnan(m.strike), np.nan, 0.0)
    z = np.random.default_rng(200 + seed).standard_normal((3, nf * d))
    got = O.lmm_paths(m, z)
    scale = m.delta * np.nanmax(m.L0)
    for row, zz in zip(got, z):
        slip = np.array([float(v) for v in direct_path(m, zz, post_step=True)])
        assert (np.abs(row - slip) / (np.abs(slip) + scale)).max() > 1e-9


def _phi_inv(x):
    """Inverse normal CDF from mpmath's erfinv (independent of AS241), with
    the oracle's clamp of the fold min(x, 1-x) at 2^-64."""
    x = mp.mpf(x)
    r = min(x, 1 - x)
    if r < mp.mpf(2) ** -64:
        x = mp.mpf(2) ** -64 if x < mp.mpf(0.5) else 1 - mp.mpf(2) ** -64
    return mp.sqrt(2) * mp.erfinv(2 * x - 1)


@pytest.mark.parametrize("nf,d,seed", [(4, 3, 7), (6, 2, 8)])
def test_tiny_n_theta_is_brute_force(nf, d, seed):
    m = random_model(nf, d, seed)
    N, M = 8, 2
    x, _ = O.sequence(nf * d, N, M, seed)
    th = O.price_caplets(m, N, M, seed)
    scale = m.delta * np.nanmax(m.L0)
    for r in range(M):
        rows = [direct_path(m, [_phi_inv(v) for v in x[r, i]]) for i in range(N)]
        want = np.array([float(mp.fsum(row[o] for row in rows) / N) for o in range(nf + 1)])
        assert (np.abs(th[r] - want) / (np.abs(want) + scale)).max() <= 1e-14


@pytest.mark.parametrize("mk", [lambda: I.cfg1().model, lambda: I.small_lmm(6, 2),
                                lambda: random_model(5, 3, 9)], ids=["cfg1", "nf6d2", "random5"])
def test_black_greek_formulas_are_derivatives_of_black_price(mk):
    m = mk()
    g = black_book_greeks(m)
    nf = m.n_fwd
    fd = np.zeros_like(g)
    for n in range(nf + 1):
        h = 1e-6 * m.L0[n]
        up, dn = m.copy(), m.copy()
        up.L0[n] += h
        dn.L0[n] -= h
        fd[nf if n == 0 else n - 1] = (black_caplets(up).sum() - black_caplets(dn).sum()) / (2 * h)
    for n in range(1, nf + 1):
        h = 1e-6 * m.sigma[n]
        up, dn = m.copy(), m.copy()
        up.sigma[n] += h
        dn.sigma[n] -= h
        fd[nf + n] = (black_caplets(up).sum() - black_caplets(dn).sum()) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())


def _fd_book_greeks(model, N, M, seed, h_rel):
    """theta-level central differences of the oracle's book (same points),
    layout [dL_1..dL_n, dL_0, dsigma_1..dsigma_n] per replication."""
    nf = model.n_fwd
    out = np.zeros((M, 2 * nf + 1))
    for n in range(nf + 1):
        h = h_rel * model.L0[n]
        up, dn = model.copy(), model.copy()
        up.L0[n] += h
        dn.L0[n] -= h
        out[:, nf if n == 0 else n - 1] = (O.price_caplets(up, N, M, seed)[:, -1] -
                                           O.price_caplets(dn, N, M, seed)[:, -1]) / (2 * h)
    for n in range(1, nf + 1):
        h = h_rel * model.sigma[n]
        up, dn = model.copy(), model.copy()
        up.sigma[n] += h
        dn.sigma[n] -= h
        out[:, nf + n] = (O.price_caplets(up, N, M, seed)[:, -1] -
                          O.price_caplets(dn, N, M, seed)[:, -1]) / (2 * h)
    return out


@pytest.mark.parametrize("mk,N,M,seed", [(lambda: I.cfg1().model, 4096, 32, 1),
                                         (lambda: I.small_lmm(6, 2), 1 << 13, 32, 17)],
                         ids=["cfg1", "nf6d2"])
def test_oracle_fd_greeks_match_black_within_se_plus_bias(mk, N, M, seed):
    # the finite-difference Greeks the GPU adjoint is compared with, checked
    # against Black's Greeks plus the scheme's Richardson bias estimate
    m = mk()
    rqv, sd, se = O.finalize(_fd_book_greeks(m, N, M, seed, 1e-6))
    b, se_b = crn_bias_greeks(m, 100_000, seed=3)
    z = (rqv - black_book_greeks(m) - b) / np.sqrt(se ** 2 + se_b ** 2)
    assert (np.abs(z) <= 3.0).all(), z
