"""Black's caplet formula and the Greeks of a caplet book (test helper).

In the LIBOR market model with constant volatility each forward is
lognormal under its own forward measure, so caplet n (fixing at T_n = n
delta, paying delta (L_n(T_n) - K_n)^+ at T_{n+1}) is worth Black's price
(caplet section):
    C_n = delta B_{n+1}(0) [L_n(0) Phi(d1) - K_n Phi(d2)],
    d1,2 = (ln(L_n(0)/K_n) +- sigma_n^2 T_n / 2) / (sigma_n sqrt(T_n)),
    B_{n+1}(0) = prod_{j=0..n} 1 / (1 + delta L_j(0)).
Its Greeks with the strikes held fixed follow by differentiation:
    dC_n/dL_n(0)   = delta B_{n+1}(0) Phi(d1)  (the d1, d2 terms cancel),
    dC_n/dL_i(0)   = -delta / (1 + delta L_i(0)) C_n  for i <= n (discount),
    dC_n/dsigma_n  = delta B_{n+1}(0) L_n(0) phi(d1) sqrt(T_n).
These are test-side closed forms; tests/test_oracle_lmm_direct.py pins them
against central differences of the price.
"""
import math

import numpy as np
from scipy.stats import norm

import oracle as O


def black_caplets(model):
    """C_n for n = 1..n_fwd (0 where the strike is NaN)."""
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


def black_book_greeks(model):
    """Greeks of the book sum_n C_n in the library's layout:
    [dL_1(0)..dL_n(0), dL_0(0), dsigma_1..dsigma_n]."""
    d, nf = model.delta, model.n_fwd
    C = black_caplets(model)
    tail = np.cumsum(C[::-1])[::-1]          # tail[i-1] = sum_{n >= i} C_n
    out = np.zeros(2 * nf + 1)
    B = 1.0 / (1.0 + d * model.L0[0])
    out[nf] = -d / (1.0 + d * model.L0[0]) * C.sum()
    for n in range(1, nf + 1):
        B /= 1.0 + d * model.L0[n]
        disc = -d / (1.0 + d * model.L0[n]) * tail[n - 1]
        K = model.strike[n - 1]
        if np.isnan(K):
            out[n - 1] = disc
            continue
        L, s, T = model.L0[n], model.sigma[n], n * d
        d1 = (math.log(L / K) + 0.5 * s * s * T) / (s * math.sqrt(T))
        out[n - 1] = d * B * norm.cdf(d1) + disc
        out[nf + n] = d * B * L * norm.pdf(d1) * math.sqrt(T)
    return out


def crn_bias_greeks(model, n_paths, seed, h_rel=1e-5):
    """Richardson estimate of the scheme's bias in each book Greek:
    b = 2 (G_delta - G_delta/2), G by central differences of the oracle's
    paths on shared pseudo-random normals (the coarse normal of a period is
    (z_a + z_b)/sqrt 2 of its two halves).  Returns (b, SE of b)."""
    rng = np.random.default_rng(seed)
    nf, d = model.n_fwd, model.n_factors
    zf = rng.standard_normal((n_paths, nf, 2, d))
    zc = ((zf[:, :, 0, :] + zf[:, :, 1, :]) / math.sqrt(2.0)).reshape(n_paths, -1)
    zf = zf.reshape(n_paths, -1)

    def diff(mm):
        return 2.0 * (O.lmm_paths(mm, zc, n_sub=1)[:, -1] - O.lmm_paths(mm, zf, n_sub=2)[:, -1])

    mean, se = np.zeros(2 * nf + 1), np.zeros(2 * nf + 1)

    def put(col, up, dn, h):
        v = (diff(up) - diff(dn)) / (2 * h)
        mean[col], se[col] = v.mean(), v.std(ddof=1) / math.sqrt(n_paths)

    for n in range(nf + 1):
        h = h_rel * model.L0[n]
        up, dn = model.copy(), model.copy()
        up.L0[n] += h
        dn.L0[n] -= h
        put(nf if n == 0 else n - 1, up, dn, h)
    for n in range(1, nf + 1):
        h = h_rel * max(model.sigma[n], 0.01)
        up, dn = model.copy(), model.copy()
        up.sigma[n] += h
        dn.sigma[n] -= h
        put(nf + n, up, dn, h)
    return mean, se
