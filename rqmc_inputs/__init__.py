"""Seeded synthetic workloads shaped like the paper's two pricing problems.

This module only builds *inputs*: model parameters (tenor grid, initial
forward curve, volatility vector, factor loadings, strikes) and MBS
parameters, plus the seeded instrument list of the batching workload.  It
holds none of the method's arithmetic (no sequence, no normal map, no path
simulation, no estimator); both the CPU oracle and the GPU library consume
exactly the arrays returned here.

Sources for the shapes:
  * LIBOR market model caplets: Section "Pricing caplets in the LIBOR model"
    (tenor structure, forward rates, SDE under the spot measure, caplet
    payoff).  The paper prices a 1-factor constant-vol caplet; the larger
    workloads below keep its structure with 80 quarterly forwards and a
    3-factor PCA-reduced correlation.
  * The paper's own LIBOR test case: the daily Treasury yield curve of
    02/24/2012 (Table 3), interpolated by a cubic spline to 6-month points,
    turned into bond prices and into initial forwards by eq. (BL), with
    (t, T, delta, K, sigma) = (0, 5, 0.5, 0.01, 0.04).
  * Mortgage-backed security: Section "Pricing Mortgage-Backed Securities"
    with the paper's constants (i0, K1, K2, K3, K4, sigma^2) =
    (0.007, 0.01, -0.005, 10, 0.5, 0.0004).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

__all__ = [
    "LmmModel", "MbsParams", "Instrument",
    "lmm_flat", "lmm_curve80", "pca_loadings",
    "mbs_paper", "cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "small_lmm",
    "TREASURY_2012_02_24", "natural_cubic_spline", "treasury_bond_prices", "lmm_treasury_caplet",
    "cfg_paper_libor",
]


@dataclass
class LmmModel:
    """LIBOR market model inputs (spot measure, constant vols).

    n_fwd forwards L_1..L_nfwd over [T_n, T_n + delta], T_n = n*delta.
    L0[0..n_fwd]: initial forwards L_0(0)..L_nfwd(0); L_0(0) is the spot
    period's rate and only enters the numeraire.
    sigma[0..n_fwd]: scalar vol of each forward (sigma[0] unused).
    loadings[n_fwd][n_factors]: unit-norm factor loadings b_n; the vol
    vector of forward n is a_n = sigma_n * b_n.
    strike[n_fwd]: K_1..K_nfwd; NaN means no caplet on that forward.
    """
    n_fwd: int
    n_factors: int
    delta: float
    L0: np.ndarray
    sigma: np.ndarray
    loadings: np.ndarray
    strike: np.ndarray

    @property
    def s(self) -> int:
        return self.n_fwd * self.n_factors

    @property
    def n_out(self) -> int:
        return self.n_fwd + 1

    def copy(self) -> "LmmModel":
        return replace(self, L0=self.L0.copy(), sigma=self.sigma.copy(),
                       loadings=self.loadings.copy(), strike=self.strike.copy())


@dataclass
class MbsParams:
    """Caflisch MBS model inputs: mortgage of `months` months."""
    months: int
    i0: float
    sigma: float
    K1: float
    K2: float
    K3: float
    K4: float

    @property
    def s(self) -> int:
        return self.months

    @property
    def n_out(self) -> int:
        return 1


@dataclass
class Instrument:
    kind: str                      # "lmm" or "mbs"
    model: object                  # LmmModel or MbsParams
    N: int
    M: int
    seed: int


def lmm_flat(n_fwd: int, delta: float, L: float, vol: float, K: float,
             caplets: Optional[List[int]] = None) -> LmmModel:
    """One-factor flat-curve, flat-vol model; caplets on the listed forwards
    (1-based; default: only the last one)."""
    caplets = [n_fwd] if caplets is None else caplets
    strike = np.full(n_fwd, np.nan)
    for n in caplets:
        strike[n - 1] = K
    return LmmModel(n_fwd=n_fwd, n_factors=1, delta=delta,
                    L0=np.full(n_fwd + 1, L, dtype=np.float64),
                    sigma=np.full(n_fwd + 1, vol, dtype=np.float64),
                    loadings=np.ones((n_fwd, 1), dtype=np.float64),
                    strike=strike)


def pca_loadings(T: np.ndarray, beta: float, d: int) -> np.ndarray:
    """Unit-row loadings from the top-d principal components of
    rho_ij = exp(-beta |T_i - T_j|).  B = E_d Lambda_d^{1/2}, each row then
    rescaled to unit length so that forward n's total vol is exactly
    sigma_n.  Sign convention: first component of each eigenvector > 0."""
    T = np.asarray(T, dtype=np.float64)
    rho = np.exp(-beta * np.abs(T[:, None] - T[None, :]))
    w, E = np.linalg.eigh(rho)
    order = np.argsort(w)[::-1][:d]
    w, E = w[order], E[:, order].copy()
    for f in range(d):
        if E[0, f] < 0:
            E[:, f] = -E[:, f]
    B = E * np.sqrt(w)[None, :]
    B /= np.linalg.norm(B, axis=1)[:, None]
    return np.ascontiguousarray(B)


def lmm_curve80(n_fwd: int = 80, n_factors: int = 3, delta: float = 0.25,
                beta: float = 0.1) -> LmmModel:
    """The 80-forward workload: linear 4%->6% curve over 20y, humped vol
    sigma(T) = (0.1 + 0.5T)e^{-0.5T} + 0.1, exponential correlation with
    decay beta reduced to n_factors PCA factors, ATM caplets on every
    forward.  Truncating to n_fwd < 80 keeps the same curve and vol
    function on the shorter grid."""
    T = np.arange(n_fwd + 1, dtype=np.float64) * delta
    L0 = 0.04 + 0.02 * T / 20.0
    sigma = (0.1 + 0.5 * T) * np.exp(-0.5 * T) + 0.1
    sigma[0] = 0.0
    B = pca_loadings(T[1:], beta, n_factors)
    strike = L0[1:].copy()
    return LmmModel(n_fwd=n_fwd, n_factors=n_factors, delta=delta,
                    L0=L0, sigma=sigma, loadings=B, strike=strike)


def mbs_paper(months: int = 360, sigma: float = 0.02) -> MbsParams:
    """The paper's MBS constants; sigma is the standard deviation of the
    monthly log-rate shock (sigma^2 = 0.0004)."""
    return MbsParams(months=months, i0=0.007, sigma=sigma,
                     K1=0.01, K2=-0.005, K3=10.0, K4=0.5)


def lmm_stress(n_fwd: int = 12, n_factors: int = 2) -> LmmModel:
    """An extreme-regime model for robustness tests: semi-annual forwards
    from 1e-4 up to 15% (log-spaced), volatilities up to 120% with two zero
    volatilities, ATM caplets except on two forwards."""
    delta = 0.5
    T = np.arange(n_fwd + 1, dtype=np.float64) * delta
    L0 = 10.0 ** np.linspace(-4.0, math.log10(0.15), n_fwd + 1)
    sigma = 0.3 + 0.9 * np.abs(np.sin(1.7 * np.arange(n_fwd + 1)))
    sigma[0] = 0.0
    sigma[[3, 8]] = 0.0
    B = pca_loadings(T[1:], 0.3, n_factors)
    strike = L0[1:].copy()
    strike[[1, 6]] = np.nan
    return LmmModel(n_fwd=n_fwd, n_factors=n_factors, delta=delta, L0=L0, sigma=sigma,
                    loadings=B, strike=strike)


def small_lmm(n_fwd: int = 6, n_factors: int = 2, delta: float = 0.25) -> LmmModel:
    """A small multi-factor model on the 80-forward curve family, for tests."""
    return lmm_curve80(n_fwd=n_fwd, n_factors=n_factors, delta=delta)


def cfg1() -> Instrument:
    """1-factor LMM: 10 quarterly forwards, flat 5% curve, flat 20% vol,
    one caplet on L_10 struck at 5%; s = 10, N = 4096, M = 32."""
    return Instrument("lmm", lmm_flat(10, 0.25, 0.05, 0.2, 0.05), 4096, 32, 1)


def cfg2() -> Instrument:
    """MBS, 360 months, the paper's constants; s = 360, N = 2^14, M = 64."""
    return Instrument("mbs", mbs_paper(360), 1 << 14, 64, 2)


def cfg3() -> Instrument:
    """3-factor LMM, 80 quarterly forwards, 80 ATM caplets + book;
    s = 240, N = 2^16, M = 1024."""
    return Instrument("lmm", lmm_curve80(), 1 << 16, 1024, 3)


def cfg4() -> List[Instrument]:
    """Greeks workload: the 80-forward book and the 360-month MBS,
    N = 2^16, M = 256."""
    return [Instrument("lmm", lmm_curve80(), 1 << 16, 256, 4),
            Instrument("mbs", mbs_paper(360), 1 << 16, 256, 4)]


def cfg5(n_inst: int = 256, seed: int = 5) -> List[Instrument]:
    """256 heterogeneous instruments drawn from a seeded numpy Generator:
    half MBS (120/240/360 months, sigma ~ U[0.01, 0.03]), half LMM books
    (20..80 forwards, 1..3 factors, the 80-forward curve family truncated);
    N = 2^U{12..18}, M = 2^U{4..9}."""
    rng = np.random.default_rng(seed)
    out: List[Instrument] = []
    for k in range(n_inst):
        N = 1 << int(rng.integers(12, 19))
        M = 1 << int(rng.integers(4, 10))
        if rng.random() < 0.5:
            months = int(rng.choice([120, 240, 360]))
            sig = float(rng.uniform(0.01, 0.03))
            out.append(Instrument("mbs", mbs_paper(months, sig), N, M, 1000 + k))
        else:
            nf = int(rng.integers(20, 81))
            d = int(rng.integers(1, 4))
            out.append(Instrument("lmm", lmm_curve80(n_fwd=nf, n_factors=d), N, M, 1000 + k))
    return out


# ---------------------------------------------------------------------------
# The paper's LIBOR test case (section "Pricing caplets in the LIBOR model")
# ---------------------------------------------------------------------------
# Table 3: daily Treasury yield curve rates on 02/24/2012, percent, at
# maturities (years) 1/12, 1/4, 1/2, 1, 2, 3, 5, 7, 10, 20, 30.
TREASURY_2012_02_24 = (
    (1.0 / 12.0, 0.25, 0.5, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0, 20.0, 30.0),
    (0.08, 0.10, 0.14, 0.18, 0.31, 0.43, 0.89, 1.41, 1.98, 2.75, 3.10),
)


def natural_cubic_spline(x, y):
    """The natural cubic spline through (x_i, y_i) (second derivative 0 at
    both ends), returned as a function of t (array-like, inside [x_0, x_n]).
    The second derivatives m_i solve the tridiagonal system
    h_{i-1} m_{i-1} + 2 (h_{i-1} + h_i) m_i + h_i m_{i+1}
        = 6 ((y_{i+1} - y_i)/h_i - (y_i - y_{i-1})/h_{i-1}),  m_0 = m_n = 0."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x) - 1
    h = np.diff(x)
    A = np.zeros((n + 1, n + 1))
    r = np.zeros(n + 1)
    A[0, 0] = A[n, n] = 1.0
    for i in range(1, n):
        A[i, i - 1] = h[i - 1]
        A[i, i] = 2.0 * (h[i - 1] + h[i])
        A[i, i + 1] = h[i]
        r[i] = 6.0 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1])
    m = np.linalg.solve(A, r)

    def f(t):
        t = np.asarray(t, dtype=np.float64)
        i = np.clip(np.searchsorted(x, t, side="right") - 1, 0, n - 1)
        a, b = x[i + 1] - t, t - x[i]
        hi = h[i]
        return (m[i] * a ** 3 + m[i + 1] * b ** 3) / (6.0 * hi) \
            + (y[i] / hi - m[i] * hi / 6.0) * a + (y[i + 1] / hi - m[i + 1] * hi / 6.0) * b

    return f


def treasury_bond_prices(T):
    """Zero-coupon bond prices B(0, T) from the Table 3 curve: the spline's
    yield y(T) (percent) read as a semi-annually compounded rate,
    B = (1 + y/200)^(-2T); B(0, 0) = 1."""
    T = np.asarray(T, dtype=np.float64)
    xs, ys = TREASURY_2012_02_24
    y = natural_cubic_spline(xs, ys)(np.maximum(T, xs[0])) / 100.0
    return np.where(T > 0, (1.0 + y / 2.0) ** (-2.0 * T), 1.0)


def lmm_treasury_caplet(T: float = 5.0, delta: float = 0.5, K: float = 0.01, vol: float = 0.04) -> LmmModel:
    """The paper's caplet: one factor, constant vol, forwards on the 6-month
    grid initialised from the Treasury bond prices by eq. (BL),
    L_n(0) = (B_n - B_{n+1}) / (delta B_{n+1}), and one caplet on the period
    [T, T + delta] (forward n = T/delta) struck at K."""
    nf = int(round(T / delta))
    grid = np.arange(nf + 2, dtype=np.float64) * delta
    B = treasury_bond_prices(grid)
    L0 = (B[:-1] - B[1:]) / (delta * B[1:])
    strike = np.full(nf, np.nan)
    strike[nf - 1] = K
    return LmmModel(n_fwd=nf, n_factors=1, delta=delta, L0=L0,
                    sigma=np.full(nf + 1, vol, dtype=np.float64),
                    loadings=np.ones((nf, 1), dtype=np.float64), strike=strike)


def cfg_paper_libor(N: int = 1 << 16, M: int = 100, seed: int = 6) -> Instrument:
    """The paper's LIBOR case (Table 3 curve, caplet on [5, 5.5], K = 1%,
    sigma = 4%) with M = 100 replications as in the paper; s = 10."""
    return Instrument("lmm", lmm_treasury_caplet(), N, M, seed)
