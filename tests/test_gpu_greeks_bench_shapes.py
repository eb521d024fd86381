"""GPU parity of the adjoint Greeks at the capacities the benchmark runs
(the 64- and 80-forward instantiations of the forward and reverse adjoint
kernels), and the adjoint's estimates against Black's caplet Greeks.

Finite-difference references are theta-level central differences of the
oracle with common random numbers (the same seed, hence the same points):
for strike 0 the payoffs are smooth and the difference is exact to O(h^2),
so the FP64 adjoint must agree to 1e-7 and the FP32 adjoint to 1e-4
(relative to the largest Greek).  At-the-money strikes put a kink in every
payoff; a 1e-8 relative bump keeps kink crossings out of the difference
(their noise falls like sqrt(h)) and the bar is 2e-3.

Black's Greeks (caplet section; closed forms in tests/black_caplet.py,
pinned there against differences of Black's price) hold for the
continuous-time model.  The log-Euler scheme differs by a bias of order
delta, estimated from the oracle by the common-random-number Richardson
difference b = 2 (G_delta - G_delta/2) of the same central differences on
pseudo-random normals.  Every Greek's RQMC estimate must lie within
3 sqrt(SE^2 + SE_b^2) of Black + b.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1408_5526_amd as rq
import rqmc_inputs as I
from black_caplet import black_book_greeks, crn_bias_greeks
from test_gpu_greeks import fd_caplet_greeks

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


# (name, n_fwd, n_factors, N, M, seed): 80 and 64 forwards fill their
# capacities; 70, 57 and 49 leave the top groups of 80 and 64 partly empty
# (ragged last block too: N not a multiple of 64)
FULL = [("nf80d3", 80, 3, 256, 2, 31), ("nf64d3", 64, 3, 200, 2, 32),
        ("nf70d3", 70, 3, 192, 1, 36),
        ("nf57d3", 57, 3, 130, 1, 33), ("nf49d2", 49, 2, 256, 1, 34)]


@pytest.mark.parametrize("name,nf,d,N,M,seed", FULL, ids=[c[0] for c in FULL])
def test_adjoint_at_benchmark_capacity_matches_oracle_fd(name, nf, d, N, M, seed):
    model = I.lmm_curve80(nf, d)
    model.strike = np.zeros(nf)                 # smooth payoffs
    _say("adjoint capacity", name, N, M, seed)
    th_o, pp_o = O.price_caplets(model, N, M, seed, per_path=True)
    fd = fd_caplet_greeks(model, N, M, seed, h_rel=1e-5)
    scale = np.abs(fd).max(axis=1, keepdims=True)
    sc = model.delta * 0.06 * (nf + 1)
    r64 = rq.price_caplets(model, N, M, seed, precision="fp64", greeks=True, per_path=True)
    # the with-Greeks forward pass's prices: the FP64 per-path bar
    assert (np.abs(_np(r64.per_path) - pp_o) <= 1e-12 * (np.abs(pp_o) + sc)).all()
    err64 = np.abs(_np(r64.greeks.theta) - fd) / scale
    _say("fp64 adjoint vs FD max rel", float(err64.max()))
    assert err64.max() < 1e-7
    r32 = rq.price_caplets(model, N, M, seed, precision="fp32", greeks=True)
    err32 = np.abs(_np(r32.greeks.theta) - fd) / scale
    _say("fp32 adjoint vs FD max rel", float(err32.max()))
    assert err32.max() < 1e-4
    # FP32 prices of the with-Greeks call against the oracle's theta
    rel = np.abs(_np(r32.theta) - th_o)[:, -1] / np.abs(th_o[:, -1])
    assert rel.max() < 1e-5


ATM = [("nf8d2", lambda: I.small_lmm(8, 2), 4096, 2, 11), ("nf80d3", lambda: I.lmm_curve80(80, 3), 256, 2, 35)]


@pytest.mark.parametrize("name,mk,N,M,seed", ATM, ids=[c[0] for c in ATM])
def test_fp32_adjoint_at_the_money_matches_oracle_fd(name, mk, N, M, seed):
    model = mk()                                # ATM strikes: every payoff has a kink
    _say("fp32 adjoint atm", name, N, M, seed)
    fd = fd_caplet_greeks(model, N, M, seed, h_rel=1e-8)
    scale = np.abs(fd).max(axis=1, keepdims=True)
    g32 = _np(rq.price_caplets(model, N, M, seed, precision="fp32", greeks=True).greeks.theta)
    err = np.abs(g32 - fd) / scale
    _say("atm fp32 adjoint vs FD max rel", float(err.max()))
    assert err.max() < 2e-3


BLACK = [("cfg1", lambda: I.cfg1().model, 4096, 32, 1), ("nf6d2", lambda: I.small_lmm(6, 2), 1 << 13, 32, 17)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,mk,N,M,seed", BLACK, ids=[c[0] for c in BLACK])
def test_adjoint_greeks_match_black_within_se_plus_bias(name, mk, N, M, seed, precision):
    model = mk()
    _say("black greeks", name, precision, N, M, seed)
    r = rq.price_caplets(model, N, M, seed, precision=precision, greeks=True)
    g, se = _np(r.greeks.mean), _np(r.greeks.se)
    b, se_b = crn_bias_greeks(model, 100_000, seed=3)
    blk = black_book_greeks(model)
    # FP32: the adjoint's own rounding (its bar against the FP64 differences,
    # 1e-4 of the largest Greek) is added to the statistical bound
    tol = 1e-4 * np.abs(blk).max() if precision == "fp32" else 0.0
    dev = np.abs(g - blk - b)
    bound = 3.0 * np.sqrt(se ** 2 + se_b ** 2) + tol
    _say("black worst dev/bound", float((dev / bound).max()))
    assert (dev <= bound).all(), (dev / bound)


def test_adjoint_full_size_sampled_replications_match_oracle_fd():
    # The benchmark's launch: the 80-forward, 3-factor book with Greeks at
    # N = 2^16, M = 1024 (FP32: two chunks of tasks; FP64: three).  On two
    # sampled replications, seven sampled Greeks (deltas of forwards 1, 40
    # and 80, the spot delta, vegas of forwards 1, 40 and 80) against the
    # oracle's central differences of that replication alone (m_offset), the
    # bumped pricings run side by side (the oracle releases the GIL).  ATM
    # strikes: the kink-aware bump and bar of the at-the-money tests above.
    from concurrent.futures import ThreadPoolExecutor
    c = I.cfg3()
    model, N, M, seed = c.model, c.N, c.M, c.seed
    nf = model.n_fwd
    _say("adjoint full size", N, M)
    g32 = _np(rq.price_caplets(model, N, M, seed, precision="fp32", greeks=True).greeks.theta)
    g64 = _np(rq.price_caplets(model, N, M, seed, precision="fp64", greeks=True).greeks.theta)
    cols = {"dL1": (0, "L0", 1), "dL40": (39, "L0", 40), "dL80": (79, "L0", 80), "dL0": (nf, "L0", 0),
            "ds1": (nf + 1, "sigma", 1), "ds40": (nf + 40, "sigma", 40), "ds80": (nf + 80, "sigma", 80)}
    reps = (5, 871)

    def bumped(m, field, n, sgn):
        mm = model.copy()
        arr = getattr(mm, field)
        h = 1e-8 * (arr[n] if field == "L0" else max(arr[n], 0.01))
        arr[n] += sgn * h
        return O.price_caplets(mm, N, 1, seed, m_offset=m)[0, -1], h

    jobs = [(m, k, sgn) for m in reps for k in cols for sgn in (1, -1)]
    with ThreadPoolExecutor(max_workers=16) as ex:
        res = list(ex.map(lambda j: bumped(j[0], cols[j[1]][1], cols[j[1]][2], j[2]), jobs))
    val = {(m, k, sgn): r for (m, k, sgn), r in zip(jobs, res)}
    for m in reps:
        fd = {k: (val[(m, k, 1)][0] - val[(m, k, -1)][0]) / (2 * val[(m, k, 1)][1]) for k in cols}
        scale = max(abs(v) for v in fd.values())
        for k, (col, _, _) in cols.items():
            e32 = abs(g32[m, col] - fd[k]) / scale
            e64 = abs(g64[m, col] - fd[k]) / scale
            _say("full size", m, k, "fd", fd[k], "fp32 err", e32, "fp64 err", e64)
            assert e64 < 2e-3 and e32 < 2e-3, (m, k)
