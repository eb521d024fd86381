"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars:
  * sequence points and digit integers: bit-exact;
  * FP64 pricing, every path:  |gpu - oracle| <= 1e-12 (|oracle| + scale_o)
    with scale_o = delta*K_n for the caplet on L_n (the payoff's natural
    size; it absorbs the kink where L_n ~ K_n), the sum of those for the
    book, and 1 for the MBS PV;  estimates theta, RQ to the same bar, sd/SE
    to 1e-9 relative (they difference nearly equal numbers);
  * FP32 form: estimates theta and RQ within 1e-6 relative of the oracle
    at N >= 4096.
Shapes span several blocks with ragged tails; the full-size workloads are
checked on sampled replications the oracle computes one by one.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import paper_1408_5526_amd as rq
import rqmc_inputs as I

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _scales_lmm(model):
    s = model.delta * np.nan_to_num(np.asarray(model.strike, dtype=np.float64), nan=0.0)
    return np.append(s, s.sum())


# ---------------------------------------------------------------------------
# sequence
# ---------------------------------------------------------------------------
SEQ = [
    (10, 4096, 32, 1, 0),
    (37, 1000, 3, 7, 0),
    (37, 1000, 3, 7, rq.PERM_RANDOM),
    (12, 300, 2, 5, rq.START_ZERO),
    (12, 300, 2, 5, rq.START_ZERO | rq.PERM_RANDOM),
    (360, 700, 2, 2, 0),
    (1, 1, 1, 3, 0),
    (37, 1000, 3, 7, rq.MC_PHILOX),
    (37, 1000, 3, 7, rq.PERM_PER_REP),
    (12, 300, 4, 5, rq.PERM_PER_REP | rq.START_ZERO),
]


@pytest.mark.parametrize("s,N,M,seed,flags", SEQ)
def test_sequence_bit_exact(s, N, M, seed, flags):
    _say("sequence", s, N, M, seed, flags)
    xg = _np(rq.sequence(s, N, M, seed, flags))
    xo, Ro = O.sequence(s, N, M, seed, flags)
    if not flags & rq.MC_PHILOX:   # pseudo-random points have no digit form
        Rg = _np(rq.sequence(s, N, M, seed, flags | rq.OUT_DIGITS)).astype(np.uint64)
        assert np.array_equal(Rg, Ro)
    assert np.array_equal(xg.view(np.uint64), xo.view(np.uint64))


def test_sequence_m_offset_and_rerun():
    _say("sequence m_offset")
    a = _np(rq.sequence(9, 513, 5, 11))
    b = np.concatenate([_np(rq.sequence(9, 513, 2, 11, m_offset=0)),
                        _np(rq.sequence(9, 513, 3, 11, m_offset=2))])
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    c = _np(rq.sequence(9, 513, 5, 11))
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))


def test_sequence_many_segments_sampled():
    # s = 4096 bases (largest prime 38873) forces segments of 2^15 indices:
    # N = 70000 spans three segments; sampled elements against the oracle's
    # definition-based radical inverse, including the segment seams.
    s, N, M, seed = 4096, 70000, 1, 23
    _say("sequence segments", s, N)
    import torch
    R = rq.sequence(s, N, M, seed, rq.OUT_DIGITS)
    rng = np.random.default_rng(0)
    dims = np.unique(np.concatenate([rng.integers(0, s, 40), [0, 1, 7, 2048, 3512, 4000, 4095]]))
    ii = np.concatenate([rng.integers(0, N, 2000), [0, 1, 32767, 32768, 32769, 65535, 65536, N - 1]])
    jj = dims[rng.integers(0, len(dims), len(ii))]
    got = R[0, torch.as_tensor(ii, device=R.device), torch.as_tensor(jj, device=R.device)]
    got = _np(got).astype(np.uint64)
    starts = {}
    for j in dims:
        p = O.nth_prime(int(j))
        D, P = O.digits(p)
        starts[int(j)] = (p, P, O.start(seed, 0, int(j)))
    for i, j, g in zip(ii, jj, got):
        p, P, n = starts[int(j)]
        assert int(g) == O.radinv_R(p, (n + int(i)) % P), (i, j)
    del R


# ---------------------------------------------------------------------------
# inverse normal
# ---------------------------------------------------------------------------
def _inv_normal_points():
    rng = np.random.default_rng(3)
    return np.concatenate([rng.random(200000), 10.0 ** rng.uniform(-19, -1, 20000),
                           1 - 10.0 ** rng.uniform(-16, -1, 20000),
                           [0.0, 2.0 ** -64, 2.0 ** -70, 0.5, 0.0017, 0.00169, 0.9983, 0.075, 0.925]])


def test_inv_normal_fp64_matches_oracle():
    import torch
    _say("inv_normal fp64")
    u = _inv_normal_points()
    z = _np(rq.inv_normal(torch.as_tensor(u, device="cuda")))
    zo = O.ppnd16(u)
    assert np.allclose(z, zo, rtol=2e-15, atol=1e-300)


def test_inv_normal_fp32_error_bound():
    import torch
    _say("inv_normal fp32")
    u = _inv_normal_points()
    z = _np(rq.inv_normal(torch.as_tensor(u, device="cuda"), "fp32")).astype(np.float64)
    zo = O.ppnd16(u)
    err = np.abs(z - zo) / np.maximum(np.abs(zo), 1e-3)
    _say("fp32 inverse normal max rel err", float(err.max()))
    assert err.max() < 5e-7


# ---------------------------------------------------------------------------
# LIBOR market model
# ---------------------------------------------------------------------------
def _one_fwd():
    return I.LmmModel(n_fwd=1, n_factors=1, delta=0.5, L0=np.array([0.05, 0.055]),
                      sigma=np.array([0.0, 0.3]), loadings=np.ones((1, 1)), strike=np.array([0.05]))


LMM = [
    ("cfg1", lambda: I.cfg1().model, 4096, 32, 1, 0),
    ("nf6d2-ragged", lambda: I.small_lmm(6, 2), 1000, 3, 17, 0),
    ("nf20d3", lambda: I.lmm_curve80(20, 3), 513, 2, 5, 0),
    ("nf80d3", lambda: I.lmm_curve80(), 300, 2, 3, 0),
    ("nf71d2", lambda: I.lmm_curve80(71, 2), 300, 2, 6, 0),      # capacity 80, top group partly empty
    ("nf33d1-perm", lambda: I.lmm_curve80(33, 1), 257, 2, 9, rq.PERM_RANDOM),
    ("nf48d2-zero", lambda: I.lmm_curve80(48, 2), 256, 1, 4, rq.START_ZERO),
    ("nf1", _one_fwd, 100, 2, 3, 0),
    ("nf64d3-n1", lambda: I.lmm_curve80(64, 3), 1, 1, 8, 0),
    ("nf20d3-mc", lambda: I.lmm_curve80(20, 3), 513, 2, 5, rq.MC_PHILOX),
    ("nf80d3-mc", lambda: I.lmm_curve80(), 300, 2, 3, rq.MC_PHILOX),
    ("nf20d3-permrep", lambda: I.lmm_curve80(20, 3), 513, 3, 5, rq.PERM_PER_REP),
    ("stress", I.lmm_stress, 700, 2, 21, 0),      # rates 1e-4..15%, vols to 120% and 0
]


@pytest.mark.parametrize("name,mk,N,M,seed,flags", LMM, ids=[c[0] for c in LMM])
def test_caplets_fp64_per_path(name, mk, N, M, seed, flags):
    model = mk()
    _say("caplets fp64", name, N, M, seed, flags)
    r = rq.price_caplets(model, N, M, seed, flags=flags, precision="fp64", per_path=True)
    th_o, pp_o = O.price_caplets(model, N, M, seed, flags=flags, per_path=True)
    sc = _scales_lmm(model)
    pp_g = _np(r.per_path)
    err = np.abs(pp_g - pp_o) - 1e-12 * (np.abs(pp_o) + sc)
    assert (err <= 0).all(), float(err.max())
    th_g = _np(r.theta)
    assert (np.abs(th_g - th_o) <= 1e-12 * (np.abs(th_o) + sc)).all()
    mo, so, eo = O.finalize(th_o)
    assert np.allclose(_np(r.mean), mo, rtol=1e-12, atol=1e-12 * sc.max())
    if M > 1:
        assert np.allclose(_np(r.sd), so, rtol=1e-9, atol=1e-13 * sc.max())
        assert np.allclose(_np(r.se), eo, rtol=1e-9, atol=1e-13 * sc.max())
    else:
        assert np.isnan(_np(r.sd)).all() and np.isnan(_np(r.se)).all()


# FP32 estimates are checked at N >= 4096 (ragged tails kept): each path's
# FP32 state rounds to a few 1e-7 relative, so at a few hundred paths the
# noise in theta alone approaches 1e-6; it falls like 1/sqrt(N).
LMM32 = [
    ("cfg1", lambda: I.cfg1().model, 4096, 32, 1, 0),
    ("nf6d2-ragged", lambda: I.small_lmm(6, 2), 4133, 3, 17, 0),
    ("nf20d3", lambda: I.lmm_curve80(20, 3), 4200, 2, 5, 0),
    ("nf80d3", lambda: I.lmm_curve80(), 4133, 2, 3, 0),
    # capacity 80 below its top: the FP32 form keeps the 24 lowest forwards'
    # states in LDS there, with Halton and with Philox points
    ("nf71d2", lambda: I.lmm_curve80(71, 2), 4133, 2, 6, 0),
    ("nf67d3-mc", lambda: I.lmm_curve80(67, 3), 4133, 2, 7, rq.MC_PHILOX),
    ("nf33d1-perm", lambda: I.lmm_curve80(33, 1), 4097, 2, 9, rq.PERM_RANDOM),
    ("nf20d3-mc", lambda: I.lmm_curve80(20, 3), 4200, 2, 5, rq.MC_PHILOX),
    ("nf33d1-permrep", lambda: I.lmm_curve80(33, 1), 4097, 3, 9, rq.PERM_PER_REP),
    ("stress", I.lmm_stress, 4133, 2, 21, 0),
]


@pytest.mark.parametrize("name,mk,N,M,seed,flags", LMM32, ids=[c[0] for c in LMM32])
def test_caplets_fp32_estimates(name, mk, N, M, seed, flags):
    model = mk()
    _say("caplets fp32", name, N, M, seed, flags)
    r = rq.price_caplets(model, N, M, seed, flags=flags, precision="fp32")
    th_o = O.price_caplets(model, N, M, seed, flags=flags)
    th_g = _np(r.theta)
    live = np.abs(th_o) > 0
    rel = np.abs(th_g - th_o)[live] / np.abs(th_o)[live]
    _say("fp32 max rel err on theta", float(rel.max()))
    assert rel.max() <= 1e-6
    mo = th_o.mean(axis=0)
    lm = np.abs(mo) > 0
    assert (np.abs(_np(r.mean) - mo)[lm] <= 1e-6 * np.abs(mo)[lm]).all()


def test_caplets_deterministic_and_m_offset():
    model = I.small_lmm(7, 3)
    _say("caplets determinism")
    a = rq.price_caplets(model, 700, 4, 13)
    b = rq.price_caplets(model, 700, 4, 13)
    assert np.array_equal(_np(a.theta).view(np.uint64), _np(b.theta).view(np.uint64))
    c1 = rq.price_caplets(model, 700, 1, 13, m_offset=0)
    c2 = rq.price_caplets(model, 700, 3, 13, m_offset=1)
    cat = np.concatenate([_np(c1.theta), _np(c2.theta)])
    assert np.array_equal(_np(a.theta).view(np.uint64), cat.view(np.uint64))


def test_caplets_full_size_sampled_replications():
    # the 80-forward book at N = 2^16, M = 1024 (the benchmark launch); the
    # oracle recomputes three replications one by one
    c = I.cfg3()
    _say("caplets full size", c.N, c.M)
    r64 = rq.price_caplets(c.model, c.N, c.M, c.seed, precision="fp64")
    r32 = rq.price_caplets(c.model, c.N, c.M, c.seed, precision="fp32")
    th64, th32 = _np(r64.theta), _np(r32.theta)
    sc = _scales_lmm(c.model)
    for m in (0, 517, 1023):
        th_o = O.price_caplets(c.model, c.N, 1, c.seed, m_offset=m)[0]
        assert (np.abs(th64[m] - th_o) <= 1e-12 * (np.abs(th_o) + sc)).all(), m
        rel = np.abs(th32[m] - th_o) / np.abs(th_o)
        _say("full fp32 replication", m, "max rel", float(rel.max()))
        assert rel.max() <= 1e-6
    # equal standard error: same points, both forms
    se64, se32 = _np(r64.se)[-1], _np(r32.se)[-1]
    assert abs(se32 / se64 - 1) < 0.01


# ---------------------------------------------------------------------------
# MBS
# ---------------------------------------------------------------------------
MBS = [
    ("cfg2-small", lambda: I.mbs_paper(360), 1000, 3, 2, 0),
    ("m120-perm", lambda: I.mbs_paper(120, 0.03), 513, 2, 4, rq.PERM_RANDOM),
    ("m1", lambda: I.mbs_paper(1), 64, 2, 5, 0),
    ("m240-zero", lambda: I.mbs_paper(240, 0.01), 300, 1, 6, rq.START_ZERO),
    ("m360-mc", lambda: I.mbs_paper(360), 700, 2, 8, rq.MC_PHILOX),
    ("m120-permrep", lambda: I.mbs_paper(120), 600, 3, 8, rq.PERM_PER_REP),
]


@pytest.mark.parametrize("name,mk,N,M,seed,flags", MBS, ids=[c[0] for c in MBS])
def test_mbs_fp64_per_path_and_fp32(name, mk, N, M, seed, flags):
    p = mk()
    _say("mbs", name, N, M, seed, flags)
    r = rq.price_mbs(p, N, M, seed, flags=flags, precision="fp64", per_path=True)
    th_o, pp_o = O.price_mbs(p, N, M, seed, flags=flags, per_path=True)
    assert (np.abs(_np(r.per_path) - pp_o) <= 1e-12 * (np.abs(pp_o) + 1)).all()
    assert (np.abs(_np(r.theta) - th_o) <= 1e-12 * (np.abs(th_o) + 1)).all()
    r32 = rq.price_mbs(p, N, M, seed, flags=flags, precision="fp32")
    rel = np.abs(_np(r32.theta) - th_o) / np.abs(th_o)
    _say("mbs fp32 max rel", float(rel.max()))
    assert rel.max() <= 1e-6


def test_mbs_zero_vol_is_par():
    p = I.mbs_paper(360, 0.0)
    r = rq.price_mbs(p, 512, 2, 1)
    assert np.allclose(_np(r.theta), 1.0, atol=1e-13, rtol=0)


def test_mbs_full_size():
    c = I.cfg2()
    _say("mbs full size", c.N, c.M)
    r = rq.price_mbs(c.model, c.N, c.M, c.seed)
    th_o = O.price_mbs(c.model, c.N, c.M, c.seed)
    assert (np.abs(_np(r.theta) - th_o) <= 1e-12 * (np.abs(th_o) + 1)).all()
    r32 = rq.price_mbs(c.model, c.N, c.M, c.seed, precision="fp32")
    assert (np.abs(_np(r32.theta) - th_o) <= 1e-6 * np.abs(th_o)).all()


# ---------------------------------------------------------------------------
# plain Euler scheme (the paper's discretisation) on the paper's own caplet
# ---------------------------------------------------------------------------
EULER = [
    ("paper-caplet", lambda: I.lmm_treasury_caplet(), 1000, 3, 6, rq.LMM_EULER),
    ("paper-caplet-mc", lambda: I.lmm_treasury_caplet(), 777, 2, 6, rq.LMM_EULER | rq.MC_PHILOX),
    ("nf80d3", lambda: I.lmm_curve80(), 300, 2, 3, rq.LMM_EULER),
    ("nf33d2", lambda: I.lmm_curve80(33, 2), 513, 2, 4, rq.LMM_EULER),
]


@pytest.mark.parametrize("name,mk,N,M,seed,flags", EULER, ids=[c[0] for c in EULER])
def test_caplets_euler_fp64_per_path_and_fp32(name, mk, N, M, seed, flags):
    model = mk()
    _say("caplets euler", name, N, M, seed, flags)
    r = rq.price_caplets(model, N, M, seed, flags=flags, precision="fp64", per_path=True)
    th_o, pp_o = O.price_caplets(model, N, M, seed, flags=flags, per_path=True)
    sc = _scales_lmm(model)
    err = np.abs(_np(r.per_path) - pp_o) - 1e-12 * (np.abs(pp_o) + sc)
    assert (err <= 0).all(), float(err.max())
    assert (np.abs(_np(r.theta) - th_o) <= 1e-12 * (np.abs(th_o) + sc)).all()


def test_caplets_euler_fp32_estimates():
    model = I.lmm_treasury_caplet()
    for flags in (rq.LMM_EULER, rq.LMM_EULER | rq.MC_PHILOX):
        r = rq.price_caplets(model, 4133, 3, 6, flags=flags, precision="fp32")
        th_o = O.price_caplets(model, 4133, 3, 6, flags=flags)
        live = np.abs(th_o) > 0
        rel = np.abs(_np(r.theta) - th_o)[live] / np.abs(th_o)[live]
        _say("euler fp32 max rel", flags, float(rel.max()))
        assert rel.max() <= 1e-6


def test_per_replication_permutations_m_offset_and_large_bases():
    # the replication key is m_global: an m_offset split reproduces the
    # whole; s = 600 reaches bases above 4096 (the counter stride)
    _say("perm per rep m_offset")
    a = _np(rq.sequence(600, 300, 3, 17, rq.PERM_PER_REP | rq.OUT_DIGITS))
    b = np.concatenate([_np(rq.sequence(600, 300, 1, 17, rq.PERM_PER_REP | rq.OUT_DIGITS, m_offset=0)),
                        _np(rq.sequence(600, 300, 2, 17, rq.PERM_PER_REP | rq.OUT_DIGITS, m_offset=1))])
    assert np.array_equal(a, b)
    xo, Ro = O.sequence(600, 300, 3, 17, O.PERM_PER_REP)
    assert np.array_equal(a.astype(np.uint64), Ro)
