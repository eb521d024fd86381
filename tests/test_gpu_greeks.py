"""GPU parity of the pathwise Greeks (adjoint kernel for the LIBOR book,
forward tangent for the MBS) against central finite differences of the
oracle with common random numbers (same seed, hence the same points).

Smooth payoffs (strike 0 for caplets; the MBS PV is smooth in i0) make the
central difference exact to O(h^2), so the bar is tight there.  For
at-the-money caplets a bumped path may cross the payoff kink; such paths
make the difference deviate from the pathwise derivative by noise that
shrinks like sqrt(h), so those cases use a small bump and a looser bar.
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


def fd_caplet_greeks(model, N, M, seed, h_rel, flags=0):
    """theta-level central differences of the book, GPU Greek layout:
    [dL_1..dL_n, dL_0, dsigma_1..dsigma_n], shape [M][2n+1]."""
    nf = model.n_fwd
    out = np.zeros((M, 2 * nf + 1))

    def book(mm):
        return O.price_caplets(mm, N, M, seed, flags=flags)[:, -1]

    for n in range(nf + 1):
        h = h_rel * model.L0[n]
        up, dn = model.copy(), model.copy()
        up.L0[n] += h
        dn.L0[n] -= h
        col = nf if n == 0 else n - 1
        out[:, col] = (book(up) - book(dn)) / (2 * h)
    for n in range(1, nf + 1):
        h = h_rel * max(model.sigma[n], 0.01)
        up, dn = model.copy(), model.copy()
        up.sigma[n] += h
        dn.sigma[n] -= h
        out[:, nf + n] = (book(up) - book(dn)) / (2 * h)
    return out


SMOOTH = [
    ("nf6d2", lambda: I.small_lmm(6, 2), 512, 2, 7),
    ("nf20d3", lambda: I.lmm_curve80(20, 3), 300, 2, 9),
    ("nf33d1", lambda: I.lmm_curve80(33, 1), 256, 1, 4),
    ("nf12d2-mc", lambda: I.lmm_curve80(12, 2), 300, 2, 6, rq.MC_PHILOX),
    ("nf12d2-permrep", lambda: I.lmm_curve80(12, 2), 300, 2, 6, rq.PERM_PER_REP),
    # edge shapes of the grouped sweeps: one forward; two forwards, two
    # factors; one past a capacity boundary (17 -> 32); a ragged last block.
    # The FP32 sweep runs steps in pairs after a lone first step when n_fwd
    # is odd: 3, 4 and 5 forwards put the pairs' last group at every offset
    ("nf1d1", lambda: I.lmm_curve80(1, 1), 200, 2, 11),
    ("nf2d2", lambda: I.lmm_curve80(2, 2), 130, 2, 12),
    ("nf3d3", lambda: I.lmm_curve80(3, 3), 200, 2, 14),
    ("nf4d1", lambda: I.lmm_curve80(4, 1), 150, 2, 15),
    ("nf5d2", lambda: I.lmm_curve80(5, 2), 180, 2, 16),
    ("nf17d3", lambda: I.lmm_curve80(17, 3), 333, 2, 13),
    # rates 1e-4..15%, vols to 120%, two zero vols (carried as 2^-60)
    ("stress", I.lmm_stress, 300, 2, 22),
]


@pytest.mark.parametrize("name,mk,N,M,seed,flags", [c if len(c) == 6 else c + (0,) for c in SMOOTH],
                         ids=[c[0] for c in SMOOTH])
def test_caplet_adjoint_smooth_payoff_matches_fd(name, mk, N, M, seed, flags):
    model = mk()
    model.strike = np.zeros(model.n_fwd)          # no kink: delta*L_n(T_n)/numeraire
    _say("adjoint smooth", name, N, M, seed, flags)
    r64 = rq.price_caplets(model, N, M, seed, flags=flags, precision="fp64", greeks=True, per_path=True)
    th_o, pp_o = O.price_caplets(model, N, M, seed, flags=flags, per_path=True)
    sc = model.delta * 0.06
    # prices from the adjoint kernel's forward pass: same per-path bar
    assert (np.abs(_np(r64.per_path) - pp_o) <= 1e-12 * (np.abs(pp_o) + sc * (model.n_fwd + 1))).all()
    fd = fd_caplet_greeks(model, N, M, seed, h_rel=1e-5, flags=flags)
    g64 = _np(r64.greeks.theta)
    scale = np.abs(fd).max(axis=1, keepdims=True)
    err64 = np.abs(g64 - fd) / scale
    _say("fp64 adjoint vs FD max rel", float(err64.max()))
    assert err64.max() < 1e-7
    r32 = rq.price_caplets(model, N, M, seed, flags=flags, precision="fp32", greeks=True)
    err32 = np.abs(_np(r32.greeks.theta) - fd) / scale
    _say("fp32 adjoint vs FD max rel", float(err32.max()))
    assert err32.max() < 1e-4


def test_caplet_adjoint_atm_book_against_fd():
    model = I.small_lmm(8, 2)                      # ATM strikes: kinks present
    N, M, seed = 4096, 2, 11
    _say("adjoint atm", N, M)
    g = _np(rq.price_caplets(model, N, M, seed, precision="fp64", greeks=True).greeks.theta)
    fd = fd_caplet_greeks(model, N, M, seed, h_rel=1e-8)
    scale = np.abs(fd).max(axis=1, keepdims=True)
    err = np.abs(g - fd) / scale
    _say("atm fp64 adjoint vs FD max rel", float(err.max()))
    assert err.max() < 2e-3


def test_caplet_adjoint_spot_delta_is_book_scaling():
    # every payoff carries 1/(1 + delta L_0(0)): dbook/dL_0(0) = -delta book / num0
    model = I.small_lmm(5, 2)
    r = rq.price_caplets(model, 1000, 2, 3, precision="fp64", greeks=True)
    book = _np(r.theta)[:, -1]
    want = -model.delta * book / (1 + model.delta * model.L0[0])
    assert np.allclose(_np(r.greeks.theta)[:, model.n_fwd], want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-7), ("fp32", 1e-4)])
def test_caplet_adjoint_zero_vol_closed_form(precision, rtol):
    # sigma = 0: L stays at L(0); delta of an ITM caplet is delta B_{n+1}(0)
    # minus the numeraire terms, and vega is 0 only in the limit -- compare to FD
    model = I.small_lmm(4, 1)
    model.sigma[:] = 0.0
    model.strike = model.L0[1:] - 0.002
    N, M, seed = 128, 1, 5
    g = _np(rq.price_caplets(model, N, M, seed, precision=precision, greeks=True).greeks.theta)[0]
    fd = fd_caplet_greeks(model, N, M, seed, h_rel=1e-5)[0]
    assert np.allclose(g, fd, rtol=rtol, atol=rtol * 1e-3 * np.abs(fd).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_caplet_adjoint_chunks_do_not_change_results(precision):
    # 3 replications x 16 blocks = 48 tasks; a store limit of 7 FP64 tasks
    # gives 7 chunks in FP64 (6 of 7 tasks, the last of 6) and 4 in FP32 (12
    # each): prices and Greeks bit-identical to the single-chunk call
    m = I.lmm_curve80(20, 3)
    _say("adjoint chunks", precision)
    ref = rq.price_caplets(m, 1000, 3, 7, flags=rq.PERM_RANDOM, precision=precision, greeks=True)
    try:
        rq.set_adjoint_store_limit(7 * (20 * 3 + 32) * 64 * 8)
        got = rq.price_caplets(m, 1000, 3, 7, flags=rq.PERM_RANDOM, precision=precision, greeks=True)
    finally:
        rq.set_adjoint_store_limit(0)
    for a, b in ((got.theta, ref.theta), (got.greeks.theta, ref.greeks.theta)):
        assert np.array_equal(_np(a).view(np.uint64), _np(b).view(np.uint64))


def test_caplet_adjoint_full_size_greeks_run():
    # the 80-forward book with Greeks, FP32, at N = 2^16, M = 256 (two chunks
    # of 131,072 tasks): finite, and the sampled replication matches the FP64
    # adjoint of that replication alone
    c = I.cfg4()[0]
    _say("adjoint full", c.N, c.M)
    r = rq.price_caplets(c.model, c.N, c.M, c.seed, precision="fp32", greeks=True)
    g = _np(r.greeks.theta)
    assert np.isfinite(g).all()
    r2 = rq.price_caplets(c.model, c.N, 1, c.seed, m_offset=100, precision="fp64", greeks=True)
    g64 = _np(r2.greeks.theta)[0]
    rel = np.abs(g[100] - g64) / np.abs(g64).max()
    _say("full fp32 vs fp64 adjoint max rel", float(rel.max()))
    assert rel.max() < 1e-4


MBS = [("m360", lambda: I.mbs_paper(360), 512, 2, 2), ("m120", lambda: I.mbs_paper(120, 0.03), 300, 2, 3),
       ("m12-sig0", lambda: I.mbs_paper(12, 0.0), 64, 1, 4)]


@pytest.mark.parametrize("name,mk,N,M,seed", MBS, ids=[c[0] for c in MBS])
def test_mbs_tangent_matches_fd(name, mk, N, M, seed):
    from dataclasses import replace
    p = mk()
    _say("mbs tangent", name)
    r = rq.price_mbs(p, N, M, seed, precision="fp64", greeks=True, per_path=True)
    th_o, pp_o = O.price_mbs(p, N, M, seed, per_path=True)
    assert (np.abs(_np(r.per_path) - pp_o) <= 1e-12 * (np.abs(pp_o) + 1)).all()
    h = 1e-4 * p.i0          # smooth in i0: O(h^2) ~ 1e-9; smaller h only adds rounding
    up = O.price_mbs(replace(p, i0=p.i0 + h), N, M, seed)
    dn = O.price_mbs(replace(p, i0=p.i0 - h), N, M, seed)
    fd = (up - dn) / (2 * h)
    g = _np(r.greeks.theta)
    if p.sigma == 0.0:
        assert np.abs(g).max() < 1e-9          # PV = 1 for every i0
        return
    assert np.allclose(g, fd, rtol=1e-6, atol=0)
    g32 = _np(rq.price_mbs(p, N, M, seed, precision="fp32", greeks=True).greeks.theta)
    assert np.allclose(g32, fd, rtol=1e-4, atol=0)


def test_autograd_functions():
    import torch
    model = I.small_lmm(5, 2)
    L0 = torch.tensor(model.L0, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(model.sigma, dtype=torch.float64, requires_grad=True)
    v = rq.CapletBook.apply(L0, sig, model, 1024, 4, 21, "fp64")
    v.backward()
    r = rq.CapletBook.last
    gm = _np(r.greeks.mean)
    assert abs(float(v) - float(_np(r.mean)[-1])) == 0.0
    assert np.allclose(L0.grad.numpy()[1:], gm[:5]) and L0.grad.numpy()[0] == gm[5]
    assert np.allclose(sig.grad.numpy()[1:], gm[6:]) and sig.grad.numpy()[0] == 0.0
    i0 = torch.tensor(0.007, dtype=torch.float64, requires_grad=True)
    pv = rq.MBSPrice.apply(i0, I.mbs_paper(60), 512, 2, 5, "fp64")
    pv.backward()
    assert i0.grad.item() == float(_np(rq.MBSPrice.last.greeks.mean)[0])


def test_mbs_tangent_full_size_sampled_replications():
    # the Greeks workload's MBS pool (360 months, N = 2^16, M = 256, the
    # launch the benchmark's Greeks configuration makes): dPV/di0 of three
    # sampled replications against the oracle's central difference of each
    # replication alone (m_offset), in both precisions
    from dataclasses import replace
    c = [x for x in I.cfg4() if x.kind == "mbs"][0]
    p, N, M, seed = c.model, c.N, c.M, c.seed
    _say("mbs tangent full size", N, M)
    g64 = _np(rq.price_mbs(p, N, M, seed, precision="fp64", greeks=True).greeks.theta)
    g32 = _np(rq.price_mbs(p, N, M, seed, precision="fp32", greeks=True).greeks.theta)
    h = 1e-4 * p.i0
    for m in (0, 131, 255):
        up = O.price_mbs(replace(p, i0=p.i0 + h), N, 1, seed, m_offset=m)[0, 0]
        dn = O.price_mbs(replace(p, i0=p.i0 - h), N, 1, seed, m_offset=m)[0, 0]
        fd = (up - dn) / (2 * h)
        _say("mbs full size", m, "fd", fd, "fp64", g64[m, 0], "fp32", g32[m, 0])
        assert abs(g64[m, 0] - fd) <= 1e-6 * abs(fd)
        assert abs(g32[m, 0] - fd) <= 1e-4 * abs(fd)
