"""GPU checks of the batch entry point (one persistent launch over many
instruments, work taken from an atomic queue).

Bars:
  * FP64 estimates of every instrument against the oracle on the same seeded
    inputs, to the single-instrument bar |gpu - o| <= 1e-12 (|o| + scale);
  * FP32 estimates within 1e-6 relative of the oracle at N >= 4096;
  * with Greeks, every instrument's estimates and Greeks equal those of the
    single-instrument entry point (same per-path code, block sums in the
    same or a different fixed order) to 1e-13 relative;
  * results are bit-identical for every launch shape (chunk, blocks per CU,
    instrument order, windows of the two-phase Greeks form), since each work
    item writes its own partial row;
  * timestamps bracket every instrument's work.
"""
import dataclasses
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


@dataclasses.dataclass
class Ins:
    kind: str
    model: object
    N: int
    M: int
    seed: int
    m_offset: int = 0
    flags: int = 0


def _mixed():
    return [
        Ins("lmm", I.small_lmm(6, 2), 1000, 3, 17),
        Ins("mbs", I.mbs_paper(60), 700, 2, 6),
        Ins("lmm", I.lmm_curve80(20, 3), 513, 2, 5, flags=rq.PERM_RANDOM),
        Ins("lmm", I.cfg1().model, 300, 4, 1),
        Ins("mbs", I.mbs_paper(120, 0.03), 257, 3, 4, m_offset=5, flags=rq.PERM_RANDOM),
        Ins("lmm", I.lmm_curve80(80, 3), 130, 2, 3, m_offset=7),
        Ins("lmm", I.lmm_curve80(33, 1), 64, 1, 9, flags=rq.START_ZERO),
        Ins("mbs", I.mbs_paper(1), 1, 1, 2),
        Ins("lmm", I.lmm_curve80(24, 2), 200, 2, 12, flags=rq.MC_PHILOX),
        Ins("mbs", I.mbs_paper(120), 150, 2, 13, flags=rq.MC_PHILOX),
        Ins("lmm", I.lmm_curve80(1, 1), 70, 2, 14),
        Ins("lmm", I.lmm_curve80(17, 3), 129, 1, 15, m_offset=3),
    ]


def _oracle(ins):
    if ins.kind == "lmm":
        return O.price_caplets(ins.model, ins.N, ins.M, ins.seed, m_offset=ins.m_offset, flags=ins.flags)
    return O.price_mbs(ins.model, ins.N, ins.M, ins.seed, m_offset=ins.m_offset, flags=ins.flags)


def _scale(ins):
    if ins.kind == "lmm":
        s = ins.model.delta * np.nan_to_num(np.asarray(ins.model.strike, dtype=np.float64), nan=0.0)
        return np.append(s, s.sum())
    return np.ones(1)


def test_batch_fp64_matches_oracle_per_instrument():
    batch = _mixed()
    _say("batch fp64", len(batch))
    br = rq.price_batch(batch, precision="fp64")
    for k, ins in enumerate(batch):
        th_o = _oracle(ins)
        th_g = _np(br.results[k].theta)
        sc = _scale(ins)
        assert (np.abs(th_g - th_o) <= 1e-12 * (np.abs(th_o) + sc)).all(), k
        mo, so, eo = O.finalize(th_o)
        assert np.allclose(_np(br.results[k].mean), mo, rtol=1e-12, atol=1e-12 * sc.max()), k
        if ins.M > 1:
            assert np.allclose(_np(br.results[k].sd), so, rtol=1e-9, atol=1e-13 * sc.max()), k
        else:
            assert np.isnan(_np(br.results[k].sd)).all()


def test_batch_fp32_matches_oracle():
    batch = [Ins("lmm", I.lmm_curve80(20, 3), 4200, 2, 5), Ins("mbs", I.mbs_paper(120), 4097, 2, 4),
             Ins("lmm", I.small_lmm(6, 2), 4133, 3, 17, flags=rq.PERM_RANDOM)]
    _say("batch fp32")
    br = rq.price_batch(batch, precision="fp32")
    for k, ins in enumerate(batch):
        th_o = _oracle(ins)
        live = np.abs(th_o) > 0
        rel = np.abs(_np(br.results[k].theta) - th_o)[live] / np.abs(th_o)[live]
        _say("batch fp32 instrument", k, "max rel", float(rel.max()))
        assert rel.max() <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_greeks_equal_single_calls(precision):
    batch = _mixed()
    _say("batch greeks", precision)
    br = rq.price_batch(batch, precision=precision, greeks=True)
    for k, ins in enumerate(batch):
        if ins.kind == "lmm":
            r = rq.price_caplets(ins.model, ins.N, ins.M, ins.seed, m_offset=ins.m_offset, flags=ins.flags,
                                 precision=precision, greeks=True)
        else:
            r = rq.price_mbs(ins.model, ins.N, ins.M, ins.seed, m_offset=ins.m_offset, flags=ins.flags,
                             precision=precision, greeks=True)
        for a, b in ((br.results[k].theta, r.theta), (br.results[k].greeks.theta, r.greeks.theta)):
            a, b = _np(a), _np(b)
            scale = np.abs(b).max(axis=1, keepdims=True) + 1e-300
            assert (np.abs(a - b) <= 1e-13 * scale).all(), (k, float((np.abs(a - b) / scale).max()))


def test_batch_invariant_to_launch_shape():
    batch = _mixed()
    _say("batch launch shapes")
    ref = rq.price_batch(batch, precision="fp32", greeks=True, tuning=(1, 0, rq.ORDER_COST))
    for tu in ((4, 2, rq.ORDER_GIVEN), (8, 1, rq.ORDER_COST), (2, 3, rq.ORDER_GIVEN)):
        got = rq.price_batch(batch, precision="fp32", greeks=True, tuning=tu)
        for k in range(len(batch)):
            for a, b in ((got.results[k].theta, ref.results[k].theta),
                         (got.results[k].greeks.theta, ref.results[k].greeks.theta),
                         (got.results[k].se, ref.results[k].se)):
                assert np.array_equal(_np(a).view(np.uint64), _np(b).view(np.uint64)), (tu, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_windows_do_not_change_results(precision):
    # with Greeks the items run in windows (forward phase, then reverse
    # phase); a store limit of 5 FP64 item slots makes many small windows,
    # one of them ragged: prices and Greeks bit-identical to one window
    batch = _mixed()
    _say("batch windows", precision)
    ref = rq.price_batch(batch, precision=precision, greeks=True)
    try:
        rq.set_adjoint_store_limit(5 * (80 * 3 + 80) * 64 * 8)
        got = rq.price_batch(batch, precision=precision, greeks=True, tuning=(2, 1, rq.ORDER_GIVEN))
    finally:
        rq.set_adjoint_store_limit(0)
    for k in range(len(batch)):
        for a, b in ((got.results[k].theta, ref.results[k].theta),
                     (got.results[k].greeks.theta, ref.results[k].greeks.theta)):
            assert np.array_equal(_np(a).view(np.uint64), _np(b).view(np.uint64)), k


def test_batch_timestamps_bracket_every_instrument():
    batch = _mixed()
    br = rq.price_batch(batch, precision="fp32", timestamps=True)
    tf, tl = _np(br.t_first).view(np.uint64), _np(br.t_last).view(np.uint64)
    assert (tf != np.uint64(0xFFFFFFFFFFFFFFFF)).all() and (tl > 0).all()
    assert (tf <= tl).all()
    hz = rq.realtime_hz()
    span_s = float((tl.max() - tf.min())) / hz
    _say("batch span s", span_s, "counter Hz", hz)
    assert 0 < span_s < 60


def test_autotune_picks_a_candidate_and_keeps_results():
    batch = _mixed()
    _say("autotune")
    assert rq.batch_tuning(batch, precision="fp32", greeks=True) == ((0, 0, 0), False)
    (chunk, per_cu, order), ms = rq.autotune_batch(batch, precision="fp32", greeks=True)
    # (0, 0): the automatic shape, which is among the candidates
    assert (chunk, per_cu) == (0, 0) or (chunk in (1, 2, 4, 8, 16) and per_cu >= 1)
    assert order in (rq.ORDER_COST, rq.ORDER_GIVEN) and ms > 0
    # kept for this list's signature: price_batch without a tuning uses it
    assert rq.batch_tuning(batch, precision="fp32", greeks=True) == ((chunk, per_cu, order), True)
    assert rq.batch_tuning(batch, precision="fp64", greeks=True)[1] is False
    a = rq.price_batch(batch, precision="fp32", greeks=True, tuning=(chunk, per_cu, order))
    b = rq.price_batch(batch, precision="fp32", greeks=True)
    c = rq.price_batch(batch, precision="fp32", greeks=True, tuning=(1, 1, rq.ORDER_GIVEN))
    for k in range(len(batch)):
        assert np.array_equal(_np(a.results[k].theta), _np(b.results[k].theta))
        assert np.array_equal(_np(a.results[k].theta), _np(c.results[k].theta))


def test_batch_of_the_256_instrument_workload_scaled_down():
    # the seeded 256-instrument list with N capped at 2^10 and M at 4 (the
    # shapes otherwise unchanged): every result finite, sampled instruments
    # equal to their single calls
    full = I.cfg5()
    batch = [Ins(c.kind, c.model, min(c.N, 1 << 10), min(c.M, 4), c.seed) for c in full]
    _say("cfg5 scaled", len(batch))
    br = rq.price_batch(batch, precision="fp32", greeks=True)
    for k in range(len(batch)):
        assert np.isfinite(_np(br.results[k].theta)).all() and np.isfinite(_np(br.results[k].greeks.theta)).all()
    for k in (0, 1, 77, 128, 255):
        ins = batch[k]
        f = rq.price_caplets if ins.kind == "lmm" else rq.price_mbs
        r = f(ins.model, ins.N, ins.M, ins.seed, precision="fp32", greeks=True)
        assert np.allclose(_np(br.results[k].theta), _np(r.theta), rtol=1e-13, atol=0), k
        assert np.allclose(_np(br.results[k].greeks.theta), _np(r.greeks.theta), rtol=1e-13,
                           atol=1e-13 * np.abs(_np(r.greeks.theta)).max()), k


def test_batch_rejects_bad_instrument_before_launch():
    bad = I.small_lmm(4, 2)
    bad.L0 = bad.L0.copy()
    bad.L0[2] = -1.0
    batch = [Ins("mbs", I.mbs_paper(12), 64, 1, 1), Ins("lmm", bad, 64, 1, 1)]
    with pytest.raises(rq.RqError, match="instrument 1"):
        rq.price_batch(batch)


# As-drawn instruments of the 256-instrument workload, among them the
# largest shapes it draws (N = 2^18 with M = 512): a 55-forward 2-factor
# book, a 360-month pool, a 45-forward 3-factor book and a 240-month pool
DRAWN = (131, 216, 188, 6)
# sampled replications (m_global) compared with the oracle, which prices
# one replication at the full N
SAMPLED = {131: (511,), 216: (300,), 188: (0, 255, 511), 6: (0, 511)}


def _drawn():
    full = I.cfg5()
    return [Ins(full[k].kind, full[k].model, full[k].N, full[k].M, full[k].seed) for k in DRAWN]


def _oracle_rows(ins, ms):
    f = O.price_caplets if ins.kind == "lmm" else O.price_mbs
    return {m: f(ins.model, ins.N, 1, ins.seed, m_offset=m)[0] for m in ms}


def test_batch_as_drawn_matches_oracle_on_sampled_replications():
    batch = _drawn()
    _say("cfg5 as drawn", [(b.kind, b.N, b.M) for b in batch])
    b64 = rq.price_batch(batch, precision="fp64")
    b32 = rq.price_batch(batch, precision="fp32", greeks=True)
    for k, ins in zip(DRAWN, batch):
        rows = _oracle_rows(ins, SAMPLED[k])
        th64, th32 = _np(b64.results[DRAWN.index(k)].theta), _np(b32.results[DRAWN.index(k)].theta)
        assert np.isfinite(th32).all() and np.isfinite(_np(b32.results[DRAWN.index(k)].greeks.theta)).all()
        sc = _scale(ins)
        for m, want in rows.items():
            assert (np.abs(th64[m] - want) <= 1e-12 * (np.abs(want) + sc)).all(), (k, m)
            live = np.abs(want) > 0
            rel = np.abs(th32[m] - want)[live] / np.abs(want)[live]
            _say("drawn", k, "m", m, "fp32 max rel", float(rel.max()))
            assert rel.max() <= 1e-6, (k, m)


def test_batch_as_drawn_greeks_equal_single_calls():
    batch = _drawn()
    _say("cfg5 as drawn greeks")
    br = rq.price_batch(batch, precision="fp32", greeks=True)
    for j, ins in enumerate(batch):
        f = rq.price_caplets if ins.kind == "lmm" else rq.price_mbs
        r = f(ins.model, ins.N, ins.M, ins.seed, precision="fp32", greeks=True)
        for a, b in ((br.results[j].theta, r.theta), (br.results[j].greeks.theta, r.greeks.theta)):
            a, b = _np(a), _np(b)
            scale = np.abs(b).max(axis=1, keepdims=True) + 1e-300
            assert (np.abs(a - b) <= 1e-13 * scale).all(), (DRAWN[j], float((np.abs(a - b) / scale).max()))
