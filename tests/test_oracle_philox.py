"""Pins of the oracle's pseudo-random generator (the paper's Philox
baseline): Philox4x64-10 from its publication (Salmon et al., SC'11) against
numpy's independent implementation, the uniform mapping, and the
sequence/pricer wiring of the MC flag."""
import numpy as np
import pytest

import oracle as O
import rqmc_inputs as I

MASK = (1 << 64) - 1


def _numpy_block(ctr, key):
    # numpy's Philox advances its 256-bit counter before each block
    c = sum(int(w) << (64 * t) for t, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    state = np.array([(c >> (64 * t)) & MASK for t in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=state, key=np.array(key, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (1, 2)),
    ((0, 1, 0, 0), (0, 0)),                       # the counter carries into word 1 in numpy
    ((7, 123456789, 0, 0), (0x9E3779B97F4A7C15, 42)),
    ((0xFFFFFFFFFFFFFFFF, 5, 9, 1), (MASK, MASK)),
    ((3, 2**40, 0, 0), (2024, 7)),
])
def test_philox_matches_numpy(ctr, key):
    assert O.philox4x64(ctr, key) == _numpy_block(ctr, key)


def test_mc_point_mapping_and_range():
    seed, mg = 99, 5
    for i in (0, 1, 17, 2**33):
        for j in range(9):
            w = O.philox4x64((j >> 2, i, 0, 0), (seed, mg))[j & 3]
            u = O.mc_point(seed, mg, i, j)
            assert u == ((w >> 11) + 0.5) * 2.0 ** -53
            assert 0.0 < u < 1.0


def test_mc_sequence_uniform_and_wired():
    x, R = O.sequence(6, 4000, 3, 7, flags=O.MC_PHILOX, m_offset=11)
    assert R is None
    assert x[2, 3999, 5] == O.mc_point(7, 13, 3999, 5)
    # chi-square on 20 bins over 72000 draws (df = 19; 0.999 quantile ~ 43.8)
    h, _ = np.histogram(x.ravel(), bins=20, range=(0.0, 1.0))
    e = x.size / 20
    assert ((h - e) ** 2 / e).sum() < 43.8
    # replications differ, and so do dimensions
    assert not np.array_equal(x[0], x[1])
    assert abs(np.corrcoef(x[0, :, 0], x[0, :, 1])[0, 1]) < 0.05


def test_mc_flag_rejects_halton_options():
    with pytest.raises(RuntimeError):
        O.sequence(3, 10, 1, 1, flags=O.MC_PHILOX | O.PERM_RANDOM)
    with pytest.raises(RuntimeError):
        O.sequence(3, 10, 1, 1, flags=O.MC_PHILOX | O.START_ZERO)


def test_mc_caplet_prices_agree_with_black_and_converge_like_mc():
    # the 10-forward flat caplet (Black 1.3698347565e-3, log-Euler bias far
    # below the MC noise here): MC estimate within 4 SE, and its spread falls
    # like N^-1/2 while the random-start Halton spread falls faster
    inst = I.cfg1()
    th = O.price_caplets(inst.model, 4096, 32, 3, flags=O.MC_PHILOX)[:, -1]
    m, sd = th.mean(), th.std(ddof=1)
    assert abs(m - 1.3698347565e-3) < 4 * sd / np.sqrt(len(th))
    s_mc = [O.price_caplets(inst.model, n, 32, 5, flags=O.MC_PHILOX)[:, -1].std(ddof=1) for n in (256, 4096)]
    s_q = [O.price_caplets(inst.model, n, 32, 5)[:, -1].std(ddof=1) for n in (256, 4096)]
    slope_mc = np.log(s_mc[1] / s_mc[0]) / np.log(16)
    slope_q = np.log(s_q[1] / s_q[0]) / np.log(16)
    assert -0.75 < slope_mc < -0.3
    assert slope_q < slope_mc - 0.15
