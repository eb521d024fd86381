"""Pins of the per-replication reading of "random permutations" (each
replication draws its own digit permutation of every base): validity,
Fisher-Yates uniformity, the wiring into the points, stratification, and
the estimator against the Black price."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import rqmc_inputs as I


def test_permutations_are_valid_and_differ_between_replications():
    for j in (0, 3, 40, 239):
        p = O.nth_prime(j)
        a, b = O.perm_rep(9, 0, j), O.perm_rep(9, 1, j)
        assert sorted(a) == list(range(p)) and sorted(b) == list(range(p))
        if p >= 5:
            assert not np.array_equal(a, b)
        # the per-replication stream is the shared scheme under a derived seed
        assert np.array_equal(a, O.perm(O.perm_rep_seed(9, 0), j))


def test_fisher_yates_is_uniform_over_replications():
    # base 3: the 6 permutations, over 6000 replications (chi2, df 5: 0.999 quantile 20.5)
    counts = {q: 0 for q in itertools.permutations(range(3))}
    for m in range(6000):
        counts[tuple(O.perm_rep(4, m, 1))] += 1
    e = 1000.0
    assert sum((c - e) ** 2 / e for c in counts.values()) < 20.5


def test_points_use_each_replications_permutation():
    s, N, M, seed = 5, 40, 3, 13
    x, R = O.sequence(s, N, M, seed, flags=O.PERM_PER_REP, m_offset=2)
    for m in range(M):
        for j in range(s):
            p = O.nth_prime(j)
            D, P = O.digits(p)
            n = O.start(seed, 2 + m, j)
            sg = O.perm_rep(seed, 2 + m, j)
            for i in (0, 1, 17, 39):
                assert R[m, i, j] == O.radinv_R(p, (n + i) % P, sg)
                assert x[m, i, j] == O.point_from_R(int(R[m, i, j]), P)
    # Algorithm 2 agrees with the definition
    x2, R2 = O.sequence(s, N, M, seed, flags=O.PERM_PER_REP, m_offset=2, gen=1)
    assert np.array_equal(R, R2)


def test_stratification_survives_the_permutation():
    # p^L consecutive indices from a random start put one point in each
    # interval [t/p^L, (t+1)/p^L), whatever each replication's permutation
    for j, L in ((0, 8), (1, 5), (2, 3), (20, 2)):
        p = O.nth_prime(j)
        D, P = O.digits(p)
        n = p ** L
        _, R = O.sequence(j + 1, n, 3, seed=31 + j, flags=O.PERM_PER_REP)
        for m in range(3):
            cells = (R[m, :, j].astype(object) * n) // P
            assert sorted(int(c) for c in cells) == list(range(n))


def test_estimator_against_black():
    inst = I.cfg1()
    th = O.price_caplets(inst.model, 4096, 32, 3, flags=O.PERM_PER_REP)[:, -1]
    se = th.std(ddof=1) / math.sqrt(len(th))
    assert abs(th.mean() - 1.3698347565e-3) < 4 * se + 2e-6
