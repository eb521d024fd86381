"""Pins for the oracle's random-start Halton generator (CPU only).

Each test ties the oracle to something other than its own code:
  * the van der Corput leading points fixed by eqs. (1)-(2) (golden file);
  * Struckmeier's von Neumann-Kakutani transformation, eqs. (4)-(6) /
    Algorithm 1, evaluated in exact rationals (an independent construction
    of the same sequence);
  * the stratification property of p^L consecutive van der Corput terms;
  * Python's exactly rounded Fraction -> float conversion for the FP64 value;
  * a known-answer vector of SplitMix64 and chi-square uniformity of the
    random starts and permutations.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_leading():
    out = {}
    with open(os.path.join(GOLD, "vdc_leading_points.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            b, vals = line.split(":")
            out[int(b)] = [Fraction(v.strip()) for v in vals.split(",")]
    return out


def test_splitmix64_known_answer():
    with open(os.path.join(GOLD, "splitmix64_seed0.txt")) as f:
        vals = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    assert [O.splitmix64(0, k) for k in range(len(vals))] == vals


def test_primes_and_digit_counts():
    primes = [O.nth_prime(j) for j in range(360)]
    # primes by an independent sieve
    lim = 2500
    sieve = np.ones(lim + 1, dtype=bool)
    sieve[:2] = False
    for q in range(2, int(lim ** 0.5) + 1):
        if sieve[q]:
            sieve[q * q::q] = False
    assert primes == list(np.nonzero(sieve)[0][:360])
    assert primes[-1] == 2423
    for p in primes[:40] + primes[-5:]:
        D, P = O.digits(p)
        assert P == p ** D and P <= 2 ** 53 < P * p


def test_start_zero_gives_van_der_corput_leading_points():
    lead = _read_leading()
    x, R = O.sequence(3, 11, 1, seed=123, flags=O.START_ZERO)
    for j, b in enumerate([2, 3, 5]):
        want = lead[b]
        D, P = O.digits(b)
        for i, w in enumerate(want):
            assert Fraction(int(R[0, i, j]), P) == w
            assert x[0, i, j] == float(w)


def test_point_is_correctly_rounded_rational():
    x, R = O.sequence(12, 257, 3, seed=7)
    for j in range(12):
        D, P = O.digits(O.nth_prime(j))
        for m in range(3):
            for i in range(0, 257, 17):
                r = int(R[m, i, j])
                assert 0 <= r < P
                assert x[m, i, j] == float(Fraction(r, P))   # exactly rounded


def _struckmeier_step(x: Fraction, p: int) -> Fraction:
    """One von Neumann-Kakutani step, eqs. (4)-(6), in exact arithmetic.

    k = floor(-ln(1-x)/ln p) + 1 is the unique k >= 1 with
    p^{-k} < 1 - x <= p^{-(k-1)}; it is found by exact comparison instead of
    floating logarithms (the rounding hazard the paper points out)."""
    y = 1 - x
    k = 1
    while not (Fraction(1, p ** k) < y):
        k += 1
    b = Fraction(p + 1 - p ** k, p ** k)
    return x + b


@pytest.mark.parametrize("j", [0, 1, 4, 9, 30])
def test_random_start_orbit_matches_algorithm1_exactly(j):
    p = O.nth_prime(j)
    D, P = O.digits(p)
    seed, m = 11, 5
    n0 = O.start(seed, m, j)
    if n0 > P - 300:       # keep clear of the wrap at P (not part of the orbit)
        pytest.skip("start too close to P")
    x, R = O.sequence(j + 1, 200, m + 1, seed)
    xs = Fraction(int(R[m, 0, j]), P)
    for i in range(1, 200):
        xs = _struckmeier_step(xs, p)
        assert xs == Fraction(int(R[m, i, j]), P), (p, i)


def test_orbit_of_zero_is_van_der_corput():
    lead = _read_leading()
    for b in (2, 3, 5):
        x = Fraction(0)
        orbit = [x]
        for _ in range(len(lead[b]) - 1):
            x = _struckmeier_step(x, b)
            orbit.append(x)
        assert orbit == lead[b]


@pytest.mark.parametrize("flags", [0, O.PERM_RANDOM, O.START_ZERO | O.PERM_RANDOM])
def test_algorithm2_equals_definition(flags):
    s, N, M = 25, 700, 3
    x0, R0 = O.sequence(s, N, M, seed=99, flags=flags, gen=0)
    x1, R1 = O.sequence(s, N, M, seed=99, flags=flags, gen=1)
    assert np.array_equal(R0, R1)
    assert np.array_equal(x0.view(np.uint64), x1.view(np.uint64))


@pytest.mark.parametrize("j", [0, 1, 3, 50])
@pytest.mark.parametrize("perm", [False, True])
def test_algorithm2_wraps_at_P(j, perm):
    # indices P-3 .. P+4 wrap to 0 .. 4 (mod P); both generators agree there
    p = O.nth_prime(j)
    D, P = O.digits(p)
    sig = O.perm(5, j) if perm else None
    got = O.alg2_run(p, P - 3, 8, sig)
    want = [O.radinv_R(p, (P - 3 + t) % P, sig) for t in range(8)]
    assert [int(v) for v in got] == want
    assert want[3] == 0


@pytest.mark.parametrize("flags", [0, O.PERM_RANDOM])
def test_stratification_invariant(flags):
    # p^L consecutive indices from any start put exactly one point in each
    # interval [t/p^L, (t+1)/p^L): the low L digits run over all residues.
    for j, L in [(0, 10), (1, 6), (2, 4), (5, 3), (20, 2)]:
        p = O.nth_prime(j)
        D, P = O.digits(p)
        n = p ** L
        x, R = O.sequence(j + 1, n, 2, seed=5 + j, flags=flags)
        for m in range(2):
            cells = (R[m, :, j].astype(object) * n) // P
            assert sorted(int(c) for c in cells) == list(range(n))


def test_start_zero_equals_plain_halton_in_every_base():
    # start 0 + identity permutation = the Halton sequence (eq. (2) bases are
    # the first s primes); compare the first 60 points against the
    # definition evaluated with Python integers.
    s, N = 40, 60
    x, R = O.sequence(s, N, 1, seed=0, flags=O.START_ZERO)
    for j in range(s):
        p = O.nth_prime(j)
        for i in range(N):
            v, num, den = i, 0, 1
            val = Fraction(0)
            while v:
                den *= p
                val += Fraction(v % p, den)
                v //= p
            assert x[0, i, j] == float(val)


def test_starts_uniform_and_in_range():
    # chi-square on the leading base-p digit of n_j^m over many (m, j)
    rng_js = [0, 1, 2, 3, 7]
    for j in rng_js:
        p = O.nth_prime(j)
        D, P = O.digits(p)
        starts = [O.start(42, m, j) for m in range(3000)]
        assert all(0 <= n < P for n in starts)
        bins = 8
        cnt = np.bincount([(n * bins) // P for n in starts], minlength=bins)
        exp = len(starts) / bins
        chi2 = ((cnt - exp) ** 2 / exp).sum()
        assert chi2 < 30.0   # 7 dof, p ~ 1e-4


def test_starts_independent_across_replications_and_dims():
    a = [O.start(1, m, j) for m in range(4) for j in range(4)]
    assert len(set(a)) == len(a)
    assert O.start(1, 0, 0) != O.start(2, 0, 0)


def test_permutations_are_uniform_permutations():
    for j in (0, 1, 2, 10, 100):
        s = O.perm(3, j)
        assert sorted(s) == list(range(O.nth_prime(j)))
    # position of digit 0 under sigma for base 5 over many seeds: uniform
    cnt = np.zeros(5)
    for seed in range(2000):
        cnt[int(np.nonzero(O.perm(seed, 2) == 0)[0][0])] += 1
    exp = 2000 / 5
    assert ((cnt - exp) ** 2 / exp).sum() < 25.0


def test_permuted_leading_zeros_are_not_permuted():
    # eq. (3) sums sigma(a_i) only up to the top digit a_k: the index 0 maps
    # to 0 and index p^t maps to sigma(1) p^{D-1-t} alone.
    sig = O.perm(17, 1)
    p = 3
    D, P = O.digits(p)
    assert O.radinv_R(p, 0, sig) == 0
    for t in range(5):
        R = O.radinv_R(p, p ** t, sig)
        want = int(sig[1]) * p ** (D - 1 - t) + sum(int(sig[0]) * p ** (D - 1 - u) for u in range(t))
        assert R == want


def test_m_offset_split_equals_single_call():
    x4, R4 = O.sequence(7, 33, 4, seed=8)
    xa, Ra = O.sequence(7, 33, 2, seed=8, m_offset=0)
    xb, Rb = O.sequence(7, 33, 2, seed=8, m_offset=2)
    assert np.array_equal(R4, np.concatenate([Ra, Rb]))


def test_N_beyond_P_rejected():
    # base 2 carries D = 53 digits (P = 2^53); N > P_j is refused (ERANGE)
    st = O._load().orc_sequence(1, 2 ** 53 + 1, 1, 0, 0, 0, 0, None, None)
    assert st == 2
