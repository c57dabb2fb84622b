"""Pins of the CPU battery oracle (the chi-square tests of the paper's Tests
section) against brute force, closed forms and hand-built inputs."""

import cmath
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import battery as B


def test_bins_and_clamp():
    r = np.array([0.0, 0.5, 0.25, 1.0 - 2.0 ** -53, 1.0])
    assert list(B.bin_of(r, 1 << 20)) == [0, 1 << 19, 1 << 18, (1 << 20) - 1, (1 << 20) - 1]
    assert list(B.bin_of(r, 100)) == [0, 50, 25, 99, 99]
    assert list(B.bin_of(np.array([0.3, 0.7, 0.09999999999999999, 0.1]), 10)) == [3, 7, 0, 1]


def _block_with(prefix):
    r = np.full(B.M, 0.75)
    r[: len(prefix)] = prefix
    return r


def test_serial_cell_index_convention():
    # first element is the most significant digit
    r = _block_with([0.5, 0.25, 0.999, 0.001, 0.0, 0.0])
    c2 = B.serial_counts(r, 2)
    assert c2[512 * 1024 + 256] == 1 and c2[1022 * 1024 + 1] == 1 and c2[0] == 1
    assert c2[768 * 1024 + 768] == B.M // 2 - 3 and c2.sum() == B.M // 2
    c3 = B.serial_counts(r, 3)
    assert c3[(50 * 100 + 25) * 100 + 99] == 1 and c3[(0 * 100 + 0) * 100 + 0] == 1
    assert c3.sum() == B.M // 3  # the last M mod 3 uniforms are unused
    c5 = B.serial_counts(r, 5)
    assert c5.sum() == B.M // 5
    assert c5[(((8 * 16 + 4) * 16 + 15) * 16 + 0) * 16 + 0] == 1


def test_serial_block_tail_is_unused():
    r = np.full(2 * B.M, 0.75)
    r[B.M - 1] = 0.0          # last uniform of block 0: outside every triple and quintuple
    # no tuple holds it in any position (a tuple running into the next block
    # would start with it: first digit 0)
    assert B.serial_counts(r, 3)[: 100 * 100].sum() == 0 and B.serial_counts(r, 5)[: 16 ** 4].sum() == 0
    assert B.serial_counts(r, 2)[0 * 1024 + 768] == 0  # pair (0.75, 0.0) -> cell 768 * 1024
    assert B.serial_counts(r, 2)[768 * 1024 + 0] == 1


def test_poker_classifier_examples():
    hands = np.array([[0, 1, 2, 3, 4], [1, 1, 2, 3, 4], [1, 1, 2, 2, 4], [7, 7, 7, 2, 4],
                      [7, 2, 7, 2, 7], [9, 9, 9, 9, 0], [5, 5, 5, 5, 5], [3, 1, 3, 1, 0]])
    assert list(B.poker_category(hands)) == [0, 1, 2, 3, 4, 5, 6, 2]


def test_poker_law_by_enumerating_all_hands():
    hands = np.array(list(itertools.product(range(10), repeat=5)), dtype=np.int64)
    counts = np.bincount(B.poker_category(hands), minlength=7)
    assert np.array_equal(counts, np.rint(B.poker_probabilities() * 1e5).astype(np.int64))
    assert counts.sum() == 10 ** 5


@pytest.mark.parametrize("balls,urns", [(5, 7), (6, 4), (4, 9)])
def test_collision_law_brute_force(balls, urns):
    exact = np.zeros(balls + 1)
    for a in itertools.product(range(urns), repeat=balls):
        exact[balls - len(set(a))] += 1
    exact /= urns ** balls
    assert np.allclose(B.collision_law(balls, urns, balls), exact, rtol=1e-12, atol=1e-15)


def test_collision_law_moments_closed_form():
    """Occupied urns Y after n balls in m urns: E[Y] = m (1 - (1 - 1/m)^n),
    E[Y(Y-1)] = m (m-1) (1 - 2 (1 - 1/m)^n + (1 - 2/m)^n)."""
    n, m = B.COLL_BALLS, B.COLL_URNS
    law = B.collision_law(n, m, 600)
    assert abs(law.sum() - 1.0) < 1e-13
    c = np.arange(law.size)
    q1 = Fraction(m - 1, m) ** n          # exact rationals: the closed forms cancel badly in binary64
    q2 = Fraction(m - 2, m) ** n
    ey = m * (1 - q1)
    eyy = m * (m - 1) * (1 - 2 * q1 + q2)
    var_y = float(eyy + ey - ey * ey)
    mean_c = float((law * c).sum())
    var_c = float((law * (c - mean_c) ** 2).sum())
    assert abs(mean_c - float(n - ey)) < 1e-9
    assert abs(var_c - var_y) < 1e-8
    p = B.collision_probabilities()
    assert p.size == B.COLL_CATS and abs(p.sum() - 1.0) < 1e-14 and (p > 1e-3).all()


def test_collisions_per_trial_small_cases():
    r = np.random.default_rng(3).random(B.M)
    r[: B.COLL_BALLS] = 0.123            # trial 0: one urn
    r[B.COLL_BALLS: 2 * B.COLL_BALLS] = (np.arange(B.COLL_BALLS) + 0.5) / B.COLL_BALLS  # distinct urns
    got = B.collisions_per_trial(r)
    assert got[0] == B.COLL_BALLS - 1 and got[1] == 0
    t = r[5 * B.COLL_BALLS: 6 * B.COLL_BALLS]
    assert got[5] == B.COLL_BALLS - len({int(x * (1 << 20)) for x in t})


def test_runs_exact_counts_by_enumeration():
    m = 12
    counts = np.zeros(m + 1)
    for bits in itertools.product((0, 1), repeat=m):
        for L in B.interior_run_lengths(np.array(bits)):
            counts[L] += 1
    for L in range(1, m):
        assert counts[L] == max(m - 1 - L, 0) * 2 ** (m - L - 1)
    w = B.runs_weights(m)
    assert np.allclose(w[: m - 1] * 2 ** m, counts[1:m])
    assert w[m - 1:].sum() == 0


def test_runs_interior_only():
    bits = np.array([1, 1, 0, 0, 0, 1, 0, 1, 1, 1])
    assert list(B.interior_run_lengths(bits)) == [3, 1, 1]
    r = np.full(B.M, 0.25)
    r[10:13] = 0.75
    r[20] = 0.75
    # interior runs: ones at 10..12 (3), zeros at 13..19 (7), the one at 20 (1)
    got = B.runs_counts(r)
    assert list(np.flatnonzero(got)) == [0, 2, 6] and got[[0, 2, 6]].tolist() == [1, 1, 1]


def test_fourier_matches_paper_sum():
    m = 64
    x = np.random.default_rng(1).random(m) - 0.5
    got = B.fourier_coefficients(x)
    for k in range(m):
        s = sum(x[j] * cmath.exp(2j * math.pi * j * k / m) for j in range(m)) / math.sqrt(m)
        assert abs(got[k] - s) < 1e-13
    # Parseval with this normalisation, and real input gives conjugate symmetry
    assert abs(np.sum(np.abs(got) ** 2) - np.sum(x * x)) < 1e-12
    assert abs(got[5] - np.conj(got[m - 5])) < 1e-14


def test_fourier_categories_and_law():
    s = B.FOURIER_SCALE
    v = np.array([0.0, -1e-300, 4.0 / math.sqrt(24.0) + 1e-12, -4.0 / math.sqrt(24.0) - 1e-12, 1.0 / s, -1.0 / s])
    assert list(B.fourier_category(v)) == [33, 32, 65, 0, 34, 32]
    p = B.fourier_probabilities()
    assert p.size == 66 and abs(p.sum() - 1.0) < 1e-15
    assert np.allclose(p, p[::-1], rtol=1e-12, atol=0)
    assert abs(p[-1] - 3.1671241833119863e-05) < 1e-18   # upper tail of the normal law beyond 4
    assert abs(p[33] - (math.erf(1 / 8 / math.sqrt(2)) / 2)) < 1e-16


def test_uniform_variance_is_one_over_24():
    """Each of Re, Im of a coefficient of uniform noise has variance 1/24."""
    x = np.random.default_rng(2).random(B.M) - 0.5
    xh = B.fourier_coefficients(x)[1: B.M // 2]
    assert abs(np.var(xh.real) - 1 / 24) < 3e-4 and abs(np.var(xh.imag) - 1 / 24) < 3e-4


def test_p_value_closed_forms():
    for x in (0.1, 1.386, 3.0, 10.0, 50.0):
        q2 = math.exp(-x / 2)
        assert B.p_value(x, 2) == pytest.approx(min(q2, 1 - q2), rel=1e-12)
        q1 = math.erfc(math.sqrt(x / 2))
        assert B.p_value(x, 1) == pytest.approx(min(q1, 1 - q1), rel=1e-12)
        q4 = math.exp(-x / 2) * (1 + x / 2)
        assert B.p_value(x, 4) == pytest.approx(min(q4, 1 - q4), rel=1e-12)
    assert B.chi_square([10, 20], np.array([15.0, 15.0])) == pytest.approx(25 / 15 * 2)


def test_interleave_order():
    s = np.array([[1.0, 2.0, 3.0], [10.0, 20.0, 30.0]])
    assert list(B.interleave(s)) == [1.0, 10.0, 2.0, 20.0, 3.0, 30.0]


def test_battery_accepts_good_and_rejects_bad():
    rng = np.random.default_rng(12345)
    good = rng.random(8 * B.M)
    res = B.run_battery(good)
    assert set(res) == set(B.TESTS)
    assert min(r[4] for r in res.values()) > 1e-6, {k: v[4] for k, v in res.items()}
    bad = good.copy()
    bad[1::2] = bad[0::2]            # every pair repeats its first element
    rb = B.run_battery(bad)
    assert rb["serial2"][4] < 1e-8 and rb["runs"][4] < 1e-8 and rb["collision"][4] < 1e-8
    # a permutation of equally spaced points fills every frequency bin exactly:
    # chi^2 = 0 lies far below the median, which the one-sided P-value flags too
    even = np.concatenate([rng.permutation((np.arange(B.M) + 0.5) / B.M) for _ in range(2)])
    assert B.chi_square(B.frequency_counts(even), np.full(B.FREQ_BINS, 2.0)) == 0.0
    assert B.run_battery(even)["frequency"][4] < 1e-8


def test_generator_passes_battery_intrastream_and_interstream(orc, paper):
    """Algorithm (9) on the paper's example instance (n = 4294967087, e = 9,
    L'Ecuyer's skip) passes all nine tests on 8 blocks, and so does the
    interstream order of 64 seeded instances (the paper reports passes far
    beyond these sizes)."""
    p, a = orc.lcg_params(32)
    _, r, _, _ = orc.generate(p, a, 4294967087, 9, 0, 1, 8 * B.M, want_c=False)
    res = B.run_battery(r)
    assert min(v[4] for v in res.values()) > 1e-8, {k: v[4] for k, v in res.items()}
    n, e, k0 = orc.seed(32, 0x14112484 + 7, 64)
    per = 8 * B.M // 64
    _, r, _, _, _ = orc.generate_many(p, a, n, e, 0, 1, per, want_c=False)
    res = B.run_battery(B.interleave(r.reshape(64, per)))
    assert min(v[4] for v in res.values()) > 1e-8, {k: v[4] for k, v in res.items()}
