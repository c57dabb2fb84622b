"""Pins of the full-period local pattern oracle (Sec. II, Figs. 3-4): the O(p L0)
enumeration equals the histogram of every window of D consecutive ciphertexts
over one whole period generated step by step (tiny instances), plus counting
identities of the cell widths and totals."""

import numpy as np
import pytest

from oracle import pattern as PT

# tiny instances: n prime, p prime < n, a a primitive root mod p, e coprime to n-1
TINY = [
    (1019, 3, 11, 2),
    (2003, 5, 13, 2),
    (1009, 5, 7, 3),
]


def full_period_windows(orc, n, e, p, a, dim):
    """Every window (c_k, ..., c_{k+D-1}), k = 0 .. n(p-1) - 1 (indices mod
    the period), from one step-by-step pass of algorithm (9) from (0, 1)."""
    period = n * (p - 1)
    c, _, m, s = orc.generate(p, a, n, e, 0, 1, period, want_r=False)
    assert (m, s) == (0, 1)                  # the state returns after n (p - 1) steps
    cyc = np.concatenate([[0], c[:-1]]).astype(np.int64)   # c_0 = 0^e = 0, c_1, ..., c_{P-1}
    assert c[-1] == 0
    return np.stack([np.roll(cyc, -j) for j in range(dim)], axis=1)


@pytest.mark.parametrize("n,e,p,a", TINY)
@pytest.mark.parametrize("dim,bins,x0,l0", [(2, 16, 0, 40), (3, 8, 5, 20), (4, 4, 300, 50), (5, 3, 0, 1000)])
def test_enumeration_equals_full_period_windows(orc, n, e, p, a, dim, bins, x0, l0):
    l0 = min(l0, n - x0)
    win = full_period_windows(orc, n, e, p, a, dim)
    sel = win[(win[:, 0] >= x0) & (win[:, 0] < x0 + l0)]
    cell = np.zeros(sel.shape[0], dtype=np.int64)
    for j in range(1, dim):
        cell = cell * bins + (sel[:, j] * bins) // n
    want = np.bincount(cell, minlength=bins ** (dim - 1))
    got = orc.pattern_hist(n, e, p, a, x0, l0, dim, bins, 1, p).astype(np.int64)
    assert np.array_equal(got, want)
    # every first point occurs p - 1 times in the period
    assert got.sum() == l0 * (p - 1)


def test_skip_ranges_add_up(orc):
    p, a = orc.lcg_params(32)
    n, e = 4294967087, 9
    whole = orc.pattern_hist(n, e, p, a, 7, 3, 3, 32, 1, 1 + 30000)
    parts = orc.pattern_hist(n, e, p, a, 7, 3, 3, 32, 1, 1 + 12345) + \
        orc.pattern_hist(n, e, p, a, 7, 3, 3, 32, 1 + 12345, 1 + 30000)
    assert np.array_equal(whole, parts) and whole.sum() == 3 * 30000


def test_first_following_point_is_a_permutation(orc):
    """For one first point and all skips of a tiny instance, the next points
    (m + s)^e are distinct (encryption is a permutation)."""
    n, e, p, a = 1019, 3, 11, 2
    h = orc.pattern_hist(n, e, p, a, 17, 1, 2, n, 1, p)
    assert h.max() == 1 and h.sum() == p - 1


@pytest.mark.parametrize("n,bins", [(4294967087, 4096), (4294967087, 64), (1019, 7), (2147483659, 100)])
def test_cell_widths(n, bins):
    w = PT.cell_widths(n, bins)
    assert w.sum() == n and w.max() - w.min() <= 1
    for b in (0, bins // 3, bins - 1):
        lo = -(-(b * n) // bins)
        assert (lo * bins) // n == b and ((lo - 1) * bins) // n == b - 1 if b else True


def test_expected_counts_total():
    e = PT.expected_counts(4294967087, 4, 64, 1000)
    assert e.size == 64 ** 3 and abs(e.sum() - 1000) < 1e-8
