"""CPU oracle of the full-period local pattern analysis (Sec. II, Figs. 3-4: the
D-dimensional pattern of consecutive ciphertexts over the whole period in
O(p L0) steps; the Tests section applies chi-square tests to its histogram).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The histogram itself comes from
``pho_pattern_hist`` in phoracle.c; this module adds the expected counts and
the chi-square statistic, in plain Python integers and numpy binary64.

Readings: the following points are binned into B cells per axis by
floor(c B / n), so cell b holds the w_b = ceil((b+1) n / B) - ceil(b n / B)
ciphertexts c with that bin; under the ideal model each following point is
uniform over Z/nZ, and a cell's expected count is T * prod_j (w_{b_j} / n)
for T = l0 (s_hi - s_lo) tuples.  chi^2 = sum (O - E)^2 / E over all
B^(D-1) cells, with B^(D-1) - 1 degrees of freedom and the one-sided P-value
about the median of the battery.
"""

from __future__ import annotations

import numpy as np

from . import battery
from . import pattern_hist  # noqa: F401  (re-exported for callers)


def cell_widths(n, bins):
    """w_b for b = 0 .. bins-1: how many c in [0, n) have floor(c bins / n) = b."""
    edges = [-(-(b * n) // bins) for b in range(bins + 1)]   # ceil(b n / bins)
    return np.array([edges[b + 1] - edges[b] for b in range(bins)], dtype=np.float64)


def expected_counts(n, dim, bins, tuples):
    """Expected count of every cell (first following point most significant)."""
    q = cell_widths(n, bins) / float(n)
    e = np.array([float(tuples)])
    for _ in range(dim - 1):
        e = np.outer(e, q).ravel()
    return e


def chi_square(hist, n, dim, bins, tuples):
    exp = expected_counts(n, dim, bins, tuples)
    chi2 = battery.chi_square(hist, exp)
    dof = hist.size - 1
    return chi2, dof, battery.p_value(chi2, dof)
