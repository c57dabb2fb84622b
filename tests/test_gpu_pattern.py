"""GPU parity of the full-period local pattern analysis (Sec. II, Figs. 3-4) against the
CPU oracle: histograms bit for bit, chi^2 and P to floating tolerance, the
full skip range checked through additivity and totals."""

import numpy as np
import pytest

from oracle import pattern as PT

pytestmark = pytest.mark.gpu

P31 = (1 << 31) - 1
A31 = 784588716
PAPER_N = 4294967087   # the safe prime of the paper's pattern figures


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ph(torch):
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


def _run(ph, torch, n, e, x0, l0, dim, bins, s_lo, s_hi, hist=None):
    spec = ph.pattern_spec(n, e, x0, l0, dim, bins, s_lo, s_hi)
    if hist is None:
        hist = torch.zeros(bins ** (dim - 1), dtype=torch.int64, device="cuda:0")
    print("pattern case n=%d e=%d x0=%d l0=%d D=%d bins=%d s=[%d,%d)" % (n, e, x0, l0, dim, bins, s_lo, s_hi),
          flush=True)
    ph.pattern_histogram(spec, hist)
    torch.cuda.synchronize()
    return spec, hist


def _instances(ph):
    n, e, _ = ph.phprng_draw_instances(32, 0x14112484 + 9, 3, (9, 17))
    out = [(PAPER_N, 9)] + list(zip(n.tolist(), e.tolist()))
    # other exponent chains: 3, 5 and a generic one (7 or 11)
    for want in (3, 5, 7, 11):
        for nn in n.tolist() + [PAPER_N]:
            if ph.phprng_check_instance(32, nn, want) == 0:
                out.append((nn, want))
                break
    return out


CASES = [  # x0, l0, dim, bins, s_lo, s_hi
    (0, 8, 2, 1 << 12, 1, 1 + (1 << 17)),
    (0, 8, 3, 64, 1, 1 + (1 << 17)),
    (100, 4, 4, 16, 777, 777 + 100001),
    (5, 3, 5, 8, 1, 1 + 50000),
    (0, 2, 3, 4096, 1, 1 + 40000),    # the 2^24 cells of the Tests section (D = 3)
    (0, 2, 5, 64, P31 - 30000, P31),  # the last skips of the period, 2^24 cells (D = 5)
    (7, 5, 3, 100, 1, 1 + 60000),     # bins that are not powers of two
    (0, 3, 5, 7, 1000, 1000 + 40000),
    (0, 4, 2, 1000003, 1, 1 + 50000),
]


@pytest.mark.parametrize("case", CASES)
def test_pattern_histogram_matches_oracle(ph, torch, orc, case):
    x0, l0, dim, bins, s_lo, s_hi = case
    for n, e in _instances(ph)[:3] if bins ** (dim - 1) > (1 << 20) else _instances(ph):
        spec, hist = _run(ph, torch, n, e, x0, l0, dim, bins, s_lo, s_hi)
        got = hist.cpu().numpy().view(np.uint64)
        want = orc.pattern_hist(n, e, P31, A31, x0, l0, dim, bins, s_lo, s_hi)
        assert np.array_equal(got, want), (n, e, np.flatnonzero(got != want)[:8])
        chi2, p, total = ph.pattern_chi2(spec, hist)
        w2, wdof, wp = PT.chi_square(want.astype(np.int64), n, dim, bins, l0 * (s_hi - s_lo))
        assert total == l0 * (s_hi - s_lo)
        assert chi2 == pytest.approx(w2, rel=1e-9)
        if wp > 1e-300:
            assert p == pytest.approx(wp, rel=1e-6, abs=1e-12)


def test_window_at_the_top_of_the_range(ph, torch, orc):
    n, e = PAPER_N, 9
    spec, hist = _run(ph, torch, n, e, n - 5, 5, 3, 32, 1, 20001)
    want = orc.pattern_hist(n, e, P31, A31, n - 5, 5, 3, 32, 1, 20001)
    assert np.array_equal(hist.cpu().numpy().view(np.uint64), want)


def test_full_period_by_parts(ph, torch, orc):
    """One first point over the whole skip period [1, p): the histogram of the
    full range equals the sum of three part ranges (bit for bit), its total is
    p - 1, and the oracle agrees on a part."""
    n, e = PAPER_N, 9
    cuts = [1, 1 + 123456, 1 + (1 << 30), P31]
    spec, full = _run(ph, torch, n, e, 0, 1, 3, 4096, 1, P31)
    parts = torch.zeros_like(full)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        _run(ph, torch, n, e, 0, 1, 3, 4096, lo, hi, parts)
    assert torch.equal(full, parts)
    chi2, p, total = ph.pattern_chi2(spec, full)
    assert total == P31 - 1 and chi2 > 0
    _, small = _run(ph, torch, n, e, 0, 1, 3, 4096, 1, 1 + 123456)
    want = orc.pattern_hist(n, e, P31, A31, 0, 1, 3, 4096, 1, 1 + 123456)
    assert np.array_equal(small.cpu().numpy().view(np.uint64), want)


def test_pattern_argument_errors(ph, torch):
    hist = torch.zeros(64, dtype=torch.int64, device="cuda:0")
    bad = [
        ph.pattern_spec(PAPER_N, 9, 0, 1, 6, 2, 1, 10),          # D > 5
        ph.pattern_spec(PAPER_N, 9, 0, 1, 3, 1 << 15, 1, 10),    # 2^30 cells
        ph.pattern_spec(PAPER_N, 9, 0, 1, 3, 8, 0, 10),          # s_lo = 0
        ph.pattern_spec(PAPER_N, 9, 0, 1, 3, 8, 1, P31 + 1),     # beyond p
        ph.pattern_spec(PAPER_N, 9, PAPER_N - 1, 2, 3, 8, 1, 9),  # window beyond n
        ph.pattern_spec(PAPER_N + 2, 9, 0, 1, 3, 8, 1, 9),       # n not prime
        ph.pattern_spec(PAPER_N, 2, 0, 1, 3, 8, 1, 9),           # e < 3
    ]
    for spec in bad:
        with pytest.raises(ph.PhprngError):
            ph.pattern_histogram(spec, hist)
    torch.cuda.synchronize()
    assert int(hist.sum()) == 0
