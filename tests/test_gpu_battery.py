"""GPU parity of the statistical battery (the chi-square tests of the paper's
Tests section) against the CPU oracle on the same uniforms: every integer
histogram bit for bit, the Fourier histogram up to coefficients within
rounding distance of a bin edge, chi^2 and P to floating tolerance."""

import math

import numpy as np
import pytest

from oracle import battery as B

pytestmark = pytest.mark.gpu

M = B.M


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _edge_sequence(nblocks, seed):
    """Uniforms with many exact bin edges, R = 1.0, R = 1/2 and long runs."""
    rng = np.random.default_rng(seed)
    r = rng.random(nblocks * M)
    k = rng.integers(0, 1 << 20, 4000)
    r[rng.integers(0, r.size, 4000)] = k / float(1 << 20)           # frequency / collision edges
    r[rng.integers(0, r.size, 2000)] = rng.integers(1, 100, 2000) / 100.0  # 3-D serial edges
    r[rng.integers(0, r.size, 2000)] = rng.integers(1, 10, 2000) / 10.0    # poker edges
    r[rng.integers(0, r.size, 500)] = 1.0
    r[rng.integers(0, r.size, 2000)] = 0.5
    r[3 * M + 1000: 3 * M + 1300] = 0.75                              # a run of 300 ones
    r[5 * M - 70: 5 * M] = 0.25                                       # a run reaching a block end
    return r


def _check_against_oracle(ph, torch, bat, r_host):
    want = B.run_battery(r_host)
    got = bat.report()
    for i, name in enumerate(ph.BATTERY_TESTS):
        counts = bat.counts(i).astype(np.int64)
        wc, we, wchi2, wdof, wp = want[name]
        if name != "fourier":
            assert np.array_equal(counts, wc), (name, np.flatnonzero(counts != wc)[:10])
        chi2, dof, p, samples = got[name]
        assert dof == wdof and samples == counts.sum()
        if name != "fourier":
            assert chi2 == pytest.approx(wchi2, rel=1e-9), name
            if wp > 1e-300:
                assert p == pytest.approx(wp, rel=1e-6, abs=1e-12), (name, p, wp)
    return want


def _fourier_check(ph, torch, bat, r_host, want_counts):
    """GPU coefficients within 1e-13 of the oracle's; the GPU histogram is the
    category count of its own coefficients; oracle and GPU categories differ
    only for coefficients within 1e-13 of a bin edge."""
    n = r_host.size
    r = _dev(torch, r_host)
    coef = torch.empty(n, dtype=torch.float64, device="cuda:0")
    bat.fourier(r, coef)
    torch.cuda.synchronize()
    g = coef.cpu().numpy()
    o = B.fourier_values(r_host)
    assert np.max(np.abs(g - o)) < 1e-13
    gcat = B.fourier_category(g)
    ocat = B.fourier_category(o)
    assert np.array_equal(np.bincount(gcat, minlength=B.FOURIER_CATS), bat.counts(8).astype(np.int64))
    differ = gcat != ocat
    if differ.any():
        near = np.abs(o * B.FOURIER_SCALE - np.rint(o * B.FOURIER_SCALE)) < 1e-11
        assert (near | ~differ).all()
    assert np.array_equal(np.bincount(ocat, minlength=B.FOURIER_CATS), want_counts)


def test_battery_random_uniforms(ph, torch):
    r_host = np.random.default_rng(20240611).random(8 * M)
    bat = ph.Battery(0)
    bat.accumulate(_dev(torch, r_host))
    want = _check_against_oracle(ph, torch, bat, r_host)
    _fourier_check(ph, torch, bat, r_host, want["fourier"][0])
    fc = bat.counts(8).astype(np.int64)
    chi2 = B.chi_square(fc, want["fourier"][1])
    assert bat.report()["fourier"][0] == pytest.approx(chi2, rel=1e-9)
    bat.close()


def test_battery_edges_and_degenerate_values(ph, torch):
    r_host = _edge_sequence(6, 7)
    bat = ph.Battery(0)
    bat.accumulate(_dev(torch, r_host))
    want = _check_against_oracle(ph, torch, bat, r_host)
    _fourier_check(ph, torch, bat, r_host, want["fourier"][0])
    bat.close()


def test_battery_constant_block(ph, torch):
    """A constant block: one frequency bin, no interior runs, every trial
    collides 2^14 - 1 times, all coefficients but k = 0 vanish."""
    r_host = np.full(M, 0.3)
    bat = ph.Battery(0)
    bat.accumulate(_dev(torch, r_host))
    _check_against_oracle(ph, torch, bat, r_host)
    assert bat.counts(7).sum() == 0
    assert bat.counts(6)[-1] == 64
    bat.close()


def test_battery_split_calls_and_chunks_agree(ph, torch):
    """130 blocks (more than one internal pass of 128 blocks) in one call, or
    in calls of 1, 7 and 122 blocks, give the same histograms."""
    nb = 130
    g = torch.Generator(device="cuda:0")
    g.manual_seed(99)
    r = torch.rand(nb * M, dtype=torch.float64, device="cuda:0", generator=g)
    one, split = ph.Battery(0), ph.Battery(0)
    one.accumulate(r)
    for a, b in ((0, 1), (1, 8), (8, nb)):
        split.accumulate(r[a * M: b * M])
    for i in range(len(ph.BATTERY_TESTS)):
        assert np.array_equal(one.counts(i), split.counts(i)), ph.BATTERY_TESTS[i]
    ra, rb = one.report(), split.report()
    for name in ph.BATTERY_TESTS:
        assert ra[name][3] == rb[name][3]
    # totals that hold at any size
    assert ra["frequency"][3] == nb * M and ra["serial3"][3] == nb * (M // 3)
    assert ra["serial5"][3] == nb * (M // 5) and ra["poker"][3] == nb * (M // 5)
    assert ra["collision"][3] == nb * 64 and ra["fourier"][3] == nb * M
    t = one.timing()
    assert all(v[0] > 0 and v[1] == 2 for v in t.values()), t
    one.reset()
    torch.cuda.synchronize()
    assert one.counts(0).sum() == 0 and one.report()["frequency"][3] == 0
    one.close()
    split.close()


def test_battery_on_generator_streams_and_interleave(ph, torch, orc):
    """Uniforms of the GPU generator: 8 streams of one block each
    (intrastream), and 64 streams of 2^17 draws in the interstream order made
    by the interleave kernel."""
    ctx = ph.Context(0, max_instances=72)
    intra_ids = ctx.seed_instances(32, 0x14112484 + 8, 8, (9, 17), 0, 0)
    ids = ctx.seed_instances(32, 0x14112484 + 7, 64, (9, 17), 0, 0)
    per = 8 * M // 64
    intra = torch.empty(8 * M, dtype=torch.float64, device="cuda:0")
    ctx.generate(ph.make_requests(intra_ids, [M] * 8, np.arange(8, dtype=np.uint64) * M), None, None, intra)
    multi = torch.empty(8 * M, dtype=torch.float64, device="cuda:0")
    ctx.generate(ph.make_requests(ids, [per] * 64, np.arange(64, dtype=np.uint64) * per), None, None, multi)
    inter = torch.empty_like(multi)
    ph.interleave(multi, inter, 64, per)
    torch.cuda.synchronize()
    mh = multi.cpu().numpy()
    ih = inter.cpu().numpy()
    assert np.array_equal(ih.view(np.uint64), B.interleave(mh.reshape(64, per)).view(np.uint64))
    for seq in (intra, inter):
        bat = ph.Battery(0)
        bat.accumulate(seq)
        _check_against_oracle(ph, torch, bat, seq.cpu().numpy())
        got = bat.report()
        assert min(v[2] for v in got.values()) > 1e-8, got
        bat.close()
    ctx.close()


@pytest.mark.parametrize("S,L", [(1, 1), (3, 1000), (64, 64), (100, 77), (1000, 65), (5000, 3)])
def test_interleave_ragged_shapes(ph, torch, S, L):
    src = np.random.default_rng(S * 7 + L).random(S * L)
    a = _dev(torch, src)
    out = torch.full((S * L,), -1.0, dtype=torch.float64, device="cuda:0")
    ph.interleave(a, out, S, L)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), B.interleave(src.reshape(S, L)))


def test_battery_argument_errors(ph, torch):
    bat = ph.Battery(0)
    r = torch.zeros(M + 1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ph.PhprngError):
        bat.accumulate(r, count=M + 1)
    with pytest.raises(ph.PhprngError):
        bat.accumulate(r[1:], count=M)       # 8-byte but not 16-byte aligned
    bat.accumulate(r, count=0)
    assert bat.report()["frequency"][3] == 0
    with pytest.raises(ph.PhprngError):
        ph.interleave(r, r, 2, 4)
    bat.close()


def test_battery_on_width64_generator_output(ph, torch):
    """Uniforms of 64-bit moduli (R in (0, 1]) through the battery: histograms
    equal the oracle's on the same values."""
    ctx = ph.Context(0, max_instances=4)
    ids = ctx.seed_instances(64, 0x14112484 + 11, 4, (9, 17), 0, 1 << 30)
    r = torch.empty(4 * M, dtype=torch.float64, device="cuda:0")
    ctx.generate(ph.make_requests(ids, [M] * 4, np.arange(4, dtype=np.uint64) * M), None, None, r)
    bat = ph.Battery(0)
    bat.accumulate(r)
    _check_against_oracle(ph, torch, bat, r.cpu().numpy())
    bat.close()
    ctx.close()
