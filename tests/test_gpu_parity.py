"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle,
element by element, bit-exact for ciphertexts and uniforms.

Sizes span several 2048-draw tiles with ragged heads and tails; the
full-size workloads are checked on seeded samples the oracle computes one
by one.  Every case runs in one process on cuda:0."""

import math
import random

import numpy as np
import pytest

from tests.gpu_helpers import alloc_outputs, compare_request, oracle_draws, to_host

pytestmark = pytest.mark.gpu

SEED0 = 0x14112484


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


@pytest.fixture(scope="module")
def ctx(ph):
    c = ph.Context(0, max_instances=1 << 17)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tabs(tab32, tab64):
    return {32: tab32, 64: tab64}


def _run(ph, ctx, specs, mode=0, want=(True, True, True), gap=0, shuffle_seed=None):
    """specs: list of (inst_id, count).  Returns host outputs and offsets."""
    counts = [c for _, c in specs]
    order = list(range(len(specs)))
    if shuffle_seed is not None:
        random.Random(shuffle_seed).shuffle(order)
    offs = [0] * len(specs)
    cur = 0
    for i in order:
        offs[i] = cur
        cur += counts[i] + gap
    total = cur
    c32, c64, r = alloc_outputs(total, *want)
    reqs = ph.make_requests([s[0] for s in specs], counts, offs)
    ctx.generate(reqs, c32, c64, r, capacity=max(total, 1), mode=mode)
    return to_host(c32, c64, r), offs


def _check(orc, tabs, ctx, specs, starts, host, offs, label):
    hc32, hc64, hr = host
    for (iid, count), k0, off in zip(specs, starts, offs):
        n, e, p, a, w = ctx.get_params(iid)
        want_c, want_r, _ = oracle_draws(orc, tabs, w, n, e, k0, count)
        got_c = hc32 if w == 32 else hc64
        compare_request(got_c, hr, off, count, want_c, want_r, "%s inst %d (n=%d e=%d k=%d)" % (label, iid, n, e, k0))


def _positions(ctx, ids):
    return [ctx.get_state(i)[3] for i in ids]


@pytest.mark.parametrize("mode", [0, 1])
def test_single_instance_million_draws(ph, ctx, orc, tabs, mode):
    """One seeded 32-bit instance, 10^6 draws from position 0."""
    ids = ctx.seed_instances(32, SEED0 + mode, 1, (9, 17), 0, 0)
    specs = [(int(ids[0]), 10 ** 6)]
    starts = _positions(ctx, ids)
    host, offs = _run(ph, ctx, specs, mode=mode)
    _check(orc, tabs, ctx, specs, starts, host, offs, "A mode%d" % mode)
    assert ctx.get_state(int(ids[0]))[3] == 10 ** 6


@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_requests_random_starts(ph, ctx, orc, tabs, mode):
    rng = random.Random(100 + mode)
    ids = ctx.seed_instances(32, SEED0 + 10 + mode, 40, (9, 17), 0, 1 << 40)
    counts = [rng.choice([1, 2, 63, 64, 65, 2047, 2048, 2049, 4096, 6143]) if i % 3 == 0 else rng.randrange(1, 9000)
              for i in range(40)]
    specs = list(zip([int(x) for x in ids], counts))
    starts = _positions(ctx, ids)
    host, offs = _run(ph, ctx, specs, mode=mode, gap=5, shuffle_seed=mode)
    _check(orc, tabs, ctx, specs, starts, host, offs, "ragged")


@pytest.mark.parametrize("mode", [0, 1])
def test_requests_across_the_skip_period_boundary(ph, ctx, orc, tabs, mode):
    p = 2147483647
    n_arr, e_arr, _ = orc.seed(32, SEED0 + 20 + mode, 8, (9, 17))
    ks = [(p - 1) - 1, (p - 1) - 3000, 5 * (p - 1) - 2047, 7 * (p - 1), 3 * (p - 1) - 2046, (p - 1) + 1,
          11 * (p - 1) - 4095, 2 * (p - 1) - 2048]
    ids = ctx.add_instances(32, n_arr, e_arr, k0=ks)
    specs = [(int(i), 6000) for i in ids]
    host, offs = _run(ph, ctx, specs, mode=mode)
    _check(orc, tabs, ctx, specs, ks, host, offs, "period")


def test_same_instance_in_several_requests(ph, ctx, orc, tabs):
    ids = ctx.seed_instances(32, SEED0 + 30, 2, (9, 17), 0, 1 << 33)
    a, b = int(ids[0]), int(ids[1])
    k_a, k_b = _positions(ctx, ids)
    specs = [(a, 1000), (b, 3000), (a, 5000), (a, 1), (b, 2048)]
    host, offs = _run(ph, ctx, specs)
    starts = [k_a, k_b, k_a + 1000, k_a + 6000, k_b + 3000]
    _check(orc, tabs, ctx, specs, starts, host, offs, "continuation")
    assert _positions(ctx, [a, b]) == [k_a + 6001, k_b + 5048]


@pytest.mark.parametrize("mode", [0, 1])
def test_plan_groups_ragged_and_empty(ph, ctx, orc, tabs, mode):
    """700 requests, planned in groups of 256, 256 and a ragged 188: the
    whole second group asks for nothing, empty requests are scattered through
    the others, and every instance appears twice, the second time in a later
    group, so that positions carry across groups.  Nothing outside the
    requested ranges is written."""
    rng = random.Random(300 + mode)
    ids = [int(x) for x in ctx.seed_instances(32, SEED0 + 300 + mode, 350, (9, 17), 0, 1 << 40)]
    pos = dict(zip(ids, _positions(ctx, ids)))
    order = ids + ids[::-1]
    counts = []
    for j in range(len(order)):
        if 256 <= j < 512:
            counts.append(0)
        elif j % 7 == 0:
            counts.append(rng.choice([0, 1, 2047, 2048, 2049]))
        else:
            counts.append(rng.randrange(1, 5000))
    specs = list(zip(order, counts))
    starts = []
    for iid, c in specs:
        starts.append(pos[iid])
        pos[iid] += c
    host, offs = _run(ph, ctx, specs, mode=mode, gap=3)
    keep = [i for i, c in enumerate(counts) if c > 0]
    _check(orc, tabs, ctx, [specs[i] for i in keep], [starts[i] for i in keep], host, [offs[i] for i in keep],
           "plan groups")
    assert _positions(ctx, ids) == [pos[i] for i in ids]
    covered = np.zeros(host[2].size, dtype=bool)
    for (iid, c), off in zip(specs, offs):
        covered[off:off + c] = True
    assert np.all(host[0][~covered] == np.uint32(0xffffffff))
    assert np.all(host[2][~covered] == -1.0)


def test_exponents_fixed_and_generic_chains(ph, ctx, orc, tabs):
    rng = random.Random(7)
    ns, es = [], []
    wanted = [3, 5, 7, 9, 11, 13, 17, 65537, 19, 23]
    for ew in wanted:
        while True:
            n = rng.randrange(1 << 31, 1 << 32) | 1
            if orc.check_instance(32, n, ew) == 0:
                break
        ns.append(n)
        es.append(ew)
    # a large exponent (generic chain over 31 bits)
    n = 4294967087
    e_big = next(x for x in range(2 ** 31 + 1, 2 ** 31 + 1000, 2) if math.gcd(x, n - 1) == 1)
    ns.append(n)
    es.append(e_big)
    ks = [rng.randrange(0, 1 << 40) for _ in ns]
    ids = ctx.add_instances(32, ns, es, k0=ks)
    specs = [(int(i), 5000) for i in ids]
    host, offs = _run(ph, ctx, specs)
    _check(orc, tabs, ctx, specs, ks, host, offs, "exponents")


@pytest.mark.parametrize("mode", [0, 1])
def test_64bit_instances(ph, ctx, orc, tabs, mode):
    rng = random.Random(200 + mode)
    n_arr, e_arr, k_arr = orc.seed(64, SEED0 + 40 + mode, 12, (3, 5, 9, 17, 7), 0, 1 << 28)
    ids = ctx.add_instances(64, n_arr, e_arr, k0=k_arr)
    counts = [rng.choice([1, 2047, 2049, 30000, rng.randrange(1, 20000)]) for _ in ids]
    specs = list(zip([int(i) for i in ids], counts))
    host, offs = _run(ph, ctx, specs, mode=mode, want=(False, True, True), gap=3)
    _check(orc, tabs, ctx, specs, [int(k) for k in k_arr], host, offs, "w64")


def test_mixed_width_batch(ph, ctx, orc, tabs):
    rng = random.Random(300)
    n64, e64, k64 = orc.seed(64, SEED0 + 50, 10, (9, 17), 0, 1 << 27)
    n32, e32, k32 = orc.seed(32, SEED0 + 51, 10, (9, 17), 0, 1 << 40)
    i64 = ctx.add_instances(64, n64, e64, k0=k64)
    i32 = ctx.add_instances(32, n32, e32, k0=k32)
    specs, starts = [], []
    for a, b, ka, kb in zip(i64, i32, k64, k32):
        specs += [(int(b), rng.randrange(1, 12000)), (int(a), rng.randrange(1, 12000))]
        starts += [int(kb), int(ka)]
    host, offs = _run(ph, ctx, specs, shuffle_seed=3)
    _check(orc, tabs, ctx, specs, starts, host, offs, "mixed")


@pytest.mark.parametrize("want", [(True, False, False), (False, False, True), (False, True, False)])
def test_optional_outputs(ph, ctx, orc, tabs, want):
    n32, e32, k32 = orc.seed(32, SEED0 + 60, 3, (9, 17), 0, 1 << 40)
    n64, e64, k64 = orc.seed(64, SEED0 + 61, 3, (9, 17), 0, 1 << 20)
    ids = list(ctx.add_instances(32, n32, e32, k0=k32)) + list(ctx.add_instances(64, n64, e64, k0=k64))
    starts = [int(k) for k in k32] + [int(k) for k in k64]
    specs = [(int(i), 3000) for i in ids]
    (hc32, hc64, hr), offs = _run(ph, ctx, specs, want=want)
    for (iid, count), k0, off in zip(specs, starts, offs):
        n, e, p, a, w = ctx.get_params(iid)
        wc, wr, _ = oracle_draws(orc, tabs, w, n, e, k0, count)
        gc = hc32 if w == 32 else hc64
        compare_request(gc, hr, off, count, wc, wr, "optional")
    # an array that was not requested stays untouched (width-32 c in c64 etc.)
    if hc64 is not None:
        assert (hc64[offs[0]:offs[0] + 3000] == np.uint64(2 ** 64 - 1)).all()


def test_start_from_supplied_m0_s0(ph, ctx, orc, tabs):
    rng = random.Random(400)
    n32, e32, _ = orc.seed(32, SEED0 + 70, 6, (9, 17))
    p32, a32 = orc.lcg_params(32)
    m0 = [rng.randrange(int(n)) for n in n32]
    s0 = [rng.randrange(1, p32) for _ in n32]
    k0 = [rng.randrange(0, 300000) for _ in n32]
    ids = ctx.add_instances(32, n32, e32, m0=m0, s0=s0, k0=k0)
    n64, e64, _ = orc.seed(64, SEED0 + 71, 4, (9, 17))
    p64, a64 = orc.lcg_params(64)
    t64 = [rng.randrange(0, 1 << 24) for _ in n64]
    s064 = [pow(a64, t, p64) for t in t64]
    m064 = [rng.randrange(int(n)) for n in n64]
    k064 = [rng.randrange(0, 100000) for _ in n64]
    ids64 = ctx.add_instances(64, n64, e64, m0=m064, s0=s064, k0=k064)
    specs = [(int(i), 4000) for i in list(ids) + list(ids64)]
    (hc32, hc64, hr), offs = _run(ph, ctx, specs)
    allp = list(zip(n32, e32, m0, s0, k0)) + list(zip(n64, e64, m064, s064, k064))
    for (iid, count), (n, e, mm, ss, kk), off in zip(specs, allp, offs):
        w = 32 if int(n) < 2 ** 32 else 64
        wc, wr, _ = oracle_draws(orc, tabs, w, int(n), int(e), kk, count, m0=mm, s0=ss)
        compare_request(hc32 if w == 32 else hc64, hr, off, count, wc, wr, "m0s0")
        # get_state reports the supplied start, advanced by the draws
        st = ctx.get_state(iid)
        assert st[3] == kk + count


def test_state_get_set_and_jumps(ph, ctx, orc, tabs):
    rng = random.Random(500)
    n32, e32, k32 = orc.seed(32, SEED0 + 80, 4, (9, 17), 0, 1 << 40)
    ids = ctx.add_instances(32, n32, e32, k0=k32)
    p, a = orc.lcg_params(32)
    for iid, n, e, k in zip(ids, n32, e32, k32):
        iid, n, e, k = int(iid), int(n), int(e), int(k)
        # state reported at the start position equals eq. (7)
        m, s, c, kk = ctx.get_state(iid)
        assert kk == k
        assert (m, s) == orc.position(tabs[32], p, a, n, 0, 1, k)
        assert c == orc.encrypt(m, e, n)
        # forward and backward jumps
        d = rng.randrange(1, 10 ** 6)
        ctx.jump(iid, d)
        assert ctx.get_state(iid)[:2] == orc.position(tabs[32], p, a, n, 0, 1, k + d)
        ctx.jump(iid, -d - 5)
        assert ctx.get_state(iid)[:2] == orc.position(tabs[32], p, a, n, 0, 1, k - 5)
        # restore an arbitrary state, then draw: equals the oracle stepping from it
        m1, s1, k1 = rng.randrange(n), rng.randrange(1, p), rng.randrange(0, 1 << 50)
        ctx.set_state(iid, m1, s1, k1)
        assert ctx.get_state(iid)[:2] == (m1, s1) and ctx.get_state(iid)[3] == k1
        (hc32, _, hr), offs = _run(ph, ctx, [(iid, 7000)])
        cc, rr, (m2, s2) = oracle_draws(orc, tabs, 32, n, e, 0, 7000, m0=m1, s0=s1)
        compare_request(hc32, hr, 0, 7000, cc, rr, "restored")
        st = ctx.get_state(iid)
        assert (st[0], st[1], st[3]) == (m2, s2, k1 + 7000)
    # 64-bit: restore to any state (m, s): small and arbitrary skip logarithms
    n64, e64, _ = orc.seed(64, SEED0 + 81, 2, (9, 17))
    ids64 = ctx.add_instances(64, n64, e64)
    p64, a64 = orc.lcg_params(64)
    for iid, n, e in zip(ids64, n64, e64):
        iid, n, e = int(iid), int(n), int(e)
        for s1, k1 in ((pow(a64, rng.randrange(0, 1 << 26), p64), 12345), (rng.randrange(2, p64), (1 << 63) + 5)):
            m1 = rng.randrange(n)
            ctx.set_state(iid, m1, s1, k1)
            assert ctx.get_state(iid) == (m1, s1, orc.encrypt(m1, e, n), k1)
            (_, hc64, hr), _ = _run(ph, ctx, [(iid, 3000)])
            cc, rr, (m2, s2) = oracle_draws(orc, tabs, 64, n, e, 0, 3000, m0=m1, s0=s1)
            compare_request(hc64, hr, 0, 3000, cc, rr, "restored64")
            assert ctx.get_state(iid) == (m2, s2, orc.encrypt(m2, e, n), k1 + 3000)


def test_graph_replays_continue_streams(ph, ctx, orc, tabs):
    import torch
    n32, e32, k32 = orc.seed(32, SEED0 + 90, 6, (9, 17), 0, 1 << 40)
    n64, e64, k64 = orc.seed(64, SEED0 + 91, 2, (9, 17), 0, 1 << 22)
    ids = list(ctx.add_instances(32, n32, e32, k0=k32)) + list(ctx.add_instances(64, n64, e64, k0=k64))
    starts = [int(k) for k in k32] + [int(k) for k in k64]
    count = 5000
    offs = [i * count for i in range(len(ids))]
    total = count * len(ids)
    c32, c64, r = alloc_outputs(total)
    reqs = ph.make_requests(ids, [count] * len(ids), offs)
    g = ctx.graph(reqs, c32, c64, r)
    scratch = torch.zeros(1 << 20, device="cuda:0")
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        hc32, hc64, hr = to_host(c32, c64, r)
        for iid, k0, off in zip(ids, starts, offs):
            n, e, p, a, w = ctx.get_params(int(iid))
            wc, wr, _ = oracle_draws(orc, tabs, w, n, e, k0 + rep * count, count)
            compare_request(hc32 if w == 32 else hc64, hr, off, count, wc, wr, "graph rep %d" % rep)
            assert ctx.get_state(int(iid))[3] == k0 + (rep + 1) * count
        scratch.add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
    g.close()


def test_tuning_does_not_change_results(ph, ctx):
    import torch
    ids = ctx.seed_instances(32, SEED0 + 100, 16, (9, 17, 5), 0, 1 << 40)
    ids64 = ctx.seed_instances(64, SEED0 + 101, 4, (9, 17, 3), 0, 1 << 24)
    allid = [int(i) for i in ids] + [int(i) for i in ids64]
    saved = [ctx.get_state(i) for i in allid]
    counts = [(i * 7919) % 20000 + 1 for i in range(len(allid))]
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    total = int(sum(counts))
    ref = None
    orig = ctx.get_tuning()
    for bt, bpc, tpc, un in [(256, 4, 4, 2), (64, 8, 1, 1), (512, 1, 16, 4), (128, 2, 64, 2)]:
        for i, st in zip(allid, saved):
            ctx.set_state(i, st[0], st[1], st[3])
        ctx.set_tuning(bt, bpc, tpc, un)
        outs = alloc_outputs(total)
        ctx.generate(ph.make_requests(allid, counts, offs), *outs)
        torch.cuda.synchronize()
        if ref is None:
            ref = outs
        else:
            for x, y in zip(ref, outs):
                assert torch.equal(x, y)
    ctx.set_tuning(**orig)


def test_timing_off_and_on(ph, ctx):
    """With per-call timing off the draws are the same, last_kernel_ms
    refuses, and the running totals count only the timed calls."""
    import torch
    ids = [int(i) for i in ctx.seed_instances(32, SEED0 + 110, 3, (9, 17), 0, 1 << 40)]
    ids += [int(i) for i in ctx.seed_instances(64, SEED0 + 111, 2, (9, 17), 0, 1 << 24)]
    saved = [ctx.get_state(i) for i in ids]
    counts = [5000, 1, 20000, 3000, 9000]
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    reqs = ph.make_requests(ids, counts, offs)
    total = int(sum(counts))
    outs = []
    try:
        for on in (False, True):
            for i, st in zip(ids, saved):
                ctx.set_state(i, st[0], st[1], st[3])
            ctx.set_timing(on)
            ctx.timing_reset()
            o = alloc_outputs(total)
            for _ in range(3):
                ctx.generate(reqs, *o)  # three calls in a row; the arrays keep the third
            torch.cuda.synchronize()
            outs.append(o)
            _, calls = ctx.timing_read()
            if on:
                assert calls == 3 and ctx.last_kernel_ms() > 0.0
            else:
                assert calls == 0
                with pytest.raises(ph.PhprngError):
                    ctx.last_kernel_ms()
    finally:
        ctx.set_timing(True)
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_rejected_calls_change_nothing(ph, ctx):
    import torch
    ids = ctx.seed_instances(32, SEED0 + 110, 2, (9, 17), 0, 1 << 40)
    before = [ctx.get_state(int(i)) for i in ids]
    c32, c64, r = alloc_outputs(100)
    with pytest.raises(ph.PhprngError) as ex:
        ctx.generate(ph.make_requests([int(ids[0]), int(ids[1])], [50, 60], [0, 50]), c32, c64, r, capacity=100)
    assert ex.value.status == ph.PHPRNG_E_RANGE
    with pytest.raises(ph.PhprngError) as ex:
        ctx.generate(ph.make_requests([int(ids[0]), 10 ** 7], [5, 5], [0, 5]), c32, c64, r, capacity=100)
    assert ex.value.status == ph.PHPRNG_E_INVALID
    assert [ctx.get_state(int(i)) for i in ids] == before
    torch.cuda.synchronize()
    assert (c32.cpu() == -1).all()
    with pytest.raises(ph.PhprngError):
        ctx.add_instances(32, [4294967087, 4294967089], [9, 9])  # second modulus composite
    with pytest.raises(ph.PhprngError):
        ctx.jump(int(ids[0]), -(before[0][3] + 1))
    assert [ctx.get_state(int(i)) for i in ids] == before


def test_many_short_log_uniform_streams(ph, orc, tabs):
    """65,536 32-bit instances with short log-uniform lengths in [2^4, 2^12]
    (mostly one or two ragged tiles each, unlike the full-size log-uniform
    workload of test_gpu_fullsize.py), random starts in [0, 2^40), one
    persistent launch; a seeded 1% of the streams is compared in full."""
    import torch
    ctx = ph.Context(0, max_instances=1 << 16)
    nin = 1 << 16
    n, e, k = orc.seed(32, SEED0 + 2, nin, (9, 17), 0, 1 << 40)
    ids = ctx.add_instances(32, n, e, k0=k)
    rng = np.random.default_rng(SEED0 + 2)
    lens = np.floor(2.0 ** (4 + 8 * rng.random(nin))).astype(np.uint64)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    total = int(lens.sum())
    c32, _, r = alloc_outputs(total, True, False, True)
    ctx.generate(ph.make_requests(ids, lens, offs), c32, None, r)
    hc32, _, hr = to_host(c32, None, r)
    sample = rng.choice(nin, size=nin // 100, replace=False)
    p, a = orc.lcg_params(32)
    ms, ss = [], []
    for i in sample:
        m, s = orc.position(tabs[32], p, a, int(n[i]), 0, 1, int(k[i]))
        ms.append(m)
        ss.append(s)
    wc, wr, _, _, woff = orc.generate_many(p, a, n[sample], e[sample], np.array(ms, dtype=np.uint64),
                                           np.array(ss, dtype=np.uint64), lens[sample])
    for j, i in enumerate(sample):
        o, L, wo = int(offs[i]), int(lens[i]), int(woff[j])
        compare_request(hc32, hr, o, L, wc[wo:wo + L], wr[wo:wo + L], "logu %d" % i)
    ctx.close()


def _cskip_expected(orc, n, e, b, m0, k, count):
    m = orc.cskip_message(n, m0, b, k)
    c, r, _ = orc.generate_cskip(n, e, b, m, count)
    return c, r


@pytest.mark.parametrize("mode", [0, 1])
def test_constant_and_unit_skip_instances(ph, ctx, orc, tabs, mode):
    """Instances on the constant-skip schedule (unit skip b = 1 included),
    both widths, mixed with pseudorandom-skip instances in one batch."""
    rng = random.Random(800 + mode)
    n32, e32, _ = orc.seed(32, SEED0 + 120 + mode, 6, (9, 17, 3, 5))
    n64, e64, _ = orc.seed(64, SEED0 + 122 + mode, 4, (9, 17, 3))
    b32 = [1, 2] + [rng.randrange(1, int(n)) for n in n32[2:]]
    b64 = [1] + [rng.randrange(1, int(n)) for n in n64[1:]]
    m32 = [0, 5] + [rng.randrange(int(n)) for n in n32[2:]]
    m64 = [rng.randrange(int(n)) for n in n64]
    k32 = [0, 1, (1 << 63) + 12345, rng.randrange(1 << 62), 2 ** 32 - 1, rng.randrange(1 << 40)]
    k64 = [0, (1 << 63) - 7, rng.randrange(1 << 50), 123]
    i32 = ctx.add_instances_skip(32, n32, e32, b32, m0=m32, k0=k32)
    i64 = ctx.add_instances_skip(64, n64, e64, b64, m0=m64, k0=k64)
    nl, el, kl = orc.seed(32, SEED0 + 124 + mode, 3, (9, 17), 0, 1 << 40)
    il = ctx.add_instances(32, nl, el, k0=kl)
    ids = [int(i) for i in i32] + [int(i) for i in i64] + [int(i) for i in il]
    counts = [rng.choice([1, 2047, 2048, 2049, 7000, rng.randrange(1, 9000)]) for _ in ids]
    specs = list(zip(ids, counts))
    (hc32, hc64, hr), offs = _run(ph, ctx, specs, mode=mode, gap=2, shuffle_seed=mode)
    allp = ([(32, int(n), int(e), b, m, k) for n, e, b, m, k in zip(n32, e32, b32, m32, k32)] +
            [(64, int(n), int(e), b, m, k) for n, e, b, m, k in zip(n64, e64, b64, m64, k64)])
    for (iid, count), off, (w, n, e, b, m0, k) in zip(specs, offs, allp):
        assert ctx.get_schedule(iid) == (1, b)
        wc, wr = _cskip_expected(orc, n, e, b, m0, k, count)
        compare_request(hc32 if w == 32 else hc64, hr, off, count, wc, wr, "cskip w%d b=%d" % (w, b))
        # state after the draws
        m, s, c, kk = ctx.get_state(iid)
        assert (m, s, kk) == (orc.cskip_message(n, m0, b, k + count), b, k + count)
        assert c == orc.encrypt(m, e, n)
    _check(orc, tabs, ctx, specs[len(allp):], [int(k) for k in kl], (hc32, hc64, hr), offs[len(allp):], "lcg-mix")
    # restore and jump on a constant-skip instance
    iid, (w, n, e, b, m0, k) = ids[3], allp[3]
    ctx.set_state(iid, 77, b, 10 ** 12)
    ctx.jump(iid, -1000)
    (hc32, _, hr), _ = _run(ph, ctx, [(iid, 5000)])
    m_start = (77 - 1000 * b) % n
    wc, wr = _cskip_expected(orc, n, e, b, m_start, 0, 5000)
    compare_request(hc32, hr, 0, 5000, wc, wr, "cskip restored")
    with pytest.raises(ph.PhprngError):
        ctx.set_state(iid, 1, b + 1 if b + 1 < n else 1, 0)


@pytest.mark.parametrize("width,count,es,klo,khi", [(32, 5000, (9, 17), 0, 1 << 40), (64, 1500, (9, 17, 3), 0, 1 << 30),
                                                     (32, 2048, (3, 5, 7), 5, 6), (64, 1024, (17,), 0, 0)])
def test_device_seeding_matches_oracle_draw(ph, orc, tabs, width, count, es, klo, khi):
    """Large seeding calls decide primality and build records on the device;
    the drawn (n, e, k) must equal the oracle's SplitMix64 draw, and the
    records must generate the oracle's streams."""
    seed = SEED0 + 900 + width + count
    c = ph.Context(0, max_instances=count)
    ids = c.seed_instances(width, seed, count, es, klo, khi)
    n_o, e_o, k_o = orc.seed(width, seed, count, es, klo, khi)
    got = np.array([c.get_params(int(i))[:2] for i in ids], dtype=np.uint64)
    assert np.array_equal(got[:, 0], n_o) and np.array_equal(got[:, 1], e_o)
    assert [c.get_position(int(i)) for i in ids] == [int(x) for x in k_o]
    rng = random.Random(count)
    pick = rng.sample(range(count), 12)
    specs = [(int(ids[i]), 3000) for i in pick]
    (hc32, hc64, hr), offs = _run(ph, c, specs)
    for (iid, cnt), i, off in zip(specs, pick, offs):
        wc, wr, _ = oracle_draws(orc, tabs, width, int(n_o[i]), int(e_o[i]), int(k_o[i]), cnt)
        compare_request(hc32 if width == 32 else hc64, hr, off, cnt, wc, wr, "device-seeded")
    c.close()


def test_64bit_positions_from_any_state(ph, ctx, orc, tabs):
    """Width-64 starts that the old skip-index bound could not reach: whole
    skip periods plus a table offset (q p(p-1)/2 of eq. (7)), an arbitrary
    supplied s0 (its skip log is ~2^60) moved on the device by millions of
    draws, a start one short of a whole period from such an s0 (summed as
    the complement), a request whose skip log crosses 2^34, a table start,
    and a move that is too far from both, which is refused."""
    rng = random.Random(1500)
    p, a = orc.lcg_params(64)
    n64, e64, _ = orc.seed(64, SEED0 + 150, 6, (9, 17, 3))
    n64, e64 = [int(x) for x in n64], [int(x) for x in e64]
    b_full = lambda n: (p * (p - 1) // 2) % n
    cases = []
    # (a) s0 = 1, k0 = 5 (p - 1) + 12345: the table plus five whole periods
    cases.append(dict(m0=0, s0=1, k0=5 * (p - 1) + 12345))
    # (b) arbitrary s0, k0 = 3e6 + 777: the skips are summed on the device
    cases.append(dict(m0=rng.randrange(n64[1]), s0=rng.randrange(2, p), k0=3 * 10 ** 6 + 777))
    # (c) arbitrary s0, k0 = (p - 1) - 2^20 - 3: a whole period less 2^20 + 3 draws
    cases.append(dict(m0=rng.randrange(n64[2]), s0=rng.randrange(2, p), k0=(p - 1) - (1 << 20) - 3))
    # (d) s0 = a^(2^34 - 1000): generation crosses skip log 2^34
    cases.append(dict(m0=rng.randrange(n64[3]), s0=pow(a, (1 << 34) - 1000, p), k0=0))
    # (e) s0 = 1, k0 = 2^26 + 5: positioned from the table
    cases.append(dict(m0=0, s0=1, k0=(1 << 26) + 5))
    ids = []
    for i, cs in enumerate(cases):
        ids += [int(x) for x in ctx.add_instances(64, [n64[i]], [e64[i]], m0=[cs["m0"]], s0=[cs["s0"]],
                                                  k0=[cs["k0"]])]
    specs = [(iid, 5000) for iid in ids]
    (_, hc64, hr), offs = _run(ph, ctx, specs, want=(False, True, True))
    for i, (cs, iid, off) in enumerate(zip(cases, ids, offs)):
        n, e = n64[i], e64[i]
        k0, m0, s0 = cs["k0"], cs["m0"], cs["s0"]
        if i == 2:
            # one whole period from (m0, s0) is (m0 + p(p-1)/2, s0); then back 2^20 + 3
            m, s = orc.jump_backward(p, a, n, (m0 + b_full(n)) % n, s0, (p - 1) - k0)
        else:
            m, s = orc.position(tabs[64] if s0 == 1 else None, p, a, n, m0, s0, k0)
        assert ctx.get_state(iid)[3] == k0 + 5000
        wc, wr, _, _ = orc.generate(p, a, n, e, m, s, 5000)
        compare_request(hc64, hr, off, 5000, wc, wr, "w64 start case %d" % i)
    # (f) too far from both the table and a whole period: refused, nothing added
    before = ctx.instance_count()
    with pytest.raises(ph.PhprngError) as ex:
        ctx.add_instances(64, [n64[5]], [e64[5]], s0=[rng.randrange(2, p)], k0=[1 << 50])
    assert ex.value.status == ph.PHPRNG_E_RANGE
    assert ctx.instance_count() == before


def test_64bit_jumps_on_each_path(ph, ctx, orc, tabs):
    """Forward and backward width-64 jumps from small and arbitrary skip
    logs: on the table, summed on the device, and as the complement of a
    whole period; each state checked against the oracle stepping."""
    rng = random.Random(1600)
    p, a = orc.lcg_params(64)
    n64, e64, _ = orc.seed(64, SEED0 + 160, 3, (9, 17))
    for j, (n, e) in enumerate(zip(n64, e64)):
        n, e = int(n), int(e)
        m0 = rng.randrange(n)
        s0 = 1 if j == 0 else rng.randrange(2, p)
        iid = int(ctx.add_instances(64, [n], [e], m0=[m0], s0=[s0])[0])
        m, s, k = m0, s0, 0
        for d in (1, 2047, 1 << 20, 3 * 10 ** 6 + 5, -(10 ** 6), -(1 << 21) - 1, 777):
            ctx.jump(iid, d)
            if d >= 0:
                m, s = orc.jump_forward(p, a, n, m, s, d)
            else:
                m, s = orc.jump_backward(p, a, n, m, s, -d)
            k += d
            assert ctx.get_state(iid) == (m, s, orc.encrypt(m, e, n), k), (j, d)
        # a whole period less 5000 forward: the complement path
        d = (p - 1) - 5000
        ctx.jump(iid, d)
        m, s = orc.jump_backward(p, a, n, (m + (p * (p - 1) // 2)) % n, s, 5000)
        k += d
        assert ctx.get_state(iid) == (m, s, orc.encrypt(m, e, n), k)
        # and back again
        ctx.jump(iid, -d)
        m, s = orc.jump_forward(p, a, n, (m - (p * (p - 1) // 2)) % n, s, 5000)
        k -= d
        assert ctx.get_state(iid) == (m, s, orc.encrypt(m, e, n), k)
        # draws continue from the jumped state
        (_, hc64, hr), _ = _run(ph, ctx, [(iid, 4000)], want=(False, True, True))
        wc, wr, _, _ = orc.generate(p, a, n, e, m, s, 4000)
        compare_request(hc64, hr, 0, 4000, wc, wr, "w64 after jumps %d" % j)


def test_graph_replays_interleaved_with_other_calls(ph, ctx, orc, tabs):
    """Between graph replays the same instances are drawn by generate,
    jumped and restored; every replay continues from where the instances
    then are, for both widths."""
    import torch
    n32, e32, k32 = orc.seed(32, SEED0 + 170, 3, (9, 17), 0, 1 << 40)
    n64, e64, k64 = orc.seed(64, SEED0 + 171, 2, (9, 17), 0, 1 << 22)
    ids = [int(x) for x in ctx.add_instances(32, n32, e32, k0=k32)] + \
          [int(x) for x in ctx.add_instances(64, n64, e64, k0=k64)]
    count = 3000
    offs = [i * count for i in range(len(ids))]
    c32, c64, r = alloc_outputs(count * len(ids))
    g = ctx.graph(ph.make_requests(ids, [count] * len(ids), offs), c32, c64, r)
    p32, a32 = orc.lcg_params(32)
    p64, a64 = orc.lcg_params(64)
    rng = random.Random(1700)

    def check(label):
        torch.cuda.synchronize()
        hc32, hc64, hr = to_host(c32, c64, r)
        for iid, off in zip(ids, offs):
            n, e, p, a, w = ctx.get_params(iid)
            m, s, _, k = expect[iid]
            wc, wr, m2, s2 = orc.generate(p, a, n, e, m, s, count)
            compare_request(hc32 if w == 32 else hc64, hr, off, count, wc, wr, label)
            expect[iid] = (m2, s2, None, k + count)

    expect = {iid: ctx.get_state(iid) for iid in ids}
    g.launch()
    check("replay 1")
    # generate on the same instances, then replay
    hc = _run(ph, ctx, [(iid, 1111) for iid in ids])
    for iid in ids:
        n, e, p, a, w = ctx.get_params(iid)
        m, s, _, k = expect[iid]
        _, _, m2, s2 = orc.generate(p, a, n, e, m, s, 1111)
        expect[iid] = (m2, s2, None, k + 1111)
    g.launch()
    check("replay after generate")
    # jumps both ways and a restore, then replay twice
    for iid in ids:
        n, e, p, a, w = ctx.get_params(iid)
        m, s, _, k = expect[iid]
        ctx.jump(iid, 5000)
        m, s = orc.jump_forward(p, a, n, m, s, 5000)
        ctx.jump(iid, -7000)
        m, s = orc.jump_backward(p, a, n, m, s, 7000)
        expect[iid] = (m, s, None, k - 2000)
    iid = ids[-1]
    n, e, p, a, w = ctx.get_params(iid)
    m1, s1 = rng.randrange(n), rng.randrange(2, p)
    ctx.set_state(iid, m1, s1, 999)
    expect[iid] = (m1, s1, None, 999)
    g.launch()
    check("replay after jumps")
    g.launch()
    check("second replay after jumps")
    for iid in ids:
        assert ctx.get_state(iid)[3] == expect[iid][3]
        assert ctx.get_state(iid)[:2] == expect[iid][:2]
    g.close()


@pytest.mark.parametrize("tiles", [3000, 20000, 45000])
def test_64bit_reduce_unit_sizes(ph, orc, tiles):
    """Width-64 batches whose tile totals make the reduce take units of 1, 2
    and 4 tiles (a batch takes the largest unit, up to 16 tiles, that still
    leaves 8192 units): ragged requests from arbitrary (m0, s0), eight
    instances asked twice in the batch (the second request continues the
    first), every draw compared with the oracle's stream."""
    rng = np.random.default_rng(SEED0 + 1700 + tiles)
    p, a = orc.lcg_params(64)
    ninst = 24
    n, e, _ = orc.seed(64, SEED0 + 1700 + tiles, ninst, (9, 17))
    n = [int(x) for x in n]
    m0 = [int(rng.integers(0, x)) for x in n]
    s0 = [int(rng.integers(2, p)) for _ in range(ninst)]
    c = ph.Context(0, max_instances=ninst)
    ids = [int(x) for x in c.add_instances(64, n, [int(x) for x in e], m0=m0, s0=s0)]
    inst_of_req = list(range(ninst)) + list(range(8))
    avg = tiles * 1024 // len(inst_of_req)
    counts = [int(x) for x in rng.integers(1, 2 * avg, len(inst_of_req))]
    counts[:4] = [1, 1023, 1024, 1025]
    specs = [(ids[i], cnt) for i, cnt in zip(inst_of_req, counts)]
    (_, hc64, hr), offs = _run(ph, c, specs, want=(False, True, True))
    per_inst = [0] * ninst
    for i, cnt in zip(inst_of_req, counts):
        per_inst[i] += cnt
    wc, wr, _, _, woff = orc.generate_many(p, a, np.array(n, dtype=np.uint64), np.array(e, dtype=np.uint64),
                                           np.array(m0, dtype=np.uint64), np.array(s0, dtype=np.uint64),
                                           np.array(per_inst, dtype=np.uint64))
    done = [0] * ninst
    for (iid, cnt), i, off in zip(specs, inst_of_req, offs):
        o = int(woff[i]) + done[i]
        compare_request(hc64, hr, off, cnt, wc[o:o + cnt], wr[o:o + cnt], "w64 reduce units, instance %d" % i)
        done[i] += cnt
    for i in range(ninst):
        assert c.get_position(ids[i]) == per_inst[i]
    c.close()


def test_64bit_table_tile_starts_and_mode_changes(ph, orc):
    """A width-64 instance whose draws in a batch all lie below the table's
    range takes its tile starts from the table (tiles at multiples of 1024
    skip logarithms, the first one entered part-way); an instance with a
    request that crosses the range end takes the reduce and scan, in the same
    batch as table instances.  Instances start at aligned and unaligned skip
    logarithms, one of them twice in a batch, one request is empty, one ends
    one draw before the range end; over four batches instances move from one
    way to the other, and every draw and the final states are compared with
    the oracle's continuing streams."""
    rng = np.random.default_rng(SEED0 + 1800)
    p, a = orc.lcg_params(64)
    n64, e64, _ = orc.seed(64, SEED0 + 1800, 7, (9, 17))
    n64 = [int(x) for x in n64]
    e64 = [int(x) for x in e64]
    top = 1 << 34
    logs = [0, 1, 1023, 1024, 12345, top - 5000, top - 1030]
    m0 = [0] + [int(rng.integers(0, n)) for n in n64[1:]]
    s0 = [pow(a, t, p) for t in logs]
    c = ph.Context(0, max_instances=16)
    ids = [int(x) for x in c.add_instances(64, n64, e64, m0=m0, s0=s0)]
    n32, e32, _ = orc.seed(32, SEED0 + 1801, 1, (9, 17))
    w32 = int(c.add_instances(32, [int(n32[0])], [int(e32[0])])[0])
    A, B, C, D, E, F, G = range(7)
    batches = [
        [(A, 3000), (B, 1), (C, 1), (C, 2048), (D, 1024), (E, 0), (E, 5000), (F, 4000), (G, 1000), (-1, 3000)],
        [(F, 3000), (A, 5000), (G, 29), (B, 1000), (-1, 100)],
        [(A, 4097), (B, 3000), (C, 100), (D, 777), (E, 2048)],
        [(F, 100), (A, 10)],
    ]
    done = [0] * 7
    got = {i: [] for i in range(7)}
    for batch in batches:
        specs = [(ids[i] if i >= 0 else w32, cnt) for i, cnt in batch]
        (_, hc64, hr), offs = _run(ph, c, specs, want=(False, True, True))
        for (i, cnt), off in zip(batch, offs):
            if i >= 0:
                got[i].append((done[i], hc64[off:off + cnt].copy(), hr[off:off + cnt].copy()))
                done[i] += cnt
    for i in range(7):
        wc, wr, wm, ws = orc.generate(p, a, n64[i], e64[i], m0[i], s0[i], done[i])
        for start, gc, gr in got[i]:
            cnt = gc.size
            compare_request(gc, gr, 0, cnt, wc[start:start + cnt], wr[start:start + cnt],
                            "w64 table/reduce instance %d draws %d..%d" % (i, start, start + cnt))
        m, s, _, k = c.get_state(ids[i])
        assert (m, s, k) == (int(wm), int(ws), done[i])
        assert s == pow(a, logs[i] + done[i], p)
    c.close()


def test_graph_replays_cross_the_table_range(ph, orc):
    """A captured graph over width-64 instances keeps up as replays carry
    one instance across skip logarithm 2^34 (table tile starts, then the
    reduce and scan from the replay that crosses it on) while another stays
    in range; every replay against the oracle's continuing streams."""
    import torch
    p, a = orc.lcg_params(64)
    n64, e64, _ = orc.seed(64, SEED0 + 1900, 2, (9, 17))
    n64, e64 = [int(x) for x in n64], [int(x) for x in e64]
    logs = [(1 << 34) - 2500, 777]
    m0 = [123456789 % n64[0], 42]
    s0 = [pow(a, t, p) for t in logs]
    c = ph.Context(0, max_instances=4)
    ids = [int(x) for x in c.add_instances(64, n64, e64, m0=m0, s0=s0)]
    count = 1000
    c64 = torch.full((2 * count,), -1, dtype=torch.int64, device="cuda:0")
    r = torch.full((2 * count,), -1.0, dtype=torch.float64, device="cuda:0")
    g = c.graph(ph.make_requests(ids, [count, count], [0, count]), None, c64, r)
    replays = 5
    streams = [orc.generate(p, a, n64[i], e64[i], m0[i], s0[i], replays * count) for i in range(2)]
    for k in range(replays):
        g.launch()
        torch.cuda.synchronize()
        hc64 = c64.cpu().numpy().view(np.uint64)
        hr = r.cpu().numpy()
        for i in range(2):
            wc, wr, _, _ = streams[i]
            compare_request(hc64, hr, i * count, count, wc[k * count:(k + 1) * count], wr[k * count:(k + 1) * count],
                            "graph replay %d instance %d" % (k, i))
    for i in range(2):
        _, _, wm, ws = streams[i]
        m, s, _, kk = c.get_state(ids[i])
        assert (m, s, kk) == (int(wm), int(ws), replays * count)
    g.close()
    c.close()
