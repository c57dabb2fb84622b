"""GPU parity on the method's edge cases, bit for bit against the oracle:

  - the cribs of Sec. II: messages 0, 1 and n - 1 encrypt to themselves, on
    unit-skip windows that run through n - 2, n - 1, 0, 1, 2 (both widths);
  - a message sum that wraps exactly at n (m + s = n gives m = 0, c = 0,
    R = 1/(n+1)) and the top message n - 1 under the pseudorandom skip;
  - R = 1.0 for the largest width-64 modulus below 2^63 (n = 2^63 - 25,
    c = n - 1): binary64(n) = binary64(n + 1) = 2^63, so the open interval
    of Sec. I closes at 1 for width 64;
  - the example instance of Sec. II from the base state: the draws, states
    and skip sums of tests/golden/crosscheck_values.json;
  - the autotuner: a legal shape, positions and width-64 messages restored,
    and the same draws with the tuned shape as with the default one;
  - positions at the top of the uint64 range: draws up to position 2^64 - 1
    for both widths, then one draw more refused;
  - width-64 moduli at both ends of [2^62, 2^63) with every exponent chain
    (3, 5, 9, 17, a generic small one, 65537 and one above 2^31), messages
    near n - 1, both launch forms: the Montgomery reduction's middle column
    carries out of 64 bits most often for the largest moduli.
"""

import json
import os
import random

import numpy as np
import pytest

from tests.gpu_helpers import alloc_outputs, compare_request, to_host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SEED0 = 0x14112484 + 3000


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


@pytest.fixture(scope="module")
def ctx(ph):
    c = ph.Context(0, max_instances=256)
    yield c
    c.close()


def _draw(ph, ctx, iid, count, want=(True, True, True)):
    c32, c64, r = alloc_outputs(count, *want)
    ctx.generate(ph.make_requests([iid], [count], [0]), c32, c64, r)
    return to_host(c32, c64, r)


def _admissible_exponent(orc, width, n, choices=(3, 5, 7, 9, 11, 13, 17, 19, 23)):
    return next(e for e in choices if orc.check_instance(width, n, e) == 0)


@pytest.mark.parametrize("width", [32, 64])
def test_unit_skip_windows_through_the_cribs(ph, ctx, orc, width):
    rng = random.Random(3001 + width)
    n_arr, _, _ = orc.seed(width, SEED0 + width, 3, (9, 17))
    for n in [int(x) for x in n_arr]:
        e = _admissible_exponent(orc, width, n)
        # messages n-2, n-1, 0, 1, 2, 3, ... (unit skip from m_0 = n - 3)
        iid = int(ctx.add_instances_skip(width, [n], [e], [1], m0=[n - 3])[0])
        hc32, hc64, hr = _draw(ph, ctx, iid, 2100)
        got_c = (hc32 if width == 32 else hc64).astype(np.uint64)
        wc, wr, _ = orc.generate_cskip(n, e, 1, n - 3, 2100)
        compare_request(got_c, hr, 0, 2100, wc, wr, "cribs w%d n=%d" % (width, n))
        # Sec. II: 0, 1 and n - 1 are fixed points of the cipher (e odd)
        assert [int(x) for x in got_c[1:4]] == [n - 1, 0, 1]
        assert hr[2] == 1.0 / float(n + 1)  # c = 0: R = 1/(n+1)
        # a window across the wrap starting at a random position
        k0 = rng.randrange(1 << 40)
        iid = int(ctx.add_instances_skip(width, [n], [e], [1], m0=[(n - 2 - k0) % n], k0=[k0])[0])
        hc32, hc64, hr = _draw(ph, ctx, iid, 5)
        got_c = (hc32 if width == 32 else hc64).astype(np.uint64)
        assert [int(x) for x in got_c] == [n - 1, 0, 1, pow(2, e, n), pow(3, e, n)]


@pytest.mark.parametrize("width", [32, 64])
def test_message_sum_wrapping_exactly_at_n(ph, ctx, orc, width):
    """States chosen so that the next skip lands the message exactly on n
    (m = 0) and, in a second instance, on n - 1."""
    rng = random.Random(3100 + width)
    p, a = orc.lcg_params(width)
    n_arr, e_arr, _ = orc.seed(width, SEED0 + 100 + width, 4, (9, 17))
    for n, e in zip([int(x) for x in n_arr], [int(x) for x in e_arr]):
        s = rng.randrange(1, p)
        s_next = a * s % p
        for target in (0, n - 1):
            m = (target - s_next) % n
            iid = int(ctx.add_instances(width, [n], [e], m0=[m], s0=[s])[0])
            hc32, hc64, hr = _draw(ph, ctx, iid, 3000)
            got_c = (hc32 if width == 32 else hc64).astype(np.uint64)
            wc, wr, _, _ = orc.generate(p, a, n, e, m, s, 3000)
            compare_request(got_c, hr, 0, 3000, wc, wr, "wrap w%d target %d" % (width, target))
            assert int(got_c[0]) == target  # 0 and n - 1 are fixed points
            if target == 0:
                assert hr[0] == 1.0 / float(n + 1)


def test_width64_uniform_reaches_one(ph, ctx, orc):
    n = (1 << 63) - 25
    assert orc.is_prime(n)
    e = _admissible_exponent(orc, 64, n)
    # unit skip: the first draw encrypts n - 1, a fixed point
    iid = int(ctx.add_instances_skip(64, [n], [e], [1], m0=[n - 2])[0])
    _, hc64, hr = _draw(ph, ctx, iid, 64, want=(False, True, True))
    assert int(hc64[0]) == n - 1 and hr[0] == 1.0
    wc, wr, _ = orc.generate_cskip(n, e, 1, n - 2, 64)
    compare_request(hc64, hr, 0, 64, wc, wr, "w64 R = 1")
    # pseudorandom skip: the message n - 1 after one draw, then a long stream
    # whose largest ciphertexts also round to 1.0
    p, a = orc.lcg_params(64)
    s = 123456789
    m = (n - 1 - a * s % p) % n
    iid = int(ctx.add_instances(64, [n], [e], m0=[m], s0=[s])[0])
    _, hc64, hr = _draw(ph, ctx, iid, 200000, want=(False, True, True))
    assert int(hc64[0]) == n - 1 and hr[0] == 1.0
    wc, wr, _, _ = orc.generate(p, a, n, e, m, s, 200000)
    compare_request(hc64, hr, 0, 200000, wc, wr, "w64 R = 1 stream")
    assert np.all(hr > 0.0) and np.all(hr <= 1.0)


def test_example_instance_crosscheck_values(ph, ctx, orc):
    with open(os.path.join(ROOT, "tests", "golden", "crosscheck_values.json")) as f:
        g = json.load(f)
    n, e = g["n"], g["e"]
    iid = int(ctx.add_instances(32, [n], [e])[0])
    hc32, _, hr = _draw(ph, ctx, iid, 10 ** 6, want=(True, False, True))
    for row in g["draws"]:
        k = row["k"]
        assert int(hc32[k - 1]) == row["c"], k
        assert hr[k - 1] == float.fromhex(row["R"]), k
    m, s, c, k = ctx.get_state(iid)
    last = g["draws"][-1]
    assert (m, s, c, k) == (last["m"], last["s"], last["c"], 10 ** 6)
    # eq. (7): position 10^6 directly, and one whole skip period later
    iid2 = int(ctx.add_instances(32, [n], [e], k0=[10 ** 6])[0])
    assert ctx.get_state(iid2)[:2] == (last["m"], last["s"])
    p = g["p"]
    iid3 = int(ctx.add_instances(32, [n], [e], k0=[10 ** 6 + (p - 1)])[0])
    assert ctx.get_state(iid3)[:2] == ((last["m"] + g["full_period_skip_sum_mod_n"]) % n, last["s"])


def test_autotune_shape_state_and_outputs(ph, orc):
    import torch
    c = ph.Context(0, max_instances=128)
    ids = [int(i) for i in c.seed_instances(32, SEED0 + 200, 48, (9, 17), 0, 1 << 40)]
    ids += [int(i) for i in c.seed_instances(64, SEED0 + 201, 16, (9, 17), 0, 1 << 24)]
    n, e, p, a, w = c.get_params(ids[-1])
    c.set_state(ids[-1], 12345 % n, 987654321, 7)
    before = [c.get_state(i) for i in ids]
    default = c.get_tuning_class(ph.PHPRNG_CLASS_MIXED)
    best = c.autotune(1 << 22)
    assert best["block_threads"] in (64, 128, 256, 512)
    assert 1 <= best["blocks_per_cu"] <= 64 and best["block_threads"] * best["blocks_per_cu"] <= 2048
    assert 1 <= best["tiles_per_chunk"] <= 64 and best["unroll"] in (1, 2, 4)
    assert c.get_tuning_class(ph.PHPRNG_CLASS_MIXED) == best
    assert [c.get_state(i) for i in ids] == before
    # same draws with the tuned and the default shape, equal to the oracle
    counts = [(i * 7919) % 30000 + 1 for i in range(len(ids))]
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.uint64)
    total = int(sum(counts))
    reqs = ph.make_requests(ids, counts, offs)
    outs_t = alloc_outputs(total)
    c.generate(reqs, *outs_t)
    for i, st in zip(ids, before):
        c.set_state(i, st[0], st[1], st[3])
    c.set_tuning_class(ph.PHPRNG_CLASS_MIXED, **default)
    outs_d = alloc_outputs(total)
    c.generate(reqs, *outs_d)
    torch.cuda.synchronize()
    for x, y in zip(outs_t, outs_d):
        assert torch.equal(x, y)
    hc32, hc64, hr = to_host(*outs_t)
    for iid, cnt, off, st in zip(ids, counts, offs, before):
        nn, ee, pp, aa, ww = c.get_params(iid)
        wc, wr, _, _ = orc.generate(pp, aa, nn, ee, st[0], st[1], cnt)
        compare_request(hc32 if ww == 32 else hc64, hr, int(off), cnt, wc, wr, "autotuned %d" % iid)
    # a second context on this device starts from the tuned shape
    c2 = ph.Context(0, max_instances=4)
    assert c2.get_tuning_class(ph.PHPRNG_CLASS_MIXED) == best
    c2.close()
    c.close()


def test_positions_at_the_top_of_the_uint64_range(ph, ctx, orc, tab32):
    """Positions use the whole uint64 range: a width-32 instance (eq. (7)
    over the whole skip period) and a width-64 unit-skip instance placed
    3000 draws below 2^64 draw up to the last position, 2^64 - 1, in two
    batches; one draw more is refused with nothing changed."""
    import torch
    top = (1 << 64) - 1
    k0 = top - 2999
    p, a = orc.lcg_params(32)
    n32, e32, _ = orc.seed(32, SEED0 + 400, 1, (9, 17))
    n32, e32 = int(n32[0]), int(e32[0])
    n64, e64, _ = orc.seed(64, SEED0 + 401, 1, (9, 17))
    n64, e64 = int(n64[0]), int(e64[0])
    i32 = int(ctx.add_instances(32, [n32], [e32], k0=[k0])[0])
    b, m0 = 987654321, 12345
    i64 = int(ctx.add_instances_skip(64, [n64], [e64], [b], m0=[m0], k0=[k0])[0])
    assert ctx.get_position(i32) == k0 and ctx.get_position(i64) == k0
    m32, s32 = orc.position(tab32, p, a, n32, 0, 1, k0)
    w32c, w32r, _, _ = orc.generate(p, a, n32, e32, m32, s32, 2999)
    w64c, w64r, _ = orc.generate_cskip(n64, e64, b, (m0 + k0 * b) % n64, 2999)
    done = 0
    for cnt in (2000, 999):
        c32, c64, r = alloc_outputs(2 * cnt)
        ctx.generate(ph.make_requests([i32, i64], [cnt, cnt], [0, cnt]), c32, c64, r)
        hc32, hc64, hr = to_host(c32, c64, r)
        compare_request(hc32, hr, 0, cnt, w32c[done:done + cnt], w32r[done:done + cnt], "w32 top")
        compare_request(hc64, hr, cnt, cnt, w64c[done:done + cnt], w64r[done:done + cnt], "w64 unit skip top")
        done += cnt
    assert ctx.get_position(i32) == top and ctx.get_position(i64) == top
    before = [ctx.get_state(i32), ctx.get_state(i64)]
    c32, c64, r = alloc_outputs(2)
    for iid in (i32, i64):
        with pytest.raises(ph.PhprngError) as ex:
            ctx.generate(ph.make_requests([iid], [1], [0]), c32, c64, r)
        assert ex.value.status == ph.PHPRNG_E_RANGE
    assert [ctx.get_state(i32), ctx.get_state(i64)] == before
    torch.cuda.synchronize()


def _primes_from(orc, start, step, count):
    out, n = [], start | 1
    while len(out) < count:
        if orc.is_prime(n):
            out.append(n)
        n += 2 * step
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_width64_moduli_at_the_range_ends(ph, ctx, orc, mode):
    rng = random.Random(3300 + mode)
    p, a = orc.lcg_params(64)
    low = _primes_from(orc, (1 << 62) + 1, 1, 3)
    high = _primes_from(orc, (1 << 63) - 1, -1, 3)
    exps = [3, 5, 9, 17, 7, 65537, (1 << 31) + 11]
    ns, es, ms, ss = [], [], [], []
    for i, n in enumerate(low + high):
        for e in exps[i % 2::2] + ([exps[-1]] if i % 2 else []):
            if orc.check_instance(64, n, e) != 0:
                continue
            s = rng.randrange(1, p)
            ns.append(n)
            es.append(e)
            ms.append(n - 1 - rng.randrange(0, 1 << 20))
            ss.append(s)
    assert {x for x in es} >= {3, 5, 9, 17}
    ids = [int(i) for i in ctx.add_instances(64, ns, es, m0=ms, s0=ss)]
    count = 3000
    reqs = ph.make_requests(ids, [count] * len(ids), np.arange(len(ids), dtype=np.uint64) * count)
    c32, c64, r = alloc_outputs(count * len(ids), False, True, True)
    ctx.generate(reqs, c32, c64, r, mode=mode)
    _, hc64, hr = to_host(c32, c64, r)
    for j, (n, e, m, s) in enumerate(zip(ns, es, ms, ss)):
        wc, wr, _, _ = orc.generate(p, a, n, e, m, s, count)
        lo = j * count
        compare_request(hc64[lo:lo + count], hr[lo:lo + count], 0, count, wc, wr,
                        "w64 n=%d e=%d mode %d" % (n, e, mode))
