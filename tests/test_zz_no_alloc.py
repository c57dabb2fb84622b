"""The allocation-free generation entry point against phprng_generate, through
the C ABI: two calls in a row (the second smaller) on instances of both
widths, each output compared bit for bit with what phprng_generate writes
from the same states, and with the oracle; the limits are refused with
nothing changed."""

import random

import numpy as np
import pytest

from tests.gpu_helpers import alloc_outputs, compare_request, to_host

pytestmark = pytest.mark.gpu

SEED0 = 0x14112484 + 2000


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


def _states(ctx, ids):
    return [ctx.get_state(i) for i in ids]


def _restore(ctx, ids, states):
    for i, st in zip(ids, states):
        ctx.set_state(i, st[0], st[1], st[3])


def _layout(specs, gap):
    offs, cur = [], 0
    for _, c in specs:
        offs.append(cur)
        cur += c + gap
    return offs, max(cur, 1)


def test_noalloc_matches_generate_twice(ph, orc):
    import torch
    ctx = ph.Context(0, max_instances=512)
    rng = random.Random(2001)
    ids = [int(i) for i in ctx.seed_instances(32, SEED0, 40, (9, 17, 5), 0, 1 << 40)]
    ids += [int(i) for i in ctx.seed_instances(64, SEED0 + 1, 12, (9, 17, 3), 0, 1 << 24)]
    # one width-64 instance restored to an arbitrary state
    n, e, p, a, w = ctx.get_params(ids[-1])
    ctx.set_state(ids[-1], rng.randrange(n), rng.randrange(2, p), 77)
    for call, (nreq, lo, hi) in enumerate(((300, 1, 9000), (37, 1, 3000))):
        # requests (some instances twice, so positions carry within the call)
        specs = [(rng.choice(ids), rng.randrange(lo, hi)) for _ in range(nreq)]
        specs[0] = (specs[0][0], 0)
        offs, total = _layout(specs, 3)
        reqs = ph.make_requests([s[0] for s in specs], [s[1] for s in specs], offs)
        before = _states(ctx, ids)
        a32, a64, ar = alloc_outputs(total)
        ctx.generate_noalloc(reqs, a32, a64, ar)
        after_noalloc = _states(ctx, ids)
        _restore(ctx, ids, before)
        b32, b64, br = alloc_outputs(total)
        ctx.generate(reqs, b32, b64, br)
        torch.cuda.synchronize()
        assert _states(ctx, ids) == after_noalloc, "call %d: positions differ" % call
        for x, y in ((a32, b32), (a64, b64), (ar, br)):
            assert torch.equal(x, y), "call %d: outputs differ from phprng_generate" % call
        # and both equal the oracle, request by request
        hc32, hc64, hr = to_host(a32, a64, ar)
        pos = {i: st for i, st in zip(ids, before)}
        for (iid, cnt), off in zip(specs, offs):
            n, e, p, a, w = ctx.get_params(iid)
            m, s, _, k = pos[iid]
            wc, wr, m2, s2 = orc.generate(p, a, n, e, m, s, cnt)
            compare_request(hc32 if w == 32 else hc64, hr, off, cnt, wc, wr, "noalloc call %d inst %d" % (call, iid))
            pos[iid] = (m2, s2, None, k + cnt)
    ctx.close()


def test_noalloc_limits_refused(ph):
    import torch
    ctx = ph.Context(0, max_instances=64)
    ids = [int(i) for i in ctx.seed_instances(32, SEED0 + 5, 4, (9, 17), 0, 0)]
    ids64 = [int(i) for i in ctx.seed_instances(64, SEED0 + 6, 2, (9, 17), 0, 0)]
    before = _states(ctx, ids + ids64)
    c32, c64, r = alloc_outputs(16)
    too_many = ph.make_requests([ids[0]] * (ph.NOALLOC_MAX_REQUESTS + 1), [0] * (ph.NOALLOC_MAX_REQUESTS + 1),
                                [0] * (ph.NOALLOC_MAX_REQUESTS + 1))
    with pytest.raises(ph.PhprngError) as ex:
        ctx.generate_noalloc(too_many, c32, c64, r)
    assert ex.value.status == ph.PHPRNG_E_RANGE
    # more width-64 tiles than the scratch holds (no output is written: refused before any launch)
    big = ph.NOALLOC_MAX_TILES64 * 1024 + 1
    r_big = torch.empty(big, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ph.PhprngError) as ex:
        ctx.generate_noalloc(ph.make_requests([ids64[0]], [big], [0]), None, None, r_big)
    assert ex.value.status == ph.PHPRNG_E_RANGE
    assert _states(ctx, ids + ids64) == before
    torch.cuda.synchronize()
    ctx.close()
