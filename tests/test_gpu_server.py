"""GPU tests of the serving loop (continuous batching): every result equals
the oracle for the position range reserved for it, whether the request ran
alone or in a mix; memory admission holds requests until arena space is
released; the open-loop replay reports sane latencies."""

import random

import numpy as np
import pytest

from tests.gpu_helpers import oracle_draws

pytestmark = pytest.mark.gpu

SEED0 = 0x14112484


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available()
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


@pytest.fixture(scope="module")
def tabs(tab32, tab64):
    return {32: tab32, 64: tab64}


def _read(ptr, count):
    """Copy `count` doubles from a device pointer with hipMemcpy (device to host)."""
    import ctypes
    import torch
    torch.cuda.synchronize()
    out = np.zeros(count, dtype=np.float64)
    if count:
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.restype = ctypes.c_int
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        assert hip.hipMemcpy(out.ctypes.data, ptr, count * 8, 2) == 0
    return out


def _collect(srv, n):
    got = []
    for _ in range(20000):
        got += srv.poll(256, 2000)
        if len(got) >= n:
            break
    assert len(got) == n
    return got


def _check_completion(ph, ctx_params, orc, tabs, c, data):
    n, e, p, a, w = ctx_params[c.instance]
    assert c.status == 0
    wc, wr, _ = oracle_draws(orc, tabs, w, n, e, c.k, c.count)
    assert np.array_equal(data.view(np.uint64), wr.view(np.uint64)), (c.instance, c.k, c.count)


# (streams, batches in flight, requests per batch): the defaults; one
# stream with a second batch queued behind the first; six small batches in
# flight over three streams
LAYOUTS = [(2, 0, 0), (1, 0, 16), (3, 6, 16)]


@pytest.mark.parametrize("streams,inflight,per_batch", LAYOUTS)
def test_server_results_match_oracle_alone_and_in_mix(ph, orc, tabs, streams, inflight, per_batch):
    rng = random.Random(1 + streams)
    ctx = ph.Context(0, max_instances=64)
    ids32 = ctx.seed_instances(32, SEED0 + 200, 24, (9, 17), 0, 1 << 40)
    ids64 = ctx.seed_instances(64, SEED0 + 201, 8, (9, 17), 0, 1 << 24)
    ids = [int(i) for i in ids32] + [int(i) for i in ids64]
    params = {i: ctx.get_params(i) for i in ids}
    starts = {i: ctx.get_position(i) for i in ids}
    srv = ph.Server(ctx, arena_doubles=1 << 22, streams=streams, max_inflight=inflight,
                    max_batch_requests=per_batch)
    reqs = [(rng.choice(ids), int(2 ** rng.uniform(4, 14))) for _ in range(300)]
    for j, (i, cnt) in enumerate(reqs):
        srv.submit(i, cnt, tag=j)
    got = _collect(srv, len(reqs))
    # reserved ranges per instance are contiguous in submission order
    by_inst = {}
    for c in sorted(got, key=lambda c: c.tag):
        assert c.instance == reqs[c.tag][0] and c.count == reqs[c.tag][1]
        by_inst.setdefault(c.instance, []).append(c)
    for i, cs in by_inst.items():
        k = starts[i]
        for c in cs:
            assert c.k == k
            k += c.count
    checked = []
    for c in got:
        data = _read(c.data, c.count)
        _check_completion(ph, params, orc, tabs, c, data)
        checked.append((c.instance, c.k, c.count, data))
    # half released one by one, the rest in one call; a ticket already
    # released is refused while the others in the same call still go back
    tickets = [c.ticket for c in got]
    half = len(tickets) // 2
    for t in tickets[:half]:
        srv.release(t)
    assert srv.stats()[1] > 0
    with pytest.raises(ph.PhprngError):
        srv.release_many(tickets[half:] + [tickets[0]])
    assert srv.stats()[1] == 0
    srv.close()
    ctx.close()
    # the same ranges requested alone, one request per fresh context, give the same bits
    for inst, k, cnt, data in checked[:12 if streams == 2 else 3]:
        n, e, p, a, w = params[inst]
        solo = ph.Context(0, max_instances=1)
        sid = int(solo.add_instances(w, [n], [e], k0=[k])[0])
        s2 = ph.Server(solo, arena_doubles=1 << 16, streams=1)
        s2.submit(sid, cnt, tag=0)
        (c2,) = _collect(s2, 1)
        d2 = _read(c2.data, c2.count)
        assert np.array_equal(d2.view(np.uint64), data.view(np.uint64))
        s2.release(c2.ticket)
        s2.close()
        solo.close()


def test_server_memory_admission(ph, orc, tabs):
    """An arena smaller than the total queued output: requests wait for
    releases and every one completes correctly."""
    ctx = ph.Context(0, max_instances=8)
    ids = [int(i) for i in ctx.seed_instances(32, SEED0 + 210, 4, (9, 17), 0, 1 << 40)]
    params = {i: ctx.get_params(i) for i in ids}
    srv = ph.Server(ctx, arena_doubles=20000, streams=2, max_batch_draws=1 << 20)
    sizes = [9000, 7000, 12000, 3000, 15000, 20000, 500, 9999]
    for j, s in enumerate(sizes):
        srv.submit(ids[j % 4], s, tag=j)
    done = []
    for _ in range(20000):
        for c in srv.poll(16, 2000):
            data = _read(c.data, c.count)
            _check_completion(ph, params, orc, tabs, c, data)
            pend, used = srv.stats()
            assert used <= 20000
            srv.release(c.ticket)
            done.append(c.tag)
        if len(done) == len(sizes):
            break
    assert sorted(done) == list(range(len(sizes)))
    with pytest.raises(ph.PhprngError):
        srv.submit(ids[0], 20001)
    srv.close()
    ctx.close()


def test_server_open_loop_replay(ph):
    ctx = ph.Context(0, max_instances=1024)
    ids = ctx.seed_instances(32, SEED0 + 220, 1000, (9, 17), 0, 1 << 40)
    srv = ph.Server(ctx, arena_doubles=1 << 24, streams=2)
    rng = np.random.default_rng(5)
    n = 2000
    arr = np.zeros(n, dtype=ph.ARRIVAL_DTYPE)
    arr["t_ns"] = np.cumsum(rng.exponential(1e9 / 20000.0, n)).astype(np.int64)  # 20k req/s
    arr["instance"] = rng.integers(0, 1000, n)
    arr["count"] = np.floor(2.0 ** (8 + 8 * rng.random(n))).astype(np.uint64)
    srv.counters(reset=True)
    lat, adm, wall = srv.replay_detail(arr)
    cnt = srv.counters()
    assert cnt["requests"] == n and cnt["draws"] == int(arr["count"].sum())
    assert 1 <= cnt["batches"] <= n and cnt["launch_ns_max"] * cnt["batches"] >= cnt["launch_ns"] > 0
    assert cnt["form_ns"] > 0 and cnt["retire_ns"] > 0
    assert (lat > 0).all()
    assert (adm >= 0).all() and (adm <= lat).all()
    assert np.percentile(lat, 50) < 5e6  # well under 5 ms at this light load
    assert wall > 0
    srv.close()
    ctx.close()


def test_server_rejected_configs_leave_the_context_usable(ph):
    ctx = ph.Context(0, max_instances=4)
    ids = ctx.seed_instances(32, SEED0 + 230, 2, (9, 17), 0, 0)
    with pytest.raises(ph.PhprngError):
        ph.Server(ctx, streams=9)            # at most 8 streams
    with pytest.raises(ph.PhprngError):
        ph.Server(ctx, max_inflight=7)       # at most 6 batches in flight
    with pytest.raises(ph.PhprngError):
        ph.Server(ctx, arena_doubles=1 << 40)  # 8 TiB: the arena allocation fails
    srv = ph.Server(ctx, arena_doubles=1 << 16, streams=1)
    t = srv.submit(int(ids[0]), 1000, tag=7)
    (c,) = _collect(srv, 1)
    assert c.status == 0 and c.count == 1000 and c.tag == 7
    srv.release(t)
    srv.close()
    ctx.close()
