"""GPU parity at the workloads' full sizes, in the launch configuration that
bench.py times, with a seeded 1% (or more) of the streams compared whole,
bit for bit, against the oracle:

  - 4096 width-32 streams x 2^18 draws from position 0 (persistent and one
    launch per stream);
  - 65,536 width-32 streams with log-uniform lengths in [2^10, 2^22] and
    starts in [0, 2^40) (about 3.3e10 draws, u32 ciphertexts and FP64
    uniforms): 396 GB of outputs do not fit in device memory, so the batch
    runs as the fewest groups of streams whose outputs fit, each group one
    persistent launch into one reused arena;
  - 1024 width-64 + 1024 width-32 streams x 2^20 draws in one launch.
"""

import numpy as np
import pytest

from tests import workloads as W
from tests.gpu_helpers import compare_request

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


def _oracle_streams(orc, tabs, width, n, e, k0, lens, nthreads=0):
    """Whole streams from positions k0 (arrays), by eq. (7) then algorithm (9)."""
    p, a = orc.lcg_params(width)
    ms, ss = [], []
    for ni, ki in zip(n, k0):
        m, s = orc.position(tabs[width], p, a, int(ni), 0, 1, int(ki))
        ms.append(m)
        ss.append(s)
    wc, wr, _, _, woff = orc.generate_many(p, a, np.asarray(n, dtype=np.uint64), np.asarray(e, dtype=np.uint64),
                                           np.array(ms, dtype=np.uint64), np.array(ss, dtype=np.uint64),
                                           np.asarray(lens, dtype=np.uint64), nthreads=nthreads)
    return wc, wr, woff


@pytest.fixture(scope="module")
def tabs(tab32, tab64):
    return {32: tab32, 64: tab64}


@pytest.fixture(autouse=True)
def release_device_memory():
    """Hand the full-size outputs back to the device when each test ends:
    torch's caching allocator would otherwise keep them, and later
    allocations by the library (contexts, staging) would find no room."""
    import torch
    yield
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_config_b_whole_streams(ph, orc, tabs):
    import torch
    ctx = ph.Context(0, max_instances=4096)
    ids = ctx.seed_instances(32, W.SEED0 + 1, 4096, (9, 17), 0, 0)
    n, e, _ = orc.seed(32, W.SEED0 + 1, 4096, (9, 17), 0, 0)
    per = 1 << 18
    total = 4096 * per
    reqs = ph.make_requests(ids, [per] * 4096, np.arange(4096, dtype=np.uint64) * per)
    dev = torch.device("cuda:0")
    c32 = torch.full((total,), -1, dtype=torch.int32, device=dev)
    r = torch.full((total,), -1.0, dtype=torch.float64, device=dev)
    ctx.generate(reqs, c32, None, r)
    for i in ids:
        ctx.jump(int(i), -per)
    c32b = torch.full((total,), -1, dtype=torch.int32, device=dev)
    rb = torch.full((total,), -1.0, dtype=torch.float64, device=dev)
    ctx.generate(reqs, c32b, None, rb, mode=ph.PHPRNG_MODE_PLAIN)
    torch.cuda.synchronize()
    assert torch.equal(c32, c32b) and torch.equal(r, rb)
    del c32b, rb
    sample = np.sort(np.random.default_rng(W.SEED0 + 11).choice(4096, size=48, replace=False))
    wc, wr, woff = _oracle_streams(orc, tabs, 32, n[sample], e[sample], np.zeros(sample.size), [per] * sample.size)
    for j, i in enumerate(sample):
        lo = int(i) * per
        gc = c32[lo:lo + per].cpu().numpy().view(np.uint32)
        gr = r[lo:lo + per].cpu().numpy()
        o = int(woff[j])
        compare_request(gc, gr, 0, per, wc[o:o + per], wr[o:o + per], "B stream %d" % i)
    ctx.close()


def test_config_c_full_shape_one_percent_whole(ph, orc, tabs):
    import torch
    nin = W.C_INSTANCES
    lens = W.config_c_lengths(nin)
    sample = W.config_c_sample(nin)
    ctx = ph.Context(0, max_instances=nin)
    ids = ctx.seed_instances(32, W.C_SEED, nin, (9, 17), 0, W.C_START_HI)
    n, e, k = orc.seed(32, W.C_SEED, nin, (9, 17), 0, W.C_START_HI)
    assert [ctx.get_position(int(ids[i])) for i in sample] == [int(k[i]) for i in sample]
    free, _ = torch.cuda.mem_get_info()
    groups = W.groups_for_memory(lens, 12, free)
    arena = max(g[3] for g in groups)
    dev = torch.device("cuda:0")
    c32 = torch.empty(arena, dtype=torch.int32, device=dev)
    r = torch.empty(arena, dtype=torch.float64, device=dev)
    print("config C: %d draws in %d launches, arena %d" % (int(lens.sum()), len(groups), arena), flush=True)
    checked = 0
    for first, last, offs, draws in groups:
        ctx.generate(ph.make_requests(ids[first:last], lens[first:last], offs), c32, None, r, capacity=arena)
        torch.cuda.synchronize()
        mine = sample[(sample >= first) & (sample < last)]
        for lo in range(0, mine.size, 64):
            part = mine[lo:lo + 64]
            wc, wr, woff = _oracle_streams(orc, tabs, 32, n[part], e[part], k[part], lens[part])
            for j, i in enumerate(part):
                o, L = int(offs[i - first]), int(lens[i])
                gc = c32[o:o + L].cpu().numpy().view(np.uint32)
                gr = r[o:o + L].cpu().numpy()
                compare_request(gc, gr, 0, L, wc[int(woff[j]):int(woff[j]) + L], wr[int(woff[j]):int(woff[j]) + L],
                                "C stream %d (k=%d, len %d)" % (i, int(k[i]), L))
                checked += 1
    assert checked == sample.size == nin // 100
    # every stream advanced by its length
    assert [ctx.get_position(int(ids[i])) for i in sample] == [int(k[i] + lens[i]) for i in sample]
    ctx.close()


def test_config_d_whole_streams(ph, orc, tabs):
    import torch
    ctx = ph.Context(0, max_instances=2048)
    i64 = ctx.seed_instances(64, W.SEED0 + 3, 1024, (9, 17), 0, 0)
    i32 = ctx.seed_instances(32, W.SEED0 + 4, 1024, (9, 17), 0, 0)
    n64, e64, _ = orc.seed(64, W.SEED0 + 3, 1024, (9, 17), 0, 0)
    n32, e32, _ = orc.seed(32, W.SEED0 + 4, 1024, (9, 17), 0, 0)
    per = 1 << 20
    ids = np.concatenate([i64, i32])
    total = 2048 * per
    dev = torch.device("cuda:0")
    c32 = torch.full((total,), -1, dtype=torch.int32, device=dev)
    c64 = torch.full((total,), -1, dtype=torch.int64, device=dev)
    r = torch.full((total,), -1.0, dtype=torch.float64, device=dev)
    ctx.generate(ph.make_requests(ids, [per] * 2048, np.arange(2048, dtype=np.uint64) * per), c32, c64, r)
    torch.cuda.synchronize()
    rng = np.random.default_rng(W.SEED0 + 13)
    s64 = np.sort(rng.choice(1024, size=11, replace=False))
    s32 = np.sort(rng.choice(1024, size=11, replace=False))
    for width, sample, n, e, base, arr in ((64, s64, n64, e64, 0, c64), (32, s32, n32, e32, 1024, c32)):
        wc, wr, woff = _oracle_streams(orc, tabs, width, n[sample], e[sample], np.zeros(sample.size),
                                       [per] * sample.size)
        for j, i in enumerate(sample):
            lo = (base + int(i)) * per
            gc = arr[lo:lo + per].cpu().numpy().view(np.uint64 if width == 64 else np.uint32)
            gr = r[lo:lo + per].cpu().numpy()
            o = int(woff[j])
            compare_request(gc, gr, 0, per, wc[o:o + per], wr[o:o + per], "D w%d stream %d" % (width, i))
        # the other array of the width is untouched
        other = c32 if width == 64 else c64
        lo = (base + int(sample[0])) * per
        assert bool((other[lo:lo + per] == -1).all())
    ctx.close()
