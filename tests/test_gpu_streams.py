"""GPU parity for calls on several streams, bit for bit against the oracle.

Positions are reserved on the host when a call is made, and a width-64
instance's message is committed on the device by the call's tile-start
kernels; a later call on another stream waits for that commit (one event
between the committing kernels of successive calls).  Here the same
instances continue over calls issued back to back on three torch streams,
without synchronizing in between, then each call's outputs are compared
with the oracle's continuation of every stream.
"""

import random

import numpy as np
import pytest

from tests.gpu_helpers import compare_request

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


def test_continuation_across_streams(ph, orc, tab32, tab64):
    import torch
    rng = random.Random(0x57E4)
    ctx = ph.Context(0, max_instances=64)
    try:
        insts = []  # [id, width, n, e, m, s]
        p64, a64 = orc.lcg_params(64)
        p32, a32 = orc.lcg_params(32)
        n64, e64, k64 = orc.seed(64, 0x57E40, 4, (9, 17), 0, 1 << 26)
        for n, e, k in zip(n64, e64, k64):  # tiles from the 64-bit table
            iid = int(ctx.add_instances(64, [int(n)], [int(e)], k0=[int(k)])[0])
            m, s = orc.position(tab64, p64, a64, int(n), 0, 1, int(k))
            insts.append([iid, 64, int(n), int(e), m, s])
        n64b, e64b, _ = orc.seed(64, 0x57E41, 4, (9, 17), 0, 0)
        for n, e in zip(n64b, e64b):  # arbitrary carried states: reduce and scan
            m, s = rng.randrange(int(n)), rng.randrange(2, p64)
            iid = int(ctx.add_instances(64, [int(n)], [int(e)], m0=[m], s0=[s])[0])
            insts.append([iid, 64, int(n), int(e), m, s])
        n32, e32, k32 = orc.seed(32, 0x57E42, 4, (9, 17), 0, 1 << 40)
        for n, e, k in zip(n32, e32, k32):
            iid = int(ctx.add_instances(32, [int(n)], [int(e)], k0=[int(k)])[0])
            m, s = orc.position(tab32, p32, a32, int(n), 0, 1, int(k))
            insts.append([iid, 32, int(n), int(e), m, s])

        streams = [torch.cuda.Stream() for _ in range(3)]
        calls = []
        # six calls: each takes every instance, with long width-64 requests so
        # that the committing kernels of one call are still running when the
        # next call is issued
        plan = [[rng.choice([150000, 70001, 2049, 1]) for _ in insts] for _ in range(6)]
        outs = []
        for counts in plan:
            total = int(sum(counts))
            outs.append((torch.full((total,), -1, dtype=torch.int32, device="cuda:0"),
                         torch.full((total,), -1, dtype=torch.int64, device="cuda:0"),
                         torch.full((total,), -1.0, dtype=torch.float64, device="cuda:0")))
        torch.cuda.synchronize()
        for j, counts in enumerate(plan):
            offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
            reqs = ph.make_requests([x[0] for x in insts], counts, offs)
            st = streams[j % 3]
            ctx.generate(reqs, *outs[j], stream=st)
            calls.append((counts, offs))
        torch.cuda.synchronize()

        for j, (counts, offs) in enumerate(calls):
            hc32 = outs[j][0].cpu().numpy().view(np.uint32)
            hc64 = outs[j][1].cpu().numpy().view(np.uint64)
            hr = outs[j][2].cpu().numpy()
            for inst, cnt, off in zip(insts, counts, offs):
                iid, width, n, e, m, s = inst
                p, a = (p64, a64) if width == 64 else (p32, a32)
                wc, wr, m2, s2 = orc.generate(p, a, n, e, m, s, int(cnt))
                compare_request(hc32 if width == 32 else hc64, hr, int(off), int(cnt), wc, wr,
                                "call %d on stream %d, w%d inst %d" % (j, j % 3, width, iid))
                inst[4], inst[5] = m2, s2
        for inst in insts:
            assert ctx.get_state(inst[0])[:2] == (inst[4], inst[5])
    finally:
        ctx.close()
