"""Shared helpers for the GPU parity tests: run requests through the HIP
library (C-ABI via the binding) and compute the same draws with the oracle."""

import numpy as np


def torch_mod():
    import torch
    return torch


def alloc_outputs(total, want_c32=True, want_c64=True, want_r=True, fill=True):
    torch = torch_mod()
    dev = torch.device("cuda:0")
    c32 = torch.full((max(total, 1),), -1, dtype=torch.int32, device=dev) if want_c32 else None
    c64 = torch.full((max(total, 1),), -1, dtype=torch.int64, device=dev) if want_c64 else None
    r = torch.full((max(total, 1),), -1.0, dtype=torch.float64, device=dev) if want_r else None
    return c32, c64, r


def to_host(c32, c64, r):
    torch = torch_mod()
    torch.cuda.synchronize()
    hc32 = c32.cpu().numpy().view(np.uint32) if c32 is not None else None
    hc64 = c64.cpu().numpy().view(np.uint64) if c64 is not None else None
    hr = r.cpu().numpy() if r is not None else None
    return hc32, hc64, hr


def oracle_draws(orc, tabs, width, n, e, k, count, m0=0, s0=1):
    """Oracle draws c_{k+1..k+count}, R_{k+1..k+count} from position k."""
    p, a = orc.lcg_params(width)
    tab = tabs.get(width)
    if s0 == 1 and tab is not None and (k % (p - 1)) <= tab.max_r:
        m, s = orc.position(tab, p, a, n, m0, s0, k)
    else:
        m, s = orc.position(None, p, a, n, m0, s0, k)
    c, r, m2, s2 = orc.generate(p, a, n, e, m, s, count)
    return c, r, (m2, s2)


def compare_request(got_c, got_r, off, count, want_c, want_r, label=""):
    if got_c is not None:
        gc = got_c[off:off + count].astype(np.uint64)
        bad = np.nonzero(gc != want_c)[0]
        assert bad.size == 0, "%s: %d ciphertext mismatches, first at %d: got %d want %d" % (
            label, bad.size, bad[0], gc[bad[0]], want_c[bad[0]])
    if got_r is not None:
        gr = got_r[off:off + count]
        bad = np.nonzero(gr.view(np.uint64) != want_r.view(np.uint64))[0]
        assert bad.size == 0, "%s: %d uniform mismatches, first at %d: got %r want %r" % (
            label, bad.size, bad[0], gr[bad[0]], want_r[bad[0]])
