"""Seeded synthetic workloads shaped like the paper's (parameter splitting over
many prime moduli, Sec. I/IV): the instance seeds, stream lengths and
output layouts shared by the GPU tests and bench.py.  Instance parameters
(n, e, start) are drawn by the library's and the oracle's own SplitMix64
seeding from these seeds; nothing here computes any part of the generator.
"""

import numpy as np

SEED0 = 0x14112484

# 65,536 width-32 streams, lengths floor(2^(10 + 12 u)), u ~ U[0, 1), starts
# uniform in [0, 2^40)
C_INSTANCES = 1 << 16
C_SEED = SEED0 + 2
C_START_HI = 1 << 40


def config_c_lengths(nin=C_INSTANCES):
    """Log-uniform stream lengths in [2^10, 2^22)."""
    rng = np.random.default_rng(C_SEED)
    return np.floor(2.0 ** (10 + 12 * rng.random(nin))).astype(np.uint64)


def config_c_sample(nin=C_INSTANCES):
    """The seeded 1% of the streams compared whole against the oracle."""
    rng = np.random.default_rng(C_SEED + 10)
    return np.sort(rng.choice(nin, size=max(1, nin // 100), replace=False))


def split_groups(lens, ngroups):
    """Contiguous groups of streams with about equal draws; within a group the
    streams' outputs follow one another from offset 0.  Returns
    [(first, last_exclusive, offsets, draws)], one per group."""
    lens = np.asarray(lens, dtype=np.uint64)
    cum = np.cumsum(lens.astype(np.float64))
    total = float(cum[-1])
    groups, first = [], 0
    for g in range(ngroups):
        if g == ngroups - 1:
            last = lens.size
        else:
            last = int(np.searchsorted(cum, total * (g + 1) / ngroups, side="right"))
            last = max(first + 1, min(last, lens.size - (ngroups - 1 - g)))
        part = lens[first:last]
        offs = np.zeros(part.size, dtype=np.uint64)
        if part.size > 1:
            offs[1:] = np.cumsum(part[:-1], dtype=np.uint64)
        groups.append((first, last, offs, int(part.sum())))
        first = last
    return groups


def groups_for_memory(lens, bytes_per_draw, free_bytes, fill=0.8):
    """Fewest groups whose largest output arena fits in `fill` of the free
    device memory."""
    total = int(np.asarray(lens, dtype=np.uint64).sum())
    ng = max(1, int(np.ceil(total * bytes_per_draw / (fill * free_bytes))))
    while True:
        gs = split_groups(lens, ng)
        if max(g[3] for g in gs) * bytes_per_draw <= fill * free_bytes or ng >= len(lens):
            return gs
        ng += 1
