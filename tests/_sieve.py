"""Segmented sieve of Eratosthenes in numpy (test helper, independent of the
oracle's Rabin-Miller code)."""

import numpy as np


def small_primes(limit):
    s = np.ones(limit + 1, dtype=bool)
    s[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0].astype(np.int64)


def odd_primes_in(lo, hi, base=None):
    """Primes in [lo, hi) for 3 <= lo < hi <= 2^32 + something, as uint64."""
    assert lo >= 3
    if base is None:
        base = small_primes(int(hi ** 0.5) + 2)
    base = base[base >= 3]
    start = lo | 1
    cnt = (hi - start + 1) // 2            # odd numbers start, start+2, ...
    is_p = np.ones(cnt, dtype=bool)
    for q in base:
        q = int(q)
        if q * q >= hi:
            break
        first = max(q * q, ((start + q - 1) // q) * q)
        if first % 2 == 0:
            first += q
        if first >= hi:
            continue
        is_p[(first - start) // 2::q] = False
    return (start + 2 * np.nonzero(is_p)[0]).astype(np.uint64)
