"""The width-32 kernels form R = (c+1)/(n+1) from a precomputed reciprocal
plus one exact correction.  It is the IEEE quotient for integers
1 <= a < b <= 2^33: the residual a - b*q0 is computed exactly by the fma, the
corrected value lies within 2^-52 ulp of a/b, and a/b with such a denominator
is never that close to a rounding boundary of binary64.  This
CPU test checks that form against IEEE division on >= 10^9 seeded pairs,
near-midpoint pairs, and every a for several b, without touching the GPU.
The paper's own shortcut (multiply by 1/(n+1), Sec. IV) is shown to differ."""

import ctypes
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "recip_check.c")


@pytest.fixture(scope="module")
def rc(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("rc") / "librecip.so")
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-pthread", "-o", out,
                    SRC, "-lm"], check=True)
    L = ctypes.CDLL(out)
    L.recip_exhaustive.restype = ctypes.c_uint64
    L.recip_exhaustive.argtypes = [ctypes.c_uint64] * 3 + [ctypes.c_int]
    L.recip_sampled.restype = ctypes.c_uint64
    L.recip_sampled.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_uint64)]
    return L


def _threads():
    return max(1, min(os.cpu_count() or 1, 16))


@pytest.mark.slow
def test_random_pairs_billion(rc):
    nt = _threads()
    per = (10 ** 9 + nt - 1) // nt
    done = ctypes.c_uint64()
    bad = rc.recip_sampled(0x14112484, per, 0, nt, ctypes.byref(done))
    assert done.value >= 10 ** 9
    assert bad == 0


def test_near_midpoint_pairs(rc):
    nt = _threads()
    done = ctypes.c_uint64()
    bad = rc.recip_sampled(77, 2 * 10 ** 7 // nt, 1, nt, ctypes.byref(done))
    assert done.value > 10 ** 7
    assert bad == 0


@pytest.mark.parametrize("b", [2 ** 31 + 12, 4294967088, 2 ** 32 - 4, 3 * 2 ** 30 + 1000, 2 ** 31 + 2 ** 30 + 1])
def test_every_numerator_for_fixed_denominators(rc, b):
    # a over the first and last 2^24 numerators plus a stride through the middle
    nt = _threads()
    assert rc.recip_exhaustive(b, 1, 1 << 24, nt) == 0
    assert rc.recip_exhaustive(b, b - (1 << 24), b, nt) == 0


def test_plain_reciprocal_multiply_is_not_exact():
    """The shortcut of Sec. IV (multiply by a precomputed 1/(n+1)) is not the
    IEEE quotient, which is why the kernels correct it."""
    import random
    rng = random.Random(3)
    n = 4294967087
    y = 1.0 / (n + 1)
    diff = sum(1 for _ in range(20000) if (lambda c: (c + 1) * y != (c + 1) / (n + 1))(rng.randrange(n)))
    assert diff > 1000


@pytest.mark.slow
def test_width64_double_correction_random_pairs(rc):
    """Width-64 form (two corrections from a = RN(c+1), b = RN(n+1))."""
    nt = _threads()
    done = ctypes.c_uint64()
    bad = rc.recip_sampled(0x64, (10 ** 9 + nt - 1) // nt, 2, nt, ctypes.byref(done))
    assert done.value >= 10 ** 9
    assert bad == 0


def test_width64_double_correction_near_midpoints(rc):
    nt = _threads()
    done = ctypes.c_uint64()
    bad = rc.recip_sampled(0x65, 2 * 10 ** 7 // nt, 3, nt, ctypes.byref(done))
    assert done.value > 10 ** 7
    assert bad == 0


def test_width64_double_correction_hardest_cases(rc):
    """Quotients within ~2^-107 (relative) of a binary64 rounding midpoint,
    built from the significand of b by a modular inverse."""
    nt = _threads()
    done = ctypes.c_uint64()
    bad = rc.recip_sampled(0x66, 2 * 10 ** 6 // nt, 4, nt, ctypes.byref(done))
    assert done.value > 10 ** 6
    assert bad == 0
