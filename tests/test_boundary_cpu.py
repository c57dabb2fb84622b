"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol include/phprng.h declares, and its host-only helpers (skip
parameters, admissibility, seeded instance draws) agree with the oracle."""

import math
import os
import random
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "phprng.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phprng_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ph():
    import paper_1411_2484_amd as ph
    if not os.path.exists(ph.LIB_PATH):
        pytest.fail("libphprng.so is not built (run python -m paper_1411_2484_amd.build)")
    ph.lib()
    return ph


def test_library_exports_every_declared_symbol(ph):
    syms = _declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(ph.lib(), s), s
    # the binding knows every declared entry point and nothing else
    assert sorted(ph.SIGNATURES) == syms


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(ROOT, "paper_1411_2484_amd", "__init__.py")).read()
    assert "oracle" not in src


def test_skip_params_match_oracle(ph, orc):
    for w in (32, 64):
        assert ph.phprng_skip_params(w) == orc.lcg_params(w)
    with pytest.raises(ph.PhprngError):
        ph.phprng_skip_params(16)


def test_check_instance_matches_oracle(ph, orc):
    rng = random.Random(21)
    cases = []
    for w, lo in ((32, 1 << 31), (64, 1 << 62)):
        for _ in range(3000):
            n = rng.randrange(lo - 1000, 2 * lo + 1000)
            e = rng.choice([1, 2, 3, 5, 7, 9, 11, 17, 65537, rng.randrange(1, 1 << 40), n - 1 + 1 if n > 1 else 3])
            cases.append((w, n, e))
        cases += [(w, lo + 1, 9), (w, 2 * lo - 1, 9)]
    cases += [(32, 4294967087, 9), (32, 4294967087, 4294967087), (16, 5, 3), (64, 4294967087, 9)]
    for w, n, e in cases:
        assert ph.phprng_check_instance(w, n, e) == orc.check_instance(w, n, e), (w, n, e)


@pytest.mark.parametrize("width", [32, 64])
def test_draw_instances_match_oracle(ph, orc, width):
    for seed, count, es, klo, khi in ((0x14112484, 3000, (9, 17), 0, 1 << 40), (7, 500, (3,), 5, 6),
                                      (123, 200, (17, 9, 5), 0, 0), (99, 1000, (65537, 9), 1, 1 << 63)):
        a = ph.phprng_draw_instances(width, seed, count, es, klo, khi)
        b = orc.seed(width, seed, count, es, klo, khi)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_draw_instances_rejects_bad_arguments(ph):
    with pytest.raises(ph.PhprngError):
        ph.phprng_draw_instances(32, 1, 4, (1, 2))
    with pytest.raises(ph.PhprngError):
        ph.phprng_draw_instances(48, 1, 4)
    with pytest.raises(ph.PhprngError):
        ph.phprng_draw_instances(32, 1, 4, (9,), 10, 5)
