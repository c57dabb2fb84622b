"""Pins for the CPU oracle against what the paper and mathematics fix.

None of these tests re-types the oracle's formulas: each checks the oracle
against a printed value, an identity that holds for a different reason
(decryption, permutation, period, symmetry), a brute-force enumeration, or an
independent library routine (Python's built-in ``pow`` and exact rational
division).
"""

import math
import random
from fractions import Fraction

import numpy as np
import pytest

from tests import _sieve

P32, A32 = 2147483647, 784588716


def _tiny_primes(limit):
    return [int(q) for q in _sieve.small_primes(limit)]


def _py_sprp(n, g):
    """Strong-probable-prime check written with Python's pow (independent)."""
    t, r = n - 1, 0
    while t % 2 == 0:
        t //= 2
        r += 1
    x = pow(g, t, n)
    if x in (1, n - 1):
        return True
    for _ in range(r - 1):
        x = x * x % n
        if x == n - 1:
            return True
    return False


def _py_probable_prime(n, rng, rounds=24):
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13):
        if n % q == 0:
            return n == q
    return all(_py_sprp(n, rng.randrange(2, n - 1)) for _ in range(rounds))


def _pollard_rho(n):
    if n % 2 == 0:
        return 2
    for c in range(1, 100):
        x = y = 2
        d = 1
        while d == 1:
            x = (x * x + c) % n
            y = (y * y + c) % n
            y = (y * y + c) % n
            d = math.gcd(abs(x - y), n)
        if d != n:
            return d
    raise AssertionError("no factor found")


# --------------------------------------------------------------------------
# Worked values printed in the paper
# --------------------------------------------------------------------------

def test_decryption_exponent_of_paper_example(orc, paper):
    ex = paper["example_instance"]
    d = orc.inverse(ex["e"], ex["n"] - 1)
    assert d == ex["d"]
    assert (d * ex["e"]) % (ex["n"] - 1) == 1
    assert orc.is_prime(ex["n"]) and orc.is_safe_prime(ex["n"])


def test_fig2_unit_skip_ciphertexts(orc, paper):
    fx = paper["unit_skip_fig2"]
    got = orc.encrypt_many(np.array(fx["messages"], dtype=np.uint64), fx["e"], fx["n"])
    assert [int(v) for v in got] == fx["ciphertexts"]
    assert orc.is_prime(fx["n"])


def test_skip_multipliers_are_primitive_roots(orc, paper):
    lcg = paper["skip_lcg_32"]
    assert (lcg["p"], lcg["a"]) == orc.lcg_params(32)
    assert orc.is_primitive_root(lcg["a"], lcg["p"])
    fig1 = paper["fig1_lcg"]
    assert orc.is_primitive_root(fig1["a"], fig1["p"])
    p64, a64 = orc.lcg_params(64)
    assert p64 == (1 << 61) - 1 and orc.is_prime(p64)
    assert orc.is_primitive_root(a64, p64)
    # squares are never primitive roots
    assert not orc.is_primitive_root(lcg["a"] * lcg["a"] % lcg["p"], lcg["p"])
    assert not orc.is_primitive_root(a64 * a64 % p64, p64)


def test_primitive_root_test_against_brute_force_order(orc):
    for p in _tiny_primes(400)[1:]:
        for a in range(1, p):
            x, order = a, 1
            while x != 1:
                x = x * a % p
                order += 1
            assert orc.is_primitive_root(a, p) == (order == p - 1), (a, p)


def test_period_lower_bound_32(paper):
    p = paper["skip_lcg_32"]["p"]
    # the smallest 32-bit modulus is the first prime above 2^31; its period
    # n (p - 1) already exceeds 2^62 (Sec. IV)
    n_min = int(_sieve.odd_primes_in((1 << 31) + 1, (1 << 31) + 1000)[0])
    assert n_min * (p - 1) > 1 << paper["period_32"]["log2_lower_bound"]


# --------------------------------------------------------------------------
# Encryption (eq. (1)), decryption (eq. (2)) and their properties
# --------------------------------------------------------------------------

def test_encrypt_matches_python_pow(orc):
    rng = random.Random(1)
    for _ in range(3000):
        n = rng.randrange(3, 1 << 64)
        m = rng.randrange(0, n)
        e = rng.randrange(0, 1 << 64)
        assert orc.encrypt(m, e, n) == pow(m, e, n)
    for _ in range(2000):
        x, y = rng.randrange(1 << 64), rng.randrange(1 << 64)
        n = rng.randrange(1, 1 << 64)
        assert orc.mulmod(x, y, n) == (x * y) % n


def test_inverse_matches_python(orc):
    rng = random.Random(2)
    for _ in range(3000):
        m = rng.randrange(2, 1 << 64)
        e = rng.randrange(1, 1 << 64)
        if math.gcd(e, m) == 1:
            assert orc.inverse(e, m) == pow(e, -1, m)
        else:
            assert orc.inverse(e, m) == 0


def test_permutation_brute_force_all_exponents_small_primes(orc):
    """Eq. (1) permutes Z/nZ for every admissible e (Sec. I), checked for every
    prime n < 2^9 and every admissible exponent."""
    for n in _tiny_primes(1 << 9):
        if n < 5:
            continue
        allm = np.arange(n, dtype=np.uint64)
        for e in range(3, n - 1):
            if math.gcd(e, n - 1) != 1:
                continue
            c = orc.encrypt_many(allm, e, n)
            assert np.array_equal(np.sort(c), allm), (n, e)


def test_permutation_and_inverse_sampled_exponents_16bit(orc):
    rng = random.Random(3)
    primes = [q for q in _tiny_primes(1 << 16) if q > 1 << 12]
    for n in rng.sample(primes, 12):
        allm = np.arange(n, dtype=np.uint64)
        es = [e for e in range(3, 200) if math.gcd(e, n - 1) == 1][:4]
        for e in es:
            c = orc.encrypt_many(allm, e, n)
            assert np.array_equal(np.sort(c), allm)
            d = orc.inverse(e, n - 1)
            back = orc.encrypt_many(c, d, n)
            assert np.array_equal(back, allm)


def test_non_admissible_exponent_is_not_a_permutation(orc):
    n = 1019  # n - 1 = 2 * 509
    allm = np.arange(n, dtype=np.uint64)
    c = orc.encrypt_many(allm, 2, n)
    assert np.unique(c).size < n


def test_decryption_recovers_message(orc):
    rng = random.Random(4)
    for width, lo in ((32, 1 << 31), (64, 1 << 62)):
        for _ in range(60):
            while True:
                n = rng.randrange(lo, 2 * lo) | 1
                if _py_probable_prime(n, rng):
                    break
            e = next(x for x in (9, 17, 3, 5, 7, 11, 13) if math.gcd(x, n - 1) == 1)
            for m in [0, 1, n - 1, n - 2] + [rng.randrange(n) for _ in range(20)]:
                c = orc.encrypt(m, e, n)
                assert c == pow(m, e, n)
                assert orc.decrypt(c, e, n) == m


def test_cribs_and_symmetries(orc):
    rng = random.Random(5)
    n = 4294967087
    for e in (3, 9, 17, 5):
        if math.gcd(e, n - 1) != 1:
            continue
        # cribs m in {0, 1, n-1} (Sec. II)
        assert [orc.encrypt(m, e, n) for m in (0, 1, n - 1)] == [0, 1, n - 1]
        # m^e < n gives a trivial ciphertext
        m = 2
        while m ** e < n:
            assert orc.encrypt(m, e, n) == m ** e
            m += 1
        for _ in range(200):
            m = rng.randrange(1, n)
            b = rng.randrange(2, n - 1)
            # (n - m)^e mod n = n - m^e mod n (Sec. II)
            assert orc.encrypt(n - m, e, n) == n - orc.encrypt(m, e, n)
            # eq. (4): (k b)^e = (b^e)(k^e) mod n
            kb = m * b % n
            assert orc.encrypt(kb, e, n) == orc.encrypt(b, e, n) * orc.encrypt(m, e, n) % n


# --------------------------------------------------------------------------
# Primality and admissibility (Sec. IV)
# --------------------------------------------------------------------------

def test_strong_pseudoprimes_to_first_prime_bases(orc, paper):
    vals = paper["strong_pseudoprimes_first_k_prime_bases"]["values"]
    bases = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for k, v in enumerate(vals, start=1):
        # composite: Pollard's rho finds a proper factor
        f = _pollard_rho(v)
        assert 1 < f < v and v % f == 0
        for g in bases[:k]:
            assert _py_sprp(v, g)
            assert orc.strong_probable_prime(v, g)
        # where the next entry of the sequence is larger, this value fails
        # the next base
        if k < len(vals) and vals[k] != v:
            assert not _py_sprp(v, bases[k])
            assert not orc.strong_probable_prime(v, bases[k])
        assert not orc.is_prime(v)


def test_is_prime_against_sieve_windows(orc):
    base = _sieve.small_primes(70000)
    for lo in ((1 << 31), (1 << 32) - (1 << 18), 1 << 20):
        hi = lo + (1 << 18)
        primes = set(int(x) for x in _sieve.odd_primes_in(lo, hi, base))
        for x in range(lo, hi):
            assert orc.is_prime(x) == (x in primes), x


def test_is_prime_64bit_windows_against_random_base_rabin_miller(orc):
    rng = random.Random(6)
    for lo in (1 << 62, (1 << 63) - (1 << 12), (1 << 64) - (1 << 12)):
        for x in range(lo | 1, lo + (1 << 12), 2):
            assert orc.is_prime(x) == _py_probable_prime(x, rng), x


def test_check_instance_rules(orc):
    n = 4294967087
    assert orc.check_instance(32, n, 9) == orc.OK
    assert orc.check_instance(32, n, 17) == orc.OK
    assert orc.check_instance(32, n, 2) == orc.E_EXPONENT       # e < 3 / even
    assert orc.check_instance(32, n, 1) == orc.E_EXPONENT
    assert orc.check_instance(32, n, 1 + (n - 1)) == orc.E_EXPONENT  # identity map
    assert orc.check_instance(32, n + 2, 9) != orc.OK            # composite (n+2 = 4294967089)
    assert orc.check_instance(32, 4294967291, 9) in (orc.OK, orc.E_EXPONENT)
    assert orc.check_instance(32, 2147483647, 9) == orc.E_RANGE  # p must be < n
    assert orc.check_instance(32, 65537, 3) == orc.E_RANGE
    assert orc.check_instance(64, n, 9) == orc.E_RANGE
    assert orc.check_instance(16, n, 9) == orc.E_INVALID


@pytest.mark.slow
def test_prime_counts_in_paper(orc, paper):
    """The admissibility predicates reproduce the four counts printed in Sec. I
    and Sec. IV over all primes in [2^31, 2^32] (primes from an independent
    numpy sieve, whose own count is pinned by the first number)."""
    cnt = paper["prime_counts_2_31_to_2_32"]
    base = _sieve.small_primes(70000)
    tot = safe = c9 = c17 = 0
    step = 1 << 27
    for lo in range((1 << 31) + 1, 1 << 32, step):
        hi = min(lo + step, 1 << 32)
        pr = _sieve.odd_primes_in(lo, hi, base)
        tot += pr.size
        c9 += orc.count_many(pr, 2, 9)
        c17 += orc.count_many(pr, 2, 17)
        safe += orc.count_many(pr, 1)
        if lo == (1 << 31) + 1:
            assert orc.count_many(pr[:200000], 0) == 200000
    assert tot == cnt["primes"]
    assert c9 == cnt["coprime_e9"]
    assert c17 == cnt["coprime_e17"]
    assert safe == cnt["safe_primes"]


# --------------------------------------------------------------------------
# Skip sequence and message schedule (eqs. (3), (5)-(7))
# --------------------------------------------------------------------------

def test_full_period_skip_sum(tab32):
    """Over one skip period every value of (Z/pZ)^* occurs once, so the skip sum
    is p(p-1)/2 (Sec. II, proof of the period)."""
    p = P32
    assert tab32.prefix(p - 1) == p * (p - 1) // 2


def test_position_equals_stepping_32(orc, tab32):
    p, a = orc.lcg_params(32)
    n = 4294967087
    m, s = 0, 1
    k = 0
    rng = random.Random(7)
    targets = sorted(set([1, 2, 3, 65535, 65536, 65537, 10 ** 6] + [rng.randrange(1, 3 * 10 ** 6) for _ in range(20)]))
    for t in targets:
        m, s = orc.jump_forward(p, a, n, m, s, t - k)
        k = t
        assert orc.position(tab32, p, a, n, 0, 1, k) == (m, s)
        assert orc.position(None, p, a, n, 0, 1, k) == (m, s)


def test_position_period_structure_32(orc, tab32):
    """Eq. (7): after q full skip periods the message advanced by q p(p-1)/2."""
    p, a = orc.lcg_params(32)
    rng = random.Random(8)
    for _ in range(20):
        n = 4294967087 if _ == 0 else None
        while n is None:
            c = rng.randrange(1 << 31, 1 << 32) | 1
            n = c if orc.is_prime(c) else None
        k = rng.randrange(0, p - 1)
        q = rng.randrange(1, 1 << 20)
        m0 = rng.randrange(n)
        mk, sk = orc.position(tab32, p, a, n, m0, 1, k)
        mq, sq = orc.position(tab32, p, a, n, m0, 1, k + q * (p - 1))
        assert sq == sk
        assert mq == (mk + q * (p * (p - 1) // 2)) % n
        # and the step just before the period boundary wraps consistently
        mb, sb = orc.position(tab32, p, a, n, m0, 1, q * (p - 1) - 1)
        m1, s1 = orc.jump_forward(p, a, n, mb, sb, 1)
        assert (m1, s1) == orc.position(tab32, p, a, n, m0, 1, q * (p - 1))
        assert s1 == 1


def test_position_general_s0_equals_stepping(orc):
    p, a = orc.lcg_params(32)
    n = 4294967087
    rng = random.Random(9)
    for _ in range(10):
        m0, s0 = rng.randrange(n), rng.randrange(1, p)
        k = rng.randrange(0, 200000)
        assert orc.position(None, p, a, n, m0, s0, k) == orc.jump_forward(p, a, n, m0, s0, k)


def test_position_64_equals_stepping(orc, tab64):
    p, a = orc.lcg_params(64)
    n = (1 << 62) + 135  # prime
    assert orc.is_prime(n)
    m, s, k = 0, 1, 0
    for t in (1, 2, 65536, 65537, 300001, 10 ** 6):
        m, s = orc.jump_forward(p, a, n, m, s, t - k)
        k = t
        assert orc.position(tab64, p, a, n, 0, 1, k) == (m, s)


def test_backward_jump_inverts_forward(orc, tab32):
    p, a = orc.lcg_params(32)
    n = 4294967087
    rng = random.Random(10)
    for _ in range(10):
        k = rng.randrange(10 ** 5, 10 ** 7)
        d = rng.randrange(1, 10 ** 5)
        mk, sk = orc.position(tab32, p, a, n, 0, 1, k)
        mb, sb = orc.jump_backward(p, a, n, mk, sk, d)
        assert (mb, sb) == orc.position(tab32, p, a, n, 0, 1, k - d)
        assert orc.jump_forward(p, a, n, mb, sb, d) == (mk, sk)


def _tiny_cases():
    rng = random.Random(11)
    out = []
    primes = _tiny_primes(60)
    for n in primes:
        if n < 7:
            continue
        for p in primes:
            if p < 3 or p >= n:
                continue
            roots = [g for g in range(2, p) if all(pow(g, (p - 1) // q, p) != 1
                                                for q in range(2, p) if (p - 1) % q == 0 and all(q % r for r in range(2, q)))]
            es = [e for e in range(3, n - 1) if math.gcd(e, n - 1) == 1]
            if not roots or not es:
                continue
            out.append((n, p, rng.choice(roots), rng.choice(es), rng.randrange(n), rng.randrange(1, p)))
    return out


def test_tiny_bruteforce_period_and_uniformity(orc):
    """Sec. II: the period is n(p-1), every ciphertext appears exactly p-1
    times per period, consecutive pairs are unique and never equal; eq. (7)
    agrees with stepping at every position of the period."""
    cases = _tiny_cases()
    assert len(cases) > 50
    for n, p, a, e, m0, s0 in cases:
        P = n * (p - 1)
        c, _, _, _ = orc.generate(p, a, n, e, m0, s0, 2 * P + 1, want_r=False)
        c = [int(x) for x in c]
        # P is a period of the emitted sequence and no proper divisor of P is
        assert c[P:2 * P + 1] == c[:P + 1]
        for d in range(1, P):
            if P % d == 0:
                assert c[d:d + P] != c[:P], (n, p, a, e, d)
        counts = np.bincount(np.array(c[:P]), minlength=n)
        assert (counts == p - 1).all()
        pairs = set(zip(c[:P], c[1:P + 1]))
        assert len(pairs) == P
        assert all(c[i] != c[i + 1] for i in range(P))
        # eq. (7) vs stepping, with general (m0, s0)
        m, s = m0, s0
        for k in range(0, P + 2):
            assert orc.position(None, p, a, n, m0, s0, k) == (m, s), (n, p, a, k)
            m, s = orc.jump_forward(p, a, n, m, s, 1)


# --------------------------------------------------------------------------
# Algorithm (9) outputs
# --------------------------------------------------------------------------

def test_generate_decrypts_to_message_schedule(orc, tab32):
    """Each draw decrypts (eq. (2)) to the message of eq. (6b) at its position."""
    p, a = orc.lcg_params(32)
    rng = random.Random(12)
    for _ in range(6):
        while True:
            n = rng.randrange(1 << 31, 1 << 32) | 1
            if orc.is_prime(n) and math.gcd(9, n - 1) == 1:
                break
        k0 = rng.randrange(0, 1 << 40)
        m, s = orc.position(tab32, p, a, n, 0, 1, k0)
        c, r, m2, s2 = orc.generate(p, a, n, 9, m, s, 3000)
        d = orc.inverse(9, n - 1)
        for t in range(0, 3000, 97):
            mt, st = orc.position(tab32, p, a, n, 0, 1, k0 + 1 + t)
            assert pow(int(c[t]), d, n) == mt
        assert (m2, s2) == orc.position(tab32, p, a, n, 0, 1, k0 + 3000)


def test_step_relation_of_consecutive_ciphertexts(orc):
    """c_{k+1} = ((c_k^d mod n) + s_{k+1})^e mod n (Sec. II, Fig. 3)."""
    p, a = orc.lcg_params(32)
    n, e = 4294967087, 9
    d = orc.inverse(e, n - 1)
    s = 1
    c, _, _, _ = orc.generate(p, a, n, e, 0, 1, 2000, want_r=False)
    s_seq = []
    for _ in range(2000):
        s = s * a % p
        s_seq.append(s)
    for k in range(1999):
        assert int(c[k + 1]) == pow((pow(int(c[k]), d, n) + s_seq[k + 1]) % n, e, n)


def _exact_nearest_double(num, den):
    """Correctly rounded num/den for positive Fractions, via Python's exact
    int/int true division (round-half-even)."""
    q = Fraction(num) / Fraction(den)
    return q.numerator / q.denominator


def test_uniform_is_correctly_rounded_quotient(orc):
    rng = random.Random(13)
    p32, a32 = orc.lcg_params(32)
    p64, a64 = orc.lcg_params(64)
    for width, (p, a) in ((32, (p32, a32)), (64, (p64, a64))):
        n_arr, e_arr, _ = orc.seed(width, 77 + width, 8)
        for n, e in zip(n_arr, e_arr):
            n, e = int(n), int(e)
            c, r, _, _ = orc.generate(p, a, n, e, rng.randrange(n), 1, 4000)
            for ci, ri in zip(c, r):
                ci = int(ci)
                want = _exact_nearest_double(float(ci + 1), float(n + 1))
                assert float(ri) == want
                if width == 32:
                    assert float(ri) == (ci + 1) / (n + 1)   # both operands exact
                    assert 0.0 < ri < 1.0
                else:
                    assert 0.0 < ri <= 1.0


def test_uniform_can_round_to_one_for_64bit_moduli(orc):
    """For n near 2^63 the largest ciphertexts give R = 1.0 (reading of the
    open interval of Sec. IV: R lies in (0, 1] for 64-bit moduli)."""
    n = (1 << 63) - 25
    assert orc.is_prime(n)
    c = n - 1
    assert float(c + 1) / float(n + 1) == 1.0


def test_generate_many_equals_single_instance_loop(orc):
    p, a = orc.lcg_params(32)
    n, e, k = orc.seed(32, 5, 16)
    counts = np.array([1 + 37 * i for i in range(16)], dtype=np.uint64)
    c, r, m_after, s_after, off = orc.generate_many(p, a, n, e, 0, 1, counts, nthreads=4)
    for i in range(16):
        ci, ri, mi, si = orc.generate(p, a, int(n[i]), int(e[i]), 0, 1, int(counts[i]))
        o = int(off[i])
        assert np.array_equal(c[o:o + int(counts[i])], ci)
        assert np.array_equal(r[o:o + int(counts[i])], ri)
        assert (int(m_after[i]), int(s_after[i])) == (mi, si)


# --------------------------------------------------------------------------
# Seeding (Sec. IV)
# --------------------------------------------------------------------------

def test_splitmix64_reference_outputs(orc, paper):
    ref = paper["splitmix64_reference"]
    got = orc.splitmix64(ref["seed"], len(ref["outputs"]))
    assert [int(x) for x in got] == ref["outputs"]


@pytest.mark.parametrize("width", [32, 64])
def test_seeded_instances_are_admissible_and_distinct(orc, width):
    rng = random.Random(14)
    n, e, k = orc.seed(width, 0x14112484, 2000, (9, 17), 10, 1 << 40)
    lo = 1 << 31 if width == 32 else 1 << 62
    assert np.unique(n).size == n.size
    for ni, ei, ki in zip(n[:300], e, k):
        ni, ei, ki = int(ni), int(ei), int(ki)
        assert lo <= ni < 2 * lo
        assert _py_probable_prime(ni, rng)
        assert ei in (9, 17) and math.gcd(ei, ni - 1) == 1
        assert 10 <= ki < 1 << 40
    n2, e2, k2 = orc.seed(width, 0x14112484, 2000, (9, 17), 10, 1 << 40)
    assert np.array_equal(n, n2) and np.array_equal(e, e2) and np.array_equal(k, k2)
    # both exponents are used; e = 9 only where 3 does not divide n - 1
    assert set(int(x) for x in np.unique(e)) == {9, 17}


# --------------------------------------------------------------------------
# Unit and constant skips (Sec. II)
# --------------------------------------------------------------------------

def test_unit_skip_stream_reproduces_fig2(orc, paper):
    fx = paper["unit_skip_fig2"]
    n, e = fx["n"], fx["e"]
    # position 0 holds m_0 = 0 (c_0 = 0); draws return c_1, c_2, ...
    assert orc.encrypt(orc.cskip_message(n, 0, 1, 0), e, n) == fx["ciphertexts"][0]
    c, r, m = orc.generate_cskip(n, e, 1, 0, 4)
    assert [int(x) for x in c] == fx["ciphertexts"][1:]
    assert m == 4


def test_constant_skip_is_a_scaled_unit_skip(orc):
    """Eq. (4): (k b)^e = (b^e mod n)(k^e mod n) mod n, and the symmetry
    ((n-k) b)^e = n - (k b)^e mod n (Sec. II)."""
    rng = random.Random(31)
    n, e = 4294967087, 9
    for _ in range(5):
        b = rng.randrange(2, n - 1)
        cb, _, _ = orc.generate_cskip(n, e, b, 0, 3000, want_r=False)
        cu, _, _ = orc.generate_cskip(n, e, 1, 0, 3000, want_r=False)
        be = orc.encrypt(b, e, n)
        assert all(int(x) == be * int(y) % n for x, y in zip(cb, cu))
        for k in rng.sample(range(1, 3000), 50):
            ck = orc.encrypt(orc.cskip_message(n, 0, b, k), e, n)
            cnk = orc.encrypt(orc.cskip_message(n, 0, b, n - k), e, n)
            assert cnk == n - ck


def test_constant_skip_closed_form_and_full_period(orc):
    rng = random.Random(32)
    for n in (101, 1009, 4099):
        for e in [x for x in (3, 5, 7, 9, 11, 17) if math.gcd(x, n - 1) == 1][:2]:
            b, m0 = rng.randrange(1, n), rng.randrange(n)
            c, r, m = orc.generate_cskip(n, e, b, m0, n, want_r=True)
            # every ciphertext exactly once over the period n
            assert np.array_equal(np.sort(c), np.arange(n, dtype=np.uint64))
            assert m == m0
            for k in (1, 2, n // 2, n - 1):
                assert orc.encrypt(orc.cskip_message(n, m0, b, k), e, n) == int(c[k - 1])
            for ci, ri in zip(c[:50], r[:50]):
                assert float(ri) == (int(ci) + 1) / (n + 1)


def test_oracle_reproduces_crosscheck_values(orc, tab32):
    """The example instance of Sec. II from the base state: draws, states and
    skip sums written by tests/golden/make_crosscheck_values.py from plain
    Python integers (independent of the oracle's C code)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crosscheck_values.json")) as f:
        g = json.load(f)
    n, e, p, a = g["n"], g["e"], g["p"], g["a"]
    assert orc.lcg_params(32) == (p, a)
    c, r, m, s = orc.generate(p, a, n, e, 0, 1, 10 ** 6)
    for row in g["draws"]:
        k = row["k"]
        assert int(c[k - 1]) == row["c"] and r[k - 1] == float.fromhex(row["R"]), k
        # eq. (7) positions from the checkpoints and by looping agree with the stepped state
        assert orc.position(tab32, p, a, n, 0, 1, k) == (row["m"], row["s"])
    assert (m, s) == (g["draws"][-1]["m"], g["draws"][-1]["s"])
    assert orc.position(None, p, a, n, 0, 1, 10 ** 6) == (m, s)
    assert tab32.prefix(10 ** 6) == g["U_1e6"]
    assert tab32.prefix(p - 1) % n == g["full_period_skip_sum_mod_n"]
    assert orc.inverse(a, p) == g["a_inverse_mod_p"]
    assert orc.inverse(e, n - 1) == g["d"]
    assert orc.decrypt(g["draws"][-1]["c"], e, n) == g["draws"][-1]["m"]
