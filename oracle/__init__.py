"""CPU oracle for the Pohlig-Hellman parameter-split generator.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports
this package, and this package never imports the GPU library.

The arithmetic lives in ``phoracle.c`` (plain C, ``unsigned __int128``
products reduced with ``%``); this module is a thin ctypes wrapper.  See the
header of ``phoracle.c`` for the readings of the paper it follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phoracle.c")
_LIB_PATH = os.path.join(_HERE, "libphoracle.so")

OK, E_INVALID, E_NOT_PRIME, E_EXPONENT, E_RANGE = 0, -1, -2, -3, -4

_u64 = ctypes.c_uint64
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pdbl = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile phoracle.c into libphoracle.so (gcc, strict IEEE flags)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-pthread", "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "pho_mulmod": (_u64, [_u64, _u64, _u64]),
            "pho_powmod": (_u64, [_u64, _u64, _u64]),
            "pho_gcd": (_u64, [_u64, _u64]),
            "pho_inverse": (_u64, [_u64, _u64]),
            "pho_encrypt": (_u64, [_u64, _u64, _u64]),
            "pho_decrypt": (_u64, [_u64, _u64, _u64]),
            "pho_encrypt_many": (None, [_pu64, _u64, _u64, _u64, _pu64]),
            "pho_strong_probable_prime": (ctypes.c_int, [_u64, _u64]),
            "pho_is_prime": (ctypes.c_int, [_u64]),
            "pho_is_safe_prime": (ctypes.c_int, [_u64]),
            "pho_is_primitive_root": (ctypes.c_int, [_u64, _u64]),
            "pho_lcg_params": (ctypes.c_int, [ctypes.c_int, _pu64, _pu64]),
            "pho_check_instance": (ctypes.c_int, [ctypes.c_int, _u64, _u64]),
            "pho_skiptab_new": (ctypes.c_void_p, [_u64, _u64, _u64, _u64, ctypes.c_int]),
            "pho_skiptab_free": (None, [ctypes.c_void_p]),
            "pho_skiptab_max_r": (_u64, [ctypes.c_void_p]),
            "pho_skip_prefix": (ctypes.c_int, [ctypes.c_void_p, _u64, _pu64, _pu64]),
            "pho_position": (ctypes.c_int, [ctypes.c_void_p, _u64, _u64, _u64, _u64, _u64, _u64, _pu64, _pu64]),
            "pho_generate": (None, [_u64, _u64, _u64, _u64, _pu64, _pu64, _u64, _pu64, _pdbl]),
            "pho_generate_many": (None, [ctypes.c_int, _u64, _pu64, _pu64, _pu64, _pu64, _pu64, _pu64, _pu64,
                                         _pu64, _pu64, _pdbl]),
            "pho_jump_forward": (None, [_u64, _u64, _u64, _pu64, _pu64, _u64]),
            "pho_cskip_message": (_u64, [_u64, _u64, _u64, _u64]),
            "pho_generate_cskip": (None, [_u64, _u64, _u64, _pu64, _u64, _pu64, _pdbl]),
            "pho_jump_backward": (None, [_u64, _u64, _u64, _pu64, _pu64, _u64]),
            "pho_splitmix64": (None, [_u64, _u64, _pu64]),
            "pho_seed": (ctypes.c_int, [ctypes.c_int, _u64, _u64, _pu64, ctypes.c_int, _u64, _u64, _pu64, _pu64,
                                        _pu64]),
            "pho_count_many": (_u64, [ctypes.c_int, _pu64, _u64, ctypes.c_int, _u64]),
            "pho_pattern_hist": (None, [_u64, _u64, _u64, _u64, _u64, _u64, ctypes.c_int, _u64, _u64, _u64, _pu64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(_pu64)


def _pd(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_pdbl)


# --- scalar number theory -------------------------------------------------

def mulmod(x, y, n):
    return lib().pho_mulmod(x, y, n)


def powmod(b, e, n):
    return lib().pho_powmod(b, e, n)


def gcd(x, y):
    return lib().pho_gcd(x, y)


def inverse(e, m):
    return lib().pho_inverse(e, m)


def encrypt(m, e, n):
    return lib().pho_encrypt(m, e, n)


def encrypt_many(m, e, n):
    m = np.ascontiguousarray(m, dtype=np.uint64)
    out = np.zeros_like(m)
    lib().pho_encrypt_many(_p64(m), m.size, e, n, _p64(out))
    return out


def decrypt(c, e, n):
    return lib().pho_decrypt(c, e, n)


def strong_probable_prime(n, g):
    return bool(lib().pho_strong_probable_prime(n, g))


def is_prime(n):
    return bool(lib().pho_is_prime(n))


def is_safe_prime(n):
    return bool(lib().pho_is_safe_prime(n))


def is_primitive_root(a, p):
    return bool(lib().pho_is_primitive_root(a, p))


def lcg_params(width):
    p, a = _u64(), _u64()
    st = lib().pho_lcg_params(width, ctypes.byref(p), ctypes.byref(a))
    if st != OK:
        raise ValueError("bad width")
    return p.value, a.value


def check_instance(width, n, e):
    return lib().pho_check_instance(width, n, e)


# --- skip-sum checkpoints and positioning (eq. (7)) -----------------------

class SkipTab:
    """Checkpoints of U(r) = sum_{j<=r} (a^j mod p) every `stride` up to max_r."""

    def __init__(self, p, a, stride, max_r, nthreads=0):
        self.p, self.a, self.stride = p, a, stride
        self._h = lib().pho_skiptab_new(p, a, stride, max_r, nthreads)
        if not self._h:
            raise ValueError("skip table: bad arguments")
        self.max_r = lib().pho_skiptab_max_r(self._h)

    def prefix(self, r):
        lo, hi = _u64(), _u64()
        st = lib().pho_skip_prefix(self._h, r, ctypes.byref(lo), ctypes.byref(hi))
        if st != OK:
            raise ValueError("r out of table reach")
        return (hi.value << 64) | lo.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pho_skiptab_free(h)
            self._h = None


def position(tab, p, a, n, m0, s0, k):
    """State (m_k, s_k) at position k by eq. (7).  tab may be None (looped sum)."""
    m, s = _u64(), _u64()
    h = tab._h if tab is not None else None
    st = lib().pho_position(h, p, a, n, m0, s0, k, ctypes.byref(m), ctypes.byref(s))
    if st != OK:
        raise ValueError("position: status %d" % st)
    return m.value, s.value


# --- generation (algorithm (9)) -------------------------------------------

def generate(p, a, n, e, m, s, count, want_c=True, want_r=True):
    """Run algorithm (9) `count` times from (m, s).  Returns (c, R, m, s)."""
    mm, ss = _u64(m), _u64(s)
    c = np.zeros(count, dtype=np.uint64) if want_c else None
    r = np.zeros(count, dtype=np.float64) if want_r else None
    lib().pho_generate(p, a, n, e, ctypes.byref(mm), ctypes.byref(ss), count,
                       _p64(c) if want_c else None, _pd(r) if want_r else None)
    return c, r, mm.value, ss.value


def generate_many(p, a, n, e, m, s, count, want_c=True, want_r=True, nthreads=0):
    """Many instances at once (threaded).  Arrays are per instance; returns
    (c, R, m, s, offsets) with outputs of instance i at offsets[i]."""
    n = np.ascontiguousarray(n, dtype=np.uint64)
    ninst = n.size
    def arr(x):
        x = np.asarray(x, dtype=np.uint64)
        if x.ndim == 0:
            x = np.full(ninst, x, dtype=np.uint64)
        return np.ascontiguousarray(x.copy())
    p, a, e, m, s, count = arr(p), arr(a), arr(e), arr(m), arr(s), arr(count)
    off = np.zeros(ninst, dtype=np.uint64)
    if ninst > 1:
        off[1:] = np.cumsum(count[:-1], dtype=np.uint64)
    total = int(count.sum())
    c = np.zeros(total, dtype=np.uint64) if want_c else None
    r = np.zeros(total, dtype=np.float64) if want_r else None
    lib().pho_generate_many(nthreads, ninst, _p64(p), _p64(a), _p64(n), _p64(e), _p64(m), _p64(s), _p64(count),
                            _p64(off), _p64(c) if want_c else None, _pd(r) if want_r else None)
    return c, r, m, s, off


def cskip_message(n, m0, b, k):
    """Message at position k under the constant skip b (unit skip: b = 1)."""
    return lib().pho_cskip_message(n, m0, b, k)


def generate_cskip(n, e, b, m, count, want_c=True, want_r=True):
    """Constant-skip draws from message m.  Returns (c, R, m)."""
    mm = _u64(m)
    c = np.zeros(count, dtype=np.uint64) if want_c else None
    r = np.zeros(count, dtype=np.float64) if want_r else None
    lib().pho_generate_cskip(n, e, b, ctypes.byref(mm), count, _p64(c) if want_c else None,
                             _pd(r) if want_r else None)
    return c, r, mm.value


def jump_forward(p, a, n, m, s, delta):
    mm, ss = _u64(m), _u64(s)
    lib().pho_jump_forward(p, a, n, ctypes.byref(mm), ctypes.byref(ss), delta)
    return mm.value, ss.value


def jump_backward(p, a, n, m, s, delta):
    mm, ss = _u64(m), _u64(s)
    lib().pho_jump_backward(p, a, n, ctypes.byref(mm), ctypes.byref(ss), delta)
    return mm.value, ss.value


# --- seeding --------------------------------------------------------------

def splitmix64(seed, count):
    out = np.zeros(count, dtype=np.uint64)
    lib().pho_splitmix64(seed, count, _p64(out))
    return out


def seed(width, seed_value, count, e_set=(9, 17), k_lo=0, k_hi=0):
    """Seeded instances: returns arrays (n, e, k)."""
    es = np.ascontiguousarray(np.asarray(e_set, dtype=np.uint64))
    n = np.zeros(count, dtype=np.uint64)
    e = np.zeros(count, dtype=np.uint64)
    k = np.zeros(count, dtype=np.uint64)
    st = lib().pho_seed(width, seed_value, count, _p64(es), int(es.size), k_lo, k_hi, _p64(n), _p64(e), _p64(k))
    if st != OK:
        raise ValueError("seed: status %d" % st)
    return n, e, k


def count_many(values, mode, e=0, nthreads=0):
    """mode 0: #prime; 1: #safe prime; 2: #(gcd(e, v-1) = 1)."""
    v = np.ascontiguousarray(values, dtype=np.uint64)
    return int(lib().pho_count_many(nthreads, _p64(v), v.size, mode, e))


def pattern_hist(n, e, p, a, x0, l0, dim, bins, s_lo, s_hi):
    """Full-period local pattern histogram (Sec. II, Figs. 3-4): counts of the D-1
    points that follow every first point c in [x0, x0 + l0), over skips
    s in [s_lo, s_hi), in bins^(dim-1) cells."""
    hist = np.zeros(int(bins) ** (int(dim) - 1), dtype=np.uint64)
    lib().pho_pattern_hist(n, e, p, a, x0, l0, int(dim), bins, s_lo, s_hi, _p64(hist))
    return hist
