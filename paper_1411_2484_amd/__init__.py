"""Python binding of libphprng.so, the gfx950 library for the Pohlig-Hellman
parameter-split pseudorandom number generator (include/phprng.h).

This module only marshals arguments: every step of generation runs in the
HIP kernels of the library.  Importing it does not load the library; the
first call does, and raises if ``libphprng.so`` has not been built
(``python -m paper_1411_2484_amd.build``).  There is no CPU fallback.

Device memory and streams come from PyTorch: output arrays are CUDA (HIP)
tensors and ``stream`` defaults to ``torch.cuda.current_stream()``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphprng.so")

PHPRNG_OK = 0
PHPRNG_E_INVALID = -1
PHPRNG_E_NOT_PRIME = -2
PHPRNG_E_EXPONENT = -3
PHPRNG_E_RANGE = -4
PHPRNG_E_NOMEM = -5
PHPRNG_E_DEVICE = -6

PHPRNG_MODE_PERSISTENT = 0
PHPRNG_MODE_PLAIN = 1

PHPRNG_CLASS_W32 = 0
PHPRNG_CLASS_W64 = 1
PHPRNG_CLASS_MIXED = 2

NOALLOC_MAX_REQUESTS = 16384
NOALLOC_MAX_TILES64 = 1 << 18

_u64 = ctypes.c_uint64
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pu32 = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p


class phprng_state(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint64), ("s", ctypes.c_uint64), ("c", ctypes.c_uint64), ("k", ctypes.c_uint64)]


class phprng_request(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("count", ctypes.c_uint64),
                ("out_offset", ctypes.c_uint64)]


class phprng_tuning(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tiles_per_chunk", ctypes.c_int32), ("unroll", ctypes.c_int32)]


class phprng_server_config(ctypes.Structure):
    _fields_ = [("arena_doubles", ctypes.c_uint64), ("streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("max_batch_draws", ctypes.c_uint64)]


class phprng_test_result(ctypes.Structure):
    _fields_ = [("chi2", ctypes.c_double), ("p_value", ctypes.c_double), ("dof", ctypes.c_uint64),
                ("samples", ctypes.c_uint64)]


class phprng_pattern(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("e", ctypes.c_uint64), ("x0", ctypes.c_uint64), ("l0", ctypes.c_uint64),
                ("s_lo", ctypes.c_uint64), ("s_hi", ctypes.c_uint64), ("dim", ctypes.c_uint32),
                ("bins", ctypes.c_uint32)]


class phprng_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("instance", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("count", ctypes.c_uint64), ("k", ctypes.c_uint64),
                ("data", ctypes.c_void_p), ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class phprng_server_counters(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("requests", ctypes.c_uint64), ("draws", ctypes.c_uint64),
                ("launch_ns", ctypes.c_int64), ("launch_ns_max", ctypes.c_int64),
                ("arena_stalls", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("form_ns", ctypes.c_int64), ("retire_ns", ctypes.c_int64)]


ARRIVAL_DTYPE = np.dtype([("t_ns", np.int64), ("instance", np.uint32), ("reserved", np.uint32),
                          ("count", np.uint64)])

REQUEST_DTYPE = np.dtype([("instance", np.uint32), ("reserved", np.uint32), ("count", np.uint64),
                          ("out_offset", np.uint64)])

# name -> (restype, argtypes); every symbol declared in include/phprng.h
SIGNATURES = {
    "phprng_skip_params": (ctypes.c_int, [ctypes.c_int, _pu64, _pu64]),
    "phprng_check_instance": (ctypes.c_int, [ctypes.c_int, _u64, _u64]),
    "phprng_draw_instances": (ctypes.c_int, [ctypes.c_int, _u64, _u64, _pu64, ctypes.c_int, _u64, _u64, _pu64,
                                             _pu64, _pu64]),
    "phprng_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "phprng_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _u64]),
    "phprng_destroy": (ctypes.c_int, [_vp]),
    "phprng_last_error": (ctypes.c_char_p, [_vp]),
    "phprng_add_instances": (ctypes.c_int, [_vp, _u64, ctypes.c_int, _pu64, _pu64, _pu64, _pu64, _pu64, _pu32]),
    "phprng_seed_instances": (ctypes.c_int, [_vp, _u64, ctypes.c_int, _u64, _pu64, ctypes.c_int, _u64, _u64,
                                             _pu32]),
    "phprng_instance_count": (_u64, [_vp]),
    "phprng_add_instances_skip": (ctypes.c_int, [_vp, _u64, ctypes.c_int, _pu64, _pu64, _pu64, _pu64, _pu64,
                                                 _pu32]),
    "phprng_get_schedule": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int), _pu64]),
    "phprng_generate": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _vp, _u64, _vp, ctypes.c_int]),
    "phprng_generate_noalloc": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _vp, _u64, _vp]),
    "phprng_jump": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_int64]),
    "phprng_get_state": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.POINTER(phprng_state)]),
    "phprng_set_state": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.POINTER(phprng_state)]),
    "phprng_get_params": (ctypes.c_int, [_vp, ctypes.c_uint32, _pu64, _pu64, _pu64, _pu64,
                                         ctypes.POINTER(ctypes.c_int)]),
    "phprng_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(phprng_tuning)]),
    "phprng_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(phprng_tuning)]),
    "phprng_set_tuning_class": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(phprng_tuning)]),
    "phprng_get_tuning_class": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(phprng_tuning)]),
    "phprng_autotune": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(phprng_tuning)]),
    "phprng_graph_create": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _vp, _u64, _vp, ctypes.POINTER(_vp)]),
    "phprng_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "phprng_graph_destroy": (ctypes.c_int, [_vp]),
    "phprng_last_kernel_ms": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "phprng_get_position": (ctypes.c_int, [_vp, ctypes.c_uint32, _pu64]),
    "phprng_server_create": (ctypes.c_int, [_vp, ctypes.POINTER(phprng_server_config), ctypes.POINTER(_vp)]),
    "phprng_server_submit": (ctypes.c_int, [_vp, ctypes.c_uint32, _u64, _u64, _pu64]),
    "phprng_server_poll": (ctypes.c_int, [_vp, ctypes.POINTER(phprng_completion), _u64, _pu64, ctypes.c_int64]),
    "phprng_server_release": (ctypes.c_int, [_vp, _u64]),
    "phprng_server_release_many": (ctypes.c_int, [_vp, _vp, _u64]),
    "phprng_server_stats": (ctypes.c_int, [_vp, _pu64, _pu64]),
    "phprng_server_read_counters": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "phprng_server_destroy": (ctypes.c_int, [_vp]),
    "phprng_server_replay": (ctypes.c_int, [_vp, _vp, _u64, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "phprng_timing_reset": (ctypes.c_int, [_vp]),
    "phprng_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "phprng_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]),
    "phprng_battery_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "phprng_battery_destroy": (ctypes.c_int, [_vp]),
    "phprng_battery_last_error": (ctypes.c_char_p, [_vp]),
    "phprng_battery_reset": (ctypes.c_int, [_vp, _vp]),
    "phprng_battery_accumulate": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "phprng_battery_report": (ctypes.c_int, [_vp, ctypes.POINTER(phprng_test_result), _vp]),
    "phprng_battery_counts": (ctypes.c_int, [_vp, ctypes.c_int, _pu64, _u64, _pu64, _vp]),
    "phprng_battery_probabilities": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), _u64, _pu64]),
    "phprng_battery_fourier": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "phprng_battery_timing": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), _pu64]),
    "phprng_chi2_pvalue": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "phprng_interleave": (ctypes.c_int, [_vp, _vp, _u64, _u64, _vp]),
    "phprng_pattern_histogram": (ctypes.c_int, [ctypes.POINTER(phprng_pattern), _vp, _vp]),
    "phprng_pattern_chi2": (ctypes.c_int, [ctypes.POINTER(phprng_pattern), _vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), _pu64, _vp]),
}

BATTERY_BLOCK = 1 << 20
BATTERY_TESTS = ("frequency", "serial2", "serial3", "serial4", "serial5", "poker", "collision", "runs", "fourier")
BATTERY_KERNELS = ("hist", "collision", "runs", "fft_pass1", "fft_pass2", "hist_count")

_lib = None


def lib():
    """Load libphprng.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libphprng.so is not built: run `python -m paper_1411_2484_amd.build`")
        # torch ships its own HIP runtime under the same soname as ROCm's.
        # Loaded first, it is the one the library binds to and both share the
        # device; loaded after a context has started ROCm's, torch finds no
        # GPU.  So torch, when installed, is imported before the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PhprngError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        text = lib().phprng_status_string(status).decode()
        super().__init__("phprng status %d (%s)%s" % (status, text, ": " + message if message else ""))


def _u64arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    return a, a.ctypes.data_as(_pu64)


def _check(st, ctx=None):
    if st != PHPRNG_OK:
        msg = lib().phprng_last_error(ctx).decode() if ctx else ""
        raise PhprngError(st, msg)


# ---- host-only helpers -----------------------------------------------------

def phprng_skip_params(width):
    p, a = _u64(), _u64()
    _check(lib().phprng_skip_params(width, ctypes.byref(p), ctypes.byref(a)))
    return p.value, a.value


def phprng_check_instance(width, n, e):
    return lib().phprng_check_instance(width, n, e)


def phprng_draw_instances(width, seed, count, e_set=(9, 17), k_lo=0, k_hi=0):
    es, pes = _u64arr(e_set)
    n = np.zeros(count, dtype=np.uint64)
    e = np.zeros(count, dtype=np.uint64)
    k = np.zeros(count, dtype=np.uint64)
    _check(lib().phprng_draw_instances(width, seed, count, pes, int(es.size), k_lo, k_hi,
                                       n.ctypes.data_as(_pu64), e.ctypes.data_as(_pu64), k.ctypes.data_as(_pu64)))
    return n, e, k


def _stream_handle(stream, device=None):
    """Raw HIP stream: `stream` itself (an int or a torch stream), else the
    current torch stream of `device` (of the current device when None)."""
    if stream is None:
        import torch
        dev = torch.cuda.current_device() if device is None else int(device)
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return raw(dev)  # the handle without building a Stream object
        return torch.cuda.current_stream(dev).cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# element types each device array may have (the library writes 4-byte
# ciphertexts, 8-byte ciphertexts and binary64 uniforms)
_C32_DTYPES = ("int32", "uint32")
_C64_DTYPES = ("int64", "uint64")
_R_DTYPES = ("float64",)


def _device_array(t, dtypes, device, what):
    """Device address of tensor `t` after checking that it is a contiguous
    tensor on HIP device `device` with one of `dtypes`; None for None.
    Raises before anything is launched."""
    if t is None:
        return None
    dt = str(getattr(t, "dtype", "")).replace("torch.", "")
    if dt not in dtypes:
        raise TypeError("%s must have dtype %s, got %s" % (what, " or ".join(dtypes), dt or type(t).__name__))
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a device (cuda) tensor" % what)
    idx = getattr(getattr(t, "device", None), "index", None)
    if device is not None and idx is not None and idx != device:
        raise ValueError("%s is on device %s, the context on device %s" % (what, idx, device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return t.data_ptr()


def _outputs(out_c32, out_c64, out_r, device, capacity):
    """Checked device addresses of the three output arrays and the capacity
    (the smallest element count among the given arrays when not stated)."""
    p32 = _device_array(out_c32, _C32_DTYPES, device, "out_c32")
    p64 = _device_array(out_c64, _C64_DTYPES, device, "out_c64")
    pr = _device_array(out_r, _R_DTYPES, device, "out_r")
    caps = [t.numel() for t in (out_c32, out_c64, out_r) if t is not None]
    if capacity is None:
        capacity = min(caps) if caps else 0
    elif caps and int(capacity) > min(caps):
        raise ValueError("capacity %d exceeds an output array of %d elements" % (capacity, min(caps)))
    return p32, p64, pr, int(capacity)


def make_requests(instances, counts, offsets):
    """Request array (numpy structured, layout of phprng_request)."""
    inst = np.asarray(instances, dtype=np.uint32)
    r = np.zeros(inst.size, dtype=REQUEST_DTYPE)
    r["instance"] = inst
    r["count"] = np.asarray(counts, dtype=np.uint64)
    r["out_offset"] = np.asarray(offsets, dtype=np.uint64)
    return r


class Context:
    """A phprng_ctx on one device (owns the device instance table)."""

    def __init__(self, device=0, max_instances=1 << 16):
        h = _vp()
        _check(lib().phprng_create(ctypes.byref(h), int(device), int(max_instances)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().phprng_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st):
        _check(st, self._h)

    def add_instances(self, width, n, e, m0=None, s0=None, k0=None):
        n, pn = _u64arr(n)
        e, pe = _u64arr(e)
        count = n.size
        args = []
        keep = []
        for v in (m0, s0, k0):
            if v is None:
                args.append(None)
            else:
                a, pa = _u64arr(v)
                keep.append(a)
                args.append(pa)
        ids = np.zeros(count, dtype=np.uint32)
        self._chk(lib().phprng_add_instances(self._h, count, width, pn, pe, args[0], args[1], args[2],
                                             ids.ctypes.data_as(_pu32)))
        return ids

    def add_instances_skip(self, width, n, e, b, m0=None, k0=None):
        """Instances with the constant skip b (b = 1: unit skip)."""
        n, pn = _u64arr(n)
        e, pe = _u64arr(e)
        bb, pb = _u64arr(b)
        keep, args = [], []
        for v in (m0, k0):
            if v is None:
                args.append(None)
            else:
                a, pa = _u64arr(v)
                keep.append(a)
                args.append(pa)
        ids = np.zeros(n.size, dtype=np.uint32)
        self._chk(lib().phprng_add_instances_skip(self._h, n.size, width, pn, pe, pb, args[0], args[1],
                                                  ids.ctypes.data_as(_pu32)))
        return ids

    def get_schedule(self, inst):
        s, b = ctypes.c_int(), _u64()
        self._chk(lib().phprng_get_schedule(self._h, int(inst), ctypes.byref(s), ctypes.byref(b)))
        return s.value, b.value

    def seed_instances(self, width, seed, count, e_set=(9, 17), k_lo=0, k_hi=0):
        es, pes = _u64arr(e_set)
        ids = np.zeros(count, dtype=np.uint32)
        self._chk(lib().phprng_seed_instances(self._h, count, width, seed, pes, int(es.size), k_lo, k_hi,
                                              ids.ctypes.data_as(_pu32)))
        return ids

    def instance_count(self):
        return int(lib().phprng_instance_count(self._h))

    def generate(self, requests, out_c32=None, out_c64=None, out_r=None, capacity=None, stream=None,
                 mode=PHPRNG_MODE_PERSISTENT):
        """requests: numpy array of REQUEST_DTYPE.  Outputs are contiguous
        device tensors on this context's device (int32/uint32, int64/uint64,
        float64) or None."""
        reqs = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        p32, p64, pr, cap = _outputs(out_c32, out_c64, out_r, self.device, capacity)
        self._chk(lib().phprng_generate(self._h, reqs.ctypes.data, reqs.size, p32, p64, pr, cap,
                                        _stream_handle(stream, self.device), int(mode)))

    def generate_noalloc(self, requests, out_c32=None, out_c64=None, out_r=None, capacity=None, stream=None):
        """phprng_generate_noalloc: the persistent generation without any
        allocation (fixed per-device scratch; see include/phprng.h)."""
        reqs = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        p32, p64, pr, cap = _outputs(out_c32, out_c64, out_r, self.device, capacity)
        self._chk(lib().phprng_generate_noalloc(self._h, reqs.ctypes.data, reqs.size, p32, p64, pr, cap,
                                                _stream_handle(stream, self.device)))

    def last_kernel_ms(self):
        v = ctypes.c_double()
        self._chk(lib().phprng_last_kernel_ms(self._h, ctypes.byref(v)))
        return v.value

    def timing_reset(self):
        self._chk(lib().phprng_timing_reset(self._h))

    def set_timing(self, on):
        """phprng_set_timing: per-call kernel timing on (default) or off."""
        self._chk(lib().phprng_set_timing(self._h, 1 if on else 0))

    def timing_read(self):
        """(total generation-kernel ms, timed calls) since timing_reset."""
        ms, n = ctypes.c_double(), ctypes.c_uint64()
        self._chk(lib().phprng_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def get_position(self, inst):
        k = _u64()
        self._chk(lib().phprng_get_position(self._h, int(inst), ctypes.byref(k)))
        return k.value

    def jump(self, inst, delta):
        self._chk(lib().phprng_jump(self._h, int(inst), int(delta)))

    def get_state(self, inst):
        st = phprng_state()
        self._chk(lib().phprng_get_state(self._h, int(inst), ctypes.byref(st)))
        return st.m, st.s, st.c, st.k

    def set_state(self, inst, m, s, k):
        st = phprng_state(m, s, 0, k)
        self._chk(lib().phprng_set_state(self._h, int(inst), ctypes.byref(st)))

    def get_params(self, inst):
        n, e, p, a = _u64(), _u64(), _u64(), _u64()
        w = ctypes.c_int()
        self._chk(lib().phprng_get_params(self._h, int(inst), ctypes.byref(n), ctypes.byref(e), ctypes.byref(p),
                                          ctypes.byref(a), ctypes.byref(w)))
        return n.value, e.value, p.value, a.value, w.value

    def set_tuning(self, block_threads=0, blocks_per_cu=0, tiles_per_chunk=0, unroll=0):
        t = phprng_tuning(block_threads, blocks_per_cu, tiles_per_chunk, unroll)
        self._chk(lib().phprng_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = phprng_tuning()
        self._chk(lib().phprng_get_tuning(self._h, ctypes.byref(t)))
        return dict(block_threads=t.block_threads, blocks_per_cu=t.blocks_per_cu,
                    tiles_per_chunk=t.tiles_per_chunk, unroll=t.unroll)

    def set_tuning_class(self, cls, block_threads=0, blocks_per_cu=0, tiles_per_chunk=0, unroll=0):
        t = phprng_tuning(block_threads, blocks_per_cu, tiles_per_chunk, unroll)
        self._chk(lib().phprng_set_tuning_class(self._h, int(cls), ctypes.byref(t)))

    def get_tuning_class(self, cls):
        t = phprng_tuning()
        self._chk(lib().phprng_get_tuning_class(self._h, int(cls), ctypes.byref(t)))
        return dict(block_threads=t.block_threads, blocks_per_cu=t.blocks_per_cu,
                    tiles_per_chunk=t.tiles_per_chunk, unroll=t.unroll)

    def autotune(self, draws=1 << 26):
        t = phprng_tuning()
        self._chk(lib().phprng_autotune(self._h, int(draws), ctypes.byref(t)))
        return dict(block_threads=t.block_threads, blocks_per_cu=t.blocks_per_cu,
                    tiles_per_chunk=t.tiles_per_chunk, unroll=t.unroll)

    def graph(self, requests, out_c32=None, out_c64=None, out_r=None, capacity=None, stream=None):
        return Graph(self, requests, out_c32, out_c64, out_r, capacity, stream)


class Graph:
    """Captured repeat draws (phprng_graph_*)."""

    def __init__(self, ctx, requests, out_c32, out_c64, out_r, capacity, stream):
        reqs = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
        p32, p64, pr, cap = _outputs(out_c32, out_c64, out_r, ctx.device, capacity)
        h = _vp()
        _check(lib().phprng_graph_create(ctx.handle, reqs.ctypes.data, reqs.size, p32, p64, pr, cap,
                                         _stream_handle(stream, ctx.device), ctypes.byref(h)),
               ctx.handle)
        self._h = h
        self._ctx = ctx

    def launch(self, stream=None):
        _check(lib().phprng_graph_launch(self._h, _stream_handle(stream, self._ctx.device)), self._ctx.handle)

    def close(self):
        if getattr(self, "_h", None):
            lib().phprng_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """phprng_server_*: continuous batching over the instances of a context.
    While it exists, only the server uses the context."""

    def __init__(self, ctx, arena_doubles=1 << 28, streams=2, max_inflight=0, max_batch_requests=0,
                 max_batch_draws=0):
        cfg = phprng_server_config(int(arena_doubles), int(streams), int(max_inflight), int(max_batch_requests), 0,
                                   int(max_batch_draws))
        h = _vp()
        _check(lib().phprng_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), ctx.handle)
        self._h = h
        self._ctx = ctx

    def submit(self, instance, count, tag=0):
        t = _u64()
        _check(lib().phprng_server_submit(self._h, int(instance), int(count), int(tag), ctypes.byref(t)))
        return t.value

    def poll(self, max_items=256, timeout_us=1000):
        buf = (phprng_completion * max_items)()
        n = _u64()
        _check(lib().phprng_server_poll(self._h, buf, max_items, ctypes.byref(n), int(timeout_us)))
        return [buf[i] for i in range(n.value)]

    def release(self, ticket):
        _check(lib().phprng_server_release(self._h, int(ticket)))

    def release_many(self, tickets):
        t = np.ascontiguousarray(tickets, dtype=np.uint64)
        _check(lib().phprng_server_release_many(self._h, t.ctypes.data, t.size))

    def stats(self):
        p, u = _u64(), _u64()
        _check(lib().phprng_server_stats(self._h, ctypes.byref(p), ctypes.byref(u)))
        return p.value, u.value

    def counters(self, reset=False):
        """Launch counters (batches, requests, draws, launch_ns, launch_ns_max,
        arena_stalls, arena_peak, form_ns, retire_ns) as a dict; reset clears
        them after the read."""
        c = phprng_server_counters()
        _check(lib().phprng_server_read_counters(self._h, ctypes.byref(c), 1 if reset else 0))
        return {k: getattr(c, k) for k, _ in phprng_server_counters._fields_}

    def replay(self, arrivals):
        """arrivals: numpy array of ARRIVAL_DTYPE.  Returns (latency_ns array, wall seconds)."""
        lat, _, wall = self.replay_detail(arrivals)
        return lat, wall

    def replay_detail(self, arrivals):
        """As replay, plus the per-arrival admission delay: returns (latency_ns,
        admit_ns, wall seconds)."""
        arr = np.ascontiguousarray(arrivals, dtype=ARRIVAL_DTYPE)
        lat = np.zeros(arr.size, dtype=np.int64)
        adm = np.zeros(arr.size, dtype=np.int64)
        wall = ctypes.c_double()
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(lib().phprng_server_replay(self._h, arr.ctypes.data, arr.size, lat.ctypes.data_as(i64p),
                                          adm.ctypes.data_as(i64p), ctypes.byref(wall)))
        return lat, adm, wall.value

    def close(self):
        if getattr(self, "_h", None):
            lib().phprng_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- statistical battery (Tests section) ---------------------------------------

def chi2_pvalue(chi2, dof):
    """One-sided P-value min(Q, 1 - Q) of chi^2 with `dof` degrees of freedom."""
    p = ctypes.c_double()
    _check(lib().phprng_chi2_pvalue(float(chi2), float(dof), ctypes.byref(p)))
    return p.value


def battery_probabilities(test):
    """Category probabilities of a battery test (index into BATTERY_TESTS)."""
    n = _u64()
    _check(lib().phprng_battery_probabilities(int(test), None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.float64)
    _check(lib().phprng_battery_probabilities(int(test), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              out.size, ctypes.byref(n)))
    return out


def interleave(src, dst, nstreams, length, stream=None):
    """dst[t * nstreams + i] = src[i * length + t] (device float64 tensors)."""
    ps = _device_array(src, _R_DTYPES, None, "src")
    pd = _device_array(dst, _R_DTYPES, None, "dst")
    if src.numel() < nstreams * length or dst.numel() < nstreams * length:
        raise ValueError("interleave: arrays shorter than nstreams * length")
    _check(lib().phprng_interleave(ps, pd, int(nstreams), int(length), _stream_handle(stream)))


class Battery:
    """phprng_battery_*: device histograms of the nine chi-square tests."""

    def __init__(self, device=0):
        h = _vp()
        _check(lib().phprng_battery_create(ctypes.byref(h), int(device)))
        self._h = h

    def _chk(self, st):
        if st != PHPRNG_OK:
            raise PhprngError(st, lib().phprng_battery_last_error(self._h).decode())

    def reset(self, stream=None):
        self._chk(lib().phprng_battery_reset(self._h, _stream_handle(stream)))

    def accumulate(self, r, count=None, stream=None):
        """Add the uniforms of device tensor `r` (float64; count a multiple of 2^20)."""
        n = r.numel() if count is None else int(count)
        pr = _device_array(r, _R_DTYPES, None, "r")
        if n > r.numel():
            raise ValueError("count beyond the array")
        self._chk(lib().phprng_battery_accumulate(self._h, pr, n, _stream_handle(stream)))

    def report(self, stream=None):
        """{test name: (chi2, dof, p_value, samples)}."""
        out = (phprng_test_result * len(BATTERY_TESTS))()
        self._chk(lib().phprng_battery_report(self._h, out, _stream_handle(stream)))
        return {name: (out[i].chi2, out[i].dof, out[i].p_value, out[i].samples)
                for i, name in enumerate(BATTERY_TESTS)}

    def counts(self, test, stream=None):
        n = _u64()
        self._chk(lib().phprng_battery_counts(self._h, int(test), None, 0, ctypes.byref(n), _stream_handle(stream)))
        out = np.zeros(n.value, dtype=np.uint64)
        self._chk(lib().phprng_battery_counts(self._h, int(test), out.ctypes.data_as(_pu64), out.size,
                                              ctypes.byref(n), _stream_handle(stream)))
        return out

    def fourier(self, r, coef, count=None, stream=None):
        n = r.numel() if count is None else int(count)
        pr = _device_array(r, _R_DTYPES, None, "r")
        pc = _device_array(coef, _R_DTYPES, None, "coef")
        if n > r.numel() or coef.numel() < n:
            raise ValueError("fourier: arrays shorter than count")
        self._chk(lib().phprng_battery_fourier(self._h, pr, n, pc, _stream_handle(stream)))

    def timing(self):
        """{kernel class: (ms, launches)} since the last reset."""
        ms = (ctypes.c_double * len(BATTERY_KERNELS))()
        ln = (ctypes.c_uint64 * len(BATTERY_KERNELS))()
        self._chk(lib().phprng_battery_timing(self._h, ms, ln))
        return {k: (ms[i], ln[i]) for i, k in enumerate(BATTERY_KERNELS)}

    def close(self):
        if getattr(self, "_h", None):
            lib().phprng_battery_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- full-period local pattern (Sec. II, Figs. 3-4) ---------------------------------------

def pattern_spec(n, e, x0, l0, dim, bins, s_lo=1, s_hi=None):
    """phprng_pattern for a width-32 instance; s_hi defaults to p (the full period)."""
    if s_hi is None:
        s_hi = (1 << 31) - 1
    return phprng_pattern(int(n), int(e), int(x0), int(l0), int(s_lo), int(s_hi), int(dim), int(bins))


def pattern_histogram(spec, hist, stream=None):
    """Add the counts of `spec` to `hist` (device int64 tensor of bins^(dim-1))."""
    ph = _device_array(hist, _C64_DTYPES, None, "hist")
    # the library refuses a bad shape itself; for a shape it accepts, the
    # caller's array must hold every cell
    dim, bins = int(spec.dim), int(spec.bins)
    if 2 <= dim <= 5 and bins >= 1 and bins ** (dim - 1) <= (1 << 24) and hist.numel() < bins ** (dim - 1):
        raise ValueError("hist must hold bins^(dim-1) counts")
    _check(lib().phprng_pattern_histogram(ctypes.byref(spec), ph, _stream_handle(stream)))


def pattern_chi2(spec, hist, stream=None):
    """(chi2, p_value, total) of a pattern histogram."""
    c, p, t = ctypes.c_double(), ctypes.c_double(), _u64()
    ph = _device_array(hist, _C64_DTYPES, None, "hist")
    _check(lib().phprng_pattern_chi2(ctypes.byref(spec), ph, ctypes.byref(c), ctypes.byref(p),
                                     ctypes.byref(t), _stream_handle(stream)))
    return c.value, p.value, t.value
