"""Python binding of libzoneburn (the C ABI of include/zoneburn.h).

Argument marshalling only: every step of the burn runs in the library's HIP
kernels.  torch supplies device memory and streams; tensors are passed by
data pointer and the current (or given) torch stream.  The library must be
built (python -m paper_2608_06466_amd.build); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzoneburn.so")

OK, EINVAL, ENOMEM, EDEVICE, EZONES, EBUSY, ENOTFOUND, EUNSUPPORTED = range(8)
FP64, MIXED = 0, 1
ZONE_STATUS = {0: "OK", 1: "MAXSTEPS", 2: "ERRTEST", 3: "CONV", 4: "HMIN", 5: "NONFINITE"}
STAT_FIELDS = ("nst", "nfe", "nje", "nlu", "nni", "netf", "ncf")


class ZoneburnError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().zb_last_error().decode() if _lib is not None else ""
        super().__init__(f"{where}: {lib().zb_strerror(code).decode()} ({msg})")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("thermal", C.c_int32), ("n_reactions", C.c_int32),
                ("reactant", C.POINTER(C.c_int32)), ("product", C.POINTER(C.c_int32)),
                ("lnA", C.POINTER(C.c_double)), ("n_exp", C.POINTER(C.c_double)),
                ("E", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("precision", C.c_int32), ("mapping", C.c_int32),
                ("reserved", C.c_int32)]


class _Segment(C.Structure):
    _fields_ = [("net", C.c_void_p), ("state", C.c_void_p), ("zones", C.c_int64),
                ("dt", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("rate_scale", C.c_void_p), ("zone_status", C.c_void_p), ("stats", C.c_void_p)]


_lib = None


def lib():
    """Load libzoneburn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2608_06466_amd.build`")
        L = C.CDLL(LIB_PATH)
        e, p, i32, i64, d = C.c_int, C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "zb_context_create": [C.c_int, C.POINTER(p)],
            "zb_context_destroy": [p],
            "zb_network_create": [p, C.POINTER(_Desc), C.POINTER(p)],
            "zb_network_destroy": [p],
            "zb_network_info": [p, C.POINTER(i32), C.POINTER(i32)],
            "zb_burn": [p, p, p, i64, d, d, d, p, C.POINTER(_Opts), p, p, p],
            "zb_sync": [p, p, C.POINTER(i64)],
            "zb_burn_batch": [p, C.POINTER(_Segment), i32, C.POINTER(_Opts), p],
            "zb_get_mapping": [p, p, i32, C.POINTER(i32)],
            "zb_autotune": [p, p, p, i64, d, d, d, i32, C.POINTER(i32), C.POINTER(C.c_float)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = e
        L.zb_strerror.argtypes = [e]
        L.zb_strerror.restype = C.c_char_p
        L.zb_last_error.argtypes = []
        L.zb_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(code, where):
    if code != OK:
        raise ZoneburnError(code, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    def __init__(self, device=0):
        h = C.c_void_p()
        _check(lib().zb_context_create(int(device), C.byref(h)), "zb_context_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().zb_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    """Device copy of a network dict (see paper_2608_06466_amd.workloads)."""

    def __init__(self, ctx: Context, net):
        self.ctx = ctx
        self.ns = int(net["n_species"])
        self.thermal = int(net["thermal"])
        self._keep = [np.ascontiguousarray(net[k], dtype=dt) for k, dt in
                      (("reactant", np.int32), ("product", np.int32), ("lnA", np.float64),
                       ("n_exp", np.float64), ("E", np.float64), ("q", np.float64))]
        ra, pa, lnA, n, E, q = self._keep
        self.nr = int(lnA.shape[0])
        desc = _Desc(self.ns, self.thermal, self.nr,
                     ra.ctypes.data_as(C.POINTER(C.c_int32)), pa.ctypes.data_as(C.POINTER(C.c_int32)),
                     lnA.ctypes.data_as(C.POINTER(C.c_double)), n.ctypes.data_as(C.POINTER(C.c_double)),
                     E.ctypes.data_as(C.POINTER(C.c_double)), q.ctypes.data_as(C.POINTER(C.c_double)))
        h = C.c_void_p()
        _check(lib().zb_network_create(ctx.h, C.byref(desc), C.byref(h)), "zb_network_create")
        self.h = h
        self.nv = self.ns + self.thermal

    def close(self):
        if self.h:
            lib().zb_network_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(precision, lanes, max_steps):
    prec = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}[precision]
    return _Opts(int(max_steps or 0), prec, int(lanes or 0), 0)


def _check_state(net, state):
    import torch
    if not (isinstance(state, torch.Tensor) and state.is_cuda and state.dtype == torch.float64
            and state.dim() == 2 and state.shape[1] == net.ns + 1 and state.is_contiguous()):
        raise ValueError("state must be a contiguous float64 CUDA tensor [zones][ns+1]")


def burn(ctx, net, state, dt, rtol, atol, rate_scale=None, precision="fp64", lanes=0,
         max_steps=0, want_status=True, want_stats=True, stream=None):
    """In-place burn of state [zones][ns+1]; returns (status int32[zones], stats int32[zones,7])."""
    import torch
    _check_state(net, state)
    zones = state.shape[0]
    if rate_scale is not None and (rate_scale.dtype != torch.float64 or not rate_scale.is_cuda
                                   or tuple(rate_scale.shape) != (zones, net.nr)
                                   or not rate_scale.is_contiguous()):
        raise ValueError("rate_scale must be a contiguous float64 CUDA tensor [zones][R]")
    status = torch.empty(zones, dtype=torch.int32, device=state.device) if want_status else None
    stats = torch.empty((zones, 7), dtype=torch.int32, device=state.device) if want_stats else None
    o = _opts(precision, lanes, max_steps)
    _check(lib().zb_burn(ctx.h, net.h, _ptr(state), zones, float(dt), float(rtol), float(atol),
                         _ptr(rate_scale), C.byref(o), _ptr(status), _ptr(stats),
                         _stream_handle(stream)), "zb_burn")
    return status, stats


def burn_batch(ctx, segments, precision="fp64", lanes=0, max_steps=0, stream=None):
    """segments: list of dicts(net, state, dt, rtol, atol, rate_scale=None, status=None, stats=None)."""
    arr = (_Segment * len(segments))()
    for i, s in enumerate(segments):
        _check_state(s["net"], s["state"])
        arr[i] = _Segment(s["net"].h.value, s["state"].data_ptr(), s["state"].shape[0],
                          float(s["dt"]), float(s["rtol"]), float(s["atol"]),
                          _ptr(s.get("rate_scale")).value if s.get("rate_scale") is not None else None,
                          s["status"].data_ptr() if s.get("status") is not None else None,
                          s["stats"].data_ptr() if s.get("stats") is not None else None)
    o = _opts(precision, lanes, max_steps)
    _check(lib().zb_burn_batch(ctx.h, arr, len(segments), C.byref(o), _stream_handle(stream)),
           "zb_burn_batch")


def sync(ctx, stream=None):
    """Wait for the stream; returns the number of zones that failed since the last sync."""
    n = C.c_int64(0)
    code = lib().zb_sync(ctx.h, _stream_handle(stream), C.byref(n))
    if code not in (OK, EZONES):
        _check(code, "zb_sync")
    return int(n.value)


def get_mapping(ctx, net, precision="fp64"):
    v = C.c_int32(0)
    _check(lib().zb_get_mapping(ctx.h, net.h, _opts(precision, 0, 0).precision, C.byref(v)),
           "zb_get_mapping")
    return int(v.value)


def autotune(ctx, net, sample_state, dt, rtol, atol, precision="fp64"):
    """Times every supported lanes-per-zone mapping on sample_state; returns (best, times_ms[7])."""
    _check_state(net, sample_state)
    best = C.c_int32(0)
    times = (C.c_float * 7)()
    _check(lib().zb_autotune(ctx.h, net.h, _ptr(sample_state), sample_state.shape[0], float(dt),
                             float(rtol), float(atol), _opts(precision, 0, 0).precision,
                             C.byref(best), times), "zb_autotune")
    return int(best.value), list(times)
