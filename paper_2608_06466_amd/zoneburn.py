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
ZONE_STATUS = {0: "OK", 1: "MAXSTEPS", 2: "ERRTEST", 3: "CONV", 4: "HMIN", 5: "NONFINITE",
               6: "OK_RETRY", 7: "OK_FP64"}
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
                ("retry", C.c_int32), ("retry_rtol", C.c_double), ("retry_atol", C.c_double),
                ("retry_max_steps", C.c_int32), ("jac_policy", C.c_int32),
                ("integrator", C.c_int32), ("retry_jac", C.c_int32), ("lu", C.c_int32),
                ("fp64_fallback", C.c_int32)]


class _Segment(C.Structure):
    _fields_ = [("net", C.c_void_p), ("state", C.c_void_p), ("zones", C.c_int64),
                ("dt", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("rate_scale", C.c_void_p), ("zone_status", C.c_void_p), ("stats", C.c_void_p),
                ("source", C.c_void_p)]


class _ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("streams", C.c_int32),
                ("launches_per_stream", C.c_int32), ("slice_zones", C.c_int64),
                ("max_pending", C.c_int32), ("reserved", C.c_int32), ("burn", _Opts)]


class _TuneCand(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("lu", C.c_int32), ("ms", C.c_float),
                ("qualified", C.c_int32)]


class _ReqInfo(C.Structure):
    _fields_ = [("zones", C.c_int64), ("zones_ok", C.c_int64), ("queue_s", C.c_double),
                ("first_launch_s", C.c_double), ("latency_s", C.c_double)]


class _Totals(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("requests_done", "zones_done", "launches", "pending",
                                        "active", "bytes_in_use", "peak_bytes_in_use")]


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
            "zb_burn_batch_noalloc": [p, C.POINTER(_Segment), i32, C.POINTER(_Opts), p],
            "zb_get_mapping": [p, p, i32, C.POINTER(i32)],
            "zb_autotune": [p, p, p, i64, d, d, d, i32, C.POINTER(i32), C.POINTER(C.c_float)],
            "zb_tune_save": [p, C.c_char_p],
            "zb_tune_load": [p, C.c_char_p, C.POINTER(i32)],
            "zb_autotune_candidates": [p, p, p, i64, d, d, d, i32, C.POINTER(_TuneCand), i32,
                                       C.POINTER(i32), C.POINTER(i32)],
            "zb_graph_create": [p, C.POINTER(_Segment), i32, C.POINTER(_Opts), C.POINTER(p)],
            "zb_graph_launch": [p, p],
            "zb_graph_destroy": [p],
            "zb_server_create": [p, C.POINTER(_ServerOpts), C.POINTER(p)],
            "zb_server_submit": [p, p, p, i64, d, d, d, p, C.POINTER(C.c_uint64)],
            "zb_server_wait": [p, C.c_uint64, d, C.POINTER(i32)],
            "zb_server_fetch": [p, C.c_uint64, p, p, p, C.POINTER(_ReqInfo)],
            "zb_server_stats": [p, C.POINTER(_Totals)],
            "zb_server_destroy": [p],
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


JAC_EVERY_STEP, JAC_REUSE = 0, 1


BDF, RKC = 0, 1


def _opts(precision, lanes, max_steps, retry=None, jac_policy=0, integrator=0, lu="valu",
          fp64_fallback=False):
    """retry: None, or (rtol, atol, max_steps[, jac]) of the zone-by-zone retry of failed
    zones, jac "analytic" (default) or "fd" (finite-difference Jacobian in the retry).
    jac_policy: 0 Jacobian and LU every step attempt, 1 VODE-style reuse.
    integrator: "bdf" (0), "rkc" (1) or "bdf_variable" (2, VODE's variable-coefficient form).
    lu: "valu" (0), "mfma" (1, the blocked FP32 LU on the matrix cores; 48-row kernels) or
    "auto" (2, the pair of LU and lanes per zone autotune_candidates chose for the network).
    fp64_fallback: mixed precision only; zones that fail are burned again in FP64."""
    prec = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}[precision]
    jp = {"every_step": 0, "reuse": 1, 0: 0, 1: 1}[jac_policy]
    it = {"bdf": 0, "rkc": 1, "bdf_variable": 2, 0: 0, 1: 1, 2: 2}[integrator]
    lv = {"valu": 0, "mfma": 1, "auto": 2, 0: 0, 1: 1, 2: 2}.get(lu)
    if lv is None:
        raise ValueError("lu must be 'valu', 'mfma' or 'auto'")
    if retry is None:
        return _Opts(int(max_steps or 0), prec, int(lanes or 0), 0, 0.0, 0.0, 0, jp, it, 0, lv,
                     int(bool(fp64_fallback)))
    rjac = retry[3] if len(retry) > 3 else "analytic"
    rj = {"analytic": 0, "fd": 1, 0: 0, 1: 1}.get(rjac)
    if rj is None:
        raise ValueError("retry jac must be 'analytic' or 'fd'")
    return _Opts(int(max_steps or 0), prec, int(lanes or 0), 1, float(retry[0]), float(retry[1]),
                 int(retry[2]), jp, it, rj, lv, int(bool(fp64_fallback)))


def _check_state(net, state, cuda=True):
    import torch
    if not (isinstance(state, torch.Tensor) and (state.is_cuda or not cuda)
            and state.dtype == torch.float64 and state.dim() == 2
            and state.shape[1] == net.ns + 1 and state.is_contiguous()):
        raise ValueError("state must be a contiguous float64 CUDA tensor [zones][ns+1]")


def _check_buf(name, t, dtype, shape, device):
    """A per-zone buffer handed to the library: dtype, shape, contiguity and the state's device
    (the kernels index it by zone; anything else would read or write out of bounds)."""
    import torch
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype and tuple(t.shape) == tuple(shape)
            and t.is_contiguous() and t.device == device):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor {list(shape)} on {device}")


def _check_segment(s, cuda=True):
    """Validates one segment dict (state, rate_scale, status, stats, source)."""
    import torch
    net, st = s["net"], s["state"]
    _check_state(net, st, cuda)
    z = st.shape[0]
    _check_buf("rate_scale", s.get("rate_scale"), torch.float64, (z, net.nr), st.device)
    _check_buf("status", s.get("status"), torch.int32, (z,), st.device)
    _check_buf("stats", s.get("stats"), torch.int32, (z, 7), st.device)
    _check_buf("source", s.get("source"), torch.float64, tuple(st.shape), st.device)


def burn(ctx, net, state, dt, rtol, atol, rate_scale=None, precision="fp64", lanes=0,
         max_steps=0, want_status=True, want_stats=True, stream=None, source=None, retry=None,
         jac_policy=0, integrator="bdf", lu="valu", fp64_fallback=False):
    """In-place burn of state [zones][ns+1]; returns (status int32[zones], stats int32[zones,7]).

    source: optional constant per-zone term [zones][ns+1] added to the right-hand side
    (burned through zb_burn_batch, which takes it)."""
    import torch
    _check_state(net, state)
    if source is not None:
        zones = state.shape[0]
        status = torch.empty(zones, dtype=torch.int32, device=state.device) if want_status else None
        stats = torch.empty((zones, 7), dtype=torch.int32, device=state.device) if want_stats else None
        burn_batch(ctx, [dict(net=net, state=state, dt=dt, rtol=rtol, atol=atol, rate_scale=rate_scale,
                              status=status, stats=stats, source=source)],
                   precision=precision, lanes=lanes, max_steps=max_steps, stream=stream, retry=retry,
                   jac_policy=jac_policy, integrator=integrator, lu=lu,
                   fp64_fallback=fp64_fallback)
        return status, stats
    zones = state.shape[0]
    _check_buf("rate_scale", rate_scale, torch.float64, (zones, net.nr), state.device)
    status = torch.empty(zones, dtype=torch.int32, device=state.device) if want_status else None
    stats = torch.empty((zones, 7), dtype=torch.int32, device=state.device) if want_stats else None
    o = _opts(precision, lanes, max_steps, retry, jac_policy, integrator, lu, fp64_fallback)
    _check(lib().zb_burn(ctx.h, net.h, _ptr(state), zones, float(dt), float(rtol), float(atol),
                         _ptr(rate_scale), C.byref(o), _ptr(status), _ptr(stats),
                         _stream_handle(stream)), "zb_burn")
    return status, stats


def _src_ptr(src, state):
    return None if src is None else src.data_ptr()


def _segments(segments):
    arr = (_Segment * len(segments))()
    for i, s in enumerate(segments):
        _check_segment(s)
        arr[i] = _Segment(s["net"].h.value, s["state"].data_ptr(), s["state"].shape[0],
                          float(s["dt"]), float(s["rtol"]), float(s["atol"]),
                          _ptr(s.get("rate_scale")).value if s.get("rate_scale") is not None else None,
                          s["status"].data_ptr() if s.get("status") is not None else None,
                          s["stats"].data_ptr() if s.get("stats") is not None else None,
                          _src_ptr(s.get("source"), s["state"]))
    return arr


def burn_batch(ctx, segments, precision="fp64", lanes=0, max_steps=0, stream=None, retry=None,
               jac_policy=0, integrator="bdf", lu="valu", fp64_fallback=False):
    """segments: list of dicts(net, state, dt, rtol, atol, rate_scale=None, status=None,
    stats=None, source=None); retry: None or (rtol, atol, max_steps[, jac])."""
    arr = _segments(segments)
    o = _opts(precision, lanes, max_steps, retry, jac_policy, integrator, lu, fp64_fallback)
    _check(lib().zb_burn_batch(ctx.h, arr, len(segments), C.byref(o), _stream_handle(stream)),
           "zb_burn_batch")


def burn_batch_noalloc(ctx, segments, precision="fp64", lanes=0, max_steps=0, stream=None,
                       retry=None, jac_policy=0, integrator="bdf", lu="valu", fp64_fallback=False):
    """burn_batch through zb_burn_batch_noalloc: no device allocation, no stream or event
    creation, counters in the library's static device array (at most 4 kernel classes; every
    class on `stream` in turn)."""
    arr = _segments(segments)
    o = _opts(precision, lanes, max_steps, retry, jac_policy, integrator, lu, fp64_fallback)
    _check(lib().zb_burn_batch_noalloc(ctx.h, arr, len(segments), C.byref(o),
                                       _stream_handle(stream)), "zb_burn_batch_noalloc")


class Graph:
    """A burn of fixed buffers captured once as a HIP graph (zb_graph_*); launch() replays it."""

    def __init__(self, ctx, segments, precision="fp64", lanes=0, max_steps=0, retry=None,
                 jac_policy=0, integrator="bdf", lu="valu", fp64_fallback=False):
        self.ctx = ctx
        self._segs = segments          # the buffers must outlive the graph
        arr = _segments(segments)
        o = _opts(precision, lanes, max_steps, retry, jac_policy, integrator, lu, fp64_fallback)
        h = C.c_void_p()
        _check(lib().zb_graph_create(ctx.h, arr, len(segments), C.byref(o), C.byref(h)),
               "zb_graph_create")
        self.h = h

    def launch(self, stream=None):
        _check(lib().zb_graph_launch(self.h, _stream_handle(stream)), "zb_graph_launch")

    def close(self):
        if self.h:
            lib().zb_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching burn server (zb_server_*): host inputs in, host results out."""

    def __init__(self, ctx, hbm_budget_bytes, precision="fp64", lanes=0, max_steps=0, streams=0,
                 launches_per_stream=0, slice_zones=0, max_pending=0, retry=None, jac_policy=0,
                 integrator="bdf", lu="valu", fp64_fallback=False):
        self.ctx = ctx
        o = _ServerOpts(int(hbm_budget_bytes), int(streams), int(launches_per_stream),
                        int(slice_zones), int(max_pending), 0,
                        _opts(precision, lanes, max_steps, retry, jac_policy, integrator, lu,
                              fp64_fallback))
        h = C.c_void_p()
        _check(lib().zb_server_create(ctx.h, C.byref(o), C.byref(h)), "zb_server_create")
        self.h = h
        self._rows = {}

    def submit(self, net, state, dt, rtol, atol, rate_scale=None):
        """state: host float64 [zones][ns+1] (copied); returns a ticket."""
        st = np.ascontiguousarray(state, dtype=np.float64)
        if st.ndim != 2 or st.shape[1] != net.ns + 1:
            raise ValueError("state must be [zones][ns+1]")
        sc = None
        if rate_scale is not None:
            sc = np.ascontiguousarray(rate_scale, dtype=np.float64)
            if sc.shape != (st.shape[0], net.nr):
                raise ValueError("rate_scale must be [zones][n_reactions]")
        t = C.c_uint64(0)
        _check(lib().zb_server_submit(self.h, net.h, st.ctypes.data_as(C.c_void_p), st.shape[0],
                                      float(dt), float(rtol), float(atol),
                                      None if sc is None else sc.ctypes.data_as(C.c_void_p),
                                      C.byref(t)), "zb_server_submit")
        self._rows[t.value] = (st.shape[0], st.shape[1])
        return t.value

    def wait(self, ticket, timeout=0.0):
        d = C.c_int32(0)
        _check(lib().zb_server_wait(self.h, C.c_uint64(ticket), float(timeout), C.byref(d)),
               "zb_server_wait")
        return bool(d.value)

    def fetch(self, ticket):
        """(state, status, stats, info) of a finished request; releases it on the server."""
        if ticket not in self._rows:   # unknown here: let the library report it
            _check(lib().zb_server_fetch(self.h, C.c_uint64(ticket), None, None, None, None),
                   "zb_server_fetch")
        z, row = self._rows[ticket]
        out = np.empty((z, row), dtype=np.float64)
        status = np.empty(z, dtype=np.int32)
        stats = np.empty((z, 7), dtype=np.int32)
        info = _ReqInfo()
        _check(lib().zb_server_fetch(self.h, C.c_uint64(ticket), out.ctypes.data_as(C.c_void_p),
                                     status.ctypes.data_as(C.c_void_p),
                                     stats.ctypes.data_as(C.c_void_p), C.byref(info)),
               "zb_server_fetch")
        del self._rows[ticket]
        return out, status, stats, {k: getattr(info, k) for k, _ in _ReqInfo._fields_}

    def stats(self):
        t = _Totals()
        _check(lib().zb_server_stats(self.h, C.byref(t)), "zb_server_stats")
        return {k: getattr(t, k) for k, _ in _Totals._fields_}

    def close(self):
        if self.h:
            lib().zb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


def tune_save(ctx, path):
    """Writes the context's autotuned choices to a JSON file (zb_tune_save)."""
    _check(lib().zb_tune_save(ctx.h, os.fsencode(path)), "zb_tune_save")


def tune_load(ctx, path):
    """Loads choices saved by tune_save into the context; returns how many applied (0 for a
    file from another GPU architecture or HIP runtime)."""
    n = C.c_int32(0)
    _check(lib().zb_tune_load(ctx.h, os.fsencode(path), C.byref(n)), "zb_tune_load")
    return int(n.value)


def autotune_candidates(ctx, net, sample_state, dt, rtol, atol, precision="mixed"):
    """Times every (lanes per zone, LU) candidate on sample_state (zb_autotune_candidates);
    returns (candidates, best index), each candidate a dict with lanes, lu ('valu'/'mfma'),
    ms and qualified.  The chosen pair then serves calls with lu='auto'."""
    _check_state(net, sample_state)
    buf = (_TuneCand * 16)()
    n, best = C.c_int32(0), C.c_int32(-1)
    _check(lib().zb_autotune_candidates(ctx.h, net.h, _ptr(sample_state), sample_state.shape[0],
                                        float(dt), float(rtol), float(atol),
                                        _opts(precision, 0, 0).precision, buf, 16, C.byref(n),
                                        C.byref(best)), "zb_autotune_candidates")
    out = [{"lanes": int(c.lanes), "lu": ("valu", "mfma")[c.lu], "ms": float(c.ms),
            "qualified": bool(c.qualified)} for c in buf[:min(16, n.value)]]
    return out, int(best.value)
