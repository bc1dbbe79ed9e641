"""ctypes front end of the CPU FP64 oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  The
C sources beside it are independent of the HIP path and share nothing with it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ZB_ORACLE_LIB: another build of these sources (the mutation test loads deliberately broken
# copies this way to show that the pins catch them)
_LIB_PATH = os.environ.get("ZB_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS = {0: "OK", 1: "MAXSTEPS", 2: "ERRTEST", 3: "CONV", 4: "HMIN", 5: "NONFINITE"}
STAT_FIELDS = ("nst", "nfe", "nje", "nlu", "nni", "netf", "ncf")


class _Net(C.Structure):
    _fields_ = [("ns", C.c_int), ("thermal", C.c_int), ("nr", C.c_int),
                ("reactant", C.POINTER(C.c_int32)), ("product", C.POINTER(C.c_int32)),
                ("lnA", C.POINTER(C.c_double)), ("n_exp", C.POINTER(C.c_double)),
                ("E", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double))]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        _lib.orc_burn.restype = i
        _lib.orc_burn.argtypes = [p, p, C.c_int64, p, d, d, d, i, p, p, i]
        _lib.orc_burn_src.restype = i
        _lib.orc_burn_src.argtypes = [p, p, C.c_int64, p, p, d, d, d, i, p, p, i]
        _lib.orc_burn_retry.restype = i
        _lib.orc_burn_retry.argtypes = [p, p, C.c_int64, p, p, d, d, d, i, p, p, p, i]
        _lib.orc_rkc.restype = i
        _lib.orc_rkc.argtypes = [p, p, C.c_int64, p, p, d, d, d, i, p, p, i]
        _lib.orc_rkc_fixed.restype = i
        _lib.orc_rkc_fixed.argtypes = [p, p, p, d, i, i]
        _lib.orc_rkc_stages.restype = i
        _lib.orc_rkc_stages.argtypes = [d, d]
        _lib.orc_burn_ex.restype = i
        _lib.orc_burn_ex.argtypes = [p, p, C.c_int64, p, p, d, d, d, i, i, i, p, p, p, i]
        _lib.orc_vc_xi.argtypes = [i, d, p, i, p]
        _lib.orc_vc_lcoef.argtypes = [i, p, p]
        _lib.orc_vc_steps.restype = i
        _lib.orc_vc_steps.argtypes = [p, p, i, i, p, p, i, p, p]
        _lib.orc_burn_zone.restype = i
        _lib.orc_burn_zone.argtypes = [p, p, p, d, d, d, i, p]
        _lib.orc_rhs.argtypes = [p, p, p, p]
        _lib.orc_rhs_cplx.argtypes = [p, p, p, p]
        _lib.orc_jac.argtypes = [p, p, p, p]
        _lib.orc_fd_jac.argtypes = [p, p, p, p, d, d, p]
        _lib.orc_rates.argtypes = [p, p, p, p, p]
        _lib.orc_lu.restype = i
        _lib.orc_lu.argtypes = [i, p, p]
        _lib.orc_lu_solve.argtypes = [i, p, p, p]
        _lib.orc_lcoef.argtypes = [i, p]
        _lib.orc_stirling.argtypes = [i, p]
        _lib.orc_order_raise.argtypes = [i, i, p, p]
        _lib.orc_order_lower.argtypes = [i, i, p]
        _lib.orc_fixed_steps.restype = i
        _lib.orc_fixed_steps.argtypes = [p, p, i, d, i, p, p, p]
        _lib.orc_radau.restype = i
        _lib.orc_radau.argtypes = [p, p, p, d, C.c_int64, d]
        _lib.orc_check_net.restype = i
        _lib.orc_check_net.argtypes = [p]
    return _lib


class Net:
    """Holds the numpy arrays of a network dict alive for the C struct."""

    def __init__(self, net):
        self.ns = int(net["n_species"])
        self.thermal = int(net["thermal"])
        self.reactant = np.ascontiguousarray(net["reactant"], dtype=np.int32)
        self.product = np.ascontiguousarray(net["product"], dtype=np.int32)
        self.lnA = np.ascontiguousarray(net["lnA"], dtype=np.float64)
        self.n_exp = np.ascontiguousarray(net["n_exp"], dtype=np.float64)
        self.E = np.ascontiguousarray(net["E"], dtype=np.float64)
        self.q = np.ascontiguousarray(net["q"], dtype=np.float64)
        self.nr = int(self.lnA.shape[0])
        self.nv = self.ns + self.thermal
        self.s = _Net(self.ns, self.thermal, self.nr, _ip(self.reactant), _ip(self.product),
                      _dp(self.lnA), _dp(self.n_exp), _dp(self.E), _dp(self.q))
        if lib().orc_check_net(C.byref(self.s)):
            raise ValueError("invalid network")

    @property
    def ref(self):
        return C.byref(self.s)


def _as_net(net):
    return net if isinstance(net, Net) else Net(net)


class _Retry(C.Structure):
    _fields_ = [("enabled", C.c_int), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_steps", C.c_int), ("jac", C.c_int)]


def burn(net, state, dt, rtol, atol, scale=None, max_steps=100000, nthreads=None, source=None,
         retry=None, jac_policy=0, form="fixed"):
    """Burn a copy of state [zones][ns+1]; returns (state, status[zones], stats[zones,7]).

    source: optional constant per-zone term [zones][ns+1] added to the right-hand side.
    retry: optional (rtol, atol, max_steps[, jac]) for a second run of every failed zone
    from its input, jac "analytic" (default) or "fd" (finite-difference Jacobian); such a
    zone then reports status 6 when the retry succeeds.
    jac_policy: 0 Jacobian and LU every step attempt, 1 VODE-style reuse.
    form: "fixed" (fixed-leading-coefficient BDF) or "variable" (variable-coefficient)."""
    if form not in ("fixed", "variable"):
        raise ValueError("form must be 'fixed' or 'variable'")
    n = _as_net(net)
    st = np.array(state, dtype=np.float64, copy=True, order="C")
    zones = st.shape[0]
    if st.ndim != 2 or st.shape[1] != n.ns + 1:
        raise ValueError("state must be [zones][ns+1]")
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    if sc is not None and sc.shape != (zones, n.nr):
        raise ValueError("scale must be [zones][R]")
    status = np.zeros(zones, dtype=np.int32)
    stats = np.zeros((zones, 7), dtype=np.int32)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    src = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
    if src is not None and src.shape != st.shape:
        raise ValueError("source must be [zones][ns+1]")
    rt = None
    if retry is not None:
        rjac = retry[3] if len(retry) > 3 else "analytic"
        if rjac not in ("analytic", "fd"):
            raise ValueError("retry jac must be 'analytic' or 'fd'")
        rt = _Retry(1, float(retry[0]), float(retry[1]), int(retry[2]), int(rjac == "fd"))
    lib().orc_burn_ex(n.ref, _dp(st), zones, _dp(sc), _dp(src), dt, rtol, atol, int(max_steps),
                      int(jac_policy), int(form == "variable"), None if rt is None else C.byref(rt),
                      _ip(status), _ip(stats), int(nthreads))
    return st, status, stats


def rhs(net, y, scale=None):
    n = _as_net(net)
    y = np.ascontiguousarray(y, dtype=np.float64)
    f = np.zeros(n.nv)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    lib().orc_rhs(n.ref, _dp(sc), _dp(y), _dp(f))
    return f


def rhs_complex(net, y, scale=None):
    n = _as_net(net)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    f = np.zeros(n.nv, dtype=np.complex128)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    lib().orc_rhs_cplx(n.ref, _dp(sc), y.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p))
    return f


def jac(net, y, scale=None):
    n = _as_net(net)
    y = np.ascontiguousarray(y, dtype=np.float64)
    J = np.zeros((n.nv, n.nv))
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    lib().orc_jac(n.ref, _dp(sc), _dp(y), _dp(J))
    return J


def fd_jac(net, y, rtol, atol, scale=None, source=None):
    """Finite-difference Jacobian of the RHS (plus source) at y (the retry's alternative)."""
    n = _as_net(net)
    y = np.ascontiguousarray(y, dtype=np.float64)
    J = np.zeros((n.nv, n.nv))
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    src = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
    lib().orc_fd_jac(n.ref, _dp(sc), _dp(src), _dp(y), float(rtol), float(atol), _dp(J))
    return J


def vc_xi(q, h, hist):
    """xi_1..xi_{q+1} of the variable-coefficient form (index 0 unused)."""
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    xi = np.zeros(q + 2)
    lib().orc_vc_xi(q, float(h), _dp(hist) if hist.size else None, int(hist.size), _dp(xi))
    return xi


def vc_lcoef(q, xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    l = np.zeros(q + 1)
    lib().orc_vc_lcoef(q, _dp(xi), _dp(l))
    return l


def vc_steps(net, Z, q, hs, hist, scale=None):
    """Fixed order q over the step sizes hs with the variable-coefficient form; Z [q+1][nv]
    in units of hs[0]; hist: past step sizes, newest first.  Returns (ys [n][nv], Z)."""
    n = _as_net(net)
    Z = np.array(Z, dtype=np.float64, copy=True, order="C")
    hs = np.ascontiguousarray(hs, dtype=np.float64)
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    ys = np.zeros((len(hs), n.nv))
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    r = lib().orc_vc_steps(n.ref, _dp(sc), q, len(hs), _dp(hs), _dp(hist) if hist.size else None,
                           int(hist.size), _dp(Z), _dp(ys))
    if r:
        raise RuntimeError(f"Newton failed at step {r - 1}")
    return ys, Z


def lu(A):
    A = np.array(A, dtype=np.float64, copy=True, order="C")
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().orc_lu(n, _dp(A), _ip(piv))
    return A, piv, info


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=np.float64, copy=True)
    lib().orc_lu_solve(LU.shape[0], _dp(np.ascontiguousarray(LU)), _ip(piv), _dp(b))
    return b


def lcoef(q):
    l = np.zeros(q + 1)
    lib().orc_lcoef(q, _dp(l))
    return l


def stirling(n):
    c = np.zeros(n + 1)
    lib().orc_stirling(n, _dp(c))
    return c


def order_raise(Z, q, dy):
    """Z: [q+2][nv] (row q+1 is overwritten)."""
    Z = np.array(Z, dtype=np.float64, copy=True, order="C")
    lib().orc_order_raise(Z.shape[1], q, _dp(Z), _dp(np.ascontiguousarray(dy, dtype=np.float64)))
    return Z


def order_lower(Z, q):
    Z = np.array(Z, dtype=np.float64, copy=True, order="C")
    lib().orc_order_lower(Z.shape[1], q, _dp(Z))
    return Z


def fixed_steps(net, Z, q, h, nsteps, scale=None, with_errors=False):
    n = _as_net(net)
    Z = np.array(Z, dtype=np.float64, copy=True, order="C")
    ys = np.zeros((nsteps, n.nv))
    errs = np.zeros(nsteps)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    rc = lib().orc_fixed_steps(n.ref, _dp(sc), q, h, nsteps, _dp(Z), _dp(ys), _dp(errs))
    if rc:
        raise RuntimeError(f"Newton failed at step {rc}")
    return (ys, Z, errs) if with_errors else (ys, Z)


def radau(net, y0, dt, nsteps, h0=0.0, scale=None):
    n = _as_net(net)
    y = np.array(y0, dtype=np.float64, copy=True)[: n.nv].copy()
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    rc = lib().orc_radau(n.ref, _dp(sc), _dp(y), dt, int(nsteps), h0)
    if rc:
        raise RuntimeError(f"Radau Newton failed at step {-rc}")
    return y


def rkc(net, state, dt, rtol, atol, scale=None, max_steps=100000, nthreads=None, source=None):
    """Runge-Kutta-Chebyshev burn of a copy of state [zones][ns+1]; (state, status, stats)."""
    n = _as_net(net)
    st = np.array(state, dtype=np.float64, copy=True, order="C")
    zones = st.shape[0]
    if st.ndim != 2 or st.shape[1] != n.ns + 1:
        raise ValueError("state must be [zones][ns+1]")
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    src = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
    status = np.zeros(zones, dtype=np.int32)
    stats = np.zeros((zones, 7), dtype=np.int32)
    lib().orc_rkc(n.ref, _dp(st), zones, _dp(sc), _dp(src), dt, rtol, atol, int(max_steps),
                  _ip(status), _ip(stats), int(nthreads or os.cpu_count() or 1))
    return st, status, stats


def rkc_fixed(net, y, h, nsteps, s, scale=None):
    """nsteps RKC steps of size h with s stages from y (one zone, [nv] values); returns y."""
    n = _as_net(net)
    v = np.array(y, dtype=np.float64, copy=True)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    if lib().orc_rkc_fixed(n.ref, _dp(sc), _dp(v), float(h), int(nsteps), int(s)) != 0:
        raise ValueError("bad stage count")
    return v


def rkc_stages(h, rho):
    return int(lib().orc_rkc_stages(float(h), float(rho)))
