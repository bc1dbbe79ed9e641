"""The GPU-vs-oracle parity check (no GPU code here; the GPU tests hand it their results).

Metric: per zone, the largest gated relative error over the integrated variables,
|y_gpu - y_ref| / max(|y_ref|, atol/rtol): the true relative error for values above
atol/rtol, an absolute error below, where the integrator controls a value only absolutely.

Bars, per zone:

* Statuses are identical on both sides, for every zone (a zone that one side fails and the
  other integrates fails the test), except the zones of the committed list of
  ill-conditioned zones (below).
* A zone that takes exactly the oracle's path (all seven counters equal: steps, RHS
  evaluations, Jacobians, factorisations, Newton iterations, error-test and convergence
  failures) differs from it only by rounding: FMA contraction and the device exp/log against
  libm in FP64, and the FP32 factorisation that the FP64 Newton iteration corrects in mixed
  precision.  Such a step-lockstep zone is held to 1e-9, or to LOCK_WIDEN times the oracle's
  own error there (e_orc, below) where the zone is sensitive enough to amplify rounding
  that far, and never beyond 1e-6.
* A zone whose path differs (one rounding difference flipped an accept/reject decision)
  differs from the oracle by the integrator's own global error at the case's tolerance.
  It is held to 1e-6, widened to WIDEN times the oracle's own error there, e_orc =
  |oracle(rtol) - oracle(rtol/100)| (a quantity of the oracle alone, independent of the GPU
  result), and never beyond CAP.  Zones above 1e-6 may be at most 1 % of the case's zones
  (at least 2).
* These bars hold at rtol = 1e-8; a case at a looser rtol scales them by rtol / 1e-8.
* A zone is ill-conditioned when the oracle alone says the integrator does not resolve it:
  WIDEN e_orc > CAP, or the oracle's reference run fails where its run at the case's
  tolerance succeeds.  Those zones must be exactly the committed list
  tests/golden/ill_conditioned_zones.json (written by make_ill_conditioned.py from the oracle,
  with the evidence for each zone).  On them the check asks for a finite result and, where
  the network conserves the species count, for the species sum.
"""
from __future__ import annotations

import json
import os

import numpy as np

# Bars at rtol = 1e-8, the tolerance of the benchmark; a case run at another rtol scales
# them with rtol (1e-6 is 100 rtol: an integrator's global error is a multiple of its
# tolerance), never below these values.
RTOL_REF = 1e-8
BAR = 1e-6
CAP = 1e-4
WIDEN = 3.0
# Step-lockstep zones: rounding drift only.  It is 1e-13..1e-10 in most zones, but stiff
# zones near equilibrium sum large cancelling fluxes in f, and there the drift grows with
# the zone's sensitivity: over every parity case it stayed within 3 e_orc (and reached
# 1.1e-7 in FP64 at rtol 1e-8).  So a lockstep zone is held to LOCK_WIDEN e_orc, at least
# LOCK_FLOOR and at most BAR.
LOCK_FLOOR = 1e-9
LOCK_WIDEN = 5.0
MAX_WIDENED_FRAC = 0.01
# statuses of a finished zone: OK, OK after the zone-by-zone retry, OK after the FP64 fallback
OK_STATUSES = (0, 6, 7)


def bars(rtol):
    """(bar, cap, lockstep floor) at the case's tolerance."""
    f = max(1.0, rtol / RTOL_REF)
    return BAR * f, CAP * f, LOCK_FLOOR * f

ILL_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "ill_conditioned_zones.json")
_ILL = None


def ill_list(name):
    global _ILL
    if _ILL is None:
        _ILL = json.load(open(ILL_FILE))["cases"] if os.path.exists(ILL_FILE) else {}
    return sorted(_ILL.get(name, {}).get("zones", []))


def gated_rows(y, ref, nv, rtol, atol):
    """Per-zone max gated relative error of y against ref over the first nv variables."""
    if y.shape[0] == 0:
        return np.zeros(0)
    return (np.abs(y[:, :nv] - ref[:, :nv])
            / np.maximum(np.abs(ref[:, :nv]), atol / rtol)).max(1)


def gated(y, ref, rtol, atol):
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(y - ref) / np.maximum(np.abs(ref), atol / rtol)))


def oracle_error(ref, fine, nv, rtol, atol):
    """e_orc per zone: the oracle at the case's tolerance against its run at rtol/100
    (inf where either failed)."""
    e = np.full(len(ref[1]), np.inf)
    ok = np.isin(ref[1], OK_STATUSES) & np.isin(fine[1], OK_STATUSES)
    e[ok] = gated_rows(ref[0][ok], fine[0][ok], nv, rtol, atol)
    return e


def ill_conditioned(ref, fine, nv, rtol, atol):
    """Zones the integrator does not resolve at the case's tolerance, from the oracle alone."""
    if fine is None:
        return np.zeros(len(ref[1]), bool)
    e = oracle_error(ref, fine, nv, rtol, atol)
    return np.isin(ref[1], OK_STATUSES) & (~np.isfinite(e) | (WIDEN * e > bars(rtol)[1]))


def _diag(name, **arrays):
    d = os.environ.get("ZB_PARITY_DIAG")
    if not d:
        return
    os.makedirs(d, exist_ok=True)
    safe = "".join(ch if ch.isalnum() else "_" for ch in name)
    np.savez(os.path.join(d, safe + ".npz"), **arrays)


def check(name, gpu, ref, rtol, atol, nv, precision="fp64", fine=None, state_in=None,
          conserving=False, ill_name=None):
    """Assert parity of a GPU result (state, status, stats) with the oracle's (ref).

    fine: the oracle at rtol/100 (same method), which measures the oracle's own error and
    allows the capped widening for zones off the oracle's step path; without it every zone
    is held to 1e-6 (lockstep zones to LOCKSTEP_BAR).  state_in, conserving: the input, and
    whether the species sum is an invariant (checked on ill-conditioned zones)."""
    out, status, stats = gpu
    ref_state, ref_status, ref_stats = ref
    n = len(status)
    assert ref_state.shape == out.shape and len(ref_status) == n
    e_orc = oracle_error(ref, fine, nv, rtol, atol) if fine is not None else np.zeros(n)
    ill = ill_conditioned(ref, fine, nv, rtol, atol)
    listed = ill_list(ill_name or name)
    assert np.nonzero(ill)[0].tolist() == listed, \
        (name, "ill-conditioned zones differ from the committed list", np.nonzero(ill)[0].tolist(), listed)

    # statuses: identical everywhere but on the listed zones
    bad = np.nonzero((status != ref_status) & ~ill)[0]
    assert bad.size == 0, (name, "status", bad[:10], status[bad[:10]], ref_status[bad[:10]])

    ok = (status == 0) & (ref_status == 0) & ~ill
    err = gated_rows(out[ok], ref_state[ok], nv, rtol, atol)
    lock = np.all(stats[ok] == ref_stats[ok], axis=1)
    bar0, cap, lfloor = bars(rtol)
    eo = e_orc[ok]
    bar = np.where(lock, np.clip(LOCK_WIDEN * eo, lfloor, bar0), np.clip(WIDEN * eo, bar0, cap))
    widened = (~lock) & (err > bar0)
    max_widened = max(2, int(MAX_WIDENED_FRAC * n))
    e_lock = float(err[lock].max()) if lock.any() else 0.0
    e_free = float(err[~lock].max()) if (~lock).any() else 0.0
    print(f"{name}: zones={n} lockstep={lock.mean() if ok.any() else 1.0:.3f} "
          f"max gated lockstep={e_lock:.2e} off-path={e_free:.2e} "
          f"widened={int(widened.sum())} (max {max_widened}) ill={int(ill.sum())}", flush=True)
    _diag(name, err=err, lock=lock, e_orc=e_orc[ok], status=status, ref_status=ref_status,
          ill=ill, stats=stats, ref_stats=ref_stats)
    over = np.nonzero(~(err <= bar))[0]          # a non-finite error fails too
    assert over.size == 0, (name, "error", np.nonzero(ok)[0][over[:10]].tolist(), err[over[:10]],
                            bar[over[:10]], lock[over[:10]])
    assert widened.sum() <= max_widened, (name, "widened zones", int(widened.sum()), max_widened)

    # ill-conditioned zones: a finite result, and the species sum where it is invariant
    gi = ill & (status == 0)
    if gi.any():
        assert np.all(np.isfinite(out[gi][:, :nv])), name
        if conserving and state_in is not None:
            ns = out.shape[1] - 1            # rows are the species, then T
            drift = np.abs(out[gi][:, :ns].sum(1) - state_in[gi][:, :ns].sum(1))
            assert drift.max() < (1e-11 if precision == "fp64" else 1e-8), (name, drift.max())
    # the temperature slot of a network without heating passes through
    if out.shape[1] > nv:
        assert np.array_equal(out[:, nv:], ref_state[:, nv:])
    return float(err.max()) if err.size else 0.0


def check_case(case, gpu, ref, fine, precision="fp64", name=None):
    """check() with the inputs and settings of a parity_cases.Case."""
    return check(name or case.name, gpu, ref, case.rtol, case.atol, case.nv, precision=precision,
                 fine=fine, state_in=case.state, conserving=case.conserving, ill_name=case.name)
