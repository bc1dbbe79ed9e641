"""The GPU parity check itself, on synthetic results (CPU only): every way a wrong GPU result
can differ from the oracle's must fail it, and rounding-level agreement must pass."""
import numpy as np
import pytest

import parity
from parity import check

RT, AT, NV = 1e-8, 1e-12, 3


def _ref(n=8, seed=0):
    rng = np.random.default_rng(seed)
    y = np.zeros((n, NV + 1))
    y[:, :NV] = rng.uniform(0.1, 1.0, (n, NV))
    stats = np.tile(np.array([100, 220, 100, 100, 200, 3, 0], np.int32), (n, 1))
    return y, np.zeros(n, np.int32), stats


def _copy(r):
    return r[0].copy(), r[1].copy(), r[2].copy()


def test_identical_results_pass():
    ref = _ref()
    check("ident", _copy(ref), ref, RT, AT, NV)


def test_gpu_failing_every_zone_fails():
    ref = _ref()
    g = _copy(ref)
    g[1][:] = 2
    with pytest.raises(AssertionError, match="status"):
        check("all fail", g, ref, RT, AT, NV, fine=_copy(ref))


def test_one_sided_failure_fails_either_way():
    ref = _ref()
    for side in (0, 1):
        g, r = _copy(ref), _copy(ref)
        (g if side == 0 else r)[1][3] = 3
        with pytest.raises(AssertionError, match="status"):
            check("one-sided", g, r, RT, AT, NV, fine=_copy(ref))


def test_lockstep_zone_is_held_to_the_rounding_bar():
    ref = _ref()
    g = _copy(ref)
    g[0][2, 1] *= 1 + 5 * parity.LOCK_FLOOR
    with pytest.raises(AssertionError, match="error"):
        check("lockstep", g, ref, RT, AT, NV)
    g = _copy(ref)
    g[0][2, 1] *= 1 + 0.5 * parity.LOCK_FLOOR
    check("lockstep ok", g, ref, RT, AT, NV)
    # a sensitive zone (the oracle's own error 1e-8 there) may drift up to 5e-8, never 1e-6
    fine = _copy(ref)
    fine[0][2, 1] = ref[0][2, 1] * (1 - 1e-8)
    g = _copy(ref)
    g[0][2, 1] *= 1 + 4e-8
    check("lockstep sensitive", g, ref, RT, AT, NV, fine=fine)
    g[0][2, 1] = ref[0][2, 1] * (1 + 8e-8)
    with pytest.raises(AssertionError, match="error"):
        check("lockstep sensitive over", g, ref, RT, AT, NV, fine=fine)
    fine[0][2, 1] = ref[0][2, 1] * (1 - 3e-6)
    g[0][2, 1] = ref[0][2, 1] * (1 + 1.5e-6)
    with pytest.raises(AssertionError, match="error"):
        check("lockstep capped", g, ref, RT, AT, NV, fine=fine)


def test_off_path_zone_bar_and_oracle_widening():
    ref = _ref()
    fine = _copy(ref)
    g = _copy(ref)
    g[2][4, 0] += 1                      # another step path
    g[0][4, 0] *= 1 + 0.9e-6
    check("off path within 1e-6", g, ref, RT, AT, NV, fine=fine)
    g[0][4, 0] = ref[0][4, 0] * (1 + 5e-6)
    with pytest.raises(AssertionError, match="error"):
        check("off path over", g, ref, RT, AT, NV, fine=fine)
    # the oracle's own error at that zone (against its rtol/100 run) widens the bar to 3x it
    fine[0][4, 0] = ref[0][4, 0] * (1 - 2e-6)
    check("widened", g, ref, RT, AT, NV, fine=fine)
    # the GPU's own error never enters: a GPU result far off stays a failure
    g[0][4, 0] = ref[0][4, 0] * (1 + 2e-5)
    with pytest.raises(AssertionError, match="error"):
        check("widened over", g, ref, RT, AT, NV, fine=fine)


def test_widening_is_capped_and_counted():
    ref = _ref(n=8)
    fine = _copy(ref)
    g = _copy(ref)
    for z in range(3):                   # three off-path zones above 1e-6 (the limit is 2)
        g[2][z, 0] += 1
        g[0][z, 0] *= 1 + 3e-6
        fine[0][z, 0] = ref[0][z, 0] * (1 - 2e-6)
    with pytest.raises(AssertionError, match="widened zones"):
        check("too many", g, ref, RT, AT, NV, fine=fine)


def test_ill_conditioned_zones_must_be_the_committed_list():
    ref = _ref()
    fine = _copy(ref)
    fine[0][6, 0] = ref[0][6, 0] * (1 + 1e-3)   # the oracle does not resolve zone 6
    g = _copy(ref)
    with pytest.raises(AssertionError, match="committed list"):
        check("not listed", g, ref, RT, AT, NV, fine=fine)


def test_nonfinite_result_of_an_ok_zone_fails():
    ref = _ref()
    g = _copy(ref)
    g[0][1, 2] = np.nan
    with pytest.raises(AssertionError):
        check("nan", g, ref, RT, AT, NV)


def test_passthrough_slot_of_a_network_without_heating():
    ref = _ref()
    g = _copy(ref)
    g[0][0, NV] = 1.0
    with pytest.raises(AssertionError):
        check("T slot", g, ref, RT, AT, NV)
