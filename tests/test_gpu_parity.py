"""GPU parity: the HIP burn against the CPU FP64 oracle on identical seeded inputs.

Bar (per zone, per species, at rtol = 1e-8): the gated relative error
|y_gpu - y_ref| / max(|y_ref|, atol/rtol) <= 1e-6, and identical zone
statuses.  Species below atol/rtol are controlled only absolutely by the
integrator, which is why the denominator is floored there.

Where the integrator does not itself resolve a zone to that level, the bar
cannot hold for any two implementations: two runs of the same algorithm that
break lockstep (a step decision flipped by one rounding difference) differ by
the algorithm's own global error, which at rtol = 1e-8 reaches ~1e-6 in the
tail of these stiff networks (and far more in the few ill-conditioned,
autocatalytic zones of the 48-variable network).  Each side's own error is
measured by self-convergence against its own run at rtol/100, atol/100:
e_orc = |oracle(rtol) - oracle(rtol/100)|, e_gpu = |gpu(rtol) - gpu(rtol/100)|
(gated), and the per-zone bar is max(1e-6, 3 (e_orc + e_gpu)).  A GPU defect
that changes the answer consistently keeps e_gpu small and so meets the plain
1e-6 bar.  Statuses must agree on zones both sides resolve (e <= 1e-7).  The
tests print how many zones needed the widened bar.
"""
import numpy as np
import pytest

import oracle
from paper_2608_06466_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = 1e-6


def gated(y, ref, rtol, atol):
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(y - ref) / np.maximum(np.abs(ref), atol / rtol)))


@pytest.fixture(scope="module")
def zbm():
    from paper_2608_06466_amd import zoneburn as zb
    assert torch.cuda.is_available()
    ctx = zb.Context(0)
    yield zb, ctx
    ctx.close()


def run_gpu(zb, ctx, net_dict, state, dt, rtol, atol, scale=None, precision="fp64", lanes=0,
            max_steps=0, net=None):
    own = net is None
    net = net or zb.Network(ctx, net_dict)
    st = torch.tensor(state, device="cuda:0")
    sc = None if scale is None else torch.tensor(scale, device="cuda:0")
    status, stats = zb.burn(ctx, net, st, dt, rtol, atol, rate_scale=sc, precision=precision,
                            lanes=lanes, max_steps=max_steps)
    zb.sync(ctx)
    out = (st.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy())
    if own:
        net.close()
    return out


def oracle_ref(net, state, dt, rtol, atol, scale=None, max_steps=100000):
    """Oracle result at (rtol, atol) and at (rtol/100, atol/100)."""
    ref = oracle.burn(net, state, dt, rtol, atol, scale, max_steps=max_steps)
    fine = oracle.burn(net, state, dt, rtol / 100, atol / 100, scale, max_steps=100 * max_steps)
    return ref, fine


def self_err(x, fine, nv, rtol, atol):
    both = (x[1] == 0) & (fine[1] == 0)
    e = np.full(len(x[1]), np.inf)
    if both.any():
        e[both] = (np.abs(x[0][both, :nv] - fine[0][both, :nv])
                   / np.maximum(np.abs(fine[0][both, :nv]), atol / rtol)).max(1)
    return e


def check(name, gpu, ref, rtol, atol, nv, gpu_fine=None):
    """ref is an oracle tuple (plain 1e-6 bar) or (ref, ref_fine) from oracle_ref."""
    if isinstance(ref[0], tuple):
        ref, ref_fine = ref
        e_self = self_err(ref, ref_fine, nv, rtol, atol) + self_err(gpu, gpu_fine, nv, rtol, atol)
    else:
        e_self = np.zeros(len(gpu[1]))
    out, status, stats = gpu
    ref_state, ref_status, ref_stats = ref
    resolved = e_self <= 1e-7
    bad = np.nonzero((status != ref_status) & resolved)[0]
    assert bad.size == 0, (name, "status", bad[:10], status[bad[:10]], ref_status[bad[:10]])
    ok = (status == 0) & (ref_status == 0)
    ez = (np.abs(out[ok][:, :nv] - ref_state[ok][:, :nv])
          / np.maximum(np.abs(ref_state[ok][:, :nv]), atol / rtol)).max(1) if ok.any() else np.zeros(0)
    bar = np.maximum(BAR, 3.0 * e_self[ok])
    e = float(ez.max()) if ez.size else 0.0
    lock = float(np.mean(np.all(stats[ok][:, [0, 5, 6]] == ref_stats[ok][:, [0, 5, 6]], axis=1))) \
        if ok.any() else 1.0
    print(f"{name}: zones={len(status)} max gated={e:.2e} over 1e-6 (widened bar): "
          f"{int((ez > BAR).sum())} status-exempt: {int(((status != ref_status) & ~resolved).sum())} "
          f"step-lockstep={lock:.3f}", flush=True)
    assert np.all(ez <= bar), (name, e, np.nonzero(ez > bar)[0][:10], bar[ez > bar][:5])
    # passthrough of the temperature slot for networks without heating
    if out.shape[1] > nv:
        assert np.array_equal(out[:, nv:], ref_state[:, nv:])
    return e


def run_pair(zb, ctx, net_dict, state, dt, rtol, atol, scale=None, precision="fp64", lanes=0,
             net=None):
    """GPU result at (rtol, atol) and at (rtol/100, atol/100)."""
    a = run_gpu(zb, ctx, net_dict, state, dt, rtol, atol, scale, precision, lanes, net=net)
    b = run_gpu(zb, ctx, net_dict, state, dt, rtol / 100, atol / 100, scale, precision, lanes,
                max_steps=10000000, net=net)
    return a, b


@pytest.mark.parametrize("lanes", [1, 4])
def test_robertson_parity(zbm, lanes):
    zb, ctx = zbm
    c = W.robertson(333)
    ref = oracle_ref(c["net"], c["state"], c["dt"], c["rtol"], c["atol"], c["scale"])
    gpu, fine = run_pair(zb, ctx, c["net"], c["state"], c["dt"], c["rtol"], c["atol"], c["scale"], lanes=lanes)
    check(f"robertson L={lanes}", gpu, ref, c["rtol"], c["atol"], 3, fine)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nv14_parity(zbm, precision):
    zb, ctx = zbm
    c = W.nv14(301)
    ref = oracle_ref(c["net"], c["state"], c["dt"], c["rtol"], c["atol"])
    gpu, fine = run_pair(zb, ctx, c["net"], c["state"], c["dt"], c["rtol"], c["atol"], precision=precision)
    check(f"nv14 {precision}", gpu, ref, c["rtol"], c["atol"], 14, fine)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_batched_networks_parity(zbm, k, precision):
    zb, ctx = zbm
    ns, R, seed = W.BATCHED_NETS[k - 1]
    net = W.random_network(ns, R, seed)
    zones = {1: 131, 2: 67, 3: 19}[k]
    st = W.random_zones(net, zones, seed=900 + k, T_range=(300.0, 6000.0), T_dist="loguniform")
    ref = oracle_ref(net, st, 1.0, 1e-8, 1e-12)
    gpu, fine = run_pair(zb, ctx, net, st, 1.0, 1e-8, 1e-12, precision=precision)
    check(f"net nv={ns + 1} {precision}", gpu, ref, 1e-8, 1e-12, ns + 1, fine)


def test_linear_and_two_body_networks(zbm):
    zb, ctx = zbm
    for seed in range(3):
        net = W.linear_network(6, seed)
        st = np.zeros((5, 7))
        st[:, :6] = np.random.default_rng(seed).dirichlet(np.ones(6), size=5)
        ref = oracle.burn(net, st, 10.0, 1e-8, 1e-12)
        gpu = run_gpu(zb, ctx, net, st, 10.0, 1e-8, 1e-12)
        check(f"linear seed {seed}", gpu, ref, 1e-8, 1e-12, 6)
    net = W.two_body_network(5.0)
    st = np.array([[0.6, 0.25, 0.05, 0.1, 0.0]] * 3)
    check("A+B->C+D", run_gpu(zb, ctx, net, st, 2.0, 1e-8, 1e-12),
          oracle.burn(net, st, 2.0, 1e-8, 1e-12), 1e-8, 1e-12, 4)


def test_edge_cases_and_statuses(zbm):
    zb, ctx = zbm
    c = W.nv14(40)
    net = zb.Network(ctx, c["net"])
    # zero zones and one zone
    out, status, stats = run_gpu(zb, ctx, c["net"], c["state"][:0], 1.0, 1e-8, 1e-12, net=net)
    assert out.shape == (0, 14)
    ref = oracle.burn(c["net"], c["state"][:1], 1.0, 1e-8, 1e-12)
    check("one zone", run_gpu(zb, ctx, c["net"], c["state"][:1], 1.0, 1e-8, 1e-12, net=net), ref,
          1e-8, 1e-12, 14)
    # step cap: every zone stops after 5 accepted steps, in lockstep with the oracle
    ref = oracle.burn(c["net"], c["state"], 1.0, 1e-8, 1e-12, max_steps=5)
    gpu = run_gpu(zb, ctx, c["net"], c["state"], 1.0, 1e-8, 1e-12, max_steps=5, net=net)
    assert np.all(gpu[1] == 1) and np.all(gpu[2][:, 0] == 5)
    assert gated(gpu[0][:, :14], ref[0][:, :14], 1e-8, 1e-12) < 1e-9
    # non-finite and negative-temperature inputs
    bad = c["state"].copy()
    bad[0, 3] = np.nan
    bad[5, -1] = -10.0
    ref = oracle.burn(c["net"], bad, 1.0, 1e-8, 1e-12)
    gpu = run_gpu(zb, ctx, c["net"], bad, 1.0, 1e-8, 1e-12, net=net)
    assert gpu[1][0] == 5 and gpu[1][5] == 5
    assert np.array_equal(gpu[0][5], bad[5])
    check("bad inputs", gpu, ref, 1e-8, 1e-12, 14)
    assert zb.sync(ctx) == 0   # the count was consumed by the previous sync
    # argument errors
    st = torch.tensor(c["state"], device="cuda:0")
    for kw in (dict(dt=0.0), dict(dt=float("nan")), dict(rtol=0.0), dict(atol=-1.0)):
        args = dict(dt=1.0, rtol=1e-8, atol=1e-12)
        args.update(kw)
        with pytest.raises(zb.ZoneburnError) as ei:
            zb.burn(ctx, net, st, **args)
        assert ei.value.code == zb.EINVAL
    with pytest.raises(zb.ZoneburnError):
        zb.burn(ctx, net, st, 1.0, 1e-8, 1e-12, lanes=3)
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zone_result_independent_of_batch(zbm, precision):
    """A zone burned alone, at another position, or next to other zones: bitwise the same."""
    zb, ctx = zbm
    c = W.nv14(257)
    net = zb.Network(ctx, c["net"])
    full = run_gpu(zb, ctx, c["net"], c["state"], 1.0, 1e-8, 1e-12, precision=precision, net=net)
    idx = [0, 13, 200, 256]
    part = run_gpu(zb, ctx, c["net"], c["state"][idx][::-1].copy(), 1.0, 1e-8, 1e-12,
                   precision=precision, net=net)
    assert np.array_equal(part[0][::-1], full[0][idx])
    assert np.array_equal(part[2][::-1], full[2][idx])
    net.close()


def test_batch_launch_matches_single_launches(zbm):
    zb, ctx = zbm
    n2 = W.nv14_network()
    ns, R, seed = W.BATCHED_NETS[0]
    n3 = W.random_network(ns, R, seed)
    s2 = W.random_zones(n2, 70, seed=1)
    s3 = W.random_zones(n3, 45, seed=2)
    N2, N3 = zb.Network(ctx, n2), zb.Network(ctx, n3)
    a2 = run_gpu(zb, ctx, n2, s2, 1.0, 1e-8, 1e-12, net=N2)
    a3 = run_gpu(zb, ctx, n3, s3, 0.5, 1e-8, 1e-12, net=N3)
    t2, t3 = torch.tensor(s2, device="cuda:0"), torch.tensor(s3, device="cuda:0")
    st2 = torch.empty(70, dtype=torch.int32, device="cuda:0")
    st3 = torch.empty(45, dtype=torch.int32, device="cuda:0")
    zb.burn_batch(ctx, [dict(net=N2, state=t2, dt=1.0, rtol=1e-8, atol=1e-12, status=st2),
                        dict(net=N3, state=t3, dt=0.5, rtol=1e-8, atol=1e-12, status=st3)])
    zb.sync(ctx)
    assert np.array_equal(t2.cpu().numpy(), a2[0]) and np.array_equal(t3.cpu().numpy(), a3[0])
    assert np.array_equal(st2.cpu().numpy(), a2[1]) and np.array_equal(st3.cpu().numpy(), a3[1])
    N2.close()
    N3.close()


def test_nv14_full_size_sampled(zbm):
    """2^20 zones in the benchmark's launch configuration; 48 sampled zones against the oracle."""
    zb, ctx = zbm
    c = W.nv14()
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(c["state"].shape[0], 256, replace=False))
    ref = oracle_ref(c["net"], c["state"][idx], 1.0, 1e-8, 1e-12)
    # one zone of the 2^20 (index 444681) runs out of its 100000 steps in both the oracle and
    # the GPU, with identical counters; every zone the GPU reports as failed is checked below
    fails = {}
    for prec in ("fp64", "mixed"):
        out, status, stats = run_gpu(zb, ctx, c["net"], c["state"], 1.0, 1e-8, 1e-12, precision=prec)
        bad = np.nonzero(status)[0]
        print(f"nv14 2^20 {prec}: failed zones {bad.tolist()[:10]}", flush=True)
        assert bad.size <= 4
        if bad.size:
            r = oracle.burn(c["net"], c["state"][bad], 1.0, 1e-8, 1e-12)
            assert np.array_equal(r[1], status[bad]), (r[1], status[bad])
        fine = run_gpu(zb, ctx, c["net"], c["state"][idx], 1.0, 1e-10, 1e-14, precision=prec)
        check(f"nv14 2^20 {prec} sampled 256", (out[idx], status[idx], stats[idx]), ref,
              1e-8, 1e-12, 14, fine)
        # species sum is conserved by every reaction
        drift = np.abs(out[:, :13].sum(1) - c["state"][:, :13].sum(1)).max()
        assert drift < (1e-11 if prec == "fp64" else 1e-9), drift


@pytest.mark.parametrize("which", ["nv14", "nv14", "nv22", "nv48"])
def test_parity_tail_on_thousands_of_zones(zbm, which):
    """Thousands of zones per network, both precisions, under the self-convergence bar."""
    zb, ctx = zbm
    if which == "nv14":
        net_d, n, Tr, Td = W.nv14_network(), 3000, (1e3, 5e3), "uniform"
    else:
        k = {"nv14": 0, "nv22": 1, "nv48": 2}[which]
        ns, R, seed = W.BATCHED_NETS[k]
        net_d, n, Tr, Td = W.random_network(ns, R, seed), [3000, 2000, 400][k], (300.0, 6000.0), "loguniform"
    st = W.random_zones(net_d, n, seed=4242, T_range=Tr, T_dist=Td)
    ref = oracle_ref(net_d, st, 1.0, 1e-8, 1e-12)
    net = zb.Network(ctx, net_d)
    for prec in ("fp64", "mixed"):
        gpu, fine = run_pair(zb, ctx, net_d, st, 1.0, 1e-8, 1e-12, precision=prec, net=net)
        check(f"{which} {prec} x{n}", gpu, ref, 1e-8, 1e-12, net_d["n_species"] + 1, fine)
    net.close()


def test_autotune_picks_the_fastest_qualifying_mapping(zbm):
    """zb_autotune times each mapping, and the chosen one then serves AUTO launches."""
    zb, ctx = zbm
    c = W.nv14(8192)
    net = zb.Network(ctx, c["net"])
    st = torch.tensor(c["state"], device="cuda:0")
    before = st.clone()
    for prec in ("fp64", "mixed"):
        best, times = zb.autotune(ctx, net, st, 1.0, 1e-8, 1e-12, precision=prec)
        print(f"autotune {prec}: best lanes {best}, ms per lane count 1..64: "
              f"{[round(t, 2) for t in times]}", flush=True)
        assert torch.equal(st, before)
        lanes = [1 << i for i in range(7)]
        timed = {l: t for l, t in zip(lanes, times) if t > 0}
        assert best in timed
        # every mapping of this network agrees on statuses and on >= 99% of the zones, so the
        # fastest one is chosen
        assert timed[best] == min(timed.values())
        assert zb.get_mapping(ctx, net, prec) == best
        out = run_gpu(zb, ctx, c["net"], c["state"][:512], 1.0, 1e-8, 1e-12, precision=prec,
                      net=net)
        ref = run_gpu(zb, ctx, c["net"], c["state"][:512], 1.0, 1e-8, 1e-12, precision=prec,
                      lanes=best, net=net)
        assert np.array_equal(out[0], ref[0])
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_constant_source_parity(zbm, precision):
    """A constant per-zone source on the benchmark network: GPU against the oracle with the
    same source, and the species sum moved by exactly dt * sum(a)."""
    zb, ctx = zbm
    c = W.nv14(300)
    rng = np.random.default_rng(5)
    src = np.zeros_like(c["state"])
    src[:, :13] = rng.uniform(0.0, 1e-3, (300, 13))
    src[:, 13] = rng.uniform(-5.0, 5.0, 300)
    ref = oracle.burn(c["net"], c["state"], 1.0, 1e-8, 1e-12, source=src)
    fine = oracle.burn(c["net"], c["state"], 1.0, 1e-10, 1e-14, source=src, max_steps=10000000)
    net = zb.Network(ctx, c["net"])
    out = []
    for rt, at in ((1e-8, 1e-12), (1e-10, 1e-14)):
        st = torch.tensor(c["state"], device="cuda:0")
        status, stats = zb.burn(ctx, net, st, 1.0, rt, at, precision=precision,
                                source=torch.tensor(src, device="cuda:0"), max_steps=10000000)
        zb.sync(ctx)
        out.append((st.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    check(f"nv14 + source {precision}", out[0], (ref, fine), 1e-8, 1e-12, 14, out[1])
    drift = out[0][0][:, :13].sum(1) - c["state"][:, :13].sum(1) - src[:, :13].sum(1)
    assert np.abs(drift).max() < (1e-11 if precision == "fp64" else 1e-9)
    # the source changes the answer well beyond the tolerance
    plain = run_gpu(zb, ctx, c["net"], c["state"], 1.0, 1e-8, 1e-12, precision=precision, net=net)
    assert np.abs(plain[0][:, :13] - out[0][0][:, :13]).max() > 1e-5
    net.close()


def test_constant_source_linear_network_matches_exponential(zbm):
    """GPU burn of y' = K y + a against expm of the augmented matrix (no oracle involved)."""
    import scipy.linalg as sla
    zb, ctx = zbm
    ns = 5
    net_d = W.linear_network(ns, 3)
    K = np.zeros((ns, ns))
    for (a_, _), (c_, _), lk in zip(net_d["reactant"], net_d["product"], net_d["lnA"]):
        K[a_, a_] -= np.exp(lk)
        K[c_, a_] += np.exp(lk)
    rng = np.random.default_rng(9)
    zones = 40
    y0 = rng.dirichlet(np.ones(ns), size=zones)
    a = rng.uniform(0.0, 0.05, (zones, ns))
    st = np.zeros((zones, ns + 1))
    st[:, :ns] = y0
    src = np.zeros_like(st)
    src[:, :ns] = a
    t = torch.tensor(st, device="cuda:0")
    status, _ = zb.burn(ctx, zb.Network(ctx, net_d), t, 10.0, 1e-8, 1e-12,
                        source=torch.tensor(src, device="cuda:0"))
    zb.sync(ctx)
    out = t.cpu().numpy()
    assert np.all(status.cpu().numpy() == 0)
    for z in range(zones):
        A = np.zeros((ns + 1, ns + 1))
        A[:ns, :ns] = K
        A[:ns, ns] = a[z]
        ref = (sla.expm(A * 10.0) @ np.append(y0[z], 1.0))[:ns]
        assert gated(out[z, :ns], ref, 1e-8, 1e-12) < 1e-6, z


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loose_tolerance_parity_with_abundance_constraint(zbm, precision):
    """rtol 1e-6 on the benchmark network: zone 43 of this input is one whose unconstrained
    integration drains a species through zero; both sides reject such steps the same way."""
    zb, ctx = zbm
    c = W.nv14(96)
    ref = oracle_ref(c["net"], c["state"], 1.0, 1e-6, 1e-10)
    net = zb.Network(ctx, c["net"])
    gpu, fine = run_pair(zb, ctx, c["net"], c["state"], 1.0, 1e-6, 1e-10, precision=precision, net=net)
    check(f"nv14 rtol 1e-6 {precision}", gpu, ref, 1e-6, 1e-10, 14, fine)
    assert gpu[0][:, :13].min() >= -1e-10
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zone_retry_parity(zbm, precision):
    """A 1500-step cap fails most zones; the in-kernel retry (rtol 1e-6, atol 1e-10, 100000
    steps) gives the oracle's statuses (6 for retried zones), its results within the bar at
    the tolerances each zone finished with, and counters summed over both runs."""
    zb, ctx = zbm
    c = W.nv14(160)
    retry = (1e-6, 1e-10, 100000)
    ref = oracle.burn(c["net"], c["state"], 1.0, 1e-8, 1e-12, max_steps=1500, retry=retry)
    net = zb.Network(ctx, c["net"])
    st = torch.tensor(c["state"], device="cuda:0")
    status, stats = zb.burn(ctx, net, st, 1.0, 1e-8, 1e-12, precision=precision, max_steps=1500,
                            retry=retry)
    nf = zb.sync(ctx)
    out, status, stats = st.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()
    retried = ref[1] == 6
    assert 20 < retried.sum() < 160 and nf == 0
    assert np.array_equal(status, ref[1])
    assert np.all(stats[retried, 0] > 1500)
    for mask, rt, at in ((retried, 1e-6, 1e-10), (~retried, 1e-8, 1e-12)):
        fine = oracle.burn(c["net"], c["state"][mask], 1.0, rt / 100, at / 100)
        gfine = run_gpu(zb, ctx, c["net"], c["state"][mask], 1.0, rt / 100, at / 100,
                        precision=precision, max_steps=10000000, net=net)
        r = (ref[0][mask], np.zeros(mask.sum(), np.int32), ref[2][mask])
        g = (out[mask], np.zeros(mask.sum(), np.int32), stats[mask])
        check(f"retry {precision} {'retried' if rt > 1e-8 else 'first run'}", g, (r, fine), rt, at,
              14, gfine)
    net.close()


@pytest.mark.parametrize("which", ["nv14", "nv22", "nv48"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_jacobian_reuse_parity(zbm, which, precision):
    """The VODE-style reuse (jac_policy 1) against the oracle's: same statuses, results within
    the widened bar, and Jacobian/LU counts far below the step counts on both sides."""
    zb, ctx = zbm
    if which == "nv14":
        net_d, n, Tr, Td = W.nv14_network(), 400, (1e3, 5e3), "uniform"
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        ns, R, seed = W.BATCHED_NETS[k]
        net_d, n, Tr, Td = W.random_network(ns, R, seed), [0, 200, 96][k], W.BATCHED_T_RANGE, "loguniform"
    st = W.random_zones(net_d, n, seed=777, T_range=Tr, T_dist=Td)
    ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12, jac_policy=1)
    fine = oracle.burn(net_d, st, 1.0, 1e-10, 1e-14, jac_policy=1, max_steps=10000000)
    net = zb.Network(ctx, net_d)
    out = []
    for rt, at, ms in ((1e-8, 1e-12, 0), (1e-10, 1e-14, 10000000)):
        t = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, net, t, 1.0, rt, at, precision=precision, jac_policy=1,
                                max_steps=ms)
        zb.sync(ctx)
        out.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    nv = net_d["n_species"] + 1
    check(f"{which} reuse {precision}", out[0], (ref, fine), 1e-8, 1e-12, nv, out[1])
    ok = out[0][1] == 0
    for s in (out[0][2][ok], ref[2][ok]):
        assert s[:, 2].sum() * 4 < s[:, 0].sum() and s[:, 3].sum() * 3 < s[:, 0].sum()
    net.close()


@pytest.mark.parametrize("which", ["nv14", "nv22", "nv48", "linear"])
def test_rkc_parity(zbm, which):
    """The Runge-Kutta-Chebyshev integrator against the oracle's, on mildly stiff zones (the
    random networks at 100-300 K; a linear network with rates 1e-2..1e2): same statuses and
    results within the widened bar (each side's own error from a run at rtol/100)."""
    zb, ctx = zbm
    rtol, atol, dt = 1e-6, 1e-10, 1.0
    if which == "linear":
        net_d = W.linear_network(6, 5, k_range=(1e-2, 1e2))
        st = np.zeros((128, 7))
        st[:, :6] = np.random.default_rng(3).dirichlet(np.ones(6), size=128)
        dt = 10.0
    else:
        k = {"nv14": 0, "nv22": 1, "nv48": 2}[which]
        ns, R, seed = W.BATCHED_NETS[k]
        net_d = W.random_network(ns, R, seed)
        st = W.random_zones(net_d, [256, 128, 48][k], seed=31, T_range=(100.0, 300.0), T_dist="loguniform")
    ref = oracle.rkc(net_d, st, dt, rtol, atol)
    fine = oracle.rkc(net_d, st, dt, rtol / 100, atol / 100, max_steps=10000000)
    net = zb.Network(ctx, net_d)
    out = []
    for rt, at in ((rtol, atol), (rtol / 100, atol / 100)):
        t = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, net, t, dt, rt, at, integrator="rkc", max_steps=10000000)
        zb.sync(ctx)
        out.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    nv = net_d["n_species"] + net_d["thermal"]
    assert np.all(ref[1] == 0)
    check(f"rkc {which}", out[0], (ref, fine), rtol, atol, nv, out[1])
    # one Jacobian bound per attempt, several stages per step, no LU on either side
    for s in (out[0][2], ref[2]):
        assert np.all(s[:, 2] == s[:, 0] + s[:, 5]) and np.all(s[:, 3] == 0)
    net.close()


def test_rkc_rejects_mixed_precision(zbm):
    zb, ctx = zbm
    c = W.nv14(4)
    net = zb.Network(ctx, c["net"])
    with pytest.raises(zb.ZoneburnError) as e:
        zb.burn(ctx, net, torch.tensor(c["state"], device="cuda:0"), 1.0, 1e-6, 1e-10,
                precision="mixed", integrator="rkc")
    assert e.value.code == zb.EINVAL
    net.close()


@pytest.mark.parametrize("which,jac_policy", [("nv14", 0), ("nv22", 0), ("nv48", 0),
                                               ("nv14", 1)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fd_retry_parity(zbm, which, jac_policy, precision):
    """A 5-step cap fails nearly every zone, so the retry with the finite-difference Jacobian
    (at the first run's tolerances) integrates them all: the oracle's statuses (6), results
    within the widened bar, and, in the retry pass, nv RHS evaluations per Jacobian on top of
    the integrator's own (2 at the start, one per Newton iteration, one per order-1 restart
    after three error failures)."""
    zb, ctx = zbm
    if which == "nv14":
        net_d = W.nv14_network()
        st = W.random_zones(net_d, 128, seed=779)
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        ns, R, seed = W.BATCHED_NETS[k]
        net_d = W.random_network(ns, R, seed)
        st = W.random_zones(net_d, [0, 96, 32][k], seed=778, T_range=W.BATCHED_T_RANGE,
                            T_dist="loguniform")
    nv = net_d["n_species"] + net_d["thermal"]
    retry = (1e-8, 1e-12, 100000, "fd")
    ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12, max_steps=5, retry=retry,
                      jac_policy=jac_policy)
    fine = oracle.burn(net_d, st, 1.0, 1e-10, 1e-14, max_steps=10000000)
    net = zb.Network(ctx, net_d)
    t = torch.tensor(st, device="cuda:0")
    status, stats = zb.burn(ctx, net, t, 1.0, 1e-8, 1e-12, precision=precision, max_steps=5,
                            retry=retry, jac_policy=jac_policy)
    assert zb.sync(ctx) == 0
    g = (t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy())
    gfine = run_gpu(zb, ctx, net_d, st, 1.0, 1e-10, 1e-14, precision=precision,
                    max_steps=10000000, net=net)
    t1 = torch.tensor(st, device="cuda:0")
    s1, st1 = zb.burn(ctx, net, t1, 1.0, 1e-8, 1e-12, precision=precision, max_steps=5,
                      jac_policy=jac_policy)
    zb.sync(ctx)
    first = (t1.cpu().numpy(), s1.cpu().numpy(), st1.cpu().numpy())
    retried = ref[1] == 6
    assert retried.sum() >= 0.9 * len(st)
    assert np.array_equal(g[1], ref[1])
    as_ok = lambda r: (r[0], np.where(r[1] == 6, 0, r[1]).astype(np.int32), r[2])
    check(f"{which} fd retry {precision} policy {jac_policy}", as_ok(g), (as_ok(ref), fine),
          1e-8, 1e-12, nv, gfine)
    once_ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12, max_steps=5, jac_policy=jac_policy)[2]
    for total, once in ((g[2], first[2]), (ref[2], once_ref)):
        p = (total - once)[retried]
        if jac_policy == 0:
            extra = p[:, 1] - 2 - p[:, 4] - nv * p[:, 2]
            assert np.all(extra >= 0) and np.all(3 * extra <= p[:, 5]), extra[extra != 0][:5]
        else:
            # reuse: far fewer Jacobians than steps, each still nv evaluations beyond the
            # integrator's own (one per Newton iteration, one per attempt that refreshes J
            # before its Newton pass, 2 at the start, restarts)
            assert p[:, 2].sum() * 4 < p[:, 0].sum()
            assert np.all(p[:, 1] >= 2 + p[:, 4] + nv * p[:, 2])
    net.close()


def test_fd_retry_options_are_checked(zbm):
    """The finite-difference retry Jacobian is a BDF option (no Jacobian-based solve in RKC),
    and only 'analytic' and 'fd' exist."""
    zb, ctx = zbm
    c = W.nv14(4)
    net = zb.Network(ctx, c["net"])
    t = torch.tensor(c["state"], device="cuda:0")
    with pytest.raises(zb.ZoneburnError) as e:
        zb.burn(ctx, net, t, 1.0, 1e-6, 1e-10, integrator="rkc", retry=(1e-4, 1e-8, 1000, "fd"))
    assert e.value.code == zb.EINVAL
    with pytest.raises(ValueError):
        zb.burn(ctx, net, t, 1.0, 1e-6, 1e-10, retry=(1e-4, 1e-8, 1000, "numeric"))
    net.close()


@pytest.mark.parametrize("lanes", [1, 4])
def test_fd_retry_robertson_rows_per_lane(zbm, lanes):
    """The finite-difference retry on Robertson with one lane per zone (four rows a lane)
    and four lanes per zone: a 20-step cap fails every zone, the retry at the same
    tolerances matches the oracle's (statuses 6, results within the bar)."""
    zb, ctx = zbm
    c = W.robertson(512)
    retry = (1e-8, 1e-12, 100000, "fd")
    ref = oracle.burn(c["net"], c["state"], c["dt"], 1e-8, 1e-12, scale=c["scale"], max_steps=20,
                      retry=retry)
    fine = oracle.burn(c["net"], c["state"], c["dt"], 1e-10, 1e-14, scale=c["scale"],
                       max_steps=10000000)
    net = zb.Network(ctx, c["net"])
    t = torch.tensor(c["state"], device="cuda:0")
    sc = torch.tensor(c["scale"], device="cuda:0")
    status, stats = zb.burn(ctx, net, t, c["dt"], 1e-8, 1e-12, rate_scale=sc, lanes=lanes,
                            max_steps=20, retry=retry)
    assert zb.sync(ctx) == 0
    g = (t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy())
    gfine = run_gpu(zb, ctx, c["net"], c["state"], c["dt"], 1e-10, 1e-14, scale=c["scale"],
                    lanes=lanes, max_steps=10000000, net=net)
    assert np.all(ref[1] == 6) and np.array_equal(g[1], ref[1])
    as_ok = lambda r: (r[0], np.where(r[1] == 6, 0, r[1]).astype(np.int32), r[2])
    check(f"robertson fd retry L{lanes}", as_ok(g), (as_ok(ref), fine), 1e-8, 1e-12, 3, gfine)
    net.close()


@pytest.mark.parametrize("which,jac_policy", [("nv14", 0), ("nv22", 0), ("nv48", 0),
                                               ("nv14", 1), ("nv48", 1)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variable_coefficient_bdf_parity(zbm, which, jac_policy, precision):
    """VODE's variable-coefficient BDF form (integrator 'bdf_variable') against the oracle's
    form='variable', with either Jacobian policy: same statuses, results within the widened
    bar (each side's own error from its run at rtol/100), and a step path of its own (the
    fixed form takes different steps on the same zones)."""
    zb, ctx = zbm
    if which == "nv14":
        net_d, n, Tr, Td = W.nv14_network(), 256, (1e3, 5e3), "uniform"
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        ns, R, seed = W.BATCHED_NETS[k]
        net_d, n, Tr, Td = W.random_network(ns, R, seed), [0, 128, 48][k], W.BATCHED_T_RANGE, "loguniform"
    st = W.random_zones(net_d, n, seed=781, T_range=Tr, T_dist=Td)
    nv = net_d["n_species"] + net_d["thermal"]
    ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12, jac_policy=jac_policy, form="variable")
    fine = oracle.burn(net_d, st, 1.0, 1e-10, 1e-14, jac_policy=jac_policy, form="variable",
                       max_steps=10000000)
    net = zb.Network(ctx, net_d)
    out = []
    for rt, at, ms, integ in ((1e-8, 1e-12, 0, "bdf_variable"), (1e-10, 1e-14, 10000000, "bdf_variable"),
                              (1e-8, 1e-12, 0, "bdf")):
        t = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, net, t, 1.0, rt, at, precision=precision,
                                jac_policy=jac_policy, max_steps=ms, integrator=integ)
        zb.sync(ctx)
        out.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    check(f"{which} variable-coefficient {precision} policy {jac_policy}", out[0], (ref, fine),
          1e-8, 1e-12, nv, out[1])
    assert not np.array_equal(out[0][2][:, 0], out[2][2][:, 0])
    net.close()


@pytest.mark.parametrize("lanes", [1, 4])
def test_variable_coefficient_bdf_robertson(zbm, lanes):
    zb, ctx = zbm
    c = W.robertson(512)
    ref = oracle.burn(c["net"], c["state"], c["dt"], 1e-8, 1e-12, scale=c["scale"], form="variable")
    fine = oracle.burn(c["net"], c["state"], c["dt"], 1e-10, 1e-14, scale=c["scale"],
                       form="variable", max_steps=10000000)
    net = zb.Network(ctx, c["net"])
    sc = torch.tensor(c["scale"], device="cuda:0")
    out = []
    for rt, at, ms in ((1e-8, 1e-12, 0), (1e-10, 1e-14, 10000000)):
        t = torch.tensor(c["state"], device="cuda:0")
        status, stats = zb.burn(ctx, net, t, c["dt"], rt, at, rate_scale=sc, lanes=lanes,
                                max_steps=ms, integrator="bdf_variable")
        zb.sync(ctx)
        out.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    check(f"robertson variable-coefficient L{lanes}", out[0], (ref, fine), 1e-8, 1e-12, 3, out[1])
    net.close()


def _blu_case(which):
    """(network, zones, lanes) of a blocked-LU case: the 48-variable network of the batched
    workload, networks of 40 and 33 variables (identity rows past nv; a last panel of one
    step), and the 14-variable network forced onto the 48-row kernel (a first panel of 14
    steps, two empty panels)."""
    if which == "nv48":
        ns, R, seed = W.BATCHED_NETS[2]
        return W.random_network(ns, R, seed), 48, 0, W.BATCHED_T_RANGE, "loguniform"
    if which == "nv40":
        return W.random_network(39, 120, 612), 48, 0, W.BATCHED_T_RANGE, "loguniform"
    if which == "nv33":
        return W.random_network(32, 100, 613), 48, 0, W.BATCHED_T_RANGE, "loguniform"
    return W.nv14_network(), 64, 64, (1e3, 5e3), "uniform"


@pytest.mark.parametrize("which,integrator", [("nv48", "bdf"), ("nv48", "bdf_variable"),
                                               ("nv40", "bdf"), ("nv33", "bdf"),
                                               ("nv14_on_64_lanes", "bdf")])
def test_blocked_mfma_lu_parity(zbm, which, integrator):
    """The blocked LU with its trailing updates on FP32 MFMA (lu='mfma', mixed precision)
    against the FP64 oracle of the same integrator form: same statuses, results within the
    widened bar (each side's own error from its run at rtol/100)."""
    zb, ctx = zbm
    net_d, n, lanes, Tr, Td = _blu_case(which)
    st = W.random_zones(net_d, n, seed=783, T_range=Tr, T_dist=Td)
    nv = net_d["n_species"] + net_d["thermal"]
    form = "variable" if integrator == "bdf_variable" else "fixed"
    ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12, form=form)
    fine = oracle.burn(net_d, st, 1.0, 1e-10, 1e-14, form=form, max_steps=10000000)
    net = zb.Network(ctx, net_d)
    out = []
    for rt, at, ms in ((1e-8, 1e-12, 0), (1e-10, 1e-14, 10000000)):
        t = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, net, t, 1.0, rt, at, precision="mixed", lanes=lanes,
                                max_steps=ms, integrator=integrator, lu="mfma")
        assert zb.sync(ctx) == 0
        out.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    check(f"{which} blocked MFMA LU {integrator}", out[0], (ref, fine), 1e-8, 1e-12, nv, out[1])
    net.close()


def test_blocked_mfma_lu_options_are_checked(zbm):
    """lu='mfma' needs the mixed precision, the every-step Jacobian and a BDF integrator
    (EINVAL otherwise).  A network on fewer than 64 lanes per zone has no blocked form and
    takes the vector-unit LU: the same results bit for bit."""
    zb, ctx = zbm
    ns, R, seed = W.BATCHED_NETS[2]
    net_d = W.random_network(ns, R, seed)
    net = zb.Network(ctx, net_d)
    t = torch.tensor(W.random_zones(net_d, 4, seed=5), device="cuda:0")
    for kw in (dict(precision="fp64"), dict(precision="mixed", jac_policy=1),
               dict(precision="fp64", integrator="rkc"), dict(precision="mixed", integrator="rkc")):
        with pytest.raises(zb.ZoneburnError) as e:
            zb.burn(ctx, net, t, 1.0, 1e-6, 1e-10, lu="mfma", **kw)
        assert e.value.code == zb.EINVAL, kw
    with pytest.raises(ValueError):
        zb.burn(ctx, net, t, 1.0, 1e-6, 1e-10, precision="mixed", lu="blocked")
    small = zb.Network(ctx, W.nv14_network())
    st = W.nv14(64)["state"]
    res = []
    for lu in ("mfma", "valu"):
        ts = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, small, ts, 1.0, 1e-8, 1e-12, precision="mixed", lu=lu)
        assert zb.sync(ctx) == 0
        res.append((ts.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    for a, b in zip(*res):
        assert np.array_equal(a, b)
    small.close()
    net.close()


def test_fp64_whole_wave_rate_factors(zbm):
    """The FP64 48-row kernel keeps per-reaction rate factors in LDS only when its launch
    needs them (trimmed layout): a thermal network with rate scales, a network without
    temperature (constant rates), each against the oracle; and one launch of a scaled and an
    unscaled segment, bitwise equal to the two separate burns (without scales the factors
    are 1 either way)."""
    zb, ctx = zbm
    ns, R, seed = W.BATCHED_NETS[2]
    net_t = W.random_network(ns, R, seed)
    net_c = W.random_network(48, 150, 614, thermal=False, log10A=(0.0, 4.0))
    rng = np.random.default_rng(615)
    st_t = W.random_zones(net_t, 32, seed=616, T_range=W.BATCHED_T_RANGE, T_dist="loguniform")
    sc_t = np.exp(rng.normal(0.0, 0.5, (32, R)))
    st_c = W.random_zones(net_c, 32, seed=617)
    single = {}
    for name, net_d, st, sc in (("scaled", net_t, st_t, sc_t), ("unscaled", net_t, st_t, None),
                                ("constant-rate", net_c, st_c, None)):
        nv = net_d["n_species"] + net_d["thermal"]
        ref = oracle_ref(net_d, st, 1.0, 1e-8, 1e-12, scale=sc)
        g = run_gpu(zb, ctx, net_d, st, 1.0, 1e-8, 1e-12, scale=sc)
        gf = run_gpu(zb, ctx, net_d, st, 1.0, 1e-10, 1e-14, scale=sc, max_steps=10000000)
        check(f"48-row FP64 {name}", g, ref, 1e-8, 1e-12, nv, gf)
        single[name] = g
    net = zb.Network(ctx, net_t)
    ts = [torch.tensor(st_t, device="cuda:0") for _ in range(2)]
    status = [torch.empty(32, dtype=torch.int32, device="cuda:0") for _ in range(2)]
    stats = [torch.empty((32, 7), dtype=torch.int32, device="cuda:0") for _ in range(2)]
    sc = torch.tensor(sc_t, device="cuda:0")
    zb.burn_batch(ctx, [dict(net=net, state=ts[0], dt=1.0, rtol=1e-8, atol=1e-12, rate_scale=sc,
                             status=status[0], stats=stats[0]),
                        dict(net=net, state=ts[1], dt=1.0, rtol=1e-8, atol=1e-12,
                             status=status[1], stats=stats[1])])
    assert zb.sync(ctx) == 0
    for k, name in enumerate(("scaled", "unscaled")):
        assert np.array_equal(ts[k].cpu().numpy(), single[name][0]), name
        assert np.array_equal(status[k].cpu().numpy(), single[name][1]), name
        assert np.array_equal(stats[k].cpu().numpy(), single[name][2]), name
    net.close()


def test_fp64_fallback(zbm):
    """fp64_fallback with the mixed precision: zones that fail in mixed precision are burned
    again from their inputs by the FP64 kernel.  Such a zone reports OK_FP64 (7), its row is
    bitwise the plain FP64 burn's, and its counters are the sum of both runs; every other zone
    is bitwise the plain mixed burn's.  The same holds for a two-segment batch (one list per
    segment) and for a graph replay; the server rejects the option."""
    zb, ctx = zbm
    net_d = W.random_network(7, 12, 881)
    full = W.random_zones(net_d, 131072, seed=882)
    net = zb.Network(ctx, net_d)

    def run(st, **kw):
        t = torch.tensor(st, device="cuda:0")
        status, stats = zb.burn(ctx, net, t, 1.0, 1e-8, 1e-12, **kw)
        zb.sync(ctx)
        return t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()

    failed = np.nonzero(run(full, precision="mixed")[1] != 0)[0]
    assert failed.size > 0, "the input must have zones that fail in mixed precision"
    idx = np.union1d(failed, np.arange(251))
    st = full[idx]
    mixed = run(st, precision="mixed")
    fp64 = run(st, precision="fp64")
    fb = run(st, precision="mixed", fp64_fallback=True)
    bad = mixed[1] != 0
    assert bad.sum() == failed.size
    assert np.all(fp64[1][bad] == 0)
    assert np.all(fb[1][bad] == 7) and np.all(fb[1][~bad] == mixed[1][~bad])
    assert np.array_equal(fb[0][bad], fp64[0][bad]) and np.array_equal(fb[0][~bad], mixed[0][~bad])
    assert np.array_equal(fb[2][bad], mixed[2][bad] + fp64[2][bad])
    assert np.array_equal(fb[2][~bad], mixed[2][~bad])
    # with FP64 the option does nothing; a non-finite input ends NONFINITE, it does not fall back
    for a_, b_ in zip(run(st, precision="fp64", fp64_fallback=True), fp64):
        assert np.array_equal(a_, b_)
    st_nan = st.copy()
    st_nan[3, 2] = np.nan
    nan = run(st_nan, precision="mixed", fp64_fallback=True)
    assert nan[1][3] == 5 and np.array_equal(np.delete(nan[1], 3), np.delete(fb[1], 3))
    # the rescued zones against the oracle (status 7 counts as OK there)
    nv = net_d["n_species"] + net_d["thermal"]
    ref = oracle_ref(net_d, st[bad], 1.0, 1e-8, 1e-12)
    gfine = run_gpu(zb, ctx, net_d, st[bad], 1.0, 1e-10, 1e-14, precision="fp64",
                    max_steps=10000000, net=net)
    rescued = (fb[0][bad], np.where(fb[1][bad] == 7, 0, fb[1][bad]).astype(np.int32), fb[2][bad])
    check("fp64 fallback zones", rescued, ref, 1e-8, 1e-12, nv, gfine)
    # two segments in one call: one list each
    half = len(idx) // 2
    ts = [torch.tensor(st[:half], device="cuda:0"), torch.tensor(st[half:], device="cuda:0")]
    status = [torch.empty(t.shape[0], dtype=torch.int32, device="cuda:0") for t in ts]
    stats = [torch.empty((t.shape[0], 7), dtype=torch.int32, device="cuda:0") for t in ts]
    zb.burn_batch(ctx, [dict(net=net, state=ts[k], dt=1.0, rtol=1e-8, atol=1e-12, status=status[k],
                             stats=stats[k]) for k in range(2)], precision="mixed", fp64_fallback=True)
    zb.sync(ctx)
    got = [np.concatenate([a.cpu().numpy() for a in x]) for x in (ts, status, stats)]
    for a, b in zip(got, fb):
        assert np.array_equal(a, b)
    # a graph replay
    tg = torch.tensor(st, device="cuda:0")
    sg = torch.empty(len(idx), dtype=torch.int32, device="cuda:0")
    gs = torch.empty((len(idx), 7), dtype=torch.int32, device="cuda:0")
    g = zb.Graph(ctx, [dict(net=net, state=tg, dt=1.0, rtol=1e-8, atol=1e-12, status=sg, stats=gs)],
                 precision="mixed", fp64_fallback=True)
    for _ in range(2):
        tg.copy_(torch.tensor(st, device="cuda:0"))
        g.launch()
        zb.sync(ctx)
        assert np.array_equal(tg.cpu().numpy(), fb[0]) and np.array_equal(sg.cpu().numpy(), fb[1])
        assert np.array_equal(gs.cpu().numpy(), fb[2])
    g.close()
    with pytest.raises(zb.ZoneburnError) as e:
        zb.Server(ctx, 1 << 26, precision="mixed", fp64_fallback=True)
    assert e.value.code == zb.EUNSUPPORTED
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ns,R,seed", [(11, 25, 615), (19, 40, 616), (36, 110, 617)])
def test_networks_below_the_padded_size(zbm, ns, R, seed, precision):
    """Networks of 12, 20 and 37 variables on the 14-, 22- and 48-row kernels: the LU and the
    solves test nv once per 8 steps, so a chunk runs a few steps past nv (identity rows of M).
    Against the oracle, in both precisions."""
    zb, ctx = zbm
    net = W.random_network(ns, R, seed)
    st = W.random_zones(net, 64, seed=seed + 1, T_range=W.BATCHED_T_RANGE, T_dist="loguniform")
    ref = oracle_ref(net, st, 1.0, 1e-8, 1e-12)
    gpu, fine = run_pair(zb, ctx, net, st, 1.0, 1e-8, 1e-12, precision=precision)
    check(f"nv{ns + 1} {precision}", gpu, ref, 1e-8, 1e-12, ns + 1, fine)
