"""GPU tests of the runtime around the burn kernels: multi-class batches, HIP-graph replays,
and the continuous-batching server.  Results are compared bitwise with plain zb_burn calls,
whose parity with the oracle is covered in test_gpu_parity.py."""
import time

import numpy as np
import pytest

import oracle
from paper_2608_06466_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zbm():
    from paper_2608_06466_amd import zoneburn as zb
    assert torch.cuda.is_available()
    ctx = zb.Context(0)
    nets_d = W.batched_networks()
    nets = [zb.Network(ctx, n) for n in nets_d]
    yield zb, ctx, nets_d, nets
    for n in nets:
        n.close()
    ctx.close()


def inputs(k, nets_d, zones, seed):
    """State (and rate scales) of network k of the batched workload: 0 Robertson, 1..3 random nv 14/22/48."""
    if k == 0:
        st, sc = W.robertson_zones(zones, seed=seed)
        return st, sc, 1.0e5
    st = W.random_zones(nets_d[k], zones, seed=seed, T_range=W.BATCHED_T_RANGE, T_dist="loguniform")
    return st, None, 1.0


def burn_alone(zb, ctx, net, st, sc, dt, rtol, precision):
    t = torch.tensor(st, device="cuda:0")
    s = None if sc is None else torch.tensor(sc, device="cuda:0")
    status, stats = zb.burn(ctx, net, t, dt, rtol, 1e-12, rate_scale=s, precision=precision)
    zb.sync(ctx)
    return t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()


def make_segments(zb, nets_d, nets, sizes, seed=11):
    segs, host = [], []
    for k, nz in enumerate(sizes):
        st, sc, dt = inputs(k, nets_d, nz, seed + k)
        seg = dict(net=nets[k], state=torch.tensor(st, device="cuda:0"), dt=dt, rtol=1e-8, atol=1e-12,
                   rate_scale=None if sc is None else torch.tensor(sc, device="cuda:0"),
                   status=torch.empty(nz, dtype=torch.int32, device="cuda:0"),
                   stats=torch.empty((nz, 7), dtype=torch.int32, device="cuda:0"))
        segs.append(seg)
        host.append((st, sc, dt))
    return segs, host


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_four_kernel_classes_in_one_call_match_single_burns(zbm, precision):
    """Robertson, nv 14, 22 and 48 in one zb_burn_batch call (concurrent launches on forked
    streams): bitwise the single-network results."""
    zb, ctx, nets_d, nets = zbm
    segs, host = make_segments(zb, nets_d, nets, [700, 300, 130, 65])
    zb.burn_batch(ctx, segs, precision=precision)
    zb.sync(ctx)
    for k, seg in enumerate(segs):
        st, sc, dt = host[k]
        ref = burn_alone(zb, ctx, nets[k], st, sc, dt, 1e-8, precision)
        assert np.array_equal(seg["state"].cpu().numpy(), ref[0]), k
        assert np.array_equal(seg["status"].cpu().numpy(), ref[1]), k
        assert np.array_equal(seg["stats"].cpu().numpy(), ref[2]), k


def test_graph_replays_match_eager(zbm):
    """A captured four-class burn replayed three times, with eager burns in between, gives the
    eager result every time."""
    zb, ctx, nets_d, nets = zbm
    segs, host = make_segments(zb, nets_d, nets, [500, 200, 90, 40], seed=31)
    init = [s["state"].clone() for s in segs]
    zb.burn_batch(ctx, segs, precision="mixed")
    zb.sync(ctx)
    eager = [(s["state"].cpu().numpy(), s["status"].cpu().numpy(), s["stats"].cpu().numpy()) for s in segs]
    g = zb.Graph(ctx, segs, precision="mixed")
    other = torch.tensor(W.nv14(128)["state"], device="cuda:0")
    other0 = other.clone()
    net2 = zb.Network(ctx, W.nv14_network())
    for rep in range(3):
        for s, i0 in zip(segs, init):
            s["state"].copy_(i0)
            s["status"].fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        zb.sync(ctx)
        for k, s in enumerate(segs):
            assert np.array_equal(s["state"].cpu().numpy(), eager[k][0]), (rep, k)
            assert np.array_equal(s["status"].cpu().numpy(), eager[k][1]), (rep, k)
            assert np.array_equal(s["stats"].cpu().numpy(), eager[k][2]), (rep, k)
        # unrelated eager work between replays
        other.copy_(other0)
        zb.burn(ctx, net2, other, 1.0, 1e-8, 1e-12)
        zb.sync(ctx)
    g.close()
    net2.close()


def test_torch_graph_capture_of_zb_burn(zbm):
    """zb.burn captured by torch.cuda.graph (the kernels clear their queues with a kernel, not a
    memset node) and replayed with the state reset eagerly in between."""
    zb, ctx, nets_d, nets = zbm
    c = W.nv14(256)
    net = zb.Network(ctx, c["net"])
    ref = burn_alone(zb, ctx, net, c["state"], None, 1.0, 1e-8, "fp64")
    static = torch.tensor(c["state"], device="cuda:0")
    init = static.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up outside the capture
        zb.burn(ctx, net, static, 1.0, 1e-8, 1e-12)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        status, stats = zb.burn(ctx, net, static, 1.0, 1e-8, 1e-12)
    for rep in range(3):
        static.copy_(init)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(static.cpu().numpy(), ref[0]), rep
        assert np.array_equal(status.cpu().numpy(), ref[1]), rep
        assert np.array_equal(stats.cpu().numpy(), ref[2]), rep
    zb.sync(ctx)
    net.close()


def test_counter_ring_wraps_without_waiting_between_calls(zbm):
    """1100 calls on one stream with no synchronisation between them: the context's 1024
    zone-queue slots wrap, and a reused slot is first waited for, so every call's zones come
    out bitwise as one call over all of them."""
    zb, _, nets_d, _ = zbm
    ctx = zb.Context(0)
    net = zb.Network(ctx, nets_d[0])
    n, per = 1100, 4
    st, sc = W.robertson_zones(n * per, seed=77)
    full = torch.tensor(st, device="cuda:0")
    fsc = torch.tensor(sc, device="cuda:0")
    ref_status, ref_stats = zb.burn(ctx, net, full, 1.0e5, 1e-8, 1e-12, rate_scale=fsc)
    zb.sync(ctx)
    t = torch.tensor(st, device="cuda:0")
    outs = [zb.burn(ctx, net, t[i * per:(i + 1) * per], 1.0e5, 1e-8, 1e-12,
                    rate_scale=fsc[i * per:(i + 1) * per]) for i in range(n)]
    zb.sync(ctx)
    assert np.array_equal(t.cpu().numpy(), full.cpu().numpy())
    assert np.array_equal(torch.cat([o[0] for o in outs]).cpu().numpy(), ref_status.cpu().numpy())
    assert np.array_equal(torch.cat([o[1] for o in outs]).cpu().numpy(), ref_stats.cpu().numpy())
    net.close()
    ctx.close()


def test_fallback_list_ring_wraps_without_waiting_between_calls(zbm):
    """20 mixed-precision calls with the FP64 fallback and no synchronisation between them:
    the 16 fallback lists of the context wrap, and each call still rescues exactly its own
    failed zones (bitwise as the same call made alone)."""
    zb = zbm[0]
    ctx = zb.Context(0)
    net_d = W.random_network(7, 12, 881)
    full = W.random_zones(net_d, 131072, seed=882)
    net = zb.Network(ctx, net_d)
    t = torch.tensor(full, device="cuda:0")
    status, _ = zb.burn(ctx, net, t, 1.0, 1e-8, 1e-12, precision="mixed")
    zb.sync(ctx)
    failed = np.nonzero(status.cpu().numpy() != 0)[0]
    assert failed.size > 0, "the input must have zones that fail in mixed precision"
    st = full[np.union1d(failed, np.arange(40))]
    a = torch.tensor(st, device="cuda:0")
    ref = zb.burn(ctx, net, a, 1.0, 1e-8, 1e-12, precision="mixed", fp64_fallback=True)
    zb.sync(ctx)
    assert (ref[0].cpu().numpy() == 7).sum() == failed.size
    ts = [torch.tensor(st, device="cuda:0") for _ in range(20)]
    outs = [zb.burn(ctx, net, x, 1.0, 1e-8, 1e-12, precision="mixed", fp64_fallback=True) for x in ts]
    zb.sync(ctx)
    for x, o in zip(ts, outs):
        assert np.array_equal(x.cpu().numpy(), a.cpu().numpy())
        assert np.array_equal(o[0].cpu().numpy(), ref[0].cpu().numpy())
        assert np.array_equal(o[1].cpu().numpy(), ref[1].cpu().numpy())
    net.close()
    ctx.close()


def test_captured_calls_beyond_the_capture_slots_are_refused(zbm):
    """A call captured into a graph keeps its zone-queue slot for the context's lifetime; the
    65th captured call of a context is refused with ZB_EBUSY (no kernel is launched), and
    the captured graphs still replay correctly."""
    zb, _, nets_d, _ = zbm
    ctx = zb.Context(0)
    net = zb.Network(ctx, nets_d[0])
    st, sc = W.robertson_zones(8, seed=5)
    state = torch.tensor(st, device="cuda:0")
    scale = torch.tensor(sc, device="cuda:0")
    ref_status, _ = zb.burn(ctx, net, state.clone(), 1.0e5, 1e-8, 1e-12, rate_scale=scale)
    zb.sync(ctx)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        zb.burn(ctx, net, state.clone(), 1.0e5, 1e-8, 1e-12, rate_scale=scale)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graphs, bufs = [], []
    for i in range(64):
        buf = state.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = zb.burn(ctx, net, buf, 1.0e5, 1e-8, 1e-12, rate_scale=scale)
        graphs.append((g, buf, out))
    g = torch.cuda.CUDAGraph()
    buf = state.clone()
    with pytest.raises(zb.ZoneburnError) as ei:
        with torch.cuda.graph(g):
            zb.burn(ctx, net, buf, 1.0e5, 1e-8, 1e-12, rate_scale=scale)
    assert ei.value.code == zb.EBUSY
    torch.cuda.synchronize()
    for k in (0, 63):
        gk, bk, ok = graphs[k]
        bk.copy_(state)
        torch.cuda.synchronize()
        gk.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ok[0].cpu().numpy(), ref_status.cpu().numpy())
    # eager calls still run
    x = state.clone()
    zb.burn(ctx, net, x, 1.0e5, 1e-8, 1e-12, rate_scale=scale)
    zb.sync(ctx)
    del graphs
    net.close()
    ctx.close()


def serving_mix(nets_d, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        k = int(rng.integers(0, 4))
        zones = int(np.rint(np.exp(rng.uniform(np.log(64), np.log([3000, 1500, 600, 150][k])))))
        rtol = float(rng.choice([1e-6, 1e-8]))
        st, sc, dt = inputs(k, nets_d, zones, 1000 + i)
        reqs.append(dict(k=k, zones=zones, rtol=rtol, state=st, scale=sc, dt=dt))
    return reqs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_server_results_same_alone_and_in_the_mix(zbm, precision):
    """Requests of all four networks, two tolerances and many sizes, submitted while earlier
    ones run: each result is bitwise the result of the same request burned alone."""
    zb, ctx, nets_d, nets = zbm
    reqs = serving_mix(nets_d, 16, seed=5)
    srv = zb.Server(ctx, 256 << 20, precision=precision, slice_zones=97)
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(srv.submit(nets[r["k"]], r["state"], r["dt"], r["rtol"], 1e-12, r["scale"]))
        if i % 4 == 3:
            time.sleep(0.002)   # later requests arrive while earlier ones are on the GPU
    results = []
    for t in tickets:
        assert srv.wait(t, timeout=120.0)
        results.append(srv.fetch(t))
    tot = srv.stats()
    srv.close()
    assert tot["requests_done"] == len(reqs) and tot["bytes_in_use"] == 0
    assert tot["launches"] < sum(-(-r["zones"] // 97) for r in reqs)   # slices shared launches
    for r, (out, status, stats, info) in zip(reqs, results):
        ref = burn_alone(zb, ctx, nets[r["k"]], r["state"], r["scale"], r["dt"], r["rtol"], precision)
        assert np.array_equal(out, ref[0])
        assert np.array_equal(status, ref[1])
        assert np.array_equal(stats, ref[2])
        assert info["zones"] == r["zones"] and info["zones_ok"] == int((ref[1] == 0).sum())
        assert 0.0 <= info["queue_s"] <= info["first_launch_s"] <= info["latency_s"]


def test_server_admission_waits_for_memory(zbm):
    """A budget that holds about two requests at a time: every request still completes, resident
    bytes never exceed the budget, and the queue of waiting requests is bounded."""
    zb, ctx, nets_d, nets = zbm
    budget = 1 << 20
    st, sc, dt = inputs(1, nets_d, 2500, 77)       # 2500 zones x (112 + 4 + 28) B = 360 KB
    srv = zb.Server(ctx, budget, max_pending=4)
    tickets = [srv.submit(nets[1], st, dt, 1e-8, 1e-12) for _ in range(4)]
    with pytest.raises(zb.ZoneburnError) as e:
        for _ in range(8):            # the pending queue (4) fills before the first admissions
            tickets.append(srv.submit(nets[1], st, dt, 1e-8, 1e-12))
    assert e.value.code in (zb.EBUSY,)
    with pytest.raises(zb.ZoneburnError) as e2:
        srv.submit(nets[1], np.tile(st, (4, 1)), dt, 1e-8, 1e-12)   # larger than the budget
    assert e2.value.code == zb.EINVAL
    ref = burn_alone(zb, ctx, nets[1], st, None, dt, 1e-8, "fp64")
    for t in tickets:
        assert srv.wait(t, timeout=120.0)
        out, status, stats, info = srv.fetch(t)
        assert np.array_equal(out, ref[0]) and np.array_equal(status, ref[1])
    tot = srv.stats()
    assert 0 < tot["peak_bytes_in_use"] <= budget
    with pytest.raises(zb.ZoneburnError) as e3:
        srv.fetch(tickets[0])
    assert e3.value.code == zb.ENOTFOUND
    srv.close()


def test_small_network_with_many_reactions_gets_a_mapping_that_fits(zbm):
    """Three species and T with 80 reactions: one lane per zone would need more LDS than a
    CU has (the reaction columns are kept once per zone of the wave), so the automatic
    mapping takes wider groups; the burn runs and matches the oracle, and the autotuner
    skips the mappings that cannot launch."""
    zb, ctx = zbm[0], zbm[1]
    net_d = W.random_network(3, 80, 911)
    st = W.random_zones(net_d, 256, seed=912, T_range=(90.0, 300.0), T_dist="loguniform")
    net = zb.Network(ctx, net_d)
    lanes = zb.get_mapping(ctx, net, "fp64")
    assert lanes > 1
    t = torch.tensor(st, device="cuda:0")
    status, stats = zb.burn(ctx, net, t, 1.0, 1e-8, 1e-12)
    zb.sync(ctx)
    ref = oracle.burn(net_d, st, 1.0, 1e-8, 1e-12)
    out = t.cpu().numpy()
    status = status.cpu().numpy()
    assert np.array_equal(status, ref[1])
    ok = ref[1] == 0
    assert ok.sum() > 200
    g = np.abs(out[ok, :4] - ref[0][ok, :4]) / np.maximum(np.abs(ref[0][ok, :4]), 1e-4)
    assert g.max() < 1e-5   # accuracy proper is covered by the parity tests
    best, times = zb.autotune(ctx, net, torch.tensor(st[:64], device="cuda:0"), 1.0, 1e-8, 1e-12)
    assert best > 1 and times[0] < 0
    net.close()


def test_graph_and_server_take_the_method_options(zbm):
    """The variable-coefficient form with the Jacobian reuse (VODE's configuration) through a
    captured graph and through the server gives, bitwise, what zb_burn gives with the same
    options."""
    zb, ctx, nets_d, nets = zbm
    opts = dict(precision="mixed", jac_policy=1, integrator="bdf_variable")
    segs, host = make_segments(zb, nets_d, nets, [300, 120, 60, 24], seed=41)
    init = [s["state"].clone() for s in segs]
    ref = []
    for k, (st, sc, dt) in enumerate(host):
        t = torch.tensor(st, device="cuda:0")
        s = None if sc is None else torch.tensor(sc, device="cuda:0")
        status, stats = zb.burn(ctx, nets[k], t, dt, 1e-8, 1e-12, rate_scale=s, **opts)
        zb.sync(ctx)
        ref.append((t.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy()))
    g = zb.Graph(ctx, segs, **opts)
    for rep in range(2):
        for s, i0 in zip(segs, init):
            s["state"].copy_(i0)
        torch.cuda.synchronize()
        g.launch()
        zb.sync(ctx)
        for k, s in enumerate(segs):
            assert np.array_equal(s["state"].cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(s["stats"].cpu().numpy(), ref[k][2]), (rep, k)
    g.close()
    srv = zb.Server(ctx, 64 << 20, slice_zones=50, **opts)
    tickets = [srv.submit(nets[k], st, dt, 1e-8, 1e-12, sc) for k, (st, sc, dt) in enumerate(host)]
    for k, t in enumerate(tickets):
        assert srv.wait(t, timeout=120.0)
        out, status, stats, info = srv.fetch(t)
        assert np.array_equal(out, ref[k][0]) and np.array_equal(stats, ref[k][2]), k
    srv.close()
