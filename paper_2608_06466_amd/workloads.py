"""Seeded synthetic inputs for the per-zone burn.

This module only draws random numbers and lays them out; it holds none of the
integrator's arithmetic.  Both the HIP path and the CPU oracle read the very
same arrays it returns, so a parity test compares the two on identical bytes.

The paper (Software design section) describes the burn as a per-zone routine
looped over by the application, with a compile-time selected network that
fixes the composition.  It prints no workload, so the shapes below are the
synthetic stand-ins used throughout this project:

* Robertson's three-species kinetics (a textbook stiff test problem) with a
  per-zone log-normal scale on each of its three rate constants;
* random mass-action networks of two-body reactions A+B->C+D with Arrhenius
  rates k = A T^n exp(-E/T) and a heat release q per reaction, the temperature
  being the last integrated variable;
* zone states with T drawn uniformly or log-uniformly and abundances drawn from
  a flat Dirichlet distribution.

A network is a plain dict of numpy arrays:
  n_species (int), thermal (0/1),
  reactant int32[R,2]  (second entry -1 for a first-order reaction),
  product  int32[R,2]  (second entry -1 for a single product),
  lnA, n_exp, E, q  float64[R].
A zone state is float64[zones, n_species+1]: the abundances, then T.
"""
from __future__ import annotations

import math

import numpy as np

# Robertson's rate constants (the standard statement of the problem).
ROBERTSON_K = (0.04, 3.0e7, 1.0e4)


def _net(ns, thermal, reactant, product, lnA, n_exp, E, q):
    return {
        "n_species": int(ns),
        "thermal": int(bool(thermal)),
        "reactant": np.ascontiguousarray(reactant, dtype=np.int32).reshape(-1, 2),
        "product": np.ascontiguousarray(product, dtype=np.int32).reshape(-1, 2),
        "lnA": np.ascontiguousarray(lnA, dtype=np.float64),
        "n_exp": np.ascontiguousarray(n_exp, dtype=np.float64),
        "E": np.ascontiguousarray(E, dtype=np.float64),
        "q": np.ascontiguousarray(q, dtype=np.float64),
    }


def robertson_network():
    """Y0 -> Y1 (k1);  Y1 + Y1 -> Y1 + Y2 (k2);  Y1 + Y2 -> Y0 + Y2 (k3).  No T coupling."""
    reactant = [[0, -1], [1, 1], [1, 2]]
    product = [[1, -1], [1, 2], [0, 2]]
    lnA = [math.log(k) for k in ROBERTSON_K]
    z = [0.0, 0.0, 0.0]
    return _net(3, 0, reactant, product, lnA, z, z, z)


def robertson_zones(zones, seed=101, sigma=0.1):
    """y0 = (1, 0, 0), T slot 0, per-zone scales exp(sigma * N(0,1)) on each rate."""
    rng = np.random.default_rng(seed)
    state = np.zeros((zones, 4), dtype=np.float64)
    state[:, 0] = 1.0
    scale = np.exp(sigma * rng.standard_normal((zones, 3)))
    return state, scale


def random_network(ns, n_reactions, seed, thermal=True,
                   log10A=(2.0, 10.0), n_range=(-1.0, 2.0), E_range=(1.0e3, 4.0e4),
                   q_range=(0.0, 1.0)):
    """Random two-body network A+B->C+D over ns species.

    Draw order (fixed so the bytes are reproducible): the index table [R,4]
    (a, b, c, d i.i.d. uniform with replacement; a reaction whose product
    multiset equals its reactant multiset is redrawn), then log10 A, n, E, q.
    """
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, ns, size=(n_reactions, 4))
    for r in range(n_reactions):
        while sorted(idx[r, :2]) == sorted(idx[r, 2:]):
            idx[r] = rng.integers(0, ns, size=4)
    la = rng.uniform(*log10A, size=n_reactions)
    n = rng.uniform(*n_range, size=n_reactions)
    E = rng.uniform(*E_range, size=n_reactions)
    q = rng.uniform(*q_range, size=n_reactions)
    return _net(ns, thermal, idx[:, :2], idx[:, 2:], la * math.log(10.0), n, E, q)


def random_zones(net, zones, seed, T_range=(1.0e3, 5.0e3), T_dist="uniform"):
    """Zone states: T first (uniform or log-uniform), then Dirichlet(1) abundances."""
    rng = np.random.default_rng(seed)
    ns = net["n_species"]
    if T_dist == "uniform":
        T = rng.uniform(T_range[0], T_range[1], size=zones)
    elif T_dist == "loguniform":
        T = np.exp(rng.uniform(math.log(T_range[0]), math.log(T_range[1]), size=zones))
    else:
        raise ValueError(T_dist)
    Y = rng.dirichlet(np.ones(ns), size=zones)
    state = np.empty((zones, ns + 1), dtype=np.float64)
    state[:, :ns] = Y
    state[:, ns] = T
    return state


def linear_network(ns, seed, k_range=(1.0e-2, 1.0e8), density=0.4):
    """First-order conservative network (reactions Yi -> Yj), log-uniform rates.

    dY/dt = K Y with non-negative off-diagonals and zero column sums, so the
    exact burn is expm(K dt) y0.  Used to pin the integrator.
    """
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(ns) for j in range(ns) if i != j]
    keep = [p for p in pairs if rng.uniform() < density]
    if not keep:
        keep = pairs[:1]
    lk = rng.uniform(math.log(k_range[0]), math.log(k_range[1]), size=len(keep))
    reactant = [[i, -1] for i, _ in keep]
    product = [[j, -1] for _, j in keep]
    z = np.zeros(len(keep))
    return _net(ns, 0, reactant, product, lk, z, z, z)


def two_body_network(k, same=False):
    """A+B->C+D (species 0..3) or, with same=True, A+A->C+D, at constant k."""
    if same:
        reactant, product = [[0, 0]], [[2, 3]]
    else:
        reactant, product = [[0, 1]], [[2, 3]]
    return _net(4, 0, reactant, product, [math.log(k)], [0.0], [0.0], [0.0])


def energy_test_network(ns, n_reactions, seed, B_seed=None):
    """Random thermal network whose heat releases obey q_r = -sum_i B_i nu_ir.

    Then T + sum_i B_i Y_i is an invariant of the exact flow.  Returns the
    network and the vector B.
    """
    net = random_network(ns, n_reactions, seed, thermal=True, E_range=(1.0e3, 2.0e4))
    rng = np.random.default_rng(seed + 7 if B_seed is None else B_seed)
    B = rng.uniform(0.0, 2.0, size=ns)
    q = np.zeros(n_reactions)
    for r in range(n_reactions):
        a, b = net["reactant"][r]
        c, d = net["product"][r]
        nu = np.zeros(ns)
        nu[a] -= 1
        if b >= 0:
            nu[b] -= 1
        nu[c] += 1
        if d >= 0:
            nu[d] += 1
        q[r] = -float(B @ nu)
    net["q"] = q
    return net, B


# ---------------------------------------------------------------------------
# The benchmark workloads: Robertson, the 14-variable network, the four-network batch
# (the mixed-precision and serving workloads reuse these inputs).
# ---------------------------------------------------------------------------

NV14_NET_SEED, NV14_ZONE_SEED = 201, 202
BATCHED_NETS = ((13, 20, 301), (21, 50, 302), (47, 150, 303))
BATCHED_ZONE_SEED = 304
BATCHED_T_RANGE = (90.0, 2500.0)   # log-uniform; gives 7..~5000 BDF steps per zone (oracle)


def robertson(zones=4096):
    """Robertson, 4096 zones, t in [0, 1e5], rtol 1e-8, atol 1e-12."""
    net = robertson_network()
    state, scale = robertson_zones(zones)
    return dict(net=net, state=state, scale=scale, dt=1.0e5, rtol=1.0e-8, atol=1.0e-12)


def nv14_network():
    return random_network(13, 30, NV14_NET_SEED)


def nv14(zones=1 << 20):
    """13 species + T, 30 reactions, T ~ U(1e3, 5e3), Dirichlet(1) abundances, dt = 1."""
    net = nv14_network()
    state = random_zones(net, zones, NV14_ZONE_SEED)
    return dict(net=net, state=state, scale=None, dt=1.0, rtol=1.0e-8, atol=1.0e-12)


def batched_networks():
    nets = [robertson_network()]
    for ns, R, seed in BATCHED_NETS:
        nets.append(random_network(ns, R, seed))
    return nets


def batched(total_zones=1 << 21):
    """Four networks (nv = 3, 14, 22, 48) in zone ratio 4:2:1:1 for one batched launch."""
    nets = batched_networks()
    parts = [total_zones // 2, total_zones // 4, total_zones // 8, total_zones - total_zones // 2
             - total_zones // 4 - total_zones // 8]
    segs = []
    rng_seeds = np.random.SeedSequence(BATCHED_ZONE_SEED).spawn(4)
    for k, (net, nz) in enumerate(zip(nets, parts)):
        if k == 0:
            st, sc = robertson_zones(nz, seed=int(rng_seeds[0].generate_state(1)[0]))
            segs.append(dict(net=net, state=st, scale=sc, dt=1.0e5, rtol=1.0e-8, atol=1.0e-12))
        else:
            st = random_zones(net, nz, int(rng_seeds[k].generate_state(1)[0]),
                              T_range=BATCHED_T_RANGE, T_dist="loguniform")
            segs.append(dict(net=net, state=st, scale=None, dt=1.0, rtol=1.0e-8, atol=1.0e-12))
    return segs


def serving_requests(n_requests, seed=501, rate_hz=100.0, size_range=(1 << 10, 1 << 18),
                     rtols=(1.0e-6, 1.0e-8)):
    """Poisson arrival stream: (arrival_s, network index 0..3, zones, rtol, zone seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps)
    lo, hi = math.log(size_range[0]), math.log(size_range[1])
    sizes = np.rint(np.exp(rng.uniform(lo, hi, size=n_requests))).astype(np.int64)
    netidx = rng.integers(0, 4, size=n_requests)
    rt = np.asarray(rtols)[rng.integers(0, len(rtols), size=n_requests)]
    zseeds = rng.integers(0, 2**31 - 1, size=n_requests)
    return [dict(arrival=float(arrivals[i]), net=int(netidx[i]), zones=int(sizes[i]),
                 rtol=float(rt[i]), seed=int(zseeds[i])) for i in range(n_requests)]


def request_inputs(nets, req):
    """(state, rate scales or None, dt) of one request drawn by serving_requests(); nets are
    batched_networks() (0 Robertson, 1..3 the random networks of 14, 22, 48 variables)."""
    k = req["net"]
    if k == 0:
        st, sc = robertson_zones(req["zones"], seed=req["seed"])
        return st, sc, 1.0e5
    st = random_zones(nets[k], req["zones"], req["seed"], T_range=BATCHED_T_RANGE, T_dist="loguniform")
    return st, None, 1.0
