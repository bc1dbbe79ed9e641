"""Named GPU-parity cases: the seeded inputs of every case that the GPU parity tests compare
with the oracle, and the oracle runs that judge them.

Both the GPU tests and tests/golden/make_ill_conditioned.py build their inputs here, so
the committed list of ill-conditioned zones (zones the integrator itself does not resolve
at the case's tolerance, found from the oracle alone) is keyed by exactly these inputs.
Nothing here touches the GPU or the HIP library.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2608_06466_amd import workloads as W

FINE = 100.0              # the oracle's reference run is at rtol / FINE, atol / FINE
FINE_MAX_STEPS = 10_000_000


class Case:
    """Inputs of one parity case and the oracle options that go with them.

    okw: extra oracle.burn keywords of the case's method (jac_policy, form, retry,
    max_steps); rkc: the case runs the RKC integrator; mask: zones of the input that the
    case covers (a retry case splits its zones by the tolerances they finish with)."""

    def __init__(self, name, net, state, dt, rtol, atol, scale=None, source=None, okw=None,
                 rkc=False, fine_rtol=None, fine_atol=None, conserving=True):
        self.name, self.net, self.state, self.dt = name, net, state, dt
        self.rtol, self.atol, self.scale, self.source = rtol, atol, scale, source
        self.okw = dict(okw or {})
        self.rkc = rkc
        self.nv = net["n_species"] + net["thermal"]
        self.fine_rtol = fine_rtol if fine_rtol is not None else rtol / FINE
        self.fine_atol = fine_atol if fine_atol is not None else atol / FINE
        # every reaction keeps the number of species (two in, two out): the species sum is
        # an invariant of the exact solution unless a source feeds the zone
        self.conserving = conserving and source is None

    def oracle(self):
        """The oracle's result at the case's tolerances."""
        if self.rkc:
            return oracle.rkc(self.net, self.state, self.dt, self.rtol, self.atol, self.scale,
                              source=self.source, **self.okw)
        return oracle.burn(self.net, self.state, self.dt, self.rtol, self.atol, self.scale,
                           source=self.source, **self.okw)

    def oracle_fine(self, factor=1.0):
        """The oracle with the same method at rtol / (FINE factor): the reference that measures
        how far the integrator itself is from the solution at the case's tolerance."""
        kw = {k: v for k, v in self.okw.items() if k not in ("retry", "max_steps")}
        rt, at = self.fine_rtol / factor, self.fine_atol / factor
        if self.rkc:
            return oracle.rkc(self.net, self.state, self.dt, rt, at, self.scale, source=self.source,
                              max_steps=FINE_MAX_STEPS)
        return oracle.burn(self.net, self.state, self.dt, rt, at, self.scale, source=self.source,
                           max_steps=FINE_MAX_STEPS, **kw)


def _rand(k):
    ns, R, seed = W.BATCHED_NETS[k]
    return W.random_network(ns, R, seed)


def _batched_zones(net, n, seed):
    return W.random_zones(net, n, seed=seed, T_range=W.BATCHED_T_RANGE, T_dist="loguniform")


def robertson(n=333, **kw):
    c = W.robertson(n)
    return Case("robertson", c["net"], c["state"], c["dt"], c["rtol"], c["atol"], scale=c["scale"], **kw)


def nv14(n=301):
    c = W.nv14(n)
    return Case(f"nv14 x{n}", c["net"], c["state"], c["dt"], c["rtol"], c["atol"])


def batched_network(k):
    """Random network k (1..3: 14, 22, 48 variables) over a wide log-uniform T range."""
    net = _rand(k - 1)
    zones = {1: 131, 2: 67, 3: 19}[k]
    st = W.random_zones(net, zones, seed=900 + k, T_range=(300.0, 6000.0), T_dist="loguniform")
    return Case(f"batched net {k}", net, st, 1.0, 1e-8, 1e-12)


def full_size_sample():
    """256 zones drawn (seed 7) from the benchmark's 2^20-zone input; idx into that input."""
    c = W.nv14()
    idx = np.sort(np.random.default_rng(7).choice(c["state"].shape[0], 256, replace=False))
    case = Case("nv14 2^20 sampled 256", c["net"], c["state"][idx], 1.0, 1e-8, 1e-12)
    return case, c, idx


TAIL = {"nv14": None, "nv14b": 0, "nv22": 1, "nv48": 2}


def tail(which):
    """Thousands of zones: the benchmark network (T ~ U(1e3, 5e3)) or a network of the batched
    workload (T log-uniform on [300, 6000] K)."""
    if which == "nv14":
        net, n, Tr, Td = W.nv14_network(), 3000, (1e3, 5e3), "uniform"
    else:
        k = TAIL[which]
        net, n, Tr, Td = _rand(k), [3000, 2000, 400][k], (300.0, 6000.0), "loguniform"
    st = W.random_zones(net, n, seed=4242, T_range=Tr, T_dist=Td)
    return Case(f"tail {which} x{n}", net, st, 1.0, 1e-8, 1e-12)


def constant_source():
    c = W.nv14(300)
    rng = np.random.default_rng(5)
    src = np.zeros_like(c["state"])
    src[:, :13] = rng.uniform(0.0, 1e-3, (300, 13))
    src[:, 13] = rng.uniform(-5.0, 5.0, 300)
    return Case("nv14 + source", c["net"], c["state"], 1.0, 1e-8, 1e-12, source=src)


def loose():
    c = W.nv14(96)
    return Case("nv14 rtol 1e-6", c["net"], c["state"], 1.0, 1e-6, 1e-10)


RETRY = (1e-6, 1e-10, 100000)


def retry_parts():
    """A 1500-step cap with the zone-by-zone retry at (1e-6, 1e-10, 100000 steps): the zones
    the oracle retries (status 6) and those its first run finishes, as two cases at the
    tolerances each part ends with.  Returns (full case, retried mask, [case, case])."""
    c = W.nv14(160)
    full = Case("retry", c["net"], c["state"], 1.0, 1e-8, 1e-12,
                okw=dict(max_steps=1500, retry=RETRY))
    ref = full.oracle()
    retried = ref[1] == 6
    parts = [Case("retry retried", c["net"], c["state"][retried], 1.0, RETRY[0], RETRY[1]),
             Case("retry first run", c["net"], c["state"][~retried], 1.0, 1e-8, 1e-12)]
    return full, ref, retried, parts


def reuse(which):
    if which == "nv14":
        net, n, st_fn = W.nv14_network(), 400, None
        st = W.random_zones(net, n, seed=777, T_range=(1e3, 5e3), T_dist="uniform")
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        net = _rand(k)
        st = _batched_zones(net, [0, 200, 96][k], 777)
    return Case(f"{which} reuse", net, st, 1.0, 1e-8, 1e-12, okw=dict(jac_policy=1))


def rkc(which):
    """Mildly stiff zones for RKC: the random networks at 100-300 K, a linear network with
    rates 1e-2..1e2."""
    if which == "linear":
        net = W.linear_network(6, 5, k_range=(1e-2, 1e2))
        st = np.zeros((128, 7))
        st[:, :6] = np.random.default_rng(3).dirichlet(np.ones(6), size=128)
        return Case("rkc linear", net, st, 10.0, 1e-6, 1e-10, rkc=True)
    k = {"nv14": 0, "nv22": 1, "nv48": 2}[which]
    net = _rand(k)
    st = W.random_zones(net, [256, 128, 48][k], seed=31, T_range=(100.0, 300.0), T_dist="loguniform")
    return Case(f"rkc {which}", net, st, 1.0, 1e-6, 1e-10, rkc=True)


FD_RETRY = (1e-8, 1e-12, 100000, "fd")


def fd_retry(which, jac_policy):
    """A 5-step cap fails nearly every zone; the retry with the finite-difference Jacobian at the
    same tolerances integrates them (the reference: a plain burn at rtol / 100)."""
    if which == "nv14":
        net = W.nv14_network()
        st = W.random_zones(net, 128, seed=779)
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        net = _rand(k)
        st = _batched_zones(net, [0, 96, 32][k], 778)
    return Case(f"{which} fd retry policy {jac_policy}", net, st, 1.0, 1e-8, 1e-12,
                okw=dict(max_steps=5, retry=FD_RETRY, jac_policy=jac_policy))


def fd_retry_robertson():
    c = W.robertson(512)
    return Case("robertson fd retry", c["net"], c["state"], c["dt"], 1e-8, 1e-12, scale=c["scale"],
                okw=dict(max_steps=20, retry=FD_RETRY))


def variable(which, jac_policy):
    if which == "nv14":
        net = W.nv14_network()
        st = W.random_zones(net, 256, seed=781, T_range=(1e3, 5e3), T_dist="uniform")
    else:
        k = {"nv22": 1, "nv48": 2}[which]
        net = _rand(k)
        st = _batched_zones(net, [0, 128, 48][k], 781)
    return Case(f"{which} variable-coefficient policy {jac_policy}", net, st, 1.0, 1e-8, 1e-12,
                okw=dict(jac_policy=jac_policy, form="variable"))


def variable_robertson():
    c = W.robertson(512)
    return Case("robertson variable-coefficient", c["net"], c["state"], c["dt"], 1e-8, 1e-12,
                scale=c["scale"], okw=dict(form="variable"))


def blocked_lu(which, integrator="bdf"):
    """Blocked matrix-core LU cases: the 48-variable network of the batched workload, networks
    of 40 and 33 variables, the 14-variable network forced onto the 48-row kernel.
    Returns (case, lanes)."""
    form = "variable" if integrator == "bdf_variable" else "fixed"
    if which == "nv48":
        net, n, lanes = _rand(2), 48, 0
    elif which == "nv40":
        net, n, lanes = W.random_network(39, 120, 612), 48, 0
    elif which == "nv33":
        net, n, lanes = W.random_network(32, 100, 613), 48, 0
    else:
        net, n, lanes = W.nv14_network(), 64, 64
    if which == "nv14_on_64_lanes":
        st = W.random_zones(net, n, seed=783, T_range=(1e3, 5e3), T_dist="uniform")
    else:
        st = _batched_zones(net, n, 783)
    return Case(f"{which} blocked MFMA LU {integrator}", net, st, 1.0, 1e-8, 1e-12,
                okw=dict(form=form)), lanes


def rate_factors(which):
    """48-row FP64 kernel: a thermal network with rate scales, without, and a network without
    temperature (constant rates)."""
    net_t = _rand(2)
    R = len(net_t["lnA"])
    rng = np.random.default_rng(615)
    st_t = _batched_zones(net_t, 32, 616)
    sc_t = np.exp(rng.normal(0.0, 0.5, (32, R)))
    if which == "scaled":
        return Case("48-row FP64 scaled", net_t, st_t, 1.0, 1e-8, 1e-12, scale=sc_t)
    if which == "unscaled":
        return Case("48-row FP64 unscaled", net_t, st_t, 1.0, 1e-8, 1e-12)
    net_c = W.random_network(48, 150, 614, thermal=False, log10A=(0.0, 4.0))
    st_c = W.random_zones(net_c, 32, seed=617)
    return Case("48-row FP64 constant-rate", net_c, st_c, 1.0, 1e-8, 1e-12)


def padded(ns, R, seed):
    net = W.random_network(ns, R, seed)
    st = _batched_zones(net, 64, seed + 1)
    return Case(f"nv{ns + 1} below the padded size", net, st, 1.0, 1e-8, 1e-12)


PADDED = [(11, 25, 615), (19, 40, 616), (36, 110, 617)]


def all_cases():
    """Every registered case (name -> Case), for the ill-conditioned-zone generator."""
    cs = [robertson(), nv14(), *[batched_network(k) for k in (1, 2, 3)], full_size_sample()[0],
          *[tail(w) for w in TAIL], constant_source(), loose(), *retry_parts()[3],
          *[reuse(w) for w in ("nv14", "nv22", "nv48")],
          *[rkc(w) for w in ("nv14", "nv22", "nv48", "linear")],
          *[fd_retry(w, p) for w, p in (("nv14", 0), ("nv22", 0), ("nv48", 0), ("nv14", 1))],
          fd_retry_robertson(),
          *[variable(w, p) for w, p in (("nv14", 0), ("nv22", 0), ("nv48", 0), ("nv14", 1),
                                         ("nv48", 1))],
          variable_robertson(),
          *[blocked_lu(w, i)[0] for w, i in (("nv48", "bdf"), ("nv48", "bdf_variable"),
                                            ("nv40", "bdf"), ("nv33", "bdf"),
                                            ("nv14_on_64_lanes", "bdf"))],
          *[rate_factors(w) for w in ("scaled", "unscaled", "constant-rate")],
          *[padded(*p) for p in PADDED]]
    out = {}
    for c in cs:
        assert c.name not in out, c.name
        out[c.name] = c
    return out
