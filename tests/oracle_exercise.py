"""A spread of small oracle calls covering every entry point of the oracle library: whole
burns in every form and policy (retry, source, rate factors, failures, non-finite input),
RKC, Radau, the network functions, the LU and the Nordsieck helpers.  Run in-process with
the ordinary oracle build and, under AddressSanitizer and UndefinedBehaviorSanitizer, in a
child process with a sanitizer build (`python oracle_exercise.py out.npz`); the two result
sets must be identical."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2608_06466_amd import workloads as W  # noqa: E402


def run():
    out = {}
    rob = W.robertson_network()
    ys, rsc = W.robertson_zones(6)
    net14 = W.random_network(13, 30, seed=201)
    z14 = W.random_zones(net14, 6, seed=7)
    net8 = W.random_network(7, 12, seed=11)
    z8 = W.random_zones(net8, 5, seed=3)
    z8[4, -1] = np.nan                              # a non-finite zone
    rng = np.random.default_rng(5)
    sc8 = rng.uniform(0.5, 2.0, (5, len(net8["lnA"])))
    src8 = np.zeros_like(z8)
    src8[:, 0] = 1e-3

    def put(name, res):
        for i, a in enumerate(res if isinstance(res, tuple) else (res,)):
            out[f"{name}/{i}"] = np.asarray(a)

    put("rob", oracle.burn(rob, ys, 1e5, 1e-8, 1e-12, scale=rsc, nthreads=2))
    put("rob_var_reuse", oracle.burn(rob, ys, 1e5, 1e-8, 1e-12, scale=rsc, jac_policy=1,
                                     form="variable", nthreads=2))
    put("nv14", oracle.burn(net14, z14, 1.0, 1e-8, 1e-12, nthreads=2))
    put("nv14_reuse", oracle.burn(net14, z14, 1.0, 1e-8, 1e-12, jac_policy=1, nthreads=2))
    put("nv14_fail_retry", oracle.burn(net14, z14, 1.0, 1e-8, 1e-12, max_steps=20,
                                       retry=(1e-6, 1e-10, 100000, "fd"), nthreads=2))
    put("nv8_scale_src", oracle.burn(net8, z8, 1.0, 1e-6, 1e-12, scale=sc8, source=src8,
                                     nthreads=2))
    put("nv8_retry", oracle.burn(net8, z8, 1.0, 1e-8, 1e-12, max_steps=5,
                                 retry=(1e-6, 1e-10, 100000), nthreads=2))
    lin = W.linear_network(4, seed=2, k_range=(1e-2, 1e2))
    zl = np.zeros((3, 5))
    zl[:, :4] = 0.25
    zl[:, 4] = 1e3
    put("rkc", oracle.rkc(lin, zl, 1.0, 1e-6, 1e-12, nthreads=2))
    put("rkc_fixed", oracle.rkc_fixed(lin, zl[0, :4], 1e-3, 10, 5))
    put("radau", oracle.radau(rob, ys[0], 1e2, 200, scale=rsc[0]))
    y = z14[0]
    put("rhs", oracle.rhs(net14, y))
    put("rhs_c", oracle.rhs_complex(net14, y.astype(np.complex128) + 1e-20j))
    put("jac", oracle.jac(net14, y))
    put("fd_jac", oracle.fd_jac(net14, y, 1e-8, 1e-12))
    A = rng.standard_normal((9, 9))
    lu, piv, info = oracle.lu(A)
    put("lu", (lu, piv, info, oracle.lu_solve(lu, piv, rng.standard_normal(9))))
    S = np.zeros((4, 4))
    S[:, 0] = 1.0                                   # singular: a zero pivot
    put("lu_singular", oracle.lu(S))
    put("coef", (oracle.lcoef(5), oracle.stirling(5)))
    Z = rng.standard_normal((6, 3))
    put("raise", oracle.order_raise(Z, 3, rng.standard_normal(3)))
    put("lower", oracle.order_lower(Z, 4))
    y4 = np.array([0.4, 0.3, 0.2, 0.1])
    Z0 = np.zeros((3, 4))
    Z0[0] = y4
    Z0[1] = 0.05 * oracle.rhs(lin, np.append(y4, 1e3))[:4]
    put("fixed_steps", oracle.fixed_steps(lin, Z0[:2], 1, 0.05, 3, with_errors=True))
    put("vc_steps", oracle.vc_steps(lin, Z0, 2, [0.05, 0.06, 0.04], [0.05, 0.05]))
    put("vc_coef", oracle.vc_lcoef(3, oracle.vc_xi(3, 1e-9, np.array([1e-9, 2e-9, 0.5e-9]))))
    return out


if __name__ == "__main__":
    np.savez(sys.argv[1], **run())
