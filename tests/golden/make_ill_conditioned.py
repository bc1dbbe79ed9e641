"""Write tests/golden/ill_conditioned_zones.json: the zones of the GPU parity cases that the
integrator itself does not resolve at the case's tolerance, with the evidence for each.

Calls only the oracle (and scipy's Radau, a library integrator, as an outside reference on
the listed zones); never the GPU.  A zone is listed when the oracle at the case's
tolerance and the oracle at rtol/100 disagree by more than CAP/WIDEN in the gated metric
(tests/parity.py; scaled by rtol/1e-8 for a case at a looser rtol), or when the oracle's rtol/100 run fails where the run at the case's
tolerance succeeds.  Evidence per zone:

  e_rtol_vs_fine        gated |oracle(rtol) - oracle(rtol/100)|
  e_fine_vs_finer       gated |oracle(rtol/100) - oracle(rtol/1000)|
  e_radau11_vs_radau12  gated |Radau(rtol 1e-11) - Radau(rtol 1e-12)|: whether an outside
                        implicit Runge-Kutta integrator settles on the zone at all
  e_finer_vs_radau12    gated |oracle(rtol/1000) - Radau(rtol 1e-12)|
  e_rtol_vs_radau12     gated |oracle(rtol) - Radau(rtol 1e-12)|

Run:  python tests/golden/make_ill_conditioned.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import parity  # noqa: E402
import parity_cases  # noqa: E402


def radau(case, z, rtol):
    from scipy.integrate import solve_ivp
    y0 = case.state[z, :case.nv].astype(np.float64)
    sc = None if case.scale is None else case.scale[z]
    src = None if case.source is None else case.source[z, :case.nv]

    def f(t, y):
        v = oracle.rhs(case.net, y, sc)
        return v if src is None else v + src

    def jac(t, y):
        return oracle.jac(case.net, y, sc)

    r = solve_ivp(f, (0.0, case.dt), y0, method="Radau", rtol=rtol, atol=rtol * 1e-7, jac=jac)
    return r.y[:, -1] if r.success else None


def main():
    out = {"criterion": f"oracle(rtol) vs oracle(rtol/100) gated error > CAP/WIDEN = "
                        f"{parity.CAP / parity.WIDEN:.3g} x max(1, rtol/1e-8), or the rtol/100 "
                        "run fails",
           "cases": {}}
    for name, case in parity_cases.all_cases().items():
        ref = case.oracle()
        fine = case.oracle_fine()
        ill = np.nonzero(parity.ill_conditioned(ref, fine, case.nv, case.rtol, case.atol))[0]
        print(f"{name}: {len(ill)} ill-conditioned of {len(ref[1])}", flush=True)
        if ill.size == 0:
            continue
        e = parity.oracle_error(ref, fine, case.nv, case.rtol, case.atol)
        sub = parity_cases.Case(name, case.net, case.state[ill], case.dt, case.rtol, case.atol,
                                None if case.scale is None else case.scale[ill],
                                None if case.source is None else case.source[ill], case.okw,
                                case.rkc, case.fine_rtol, case.fine_atol)
        finer = sub.oracle_fine(factor=10.0)
        ev = []
        for j, z in enumerate(ill):
            g = lambda a, b: float(parity.gated_rows(a[None, :], b[None, :], case.nv, case.rtol,
                                                     case.atol)[0])
            rec = {"zone": int(z), "e_rtol_vs_fine": float(e[z]),
                   "fine_status": int(fine[1][z]), "finer_status": int(finer[1][j])}
            if fine[1][z] == 0 and finer[1][j] == 0:
                rec["e_fine_vs_finer"] = g(fine[0][z], finer[0][j])
            y11, y12 = radau(case, z, 1e-11), radau(case, z, 1e-12)
            if y11 is not None and y12 is not None:
                rec["e_radau11_vs_radau12"] = g(y11, y12)
                rec["e_rtol_vs_radau12"] = g(ref[0][z][:case.nv], y12)
                if finer[1][j] == 0:
                    rec["e_finer_vs_radau12"] = g(finer[0][j][:case.nv], y12)
            ev.append(rec)
            print("   ", rec, flush=True)
        out["cases"][name] = {"zones": [int(z) for z in ill], "evidence": ev}
    with open(os.path.join(HERE, "ill_conditioned_zones.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
