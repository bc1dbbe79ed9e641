"""The pins catch plausible mistakes in the oracle: each case below plants one mistake (a
dropped term, a wrong sign, a wrong index, a transposed operand, a wrong constant) in a copy
of the oracle's C sources, builds it, and runs the pins that should notice; every one of
them must make those pins fail.  CPU only; the copies live in a temporary directory."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
SOURCES = ["net.c", "lu.c", "bdf.c", "radau.c", "rkc.c"]

# (id, file, exact text, mutated text, pins (-k expression) that must fail)
MUTATIONS = [
    ("rhs-sign", "net.c",
     "        if (b >= 0) w *= (y[a] < 0.0 && y[b] < 0.0) ? -y[b] : y[b];\n        f[a] -= w;",
     "        if (b >= 0) w *= (y[a] < 0.0 && y[b] < 0.0) ? -y[b] : y[b];\n        f[a] += w;",
     "two_body_closed_forms or species_sum_invariant"),
    ("jac-index", "net.c", "dwb = sg * k[r] * y[a];", "dwb = sg * k[r] * y[b];",
     "jacobian_equals_complex_step"),
    ("dkdT-dropped-term", "net.c", "k[r] * (net->n_exp[r] + net->E[r] / T) / T",
     "k[r] * (net->n_exp[r] + net->E[r] / T)", "jacobian_equals_complex_step"),
    ("arrhenius-sign", "net.c", "net->n_exp[r] * log(T) - net->E[r] / T;",
     "net->n_exp[r] * log(T) + net->E[r] / T;", "arrhenius_rate_first_order_decay"),
    ("pivot-tie", "lu.c", "if (v > best)", "if (v >= best)", "lu_ties_choose_lowest_row"),
    ("solve-division", "lu.c", "b[i] = s / LU[i * n + i];", "b[i] = s * LU[i * n + i];",
     "linear_network_matches_matrix_exponential"),
    ("lcoef", "bdf.c", "for (int j = i; j >= 1; j--) p[j] += p[j - 1] / i;",
     "for (int j = i; j >= 1; j--) p[j] += p[j - 1] * i;", "lcoef_exact_rationals"),
    ("stirling", "bdf.c", "p[j] = p[j - 1] + m * p[j];", "p[j] = p[j - 1] + (m + 1) * p[j];",
     "stirling_numbers"),
    ("pascal-sign", "bdf.c",
     "Z[(size_t)(j - 1) * nv + i] += Z[(size_t)j * nv + i];",
     "Z[(size_t)(j - 1) * nv + i] -= Z[(size_t)j * nv + i];", "nordsieck_step_equals_classic_bdf"),
    ("raise-factorial", "bdf.c", "Zn[i] = dy[i] / fact;", "Zn[i] = dy[i] / (2.0 * fact);",
     "order_raise_is_exact"),
    ("lower-sign", "bdf.c", "Z[(size_t)j * nv + i] -= c[j] * Zq[i];",
     "Z[(size_t)j * nv + i] += c[j] * Zq[i];", "order_lower_is_exact"),
    ("error-divisor", "bdf.c", "C->ediv = q + 1;", "C->ediv = q;",
     "error_estimate_against_true_local_error"),
    ("correction-scale", "bdf.c", "double e = dy[i] / l[0];", "double e = dy[i] * l[0];",
     "nordsieck_step_equals_classic_bdf"),
    ("residual-sign", "bdf.c", "b[i] = -(dy[i] - l[0] * (h * f[i] - Z[nv + i]));",
     "b[i] = -(dy[i] - l[0] * (h * f[i] + Z[nv + i]));",
     "linear_network_matches_matrix_exponential"),
    ("iteration-matrix-transposed", "bdf.c",
     "J->LU[i * nv + j] = (i == j ? 1.0 : 0.0) - gamma * J->J[i * nv + j];",
     "J->LU[i * nv + j] = (i == j ? 1.0 : 0.0) - gamma * J->J[j * nv + i];",
     "nordsieck_step_equals_classic_bdf or counter_consistency or step_counts_comparable"),
    ("radau-tableau", "radau.c", "a21 = 3.0 / 4.0", "a21 = 3.0 / 5.0",
     "radau_is_third_order or radau_matches_matrix_exponential"),
    ("rkc-damping", "rkc.c", "const double eps = 2.0 / 13.0;", "const double eps = 2.0 / 11.0;",
     "rkc_step_is_the_damped_chebyshev_polynomial"),
]


def _build(tmp, mutation):
    _, fname, old, new, _ = mutation
    src = os.path.join(tmp, "src")
    os.makedirs(src, exist_ok=True)
    for f in SOURCES + ["oracle.h"]:
        shutil.copy(os.path.join(ORACLE, f), src)
    p = os.path.join(src, fname)
    text = open(p).read()
    assert text.count(old) == 1, (fname, old)
    open(p, "w").write(text.replace(old, new))
    lib = os.path.join(tmp, "liboracle_mut.so")
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-w", "-o", lib] + [os.path.join(src, s) for s in SOURCES]
                   + ["-lm"], check=True)
    return lib


def _pins(lib, kexpr):
    env = dict(os.environ, ZB_ORACLE_LIB=lib or "")
    if not lib:
        env.pop("ZB_ORACLE_LIB")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", kexpr],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.mark.slow
def test_unmutated_oracle_passes_the_selected_pins():
    kexpr = " or ".join(f"({m[4]})" for m in MUTATIONS)
    rc, out = _pins(None, kexpr)
    assert rc == 0, out


@pytest.mark.slow
@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_the_mutation(mutation, tmp_path):
    lib = _build(str(tmp_path), mutation)
    rc, out = _pins(lib, mutation[4])
    assert rc == 1, f"mutation {mutation[0]} survived its pins ({mutation[4]}):\n{out}"
