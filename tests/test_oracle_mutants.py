"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, index or
stride, a transposed operand, an off-by-one) in a private copy of the
oracle's C source, builds it, and runs the oracle pin tests against the
broken build in a child process.  At least one pin must fail for every
mutant; the unmodified source must pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "triot_oracle.c")
PINS = ["tests/test_oracle_index.py", "tests/test_oracle_ops.py",
        "tests/test_oracle_moments.py", "tests/test_oracle_adjoint.py",
        "tests/test_oracle_reductions.py"]

MUTANTS = {
    "stride": ("off += t[i] * trailing;", "off += t[i] * s[i];"),
    "carry_off_by_one": ("if (t[i] < c[i])\n            return 1;",
                         "if (t[i] <= c[i])\n            return 1;"),
    "column_major": ("for (int i = d - 1; i >= 0; --i) {\n        t[i] += 1;",
                     "for (int i = 0; i < d; ++i) {\n        t[i] += 1;"),
    "unflatten_digit": ("t[i] = f % s[i];", "t[i] = f / s[i];"),
    "base_dropped": ("uint64_t off = o->base + oracle_flat_index",
                     "uint64_t off = 0 * o->base + oracle_flat_index"),
    "window_start_ignored": ("oracle_unflatten(total ? o->base % total : 0",
                             "oracle_unflatten(0"),
    "mul_acc_sign": ("float prod = py * pz;\n            *px = *px + prod;",
                     "float prod = py * pz;\n            *px = *px - prod;"),
    "mul_acc_operand": ("float pz = *(const float *)at(&Z, t, d);",
                        "float pz = *(const float *)at(&Y, t, d);"),
    "fill_zero_missing": ("memset(at(&D, t, d), 0, (size_t)elem_bytes);", ";"),
    "moment_term_dropped": ("S[i] += (double)t[i] * w;", "S[i] += (double)t[i];"),
    "cov_index": ("((double)t[i] - E[i]) * ((double)t[j] - E[j]);",
                  "((double)t[i] - E[i]) * ((double)t[i] - E[j]);"),
    "cov_unnormalised": ("out[1 + d + p] = K[p] / M;", "out[1 + d + p] = K[p];"),
    "adj_sign": ("acc += gmom[1 + i] * ((double)t[i] - mom[1 + i]);",
                 "acc += gmom[1 + i] * ((double)t[i] + mom[1 + i]);"),
    "adj_cov_term": ("acc += gmom[1 + d + p] * (dij - mom[1 + d + p]);",
                     "acc += gmom[1 + d + p] * dij;"),
    "mul_adj_operand": ("*(float *)dst = *(const float *)at(&GO, t, d) *\n                                    *(const float *)at(&B, t, d);",
                        "*(float *)dst = *(const float *)at(&GO, t, d) *\n                                    *(const float *)at(&A, t, d);"),
    "dot_weight_dropped": ("            s += w;", "            s += 1.0;"),
    "xpyx_sign": ("float sum = vx + prod;", "float sum = vx - prod;"),
    "xpyx_operand": ("float prod = vy * vx;", "float prod = vy * vz;"),
    "xpyx_fused": ("float prod = vy * vx;\n            float sum = vx + prod;",
                   "float prod = 0.0f;\n            float sum = fmaf(vy, vx, vx);"),
    "marginal_overwrite": ("out[oracle_flat_index(kt, ks, dk)] += w;",
                           "out[oracle_flat_index(kt, ks, dk)] = w;"),
    "bbox_max": ("if (!found || v > out[2 * i + 1])", "if (!found || v < out[2 * i + 1])"),
    "bbox_sign": ("if (!(rd(at(&V[k], t, d), f64) != 0.0))", "if (!(rd(at(&V[k], t, d), f64) > 0.0))"),
    "conv_correlation": ("v[i] = t[i] + u[i];", "v[i] = t[i] > u[i] ? t[i] - u[i] : u[i] - t[i];"),
    "conv_rounding": ("double prod = a * rhs[oracle_flat_index(u, cr, d)];\n            double *o = &out[oracle_flat_index(v, co, d)];\n            *o = *o + prod;",
                   "double prod = a * rhs[oracle_flat_index(u, cr, d)];\n            double *o = &out[oracle_flat_index(v, co, d)];\n            *o = prod + (*o + 0.0) * 1.0000000000000002;"),
}


def _run_pins(lib_path):
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib_path
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


def _build(src_text, tmp_path, name):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    text = open(SRC).read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, "mutation anchor for %s must match exactly once" % name
    so = _build(text.replace(old, new), tmp_path, name)
    assert _run_pins(so) != 0, "no pin caught the %s mutant" % name


def test_unmodified_source_passes(tmp_path):
    so = _build(open(SRC).read(), tmp_path, "clean")
    assert _run_pins(so) == 0
