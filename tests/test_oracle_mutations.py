"""Planted-mistake check of the oracle pins (CPU only).

Each case copies the C oracle into a temporary directory, plants one plausible mistake
(a flipped sign, a dropped power, a wrong index, a wrong shape exponent ...), rebuilds it
there and runs the physics pins against it, leaving out the comparisons with the numpy
oracle.  Every mutant must fail at least one pin.  The committed oracle is never touched.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "phase_sign_of_n_dot_r": ("(t[i] - ndotr / ORC_C)", "(t[i] + ndotr / ORC_C)"),
    "denominator_power_one": ("double D2 = D * D;", "double D2 = D;"),
    "tsc_exponent": ("if (shape == ORC_SHAPE_TSC) return s2 * s2;", "if (shape == ORC_SHAPE_TSC) return s2;"),
    "qsc_exponent": ("if (shape == ORC_SHAPE_QSC) return s2 * s2 * s2;", "if (shape == ORC_SHAPE_QSC) return s2 * s2;"),
    "gauss_width": ("return exp(-a * a);", "return exp(-0.5 * a * a);"),
    "missing_sqrt_of_form_factor": ("double F = sqrt(oracle_form_factor_sq(weight[i], g));",
                                    "double F = oracle_form_factor_sq(weight[i], g);"),
    "dropped_incoherent_term": ("return N + (N * N - N) * g;", "return (N * N) * g;"),
    "prefactor_without_dt": ("double q = ORC_QE * dt;", "double q = ORC_QE;"),
    "cross_product_index": ("out[1] = a[2] * b[0] - a[0] * b[2];", "out[1] = a[0] * b[2] - a[2] * b[0];"),
    "sinc_half_argument": ("double x = omega * len / (2.0 * ORC_C);", "double x = omega * len / ORC_C;"),
    "beta_dot_n_transposed": ("double D = 1.0 - (beta[0] * n[0] + beta[1] * n[1] + beta[2] * n[2]);",
                              "double D = 1.0 - (beta[0] * n[0] + beta[1] * n[2] + beta[2] * n[1]);"),
    "phase_cos_sin_swapped": ("double cr = cos(phase), ci = sin(phase);", "double cr = sin(phase), ci = cos(phase);"),
    "cubic_cell_drops_an_axis": ("oracle_shape_g(base, len, omega * fabs(n[1])) *", "1.0 *"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "rad_oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    for d in ("oracle", "workloads", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__", "golden"))
    (tmp_path / "oracle" / "rad_oracle.c").write_text(src.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "-k", "not numpy_oracle"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (name, r.stdout[-2000:], r.stderr[-2000:])
