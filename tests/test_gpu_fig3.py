"""Synthetic analogue of the paper's Fig. 3 on the device: one macro-particle with the
coherent (N^2), incoherent (N) and form-factor (Eq. 12) weightings, and the coherent ->
incoherent transition frequency against its closed form."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fig3_analogue_scalings_and_transition():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "fig3_analogue"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    dev = out["max_rel_dev"]
    print(dev, out["transition_omega"])
    assert dev["coherent_vs_N2"] <= 1e-4
    assert dev["incoherent_vs_N"] <= 1e-4
    assert dev["form_factor_vs_Eq12"] <= 1e-4
    assert out["transition_omega"]["rel_diff"] <= 0.01
