"""The C ABI used from plain C (tests/c_abi/rad_c_demo.c: HIP runtime + librad.so, no
Python or torch in the process) against the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from workloads import TINY, FIELDS, flatten
from tests.helpers import assert_parity

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "tests", "c_abi", "rad_c_demo")


@pytest.mark.parametrize("shape,shape_id", [("gauss", 4), ("cic", 1)])
def test_c_program_matches_oracle(tmp_path, shape, shape_id):
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # library and harness as built; built first only if absent
    w = TINY.scaled(n_particles=300, n_steps=5, shape=shape, seed=61)
    st = w.steps()
    dirs = w.directions()
    blob = np.concatenate([np.ascontiguousarray(st[k], np.float64).reshape(-1) for k in FIELDS]
                          + [dirs.reshape(-1)])
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    blob.tofile(inp)
    args = [DEMO, str(inp), str(out), str(w.n_particles), str(w.n_steps), str(w.n_dir), str(w.n_omega),
            repr(w.omega0), repr(w.domega), repr(w.dt), str(shape_id), repr(w.shape_len)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    I = np.fromfile(out, np.float64).reshape(w.n_dir, w.n_omega)
    times = w.t0 + np.arange(w.n_steps) * w.dt
    Iref = oracle.spectrum(flatten(st, times), dirs, w.omegas(), shape, w.shape_len, w.dt)
    assert_parity(I, Iref, f"C program ({shape})")


def test_c_program_reports_errors(tmp_path):
    """A bad argument reaches rad_last_error() and a non-zero exit status."""
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()
    w = TINY.scaled(n_particles=8, n_steps=1, seed=62)
    st = w.steps()
    blob = np.concatenate([np.ascontiguousarray(st[k], np.float64).reshape(-1) for k in FIELDS]
                          + [w.directions().reshape(-1)])
    inp = tmp_path / "in.bin"
    blob.tofile(inp)
    args = [DEMO, str(inp), str(tmp_path / "out.bin"), "8", "1", str(w.n_dir), str(w.n_omega),
            repr(w.omega0), repr(w.domega), repr(w.dt), "99", "1e-7"]      # unknown shape
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 1 and "unknown shape" in r.stderr
