"""Full-size parity on sampled outputs: the workloads' real particle counts, step counts and
grids, launched as the bench launches them, checked against the oracle on a deterministic
subset of (direction, frequency) points that the oracle evaluates one by one."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, PRECISION, serving_bunches, flatten
from tests.helpers import error_report, to_device, step_slice

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    rad._lib.lib()
    oracle.set_threads(16)
    return rad


def check(I, Iref, what):
    rep = error_report(I, Iref)
    print(f"{what}: e_inf {rep['e_inf']:.3e}, per-frequency {rep['per_frequency_max']:.3e}", flush=True)
    assert rep["e_inf"] <= TOL and rep["per_frequency_max"] <= TOL


def test_single_bunch_all_100_steps(rad):
    """65536 particles x 100 per-step pushes on 128 x 256 with the tuned launch shape;
    oracle on every 8th direction x every 16th frequency (plus the last)."""
    w = SINGLE
    st = w.steps()
    dev = to_device(st, "f32")
    g = rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    for j, t in enumerate(w.times()):
        g.push_step(float(t), step_slice(dev, j, w.n_particles))
    I = g.spectrum()
    ds = np.arange(0, w.n_dir, 8)
    ks = np.r_[np.arange(0, w.n_omega, 16), w.n_omega - 1]
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    check(I[np.ix_(ds, ks)], Iref, f"single bunch, 100 steps, tile {g.get_tile()}")


def test_precision_grid_full_particles_from_one_picosecond(rad):
    """16384 particles on the 64 x 1024 grid to 1e20 rad/s from t = 1 ps (500 of the 10000
    steps); oracle on 4 directions x 9 frequencies including the highest."""
    w = PRECISION.scaled(n_steps=500)
    st = w.steps()
    g = rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    g.push_steps(w.t0, w.n_steps, to_device(st, "f64"))
    I = g.spectrum()
    ds = np.array([0, 9, 36, 63])
    ks = np.r_[np.arange(0, w.n_omega, 128), w.n_omega - 1]
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    check(I[np.ix_(ds, ks)], Iref, "precision grid, 16384 x 500 steps from 1 ps")


def test_serving_grid_largest_chunk(rad):
    """The largest serving bunch's one-step chunk on its 128 x 512 grid."""
    mb = serving_bunches()
    ws = mb.bunches()
    w = max(ws, key=lambda x: x.n_particles).scaled(n_steps=1)
    st = w.steps()
    g = rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    g.push_step(float(w.times()[0]), to_device(st, "f32"))
    I = g.spectrum()
    ds = np.arange(0, w.n_dir, 16)
    ks = np.r_[np.arange(0, w.n_omega, 32), w.n_omega - 1]
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    check(I[np.ix_(ds, ks)], Iref, f"serving chunk of {w.n_particles} particles on 128 x 512")
