"""Kernel variants through the C ABI: explicit (e.g. logarithmic) frequency lists evaluated
with a per-term FP64 phase, and direction-dependent cubic-cell form factors."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, TINY, flatten, direction_grid
from tests.helpers import e_inf, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    rad._lib.lib()
    return rad


def test_log_spaced_frequencies_match_oracle(rad):
    w = SINGLE.scaled(n_particles=700, n_steps=3, nx_dir=4, ny_dir=8, seed=17)
    st = w.steps()
    om = np.geomspace(1e13, 2e19, 150)
    for dtype in ("f32", "f64"):
        g = rad.Grid(w.directions(), 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=om)
        g.push_steps(w.t0, w.n_steps, to_device(st, dtype))
        I = g.spectrum()
        Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), om, w.shape, w.shape_len, w.dt)
        err = e_inf(I, Iref)
        col = np.max(np.abs(I - Iref), axis=0) / np.max(Iref, axis=0)
        print(f"log-spaced omega ({dtype}): e_inf {err:.3e}, per-frequency max {col.max():.3e}")
        assert err <= TOL and col.max() <= TOL


def test_explicit_uniform_list_equals_recurrence(rad):
    """The same uniform frequencies given as a list (per-term phase) and as (omega0, domega)
    (rotation recurrence) agree to FP32 rounding."""
    w = SINGLE.scaled(n_particles=2000, n_steps=2, nx_dir=8, ny_dir=8, n_omega=256, seed=18)
    st = w.steps()
    dev = to_device(st, "f32")
    g1 = rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    g2 = rad.Grid(w.directions(), 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=w.omegas())
    g1.push_steps(w.t0, 2, dev)
    g2.push_steps(w.t0, 2, dev)
    assert e_inf(g2.spectrum(), g1.spectrum()) <= 2e-6


@pytest.mark.parametrize("shape", ["cic3d", "tsc3d", "qsc3d"])
def test_cubic_cell_shapes_match_oracle(rad, shape):
    """Wide directions (+-0.4 rad) so the per-axis factors differ from the 1-D shape."""
    w = SINGLE.scaled(n_particles=600, n_steps=3, n_omega=96, omega_max=4e18, shape=shape, seed=19)
    dirs = direction_grid(5, 6, 0.4)
    st = w.steps()
    g = rad.Grid(dirs, w.omega0, w.domega, w.n_omega, shape=shape, shape_len=w.shape_len, dt=w.dt)
    g.push_steps(w.t0, w.n_steps, to_device(st, "f32"))
    I = g.spectrum()
    Iref = oracle.spectrum(flatten(st, w.times()), dirs, w.omegas(), shape, w.shape_len, w.dt)
    I1d = oracle.spectrum(flatten(st, w.times()), dirs, w.omegas(), shape[:-2], w.shape_len, w.dt)
    err = e_inf(I, Iref)
    col = np.max(np.abs(I - Iref), axis=0) / np.max(Iref, axis=0)
    col1d = np.max(np.abs(I1d - Iref), axis=0) / np.max(Iref, axis=0)
    print(f"{shape}: e_inf {err:.3e}, per-frequency {col.max():.3e}; 1-D shape instead differs per frequency "
          f"by up to {col1d.max():.3e}")
    assert err <= TOL and col.max() <= TOL
    assert col1d.max() > 100 * TOL      # the direction dependence is visible on this grid


def test_cubic_cell_along_axis_equals_1d_shape(rad):
    w = TINY.scaled(n_particles=256, n_steps=4, shape="cic", seed=20)
    st = w.steps()
    dirs = np.array([[0.0, 0.0, 1.0]])
    dev = to_device(st, "f64")
    g3 = rad.Grid(dirs, w.omega0, w.domega, w.n_omega, shape="cic3d", shape_len=1e-7, dt=w.dt)
    g1 = rad.Grid(dirs, w.omega0, w.domega, w.n_omega, shape="cic", shape_len=1e-7, dt=w.dt)
    g3.push_steps(w.t0, w.n_steps, dev)
    g1.push_steps(w.t0, w.n_steps, dev)
    assert e_inf(g3.spectrum(), g1.spectrum()) <= 1e-6


def test_batch_of_frequency_list_grids(rad):
    om = np.geomspace(1e14, 1e19, 64)
    ws = [SINGLE.scaled(n_particles=n, n_steps=2, nx_dir=4, ny_dir=4, seed=30 + k) for k, n in enumerate((300, 1700))]
    sts = [w.steps() for w in ws]
    grids = [rad.Grid(w.directions(), 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=om)
             for w in ws]
    devs = [to_device(st, "f32") for st in sts]
    rad.Batcher().push([(g, w.t0, w.n_steps, d) for g, w, d in zip(grids, ws, devs)])
    for g, w, st in zip(grids, ws, sts):
        Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), om, w.shape, w.shape_len, w.dt)
        assert e_inf(g.spectrum(), Iref) <= TOL
    uni = SINGLE.scaled(n_particles=100, n_steps=1, nx_dir=4, ny_dir=4, seed=40)
    gu = rad.Grid(uni.directions(), uni.omega0, uni.domega, 64, shape=uni.shape, shape_len=uni.shape_len, dt=uni.dt)
    with pytest.raises(rad.RadError):
        rad.Batcher().push([(grids[0], 0.0, 1, {k: v[:300] for k, v in devs[0].items()}),
                            (gu, 0.0, 1, to_device(uni.steps(), "f32"))])


def test_variant_grids_require_16_frequencies_per_lane(rad):
    g = rad.Grid(np.array([[0.0, 0.0, 1.0]]), 0.0, 0.0, 0, shape="cic", omegas=np.geomspace(1e14, 1e18, 40))
    assert g.get_tile()["w_per_lane"] == 16
    with pytest.raises(rad.RadError):
        g.set_tile(w_per_lane=32)
