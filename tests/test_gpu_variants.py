"""Kernel variants through the C ABI: explicit (e.g. logarithmic) frequency lists evaluated
with a per-term FP64 phase, and direction-dependent cubic-cell form factors."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, TINY, flatten, direction_grid, block_log_omegas
from tests.helpers import assert_close, assert_complex_parity, assert_parity, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
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
        assert_parity(I, Iref, f"log-spaced omega ({dtype})")


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
    assert_close(g2.spectrum(), g1.spectrum(), "uniform list (per-term phase) vs recurrence", tol_inf=2e-6,
                 tol_freq=TOL)


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
    assert_parity(I, Iref, shape)
    col1d = np.max(np.abs(I1d - Iref), axis=0) / np.max(Iref, axis=0)
    print(f"{shape}: the 1-D shape instead differs per frequency by up to {col1d.max():.3e}")
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
    assert_close(g3.spectrum(), g1.spectrum(), "cubic cell along the axis vs 1-D shape")


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
        assert_parity(g.spectrum(), Iref, "batch of log-list grids")
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


def test_frequency_lists_are_classified(rad):
    """Uniform list -> the uniform path (0); aligned piecewise-uniform -> per-block step (4);
    anything else -> per-term phase (1); with a cubic-cell shape bit 2 is added."""
    d = np.array([[0.0, 0.0, 1.0]])
    w = SINGLE
    assert rad.Grid(d, 0.0, 0.0, 0, shape="cic", omegas=w.omegas()).variant == 0
    assert rad.Grid(d, w.omega0, w.domega, w.n_omega, shape="cic").variant == 0
    assert rad.Grid(d, 0.0, 0.0, 0, shape="cic", omegas=block_log_omegas(1e14, 1e19, 100)).variant == 4
    assert rad.Grid(d, 0.0, 0.0, 0, shape="cic3d", omegas=block_log_omegas(1e14, 1e19, 100)).variant == 6
    assert rad.Grid(d, 0.0, 0.0, 0, shape="cic", omegas=np.geomspace(1e14, 1e19, 100)).variant == 1
    shifted = block_log_omegas(1e14, 1e19, 64)
    shifted[5] *= 1.0 + 1e-9                     # one entry off its block's progression
    assert rad.Grid(d, 0.0, 0.0, 0, shape="cic", omegas=shifted).variant == 1


@pytest.mark.parametrize("shape,n_omega,dtype", [("cic", 150, "f32"), ("gauss", 64, "f64"), ("tsc3d", 96, "f32")])
def test_piecewise_uniform_list_matches_oracle(rad, shape, n_omega, dtype):
    """Block-stepped recurrence on a log-like list (uniform inside each block of 16, ragged
    last block for 150) against the oracle on the listed frequencies."""
    w = SINGLE.scaled(n_particles=800, n_steps=3, nx_dir=4, ny_dir=8, shape=shape, seed=21)
    st = w.steps()
    om = block_log_omegas(1e13, 2e19, n_omega)
    dirs = direction_grid(4, 8, 0.3) if shape.endswith("3d") else w.directions()
    g = rad.Grid(dirs, 0.0, 0.0, 0, shape=shape, shape_len=w.shape_len, dt=w.dt, omegas=om)
    assert g.variant & 4
    g.push_steps(w.t0, w.n_steps, to_device(st, dtype))
    I = g.spectrum()
    Iref = oracle.spectrum(flatten(st, w.times()), dirs, om, shape, w.shape_len, w.dt)
    assert_parity(I, Iref, f"block-stepped list ({shape}, {n_omega}, {dtype})", ks=np.arange(n_omega))


def test_piecewise_uniform_list_batched(rad):
    om = block_log_omegas(1e14, 1e19, 80)
    ws = [SINGLE.scaled(n_particles=n, n_steps=2, nx_dir=4, ny_dir=4, seed=50 + k) for k, n in enumerate((500, 2300))]
    sts = [w.steps() for w in ws]
    grids = [rad.Grid(w.directions(), 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=om)
             for w in ws]
    devs = [to_device(st, "f32") for st in sts]
    rad.Batcher().push([(g, w.t0, w.n_steps, d) for g, w, d in zip(grids, ws, devs)])
    # the same batch replayed from a captured graph is bitwise equal, replay after replay
    ref = [g.get_state() for g in grids]
    gb = rad.Batcher(graph=True)
    for _ in range(3):
        for g in grids:
            g.reset()
        gb.push([(g, w.t0, w.n_steps, d) for g, w, d in zip(grids, ws, devs)])
        assert all(np.array_equal(g.get_state(), r) for g, r in zip(grids, ref))
    assert gb.graph_stats()["launches"] >= 2
    for g, w, st, d in zip(grids, ws, sts, devs):
        Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), om, w.shape, w.shape_len, w.dt)
        assert_parity(g.spectrum(), Iref, "batched block-stepped list")
        single = rad.Grid(w.directions(), 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=om)
        single.push_steps(w.t0, w.n_steps, d)
        assert_close(g.spectrum(), single.spectrum(), "batched vs single (block-stepped list)")


def test_complex_spectrum_of_variant_grid(rad):
    """Cartesian complex S (e1 S1 + e2 S2) of a log-list, cubic-cell grid over wide
    directions against the oracle's complex sum, component by component."""
    w = SINGLE.scaled(n_particles=400, n_steps=2, n_omega=48, shape="tsc3d", seed=23)
    st = w.steps()
    dirs = direction_grid(3, 4, 0.35)
    om = np.geomspace(1e14, 6e18, 48)
    g = rad.Grid(dirs, 0.0, 0.0, 0, shape="tsc3d", shape_len=w.shape_len, dt=w.dt, omegas=om)
    assert g.variant == 3
    g.push_steps(w.t0, w.n_steps, to_device(st, "f64"))
    S = g.spectrum_complex()
    Sref = oracle.spectrum_complex(flatten(st, w.times()), dirs, om, "tsc3d", w.shape_len)
    assert_complex_parity(S, Sref, "complex spectrum (variant 3)")
