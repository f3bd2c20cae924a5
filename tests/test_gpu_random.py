"""Seeded random configurations (grid sizes, particle counts, shapes, frequency kinds,
launch shapes, batch tilings) through the C ABI, each against the FP64 oracle: a sweep for
tiling and indexing mistakes that fixed sizes would not reach."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, flatten, direction_grid, block_log_omegas
from tests.helpers import assert_parity, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-4
N_CASES = 48


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    rad._lib.lib()
    return rad


def random_case(k: int):
    rng = np.random.default_rng(1000 + k)
    nx, ny = int(rng.integers(1, 9)), int(rng.integers(1, 12))
    n_omega = int(rng.integers(1, 300))
    shape = str(rng.choice(["point", "cic", "tsc", "qsc", "gauss", "cic3d", "tsc3d"]))
    kind = str(rng.choice(["uniform", "uniform", "log", "blocklog"]))
    n = int(rng.integers(1, 2500))
    steps = int(rng.integers(1, 4))
    dtype = str(rng.choice(["f32", "f64"]))
    w = SINGLE.scaled(n_particles=n, n_steps=steps, nx_dir=nx, ny_dir=ny, n_omega=n_omega,
                      omega_max=float(rng.uniform(1e18, 2e19)), shape=shape, in_dtype=dtype, seed=2000 + k)
    dirs = direction_grid(nx, ny, float(rng.uniform(0.005, 0.3)))
    om = None
    if kind == "log" and n_omega > 1:
        om = np.geomspace(1e14, w.omega_max, n_omega)
    elif kind == "blocklog" and n_omega > 1:
        om = block_log_omegas(1e14, w.omega_max, n_omega)
    variant = (om is not None) or shape.endswith("3d")
    wpl = 16 if variant else int(rng.choice([16, 32]))
    tile = dict(w_per_lane=wpl, dir_per_wave=int(rng.choice([16, 32, 64])), waves=int(rng.choice([1, 2, 4, 8])),
                wg_per_cu=int(rng.integers(1, 9)))
    btile = dict(w_per_lane=16 if variant else int(rng.choice([16, 32])), dir_per_wave=int(rng.choice([16, 32, 64])),
                 waves=int(rng.choice([1, 2, 4, 8])), wg_per_cu=int(rng.integers(1, 9)))
    return w, dirs, om, tile, btile


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_configuration(rad, k):
    w, dirs, om, tile, btile = random_case(k)
    st = w.steps()
    omegas = w.omegas() if om is None else om
    Iref = oracle.spectrum(flatten(st, w.times()), dirs, omegas, w.shape, w.shape_len, w.dt)
    dev = to_device(st, w.in_dtype)

    def grid():
        if om is None:
            return rad.Grid(dirs, w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt, tile=tile)
        return rad.Grid(dirs, 0.0, 0.0, 0, shape=w.shape, shape_len=w.shape_len, dt=w.dt, omegas=om, tile=tile)

    g = grid()
    g.push_steps(w.t0, w.n_steps, dev)
    gb = grid()
    b = rad.Batcher(tile=btile)
    b.push([(gb, w.t0, w.n_steps, dev)])
    desc = (f"case {k}: {len(dirs)} dirs x {len(omegas)} omega, {w.n_particles} x {w.n_steps} {w.in_dtype}, "
            f"{w.shape}, variant {g.variant}, tile {tile}, batch {btile}")
    assert_parity(g.spectrum(), Iref, desc)
    assert_parity(gb.spectrum(), Iref, desc + " (batched)")
