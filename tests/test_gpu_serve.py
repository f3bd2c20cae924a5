"""Serving loop (continuous batching of per-step chunks from several bunches) through the
C ABI: results match direct pushes and the oracle, a tight HBM budget defers chunks but
never drops them, and every chunk's timeline is ordered."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, flatten, FIELDS
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


def make_bunches(counts, steps, n_omega=128):
    out = []
    for i, n in enumerate(counts):
        w = SINGLE.scaled(n_particles=int(n), n_steps=steps, nx_dir=4, ny_dir=8, n_omega=n_omega,
                          gamma=("uniform", 20.0, 500.0), seed=300 + i)
        out.append((w, w.steps()))
    return out


def grid_for(rad, w):
    return rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                    shape_len=w.shape_len, dt=w.dt)


def host_chunk(st, j):
    return {k: np.ascontiguousarray(st[k][j], dtype=np.float32) for k in FIELDS}


def run_server(rad, bs, grids, **cfg):
    srv = rad.Server(**cfg)
    rng = np.random.default_rng(0)
    order = [(b, j) for b, (w, _) in enumerate(bs) for j in range(w.n_steps)]
    rng.shuffle(order)
    tickets = []
    for b, j in order:
        w, st = bs[b]
        tickets.append(srv.submit(grids[b], float(w.times()[j]), host_chunk(st, j)))
    srv.drain()
    stats = [srv.wait(t) for t in tickets]
    cnt = srv.counters()
    srv.close()
    return stats, cnt


def test_server_matches_direct_pushes_and_oracle(rad):
    bs = make_bunches([300, 2500, 90, 1200], steps=3)
    grids = [grid_for(rad, w) for w, _ in bs]
    stats, cnt = run_server(rad, bs, grids, hbm_budget=64 << 20, max_batch=8)
    assert cnt["completed"] == cnt["submitted"] == sum(w.n_steps for w, _ in bs)
    for g, (w, st) in zip(grids, bs):
        I = g.spectrum()
        direct = grid_for(rad, w)
        direct.push_steps(w.t0, w.n_steps, to_device(st, "f32"))
        assert e_inf(I, direct.spectrum()) <= 1e-6
        if w.n_particles <= 1200:
            Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape,
                                   w.shape_len, w.dt)
            err = e_inf(I, Iref)
            print(f"served bunch n={w.n_particles}: e_inf vs oracle {err:.3e}")
            assert err <= TOL
    for s in stats:
        assert s["status"] == 0
        assert s["t_submit"] <= s["t_admit"] <= s["t_launch"] <= s["t_complete"]
        assert 1 <= s["batch_size"] <= 8


def test_tight_budget_defers_but_never_drops(rad):
    bs = make_bunches([20000, 15000, 18000], steps=4)
    grids = [grid_for(rad, w) for w, _ in bs]
    biggest = 10 * ((20000 * 4 + 255) // 256 * 256)
    stats, cnt = run_server(rad, bs, grids, hbm_budget=max(1 << 20, biggest + 4096), max_batch=4)
    assert cnt["completed"] == cnt["submitted"] == 12
    assert max(s["batch_size"] for s in stats) == 1      # only one chunk fits at a time
    ref = [grid_for(rad, w) for w, _ in bs]
    for g, r, (w, st) in zip(grids, ref, bs):
        r.push_steps(w.t0, w.n_steps, to_device(st, "f32"))
        assert e_inf(g.spectrum(), r.spectrum()) <= 1e-6


def test_oversized_chunk_rejected(rad):
    (w, st), = make_bunches([40000], steps=1)
    g = grid_for(rad, w)
    srv = rad.Server(hbm_budget=1 << 20)
    with pytest.raises(rad.RadError) as ei:
        srv.submit(g, 0.0, host_chunk(st, 0))
    assert ei.value.code == rad.RAD_ERR_INVALID_ARG
    srv.close()


def test_server_launch_shape(rad):
    """An explicit launch shape for the served batches: reported back, same results."""
    bs = make_bunches([900, 2100], steps=2)
    grids = [grid_for(rad, w) for w, _ in bs]
    tile = {"w_per_lane": 16, "dir_per_wave": 16, "waves": 2, "wg_per_cu": 3}
    srv = rad.Server(hbm_budget=64 << 20, max_batch=8, tile=tile)
    assert srv.get_tile() == tile
    with pytest.raises(rad.RadError):
        srv.set_tile(w_per_lane=24, dir_per_wave=16, waves=2, wg_per_cu=1)
    tickets = [srv.submit(g, float(w.times()[j]), host_chunk(st, j))
               for g, (w, st) in zip(grids, bs) for j in range(w.n_steps)]
    srv.drain()
    for tk in tickets:
        assert srv.wait(tk)["status"] == 0
    srv.close()
    for g, (w, st) in zip(grids, bs):
        direct = grid_for(rad, w)
        direct.push_steps(w.t0, w.n_steps, to_device(st, "f32"))
        assert e_inf(g.spectrum(), direct.spectrum()) <= 1e-6
