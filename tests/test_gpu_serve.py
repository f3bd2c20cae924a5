"""Serving loop (continuous batching of per-step chunks from several bunches) through the
C ABI: results match direct pushes and the oracle, a tight HBM budget defers chunks but
never drops them, and every chunk's timeline is ordered."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, flatten, FIELDS
from tests.helpers import assert_close, assert_parity, in_block_sample, to_device

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
        assert_close(I, direct.spectrum(), f"served bunch n={w.n_particles} vs direct push")
        if w.n_particles <= 1200:
            Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape,
                                   w.shape_len, w.dt)
            assert_parity(I, Iref, f"served bunch n={w.n_particles} vs oracle")
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
        assert_close(g.spectrum(), r.spectrum(), "tight budget vs direct push")


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
        assert_close(g.spectrum(), direct.spectrum(), "explicit server launch shape vs direct push")


def test_continuous_batching(rad):
    """Requests that arrive while others are on the GPU are admitted and launched without
    waiting for the earlier work to drain.  A first set of large chunks (two bunches) is
    submitted; once the server reports a batch in flight, a second set from two other
    bunches arrives.  Some second-set chunk must be admitted before some first-set chunk
    has completed, some batched launch must mix bunches, and every bunch's served spectrum
    must equal the same bunch pushed alone (FP32 rounding) and the oracle (parity gate)."""
    import time
    from collections import defaultdict
    big = make_bunches([90000, 70000], steps=10, n_omega=512)
    small = [(w, w.steps()) for w in (SINGLE.scaled(n_particles=n, n_steps=10, nx_dir=4, ny_dir=8, n_omega=512,
                                                   gamma=("uniform", 20.0, 500.0), seed=350 + i)
                                      for i, n in enumerate((3000, 7000)))]
    bs = big + small
    grids = [grid_for(rad, w) for w, _ in bs]
    srv = rad.Server(hbm_budget=512 << 20, max_batch=4, max_inflight=2)
    tickets = []
    for j in range(10):
        for b in (0, 1):
            w, st = bs[b]
            tickets.append((srv.submit(grids[b], float(w.times()[j]), host_chunk(st, j)), b, 0))
    t_end = time.perf_counter() + 60
    while srv.counters()["inflight_batches"] < 1:
        assert time.perf_counter() < t_end, "no batch went in flight"
        time.sleep(1e-4)
    seen_inflight = srv.counters()
    for j in range(10):
        for b in (2, 3):
            w, st = bs[b]
            tickets.append((srv.submit(grids[b], float(w.times()[j]), host_chunk(st, j)), b, 1))
    srv.drain()
    stats = [(srv.wait(tk), b, s) for tk, b, s in tickets]
    srv.close()
    print("counters when the second set arrived:", seen_inflight)
    first = [st for st, _, s in stats if s == 0]
    second = [st for st, _, s in stats if s == 1]
    assert all(st["status"] == 0 for st, _, _ in stats)
    last_first_done = max(st["t_complete"] for st in first)
    early = [st for st in second if st["t_admit"] < last_first_done]
    print(f"second-set chunks admitted before the first set completed: {len(early)} of {len(second)}")
    assert early
    members = defaultdict(set)
    for st, b, _ in stats:
        members[st["batch_id"]].add(b)
    mixed = [k for k, v in members.items() if len(v) > 1]
    print(f"{len(members)} batched launches, {len(mixed)} of them mix bunches")
    assert mixed
    ds = np.arange(0, 32, 4)
    ks = in_block_sample(512, 32)
    for g, (w, st) in zip(grids, bs):
        I = g.spectrum()
        alone = grid_for(rad, w)
        alone.push_steps(w.t0, w.n_steps, to_device(st, "f32"))
        assert_close(I, alone.spectrum(), f"bunch n={w.n_particles}: served in the mix vs alone")
        Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape,
                               w.shape_len, w.dt)
        assert_parity(I[np.ix_(ds, ks)], Iref, f"served bunch n={w.n_particles} vs oracle", ks=ks)


def test_serving_workload_poisson_trace(rad):
    """The serving workload's own bunches and 128 x 512 grids, chunks arriving as its
    Poisson process at the stated 2000 chunks/s (the first 400 arrivals; each bunch's chunks
    are its successive time steps).  Every served spectrum equals the same chunks pushed
    directly (FP32 rounding) and, on a direction x frequency sample, the oracle."""
    import time
    from workloads import serving_bunches, poisson_trace
    ws = serving_bunches().bunches()
    arrivals, which = poisson_trace(2000.0, 400, len(ws), seed=0)
    n_per = [int(np.sum(which == b)) for b in range(len(ws))]
    sts = [w.steps(0, max(1, n), workers=16) for w, n in zip(ws, n_per)]
    grids = [grid_for(rad, w) for w in ws]
    srv = rad.Server(hbm_budget=2 << 30, max_batch=64)
    step_of = [0] * len(ws)
    tickets = []
    t0 = time.perf_counter()
    for i in range(len(arrivals)):
        while time.perf_counter() - t0 < arrivals[i]:
            time.sleep(1e-4)
        b = int(which[i])
        j = step_of[b]
        step_of[b] += 1
        tickets.append(srv.submit(grids[b], float(ws[b].times(j, j + 1)[0]), host_chunk(sts[b], j)))
    srv.drain()
    stats = [srv.wait(t) for t in tickets]
    srv.close()
    assert all(s["status"] == 0 for s in stats)
    sizes = [s["batch_size"] for s in stats]
    print(f"{len(stats)} chunks in {len(set(s['batch_id'] for s in stats))} batches, largest {max(sizes)}")
    ds = np.arange(0, 128, 32)
    ks = in_block_sample(512, 64)
    for b, (w, g, st, n) in enumerate(zip(ws, grids, sts, n_per)):
        if n == 0:
            continue
        part = {k: v[:n] for k, v in st.items()}
        direct = grid_for(rad, w)
        direct.push_steps(w.t0, n, to_device(part, "f32"))
        I = g.spectrum()
        # Both sides sum the same FP32 terms, grouped differently: one direct launch puts up to
        # 32768 particles of many steps into each FP32 partial, the served batches fewer.  A
        # recursive FP32 sum of n terms of random phase carries a rounding error of about
        # 2^-24 sqrt(n / 2) of its magnitude (7.6e-6 at n = 32768), so 1e-5 rather than the
        # 1e-6 of the few-chunk tests.
        assert_close(I, direct.spectrum(), f"served bunch {b} (n={w.n_particles}, {n} chunks) vs direct pushes",
                     tol_inf=1e-5, tol_freq=1e-5)
        if w.n_particles <= 40000:
            Iref = oracle.spectrum(flatten(part, w.times(0, n)), w.directions()[ds], w.omegas()[ks], w.shape,
                                   w.shape_len, w.dt)
            assert_parity(I[np.ix_(ds, ks)], Iref, f"served bunch {b} vs oracle", ks=ks)
