"""rad_push_step_noalloc -- the push for callers that cannot allocate device memory --
through the C ABI, against the allocating rad_push_step: two calls in a row on different
grids, the second with a smaller input, each equal to rad_push_step's result (bitwise where
both entry points use the same particle splits, FP32 rounding of the partial sums where the
fixed scratch holds fewer splits) and to the oracle (parity gate).  A grid larger than the
scratch is rejected with a clear error."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, flatten
from tests.helpers import assert_close, assert_parity, in_block_sample, to_device, step_slice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    rad._lib.lib()
    return rad


def grid_for(rad, w):
    return rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)


def pushed(rad, w, st, noalloc):
    g = grid_for(rad, w)
    dev = to_device(st, w.in_dtype)
    for j, t in enumerate(w.times()):
        part = step_slice(dev, j, w.n_particles)
        if noalloc:
            g.push_step_noalloc(float(t), part)
        else:
            g.push_step(float(t), part)
    return g


def test_noalloc_push_equals_push_step_twice(rad):
    import paper_1802_03972_amd._lib as L
    # first call: 64 x 256 grid whose tuned launch wants more particle splits than the
    # 64 MiB scratch holds (256 KiB per split), so the scratch path cuts fewer, longer splits
    big = SINGLE.scaled(n_particles=20000, n_steps=3, nx_dir=8, ny_dir=8, n_omega=256, seed=71)
    # second call, smaller input: 15 x 40 grid; both entry points use the same splits
    small = SINGLE.scaled(n_particles=700, n_steps=2, nx_dir=3, ny_dir=5, n_omega=40, seed=72)
    for w, same_splits in ((big, False), (small, True)):
        st = w.steps()
        a = pushed(rad, w, st, noalloc=True)
        b = pushed(rad, w, st, noalloc=False)
        Ia, Ib = a.spectrum(), b.spectrum()
        what = f"no-alloc push, {w.n_dir} x {w.n_omega}, {w.n_particles} x {w.n_steps}"
        if same_splits:
            assert np.array_equal(Ia, Ib), what
        else:
            assert_close(Ia, Ib, what + " vs rad_push_step")
        ks = in_block_sample(w.n_omega)
        Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas()[ks], w.shape, w.shape_len, w.dt)
        assert_parity(Ia[:, ks], Iref, what + " vs oracle", ks=ks)
        # mixed with allocating pushes and a reset on the same grid, in issue order
        a.reset()
        dev = to_device(st, w.in_dtype)
        a.push_step(float(w.times()[0]), step_slice(dev, 0, w.n_particles))
        for j in range(1, w.n_steps):
            a.push_step_noalloc(float(w.times()[j]), step_slice(dev, j, w.n_particles))
        assert_close(a.spectrum(), Ib, what + ", mixed with rad_push_step")
    assert L.RAD_OK == 0


def test_noalloc_at_the_scratch_limit(rad):
    """A grid of exactly RAD_NOALLOC_SCRATCH_BYTES / 16 points (2048 directions x 2048
    frequencies): one particle split per launch, and a push of more particles than one split
    holds takes two launches, each folded before the scratch is reused."""
    w = SINGLE.scaled(n_particles=40000, n_steps=1, nx_dir=32, ny_dir=64, n_omega=2048, seed=74)
    assert w.n_dir * w.n_omega * 16 == 64 << 20
    st = w.steps()
    a = pushed(rad, w, st, noalloc=True)
    b = pushed(rad, w, st, noalloc=False)
    what = f"no-alloc push at the limit, {w.n_dir} x {w.n_omega}, {w.n_particles} particles"
    # the scratch path sums at most 32768 particles per FP32 split; an allocating push may
    # cut other splits (on this grid's 512 tiles it also takes one per launch): FP32
    # rounding of sums over 32768 terms of random phase, about 2^-24 sqrt(32768 / 2) =
    # 7.6e-6 of their size, bounds the difference
    Ia = a.spectrum()
    assert_close(Ia, b.spectrum(), what + " vs rad_push_step", tol_inf=1e-5, tol_freq=1e-5)
    ds = np.arange(0, w.n_dir, 511)
    ks = in_block_sample(w.n_omega, 64)
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    assert_parity(Ia[np.ix_(ds, ks)], Iref, what + " vs oracle", ks=ks)


def test_noalloc_push_under_graph_capture(rad):
    """Captured into a graph (the call records no event under capture), the no-alloc push
    replays bitwise equal to the same push issued directly, over several replays with eager
    work, resets and synchronisation between them (no memset is recorded: the kernels
    write every partial they read)."""
    import torch
    w = SINGLE.scaled(n_particles=3000, n_steps=1, nx_dir=4, ny_dir=8, n_omega=64, seed=75)
    st = w.steps()
    part = step_slice(to_device(st, w.in_dtype), 0, w.n_particles)
    t = float(w.times()[0])
    g = grid_for(rad, w)
    g.push_step_noalloc(t, part)
    ref = g.spectrum()
    g.reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.push_step_noalloc(t, part)
    torch.cuda.synchronize()
    for rep in range(3):
        g.reset()
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(g.spectrum(), ref), rep
        del junk
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape, w.shape_len, w.dt)
    assert_parity(ref, Iref, "no-alloc push (captured and replayed) vs oracle")


def test_noalloc_rejects_grid_beyond_scratch(rad):
    w = SINGLE.scaled(n_particles=64, n_steps=1, nx_dir=32, ny_dir=64, n_omega=2049, seed=73)
    g = grid_for(rad, w)          # 2048 x 2049 points need 16 B each per split: > 64 MiB
    with pytest.raises(rad.RadError) as ei:
        g.push_step_noalloc(0.0, to_device(w.steps(), "f32"))
    assert ei.value.code == rad.RAD_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
    g.push_step(0.0, to_device(w.steps(), "f32"))    # the allocating push still works
    assert np.all(np.isfinite(g.spectrum()))
