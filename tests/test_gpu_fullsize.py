"""Full-size parity on sampled outputs: the workloads' real particle counts, step counts and
grids, launched as the bench launches them, checked against the oracle on a deterministic
subset of (direction, frequency) points that the oracle evaluates one by one.  Sampled
frequencies include, in blocks of 16, the bins a lane reaches by walking from its
FP64-seeded middle frequency (offsets 0, 7 and 15, up to eight products away)."""
import time

import numpy as np
import pytest

import oracle
from workloads import SINGLE, PRECISION, batched_uneven, serving_bunches, flatten, host_workers
from tests.helpers import assert_parity, error_report, in_block_sample, to_device, step_slice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rad():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1802_03972_amd as rad
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    rad._lib.lib()
    oracle.set_threads(host_workers())
    return rad


def grid_for(rad, w, **kw):
    return rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape, shape_len=w.shape_len,
                    dt=w.dt, **kw)


def test_single_bunch_all_100_steps(rad):
    """65536 particles x 100 per-step pushes on 128 x 256 with the tuned launch shape;
    oracle on every 8th direction x frequencies 0, 7, 15 of every block of 16, and on two
    directions x every frequency (all 16 in-block offsets of the walk, up to eight steps
    from the seed)."""
    w = SINGLE
    st = w.steps(workers=host_workers())
    dev = to_device(st, "f32")
    g = grid_for(rad, w)
    for j, t in enumerate(w.times()):
        g.push_step(float(t), step_slice(dev, j, w.n_particles))
    I = g.spectrum()
    parts = flatten(st, w.times())
    ds = np.arange(0, w.n_dir, 8)
    ks = in_block_sample(w.n_omega)
    Iref = oracle.spectrum(parts, w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    assert_parity(I[np.ix_(ds, ks)], Iref, f"single bunch, 100 steps, tile {g.get_tile()}", ks=ks)
    d2 = np.array([0, 77])
    ka = np.arange(w.n_omega)
    Iref2 = oracle.spectrum(parts, w.directions()[d2], w.omegas(), w.shape, w.shape_len, w.dt)
    # the report lists the per-frequency error by in-block offset (k mod 16)
    assert_parity(I[d2], Iref2, "single bunch, 100 steps, two directions x every frequency", ks=ka)


PRECISION_KS = np.array([0, 1, 7, 15, 135, 271, 392, 519, 655, 776, 903, 1015, 1023])


def test_precision_stress_all_10000_steps_from_one_picosecond(rad):
    """The precision-stress workload at its stated size: 16384 particles x 10000 steps from
    t = 1 ps on 64 x 1024 frequencies to 1e20 rad/s, FP64 input, in both arithmetic modes.
    Oracle on 4 directions x 13 frequencies (walked bins of every kind, the highest
    included), summed as complex S over the same steps.  FP64 geometry and phase pass the
    gate; the all-FP32 variant loses the phase at high frequency and fails it."""
    import torch
    w = PRECISION
    bunch = w.bunch()
    ds = np.array([0, 9, 36, 63])
    ks = PRECISION_KS
    grids = {"fp64_phase": grid_for(rad, w, precision=rad.PHASE_F64),
             "all_fp32": grid_for(rad, w, precision=rad.ALL_F32)}
    S_ref = 0.0
    group = 250
    t0 = time.perf_counter()
    for j0 in range(0, w.n_steps, group):
        j1 = min(w.n_steps, j0 + group)
        st = w.steps(j0, j1, bunch=bunch, workers=host_workers())
        dev = to_device(st, "f64")
        tj = float(w.times(j0, j0 + 1)[0])
        for g in grids.values():
            g.push_steps(tj, j1 - j0, dev)
        S_ref = S_ref + oracle.spectrum_complex(flatten(st, w.times(j0, j1)), w.directions()[ds], w.omegas()[ks],
                                                w.shape, w.shape_len)
        torch.cuda.synchronize()
        del dev
        if j0 % 2000 == 0:
            print(f"  steps {j1}/{w.n_steps} ({time.perf_counter() - t0:.0f} s)", flush=True)
    Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_ref) ** 2, axis=-1)
    assert_parity(grids["fp64_phase"].spectrum()[np.ix_(ds, ks)], Iref,
                  "precision stress, FP64 phase, 10000 steps from 1 ps", ks=ks)
    rep = error_report(grids["all_fp32"].spectrum()[np.ix_(ds, ks)], Iref, ks)
    print(f"precision stress, all FP32: {rep}", flush=True)
    assert rep["e_inf"] > 1e-3 and rep["per_frequency_max_top_quarter"] > 0.1


def test_batched_uneven_all_200_steps(rad):
    """The batched workload at its stated size: 12 bunches (log-uniform counts in
    [1e3, 5e5]), 200 distinct time steps, one batched persistent launch per step over all
    bunches.  Every bunch against the oracle on 3 directions x 7 frequencies (near and far
    walked bins), summed over all 200 steps."""
    import torch
    mb = batched_uneven()
    ws = mb.bunches()
    bunches = [w.bunch() for w in ws]
    grids = [grid_for(rad, w) for w in ws]
    b = rad.Batcher(max_items=len(ws))
    ds = np.array([0, 27, 63])
    ks = np.array([0, 7, 15, 100, 143, 200, 255])
    S_ref = [0.0] * len(ws)
    n_steps = ws[0].n_steps
    group = 20
    t0 = time.perf_counter()
    for j0 in range(0, n_steps, group):
        j1 = min(n_steps, j0 + group)
        sts = [w.steps(j0, j1, bunch=bb, workers=host_workers()) for w, bb in zip(ws, bunches)]
        devs = [to_device(st, "f32") for st in sts]
        times = ws[0].times(j0, j1)
        for j in range(j1 - j0):
            b.push([(g, float(times[j]), 1, step_slice(d, j, w.n_particles))
                    for g, w, d in zip(grids, ws, devs)])
        for i, (w, st) in enumerate(zip(ws, sts)):
            S_ref[i] = S_ref[i] + oracle.spectrum_complex(flatten(st, times), w.directions()[ds], w.omegas()[ks],
                                                          w.shape, w.shape_len)
        torch.cuda.synchronize()
        del devs
        print(f"  steps {j1}/{n_steps} ({time.perf_counter() - t0:.0f} s)", flush=True)
    for i, (w, g) in enumerate(zip(ws, grids)):
        Iref = oracle.prefactor(w.dt) * np.sum(np.abs(S_ref[i]) ** 2, axis=-1)
        assert_parity(g.spectrum()[np.ix_(ds, ks)], Iref, f"batched bunch {i} (n={w.n_particles}), 200 steps", ks=ks)


def test_serving_grid_largest_chunk(rad):
    """The largest serving bunch's one-step chunk on its 128 x 512 grid."""
    mb = serving_bunches()
    ws = mb.bunches()
    w = max(ws, key=lambda x: x.n_particles).scaled(n_steps=1)
    st = w.steps()
    g = grid_for(rad, w)
    g.push_step(float(w.times()[0]), to_device(st, "f32"))
    I = g.spectrum()
    ds = np.arange(0, w.n_dir, 16)
    ks = in_block_sample(w.n_omega, 32)
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions()[ds], w.omegas()[ks], w.shape, w.shape_len, w.dt)
    assert_parity(I[np.ix_(ds, ks)], Iref, f"serving chunk of {w.n_particles} particles on 128 x 512", ks=ks)
