"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element.

Gate (relative tolerance 1e-4 on the spectrum): e_inf = max |I_gpu - I_oracle| / max
I_oracle, and the per-frequency error (each frequency against its own oracle peak over
directions, so the incoherent omega > 0 band is checked as closely as the coherent peak;
tests.helpers).  The oracle always consumes exactly the values the device ingests
(float32 configs are rounded before both sides see them).
"""
import numpy as np
import pytest

import oracle
from workloads import TINY, SINGLE, PRECISION, circular_orbit, flatten, replicate, Workload
from tests.helpers import (assert_close, assert_complex_parity, assert_parity, in_block_sample, to_device,
                           step_slice)

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


def make_grid(rad, w: Workload, **kw):
    return rad.Grid(w.directions(), w.omega0, w.domega, w.n_omega, shape=w.shape,
                    shape_len=w.shape_len, dt=w.dt, **kw)


def run_gpu(rad, w: Workload, steps: dict, per_step=True, grid=None, **kw):
    g = grid or make_grid(rad, w, **kw)
    dev = to_device(steps, w.in_dtype)
    n = steps["x"].shape[1]
    times = w.times(0, steps["x"].shape[0])
    if per_step:
        for j, t in enumerate(times):
            g.push_step(float(t), step_slice(dev, j, n))
    else:
        g.push_steps(float(times[0]), len(times), dev)
    return g


def oracle_I(w: Workload, steps: dict, dirs=None, omegas=None):
    times = w.times(0, steps["x"].shape[0])
    return oracle.spectrum(flatten(steps, times), w.directions() if dirs is None else dirs,
                           w.omegas() if omegas is None else omegas, w.shape, w.shape_len, w.dt)


# ----------------------------------------------------------------------------- builtins
def test_trig_builtins_take_revolutions(rad):
    r = np.linspace(0.0, 1.0, 4097, dtype=np.float32)[:-1]
    out = rad.trig_probe(r)
    ref_s, ref_c = np.sin(2 * np.pi * r.astype(np.float64)), np.cos(2 * np.pi * r.astype(np.float64))
    err_hw = max(np.abs(out[:, 0] - ref_s).max(), np.abs(out[:, 1] - ref_c).max())
    err_lib = max(np.abs(out[:, 2] - ref_s).max(), np.abs(out[:, 3] - ref_c).max())
    print(f"hardware sin/cos(2 pi r) max abs err {err_hw:.3e}; library sincospi {err_lib:.3e}")
    assert err_lib < 5e-7
    assert err_hw < 1e-5


# ----------------------------------------------------------------------------- parity
def test_tiny_config_full_grid(rad):
    """1024 macro-particles x 64 steps, 4x4 directions x 64 omega, FP64 input, Gauss."""
    w = TINY
    st = w.steps()
    g = run_gpu(rad, w, st)
    I = g.spectrum()
    Iref = oracle_I(w, st)
    assert_parity(I, Iref, "tiny full grid", ks=np.arange(w.n_omega))
    S = g.spectrum_complex()
    Sref = oracle.spectrum_complex(flatten(st, w.times()), w.directions(), w.omegas(), w.shape, w.shape_len)
    assert_complex_parity(S, Sref, "tiny full grid, complex S")


@pytest.mark.parametrize("shape,dtype", [("cic", "f32"), ("tsc", "f64"), ("qsc", "f32"),
                                         ("gauss", "f64"), ("point", "f32")])
def test_ragged_tiles(rad, shape, dtype):
    """Sizes that leave ragged tails in every dimension: 5x8 directions, 100 omega,
    1000 particles (not a multiple of the 32-particle chunk), 3 steps."""
    w = SINGLE.scaled(n_particles=1000, n_steps=3, nx_dir=5, ny_dir=8, n_omega=100,
                      omega_max=4e18, shape=shape, in_dtype=dtype, seed=21)
    st = w.steps()
    I = run_gpu(rad, w, st).spectrum()
    assert_parity(I, oracle_I(w, st), f"ragged {shape}/{dtype}")


def test_every_tile_shape_agrees(rad):
    w = SINGLE.scaled(n_particles=700, n_steps=2, nx_dir=6, ny_dir=7, n_omega=150, omega_max=6e18, seed=5)
    st = w.steps()
    Iref = oracle_I(w, st)
    for wpl in (16, 32):
        for dpw in (16, 32, 64):
            for waves in (1, 2, 4, 8):
                for wg in ((1, 6) if wpl == 16 else (1,)):   # splits per tile also vary
                    g = make_grid(rad, w)
                    g.set_tile(w_per_lane=wpl, dir_per_wave=dpw, waves=waves, wg_per_cu=wg)
                    I = run_gpu(rad, w, st, grid=g).spectrum()
                    assert_parity(I, Iref, f"tile {wpl}, {dpw}, {waves}, {wg}")
                    g.close()


def test_push_steps_matches_per_step_pushes(rad):
    w = TINY.scaled(n_particles=300, n_steps=5, seed=2)
    st = w.steps()
    I1 = run_gpu(rad, w, st, per_step=True).spectrum()
    I2 = run_gpu(rad, w, st, per_step=False).spectrum()
    assert_close(I2, I1, "multi-step push vs per-step pushes")
    assert_parity(I2, oracle_I(w, st), "multi-step push")


def test_chunk_linearity(rad):
    """Splitting one step's particles over two pushes changes only the rounding."""
    w = SINGLE.scaled(n_particles=2000, n_steps=1, nx_dir=4, ny_dir=8, n_omega=128, seed=8)
    st = w.steps()
    dev = to_device(st, w.in_dtype)
    g1 = make_grid(rad, w)
    g1.push_step(0.0, dev)
    g2 = make_grid(rad, w)
    g2.push_step(0.0, {k: v[:777] for k, v in dev.items()})
    g2.push_step(0.0, {k: v[777:] for k, v in dev.items()})
    assert_close(g2.spectrum(), g1.spectrum(), "one step split over two pushes")


def test_deterministic_repeat(rad):
    w = SINGLE.scaled(n_particles=5000, n_steps=2, nx_dir=8, ny_dir=8, n_omega=256, seed=9)
    st = w.steps()
    a = run_gpu(rad, w, st).spectrum()
    b = run_gpu(rad, w, st).spectrum()
    assert np.array_equal(a, b)


def test_time_shift_invariance_fp64_phase(rad):
    """t -> t + 1 ps with r unchanged multiplies S by exp(i omega T): I unchanged."""
    w = PRECISION.scaled(n_particles=512, n_steps=4, n_omega=256, omega_max=1e20, t0=0.0, seed=4)
    st = w.steps()
    I0 = run_gpu(rad, w, st).spectrum()
    w1 = w.scaled(t0=1e-12)
    I1 = run_gpu(rad, w1, st).spectrum()
    assert_parity(I1, I0, "time shift 1 ps (device vs device)")
    ks = in_block_sample(w.n_omega)
    assert_parity(I1[:, ks], oracle_I(w1, st, omegas=w1.omegas()[ks]), "shifted by 1 ps vs oracle", ks=ks)


def test_checkpoint_resume(rad):
    w = SINGLE.scaled(n_particles=1500, n_steps=4, nx_dir=4, ny_dir=4, n_omega=64, seed=3)
    st = w.steps()
    dev = to_device(st, w.in_dtype)
    n = w.n_particles
    times = w.times()
    g = make_grid(rad, w)
    for j in range(4):
        g.push_step(float(times[j]), step_slice(dev, j, n))
    full = g.get_state()
    g2 = make_grid(rad, w)
    for j in range(2):
        g2.push_step(float(times[j]), step_slice(dev, j, n))
    saved = g2.get_state()
    g3 = make_grid(rad, w)
    g3.set_state(saved)
    for j in range(2, 4):
        g3.push_step(float(times[j]), step_slice(dev, j, n))
    assert np.array_equal(g3.get_state(), full)
    g.reset()
    assert np.all(g.spectrum() == 0.0)


def test_bad_data_sets_sticky_flag(rad):
    import torch
    w = TINY.scaled(n_particles=64, n_steps=1, seed=1)
    st = w.steps()
    dev = to_device(st, "f64")
    dev["bx"][5] = float("nan")
    g = make_grid(rad, w)
    g.push_step(0.0, dev)
    with pytest.raises(rad.RadError) as ei:
        g.spectrum()
    assert ei.value.code == rad.RAD_ERR_BAD_DATA
    g.reset()
    dev2 = to_device(st, "f64")
    dev2["bz"][3] = 1.0  # beta along n ~ 1: 1 - beta.n <= 0 for the on-axis direction
    dev2["bx"][3] = 0.0
    dev2["by"][3] = 0.0
    g2 = rad.Grid(np.array([[0.0, 0.0, 1.0]]), 0.0, 1e16, 8, shape="gauss", shape_len=1e-7, dt=w.dt)
    g2.push_step(0.0, dev2)
    with pytest.raises(rad.RadError):
        g2.spectrum()
    g2.reset()
    g2.push_step(0.0, to_device(st, "f64"))
    assert np.all(np.isfinite(g2.spectrum()))
    torch.cuda.synchronize()


def test_empty_push_is_noop(rad):
    import torch
    w = TINY.scaled(n_particles=32, n_steps=1)
    g = make_grid(rad, w)
    empty = {k: torch.empty(0, dtype=torch.float64, device="cuda") for k in rad.FIELDS}
    g.push_step(0.0, empty)
    assert np.all(g.spectrum() == 0.0)


def test_circular_orbit_harmonics_gpu(rad):
    """One electron on a circular orbit: device spectrum at the harmonics vs the oracle
    (which itself matches the Bessel closed form)."""
    beta, w0, K, Np = 0.9, 1e13, 512, 2
    dt = 2 * np.pi / w0 / K
    times = np.arange(K * Np) * dt
    tr = circular_orbit(beta, w0, times)
    th = np.array([0.3, 0.7, 1.2])
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    g = rad.Grid(dirs, 0.0, w0, 12, shape="point", shape_len=0.0, dt=dt)
    dev = to_device(tr, "f64")
    g.push_steps(0.0, K * Np, dev)
    I = g.spectrum()
    Iref = oracle.spectrum(flatten(tr, times), dirs, np.arange(12) * w0, "point", 0.0, dt)
    assert_parity(I[:, 1:], Iref[:, 1:], "circular orbit harmonics 1..11")
    assert_parity(I, Iref, "circular orbit incl. the omega = 0 null")


def test_coherent_and_incoherent_limits_gpu(rad):
    w = TINY.scaled(n_particles=1, n_steps=32, seed=7)
    st1 = w.steps()
    Ns = np.array([3.0, 17.5, 120.0, 1e4])
    stM = replicate(st1, Ns)
    one = dict(st1); one["w"] = np.ones_like(st1["w"])
    for shape, expect in (("point", Ns.sum() ** 2), ):
        ww = w.scaled(shape=shape, n_particles=len(Ns))
        I1 = run_gpu(rad, w.scaled(shape=shape), one).spectrum()
        IM = run_gpu(rad, ww, stM).spectrum()
        assert_parity(IM, expect * I1, "co-located copies: (sum N)^2 I_1")
    # g = 0 exactly for omega > 0 (very wide Gaussian): a single macro-particle gives N * I1
    wg = w.scaled(shape="gauss", shape_len=1.0)
    N = 4321.0
    macro = dict(st1); macro["w"] = np.full_like(st1["w"], N)
    I1 = run_gpu(rad, wg, one).spectrum()[:, 1:]
    IN = run_gpu(rad, wg, macro).spectrum()[:, 1:]
    assert_parity(IN, N * I1, "g = 0: N I_1")


def test_single_bunch_full_size_sampled(rad):
    """One full-size step of the 65536-particle single-bunch workload (launch shape of the
    bench), checked against the oracle on every direction and, in every block of 16
    frequencies, offsets 0, 7 and 15 (walked eight, one and seven products from the seed)."""
    w = SINGLE.scaled(n_steps=1)
    st = w.steps()
    I = run_gpu(rad, w, st).spectrum()
    sel = in_block_sample(w.n_omega)
    Iref = oracle_I(w, st, omegas=w.omegas()[sel])
    assert_parity(I[:, sel], Iref, "single bunch full size (1 step), sampled", ks=sel)


def test_push_split_over_several_launches(rad):
    """A single push larger than one launch holds (4 splits x 32768 particles on this
    tiling) is cut into three launches; same for a batched push over many tiles."""
    w = SINGLE.scaled(n_particles=300000, n_steps=1, nx_dir=8, ny_dir=16, n_omega=512, seed=31)
    st = w.steps()
    dev = to_device(st, "f32")
    tile = dict(w_per_lane=16, dir_per_wave=16, waves=1, wg_per_cu=1)
    g = make_grid(rad, w, tile=tile)
    g.profile(True)
    g.push_step(float(w.times()[0]), dev)
    prof = g.profile_read()
    assert prof["launches"] == 3
    gb = make_grid(rad, w)
    b = rad.Batcher(tile=tile)
    b.push([(gb, float(w.times()[0]), 1, dev)])
    ds = np.arange(0, w.n_dir, 8)
    ks = in_block_sample(w.n_omega, 64)
    Iref = oracle_I(w, st, dirs=w.directions()[ds], omegas=w.omegas()[ks])
    for name, grid in (("per-grid", g), ("batched", gb)):
        assert_parity(grid.spectrum()[np.ix_(ds, ks)], Iref, f"multi-launch push ({name})", ks=ks)


@pytest.mark.parametrize("n_dir,n_omega", [(1, 1), (1, 17), (3, 1)])
def test_degenerate_grids(rad, n_dir, n_omega):
    """One direction and/or one frequency (a single 3e18 rad/s line)."""
    w = TINY.scaled(n_particles=200, n_steps=3, seed=32)
    st = w.steps()
    dirs = w.directions()[:n_dir]
    om0, dom = 3e18, (2e17 if n_omega > 1 else 0.0)
    g = rad.Grid(dirs, om0, dom, n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    run_gpu(rad, w, st, grid=g)
    om = om0 + np.arange(n_omega) * dom
    assert_parity(g.spectrum(), oracle_I(w, st, dirs=dirs, omegas=om), f"{n_dir} dirs x {n_omega} omega")


def test_zero_and_fractional_weights(rad):
    """N = 0 contributes nothing; 0 < N < 1 is a valid weighting (F^2 = N(1-g) + N^2 g)."""
    w = SINGLE.scaled(n_particles=640, n_steps=2, nx_dir=4, ny_dir=4, n_omega=64, seed=33)
    st = w.steps()
    wts = np.random.default_rng(3).uniform(0.0, 1.0, w.n_particles)
    wts[::5] = 0.0
    st = dict(st)
    st["w"] = np.broadcast_to(wts, st["w"].shape).copy()
    I = run_gpu(rad, w, st).spectrum()
    assert_parity(I, oracle_I(w, st), "zero and fractional weights")
    only_zero = dict(st)
    only_zero["w"] = np.zeros_like(st["w"])
    assert np.all(run_gpu(rad, w, only_zero).spectrum() == 0.0)


def test_reset_push_readout_on_different_streams(rad):
    """Accumulate, reset, accumulate again, read: four streams, no host synchronisation;
    only the second accumulation may be in the result."""
    import torch
    w = SINGLE.scaled(n_particles=3000, n_steps=2, nx_dir=4, ny_dir=8, n_omega=128, seed=34)
    st = w.steps()
    other = SINGLE.scaled(n_particles=3000, n_steps=2, nx_dir=4, ny_dir=8, n_omega=128, seed=35).steps()
    dev, dev_other = to_device(st, "f32"), to_device(other, "f32")
    ref = make_grid(rad, w)
    ref.push_steps(w.t0, w.n_steps, dev)
    s1, s2, s3, s4 = (torch.cuda.Stream() for _ in range(4))
    torch.cuda.synchronize()
    g = make_grid(rad, w)
    g.push_steps(w.t0, w.n_steps, dev_other, s1)
    g.reset(s2)
    g.push_steps(w.t0, w.n_steps, dev, s3)
    assert_close(g.spectrum(s4), ref.spectrum(), "push / reset / push / read on four streams")


def test_device_readout_is_ordered_before_later_reset_and_push(rad):
    """rad_spectrum_device on one stream, then (no host synchronisation) a reset and a push
    on other streams: the read-out must see the accumulator as it was when it was issued.
    Work queued on the read-out stream first delays the read-out well past the moment the
    reset and the push could run."""
    import torch
    w = SINGLE.scaled(n_particles=3000, n_steps=2, nx_dir=4, ny_dir=8, n_omega=128, seed=37)
    st = w.steps()
    other = SINGLE.scaled(n_particles=3000, n_steps=2, nx_dir=4, ny_dir=8, n_omega=128, seed=38).steps()
    dev, dev_other = to_device(st, "f32"), to_device(other, "f32")
    ref = make_grid(rad, w)
    ref.push_steps(w.t0, w.n_steps, dev)
    I_ref = ref.spectrum()
    sa, sb, sc = (torch.cuda.Stream() for _ in range(3))
    g = make_grid(rad, w)
    out = torch.empty(w.n_dir * w.n_omega, dtype=torch.float64, device="cuda")
    x = torch.randn(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    g.push_steps(w.t0, w.n_steps, dev, sa)
    with torch.cuda.stream(sb):
        for _ in range(40):                      # delay the read-out stream
            x = torch.tanh(x @ x)
    g.spectrum_device(out, sb)
    g.reset(sc)
    g.push_steps(w.t0, w.n_steps, dev_other, sa)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy().reshape(w.n_dir, w.n_omega), I_ref, "device read-out before reset")
    later = make_grid(rad, w)
    later.push_steps(w.t0, w.n_steps, dev_other)
    assert_close(g.spectrum(), later.spectrum(), "reset then push after the read-out")


def test_recurrence_with_steps_near_zero_and_pi(rad):
    """The per-frequency phase step theta = domega*tau close to a multiple of pi is the hard
    case for the three-term walk z_{k+1} = 2 cos(theta) z_k - z_{k-1} of the uniform-grid
    kernel: there the rounding of 2 cos(theta) stands for a large angle error, and only the
    short walks from the mid-block seed (at most 8 steps, error at most ~m^2 roundings) keep
    it small.  Every frequency is checked.  Particles
    are placed so that on the axis the step is within 1e-7..1e-2 rad of 0 or pi (and within
    ~0.02 rad of it on the tilted directions); three steps a whole number of step periods
    apart."""
    w = SINGLE.scaled(n_particles=2048, n_steps=3, n_omega=256, in_dtype="f64", seed=36)
    C = 299792458.0
    dom = w.domega
    w = SINGLE.scaled(n_particles=2048, n_steps=3, n_omega=256, in_dtype="f64", seed=36,
                      dt=7 * 2 * np.pi / dom)
    rng = np.random.default_rng(36)
    n = w.n_particles
    eps = 10.0 ** rng.uniform(-7, -2, n) * rng.choice([-1.0, 1.0], n)
    theta = 2 * np.pi * rng.integers(0, 6, n) + np.pi * rng.integers(0, 2, n) + eps
    z = C * theta / dom
    gamma = 200.0
    beta = np.sqrt(1 - 1 / gamma**2)
    bx, by = 1e-3 * rng.standard_normal(n), 1e-3 * rng.standard_normal(n)
    bz = np.sqrt(beta**2 - bx**2 - by**2)
    dbx, dby = 1e12 * rng.standard_normal(n), 1e12 * rng.standard_normal(n)
    dbz = -(bx * dbx + by * dby) / bz
    fields = dict(x=np.zeros(n), y=np.zeros(n), z=z, bx=bx, by=by, bz=bz, dbx=dbx, dby=dby, dbz=dbz,
                  w=rng.uniform(1e3, 1e5, n))
    st = {k: np.broadcast_to(v, (w.n_steps, n)).copy() for k, v in fields.items()}
    tilt = np.array([0.0, 1e-4, 2e-3, 2e-2])
    dirs = np.stack([tilt, np.zeros(4), np.sqrt(1 - tilt**2)], axis=1)
    g = rad.Grid(dirs, w.omega0, dom, w.n_omega, shape=w.shape, shape_len=w.shape_len, dt=w.dt)
    I = run_gpu(rad, w, st, grid=g).spectrum()
    Iref = oracle_I(w, st, dirs=dirs)
    rep = assert_parity(I, Iref, "near-degenerate steps", ks=np.arange(w.n_omega))
    assert rep["per_direction_max"] <= TOL
