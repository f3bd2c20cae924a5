"""Seeded input generator: reproducible, physical (|beta| < 1) and self-consistent
(dr/dt = c beta, dbeta/dt matches the derivative of beta)."""
import numpy as np

from workloads import (TINY, SINGLE, PRECISION, C_LIGHT, batched_uneven, serving_bunches,
                       poisson_trace, direction_grid, omega_grid)


def test_reproducible_draws():
    a = TINY.steps(0, 3)
    b = TINY.steps(0, 3)
    for k in a:
        assert np.array_equal(a[k], b[k])
    c = TINY.scaled(seed=1).steps(0, 3)
    assert not np.array_equal(a["x"], c["x"])


def test_beta_below_one_and_float32_rounding():
    for w in (TINY, SINGLE.scaled(n_particles=4096, n_steps=4), PRECISION.scaled(n_particles=4096, n_steps=4)):
        st = w.steps()
        b2 = st["bx"] ** 2 + st["by"] ** 2 + st["bz"] ** 2
        assert np.all(b2 < 1.0)
        if w.in_dtype == "f32":
            assert np.array_equal(st["x"], st["x"].astype(np.float32).astype(np.float64))


def test_trajectory_self_consistent():
    w = PRECISION.scaled(n_particles=64)
    b = w.bunch()
    t, h = 1.2e-12, 1e-18
    s0, sp, sm = b.state(t), b.state(t + h), b.state(t - h)
    for r, v in (("x", "bx"), ("y", "by"), ("z", "bz")):
        np.testing.assert_allclose((sp[r] - sm[r]) / (2 * h), C_LIGHT * s0[v], rtol=1e-6, atol=1e-6)
    for v, dv in (("bx", "dbx"), ("bz", "dbz")):
        np.testing.assert_allclose((sp[v] - sm[v]) / (2 * h), s0[dv], rtol=1e-5,
                                   atol=1e-6 * np.abs(s0["dbx"]).max())


def test_grids():
    d = direction_grid(8, 16, 0.02)
    assert d.shape == (128, 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=0, atol=1e-15)
    assert d[0, 0] == -0.02 and d[0, 1] == -0.02 and d[15, 1] == 0.02 and d[16, 0] > d[0, 0]
    om = omega_grid(0.0, 1e19 / 255, 256)
    assert om[0] == 0.0 and abs(om[-1] - 1e19) < 1e4
    assert SINGLE.updates == 65536 * 100 * 128 * 256


def test_multi_bunch_configs():
    mb = batched_uneven()
    assert len(mb.counts) == 12 and all(1e3 <= n <= 5e5 for n in mb.counts)
    sv = serving_bunches()
    assert len(sv.counts) == 8 and all(1e4 <= n <= 2e5 for n in sv.counts)
    t, b = poisson_trace(2000.0, 4000, 8)
    assert t.shape == (4000,) and np.all(np.diff(t) > 0) and b.max() < 8
    assert abs(4000 / t[-1] - 2000) < 200
