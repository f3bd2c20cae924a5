"""The parity gate itself (CPU only): the per-frequency error sees the incoherent band
that the global-peak metric e_inf cannot see.

With omega = 0 in the grid, the coherent bin (F = N) is the global peak, while every
omega > 0 bin of a bunch with random phases is incoherent (F close to sqrt N, Eq. 12) and
sits orders of magnitude below it.  A 1 % error on every omega > 0 bin -- or a band set
to zero -- passes e_inf <= 1e-4 and must fail the per-frequency gate."""
import numpy as np
import pytest

import oracle
from workloads import SINGLE, TINY, circular_orbit, flatten
from tests.helpers import assert_parity, e_inf, error_report, in_block_sample


@pytest.fixture(scope="module")
def tiny_spectrum(orc):
    w = TINY
    st = w.steps()
    return oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape, w.shape_len, w.dt)


def test_one_percent_on_incoherent_band_is_caught(tiny_spectrum):
    Iref = tiny_spectrum
    bad = Iref.copy()
    bad[:, 1:] *= 1.01
    assert e_inf(bad, Iref) <= 1e-4            # the global-peak metric accepts it
    rep = error_report(bad, Iref)
    assert rep["per_frequency_max"] == pytest.approx(0.01, rel=1e-9)
    with pytest.raises(AssertionError):
        assert_parity(bad, Iref, "omega > 0 bins x 1.01")
    assert_parity(Iref * (1 + 1e-6), Iref, "uniform 1e-6 scaling")


def test_zeroed_band_is_caught(orc):
    """The ragged-Gauss input: its largest omega > 0 bin is below 1e-4 of the peak, so a
    result that is zero for every omega > 0 passes e_inf."""
    w = SINGLE.scaled(n_particles=1000, n_steps=3, nx_dir=5, ny_dir=8, n_omega=100, omega_max=4e18,
                      shape="gauss", in_dtype="f64", seed=21)
    st = w.steps()
    Iref = oracle.spectrum(flatten(st, w.times()), w.directions(), w.omegas(), w.shape, w.shape_len, w.dt)
    zero = Iref.copy()
    zero[:, 1:] = 0.0
    assert e_inf(zero, Iref) <= 1e-4
    with pytest.raises(AssertionError):
        assert_parity(zero, Iref, "omega > 0 band zeroed")


def test_exact_null_columns_are_skipped(orc):
    """One electron on a closed circular orbit over whole periods: the omega = 0 column is
    an exact null (zero up to rounding); a rounding-size error there must not fail the
    gate, while the harmonics are still gated."""
    beta, w0, K = 0.9, 1e13, 256
    dt = 2 * np.pi / w0 / K
    times = np.arange(K) * dt
    tr = circular_orbit(beta, w0, times)
    dirs = np.array([[np.sin(0.5), 0.0, np.cos(0.5)]])
    Iref = oracle.spectrum(flatten(tr, times), dirs, np.arange(6) * w0, "point", 0.0, dt)
    assert Iref[0, 0] < 1e-20 * Iref.max()
    noisy = Iref.copy()
    noisy[0, 0] += 1e-14 * Iref.max()
    rep = assert_parity(noisy, Iref, "null column with rounding noise")
    assert rep["null_columns_skipped"] == 1
    off = Iref.copy()
    off[0, 3] *= 1.001
    with pytest.raises(AssertionError):
        assert_parity(off, Iref, "harmonic 3 off by 1e-3")


def test_in_block_sample_hits_recurrence_bins():
    ks = in_block_sample(256)
    assert set(ks % 16) == {0, 7, 15}
    assert ks[-1] == 255 and ks[0] == 0
    assert len(in_block_sample(1)) == 1
