"""Pins of the FP64 oracle against what the paper and the mathematics fix.

No numbers are printed in the paper for a worked example, so every pin here is a closed
form, an invariant, a limit or a brute-force sum:

  * textbook harmonic spectrum of one electron on a circular orbit (Eq. 1, absolute SI);
  * no acceleration => no radiation (Eq. 1 amplitude is linear in dbeta/dt);
  * n . S = 0 (the amplitude is a cross product with n);
  * coherent limit (N^2) and incoherent limit (N) of Eq. 12 inside Eq. 13;
  * Monte-Carlo average of the configuration form factor (Eqs. 8, 10) against the closed
    form of Eqs. 11-12 for every Table 1 shape;
  * brute-force electron sums (Eq. 2) against the macro-particle result, per realisation
    (exact factorisation, Eq. 9) and on average;
  * time-shift and rotation invariance;
  * the C oracle against the independent numpy oracle.
"""
import numpy as np
import pytest
from scipy import constants as K
from scipy.special import jv, jvp

import oracle
from oracle import np_oracle
from workloads import TINY, circular_orbit, flatten, replicate, C_LIGHT

SHAPES = ("point", "cic", "tsc", "qsc", "gauss")


def both(fn_name, *args, **kw):
    return getattr(oracle, fn_name)(*args, **kw), getattr(np_oracle, fn_name)(*args, **kw)


def tiny_samples(n=64, steps=8, seed=3, **over):
    w = TINY.scaled(n_particles=n, n_steps=steps, seed=seed, **over)
    st = w.steps()
    return w, flatten(st, w.times())


# --------------------------------------------------------------------------- T5
@pytest.mark.parametrize("beta", [0.5, 0.9])
def test_circular_orbit_harmonics_absolute(orc, beta):
    """One electron, uniform circular motion, exactly Np periods sampled K times each.

    |dt sum_j A_j chi_j|^2 at omega = m omega0 equals
    Np^2 (2 pi m)^2 [cot^2(theta) J_m^2(x) + beta^2 J_m'^2(x)], x = m beta sin(theta),
    so I = e^2/(16 pi^3 eps0 c) times that (Eq. 1, Jackson ch. 14 / Landau-Lifshitz sec. 74).
    The prefactor is taken from scipy.constants, independently of the oracle's constants.
    """
    w0, K_per, Np = 1e13, 512, 2
    T0 = 2 * np.pi / w0
    dt = T0 / K_per
    times = np.arange(K_per * Np) * dt
    tr = flatten(circular_orbit(beta, w0, times), times)
    th = np.array([0.3, 0.7, 1.2])
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    om = np.arange(10) * w0
    pref = K.e ** 2 / (16 * np.pi ** 3 * K.epsilon_0 * K.c)
    for I in both("spectrum", tr, dirs, om, "point", 0.0, dt):
        for i, t in enumerate(th):
            for m in (1, 2, 5, 9):
                x = m * beta * np.sin(t)
                ref = pref * Np ** 2 * (2 * np.pi * m) ** 2 * (
                    (np.cos(t) / np.sin(t)) ** 2 * jv(m, x) ** 2 + beta ** 2 * jvp(m, x) ** 2)
                assert I[i, m] == pytest.approx(ref, rel=1e-8), (beta, t, m)
            # omega = 0: the time integral of the exact derivative over full periods is zero
            assert I[i, 0] < 1e-20 * I[i, 1]


# --------------------------------------------------------------------------- T1
def test_no_acceleration_no_radiation(orc):
    w, s = tiny_samples()
    s = dict(s)
    for k in ("dbx", "dby", "dbz"):
        s[k] = np.zeros_like(s[k])
    for I in both("spectrum", s, w.directions(), w.omegas(), "gauss", 1e-7, w.dt):
        assert np.all(I == 0.0)


# --------------------------------------------------------------------------- T2
def test_spectrum_perpendicular_to_n(orc):
    w, s = tiny_samples()
    dirs = w.directions()
    for S in both("spectrum_complex", s, dirs, w.omegas(), "cic", 1e-7):
        nS = np.einsum("dkc,dc->dk", S, dirs)
        mag = np.sqrt(np.sum(np.abs(S) ** 2, -1))
        assert np.all(np.abs(nS) <= 1e-12 * mag.max())


def test_amplitude_matches_expanded_form(orc):
    """A from the nested cross products equals the BAC-CAB expansion
    [(n - beta)(n.dbeta) - dbeta (1 - beta.n)] / (1 - beta.n)^2 for unit n."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        b = rng.normal(size=3); b *= rng.uniform(0.1, 0.999) / np.linalg.norm(b)
        db = rng.normal(size=3) * 1e12
        D = 1 - b @ n
        ref = ((n - b) * (n @ db) - db * D) / D ** 2
        assert np.allclose(oracle.amplitude(n, b, db), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
        assert np.allclose(np_oracle.amplitude(n, b[None], db[None])[0], ref, rtol=1e-10,
                           atol=1e-10 * np.abs(ref).max())


# --------------------------------------------------------------------------- T3
@pytest.mark.parametrize("shape", ["point", "cic"])
def test_coherent_limit(orc, shape):
    """M macro-particles on one trajectory with g = 1 (point shape, or omega = 0):
    I = (sum N_m)^2 I_1."""
    w, s1 = tiny_samples(n=1, steps=32, seed=7)
    st1 = w.steps()
    Ns = np.array([3.0, 17.5, 120.0, 1e4])
    stM = replicate(st1, Ns)
    sM = flatten(stM, w.times())
    om = w.omegas()[:8] if shape == "point" else np.array([0.0])
    dirs = w.directions()
    s_single = dict(s1); s_single["w"] = np.ones_like(s1["w"])
    for fn in (oracle.spectrum, np_oracle.spectrum):
        I1 = fn(s_single, dirs, om, shape, 1e-7, w.dt)
        IM = fn(sM, dirs, om, shape, 1e-7, w.dt)
        np.testing.assert_allclose(IM, Ns.sum() ** 2 * I1, rtol=1e-11)


# --------------------------------------------------------------------------- T4
def test_incoherent_single_macro_particle(orc):
    """g = 0 exactly (Gaussian so wide that exp underflows): F = sqrt(N), I = N I_1."""
    w, s1 = tiny_samples(n=1, steps=32, seed=8)
    N = 4321.0
    s_macro = dict(s1); s_macro["w"] = np.full_like(s1["w"], N)
    s_single = dict(s1); s_single["w"] = np.ones_like(s1["w"])
    om = w.omegas()[1:]
    assert oracle.shape_g("gauss", 1.0, om[0]) == 0.0
    for fn in (oracle.spectrum, np_oracle.spectrum):
        I1 = fn(s_single, w.directions(), om, "gauss", 1.0, w.dt)
        IN = fn(s_macro, w.directions(), om, "gauss", 1.0, w.dt)
        np.testing.assert_allclose(IN, N * I1, rtol=1e-12)


def test_incoherent_random_phase_average(orc):
    """Many macro-particles with identical motion, shifted along n by random offsets
    spanning many wavelengths, g = 0: E[I] = sum N_m I_1 (cross terms average out)."""
    w, s1 = tiny_samples(n=1, steps=16, seed=9)
    st1 = w.steps()
    n = w.directions()[5]
    om = np.array([2e18, 3e18, 4e18])
    s_single = dict(s1); s_single["w"] = np.ones_like(s1["w"])
    I1 = oracle.spectrum(s_single, n[None], om, "gauss", 1.0, w.dt)[0]
    rng = np.random.default_rng(11)
    Ns = rng.uniform(1e3, 1e5, 48)
    ratios = []
    for _ in range(300):
        shifts = rng.uniform(0, 2e-6, Ns.shape[0])    # >> c/omega ~ 1e-10 m
        stM = replicate(st1, Ns, shifts, n)
        IM = oracle.spectrum(flatten(stM, w.times()), n[None], om, "gauss", 1.0, w.dt)[0]
        ratios.append(IM / (Ns.sum() * I1))
    ratios = np.array(ratios).ravel()
    # I / <I> is ~ exponential (std 1): mean of K draws is within 4/sqrt(K)
    assert abs(ratios.mean() - 1.0) < 4.0 / np.sqrt(ratios.size)


# --------------------------------------------------------------------------- T8
def test_shape_identities(orc):
    om = np.array([0.0, 1e14, 3e15, 7e15, 2e16, 1e17])
    L = 0.1e-6
    for sh in SHAPES:
        assert oracle.shape_g(sh, L, 0.0) == 1.0
        assert float(np_oracle.shape_g(sh, L, 0.0)) == 1.0
        for o in om:
            assert oracle.form_factor_sq(1.0, oracle.shape_g(sh, L, o)) == 1.0
    for o in om:
        cic = oracle.shape_g("cic", L, o)
        assert oracle.shape_g("tsc", L, o) == pytest.approx(cic ** 2, rel=1e-14, abs=1e-300)
        assert oracle.shape_g("qsc", L, o) == pytest.approx(cic ** 3, rel=1e-14, abs=1e-300)
    # CIC zeros at omega Delta / 2c = k pi
    o0 = 2 * np.pi * C_LIGHT / L
    assert oracle.shape_g("cic", L, o0) < 1e-30
    # N = 0 contributes nothing; F^2 interpolates N (g = 0) .. N^2 (g = 1)
    assert oracle.form_factor_sq(0.0, 0.3) == 0.0
    assert oracle.form_factor_sq(50.0, 0.0) == 50.0
    assert oracle.form_factor_sq(50.0, 1.0) == 2500.0


# --------------------------------------------------------------------------- T6
@pytest.mark.parametrize("shape", ["cic", "tsc", "qsc", "gauss"])
def test_form_factor_monte_carlo(orc, shape):
    """Eq. 10 by Monte Carlo: electrons drawn independently from the normalised shape,
    averaged |sum_k exp(-i omega s_k/c)|^2 vs N + (N^2 - N) g(omega) (Eqs. 11-12)."""
    rng = np.random.default_rng(2024)
    N, R, L = 20, 200_000, 0.1e-6
    offs = np_oracle.sample_offsets(rng, shape, L, (R, N))
    for omega in (0.0, 1e15, 5e15, 1.2e16, 3e16):
        x = np_oracle.electron_phase_sum(offs, omega)
        mean, err = x.mean(), x.std() / np.sqrt(R)
        ref = oracle.form_factor_sq(N, oracle.shape_g(shape, L, omega))
        assert abs(mean - ref) <= 4.5 * err + 1e-9 * ref, (shape, omega, mean, ref, err)


def test_brute_force_electrons_per_realisation(orc):
    """Eq. 2 for N point electrons riding one macro trajectory at offsets s_k n equals the
    central-phase spectrum times sum_k exp(-i omega s_k / c) (Eqs. 7-9), per realisation."""
    w, s1 = tiny_samples(n=1, steps=16, seed=5)
    st1 = w.steps()
    n = w.directions()[3]
    om = np.array([0.0, 1e15, 4e15, 1e16])
    s_single = dict(s1); s_single["w"] = np.ones_like(s1["w"])
    Sbar = oracle.spectrum_complex(s_single, n[None], om, "point", 0.0)[0]     # (K, 3)
    rng = np.random.default_rng(6)
    for _ in range(5):
        offs = np_oracle.sample_offsets(rng, "gauss", 0.1e-6, 12)
        st = replicate(st1, np.ones(12), offs, n)
        Se = oracle.spectrum_complex(flatten(st, w.times()), n[None], om, "point", 0.0)[0]
        ph = np.exp(-1j * om[:, None] * offs[None, :] / C_LIGHT).sum(1)
        np.testing.assert_allclose(Se, Sbar * ph[:, None], rtol=1e-10, atol=1e-10 * np.abs(Se).max())


def test_brute_force_electrons_average_vs_macro(orc):
    """Average of brute-force electron spectra over realisations of the CIC distribution
    matches the single macro-particle spectrum with the Eq. 12 form factor."""
    w, s1 = tiny_samples(n=1, steps=8, seed=12)
    st1 = w.steps()
    n = w.directions()[6]
    om = np.array([0.0, 1e15, 6e15, 2e16])
    L, N, R = 0.1e-6, 8, 3000
    s_macro = dict(s1); s_macro["w"] = np.full_like(s1["w"], float(N))
    I_macro = oracle.spectrum(s_macro, n[None], om, "cic", L, w.dt)[0]
    rng = np.random.default_rng(13)
    offs = np_oracle.sample_offsets(rng, "cic", L, (R, N))
    times = w.times()
    acc = []
    for r in range(R):
        st = replicate(st1, np.ones(N), offs[r], n)
        acc.append(np_oracle.spectrum(flatten(st, times), n[None], om, "point", 0.0, w.dt)[0])
    acc = np.array(acc)
    mean, err = acc.mean(0), acc.std(0) / np.sqrt(R)
    assert np.all(np.abs(mean - I_macro) <= 4.5 * err + 1e-9 * I_macro), (mean, I_macro, err)


# --------------------------------------------------------------------------- T10 / T11
def test_time_shift_invariance(orc):
    w, s = tiny_samples()
    om, dirs = w.omegas(), w.directions()
    S0 = oracle.spectrum_complex(s, dirs, om, "cic", 1e-7)
    T = 1e-12
    s2 = dict(s); s2["t"] = s["t"] + T
    S1 = oracle.spectrum_complex(s2, dirs, om, "cic", 1e-7)
    np.testing.assert_allclose(S1, S0 * np.exp(1j * om * T)[None, :, None],
                               rtol=1e-7, atol=1e-7 * np.abs(S0).max())
    I0 = oracle.spectrum(s, dirs, om, "cic", 1e-7, w.dt)
    I1 = oracle.spectrum(s2, dirs, om, "cic", 1e-7, w.dt)
    np.testing.assert_allclose(I1, I0, rtol=1e-7, atol=1e-12 * I0.max())


def test_rotation_invariance(orc):
    w, s = tiny_samples()
    om, dirs = w.omegas(), w.directions()
    rng = np.random.default_rng(4)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    s2 = dict(s)
    for a, b, c in (("x", "y", "z"), ("bx", "by", "bz"), ("dbx", "dby", "dbz")):
        v = np.stack([s[a], s[b], s[c]], 1) @ q.T
        s2[a], s2[b], s2[c] = v[:, 0], v[:, 1], v[:, 2]
    I0 = oracle.spectrum(s, dirs, om, "gauss", 1e-7, w.dt)
    I1 = oracle.spectrum(s2, dirs @ q.T, om, "gauss", 1e-7, w.dt)
    np.testing.assert_allclose(I1, I0, rtol=1e-6, atol=1e-9 * I0.max())


# --------------------------------------------------------------------------- oracle vs oracle
def test_c_oracle_shape_factor_matches_numpy_oracle(orc):
    L = 0.1e-6
    for o in (0.0, 1e14, 3e15, 7e15, 2e16, 1e17):
        for sh in SHAPES:
            assert oracle.shape_g(sh, L, o) == pytest.approx(float(np_oracle.shape_g(sh, L, o)),
                                                             rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("shape", SHAPES)
def test_c_oracle_matches_numpy_oracle(orc, shape):
    w, s = tiny_samples(n=256, steps=16, seed=0)
    dirs, om = w.directions(), w.omegas()
    Ic = oracle.spectrum(s, dirs, om, shape, 0.1e-6, w.dt)
    In = np_oracle.spectrum(s, dirs, om, shape, 0.1e-6, w.dt)
    assert np.max(np.abs(Ic - In)) <= 1e-12 * np.max(In)
    Sc = oracle.spectrum_complex(s, dirs, om, shape, 0.1e-6)
    Sn = np_oracle.spectrum_complex(s, dirs, om, shape, 0.1e-6)
    assert np.max(np.abs(Sc - Sn)) <= 1e-12 * np.max(np.abs(Sn))


def test_prefactor_reading(orc):
    """C = (q_e dt)^2 / (16 pi^3 eps0 c): the rectangle-rule dt sits inside |.|^2."""
    dt = 0.05e-15
    ref = (K.e * dt) ** 2 / (16 * np.pi ** 3 * K.epsilon_0 * K.c)
    assert oracle.prefactor(dt) == pytest.approx(ref, rel=1e-8)
    assert np_oracle.prefactor(dt) == pytest.approx(ref, rel=1e-8)


def test_empty_and_zero_weight(orc):
    w, s = tiny_samples(n=8, steps=2)
    dirs, om = w.directions(), w.omegas()
    empty = {k: v[:0] for k, v in s.items()}
    assert np.all(oracle.spectrum(empty, dirs, om, "cic", 1e-7, w.dt) == 0.0)
    s0 = dict(s); s0["w"] = np.zeros_like(s["w"])
    assert np.all(oracle.spectrum(s0, dirs, om, "cic", 1e-7, w.dt) == 0.0)


# --------------------------------------------------------------------------- cubic-cell shapes
@pytest.mark.parametrize("shape", ["cic3d", "tsc3d", "qsc3d"])
def test_cubic_cell_form_factor_monte_carlo(orc, shape):
    """Eq. 10 by Monte Carlo for electrons filling a cubic cell (each axis from the 1-D
    density), observed along tilted directions, vs N + (N^2 - N) g(n, omega)."""
    rng = np.random.default_rng(77)
    N, R, L = 12, 120_000, 0.1e-6
    offs = np_oracle.sample_offsets3(rng, shape, L, (R, N))
    for n in (np.array([0.6, 0.0, 0.8]), np.array([0.48, 0.6, 0.64]), np.array([0.0, 0.0, 1.0])):
        for omega in (2e15, 6e15, 1.5e16):
            x = np_oracle.electron_phase_sum3(offs, n, omega)
            mean, err = x.mean(), x.std() / np.sqrt(R)
            ref = oracle.form_factor_sq(N, oracle.shape_g3(shape, L, n, omega))
            assert abs(mean - ref) <= 4.5 * err + 1e-9 * ref, (shape, n, omega, mean, ref, err)


def test_cubic_cell_reduces_to_1d_along_an_axis(orc):
    for base in ("cic", "tsc", "qsc"):
        for omega in (0.0, 3e15, 1e16, 4e16):
            for axis in range(3):
                n = np.zeros(3); n[axis] = 1.0
                assert oracle.shape_g3(base + "3d", 1e-7, n, omega) == pytest.approx(
                    oracle.shape_g(base, 1e-7, omega), rel=1e-14, abs=1e-300)
                assert float(np_oracle.shape_g3(base + "3d", 1e-7, n, omega)) == pytest.approx(
                    oracle.shape_g(base, 1e-7, omega), rel=1e-13, abs=1e-300)


def test_cubic_cell_spectrum_c_vs_numpy_oracle(orc):
    w, s = tiny_samples(n=128, steps=8, seed=1)
    dirs = np.array([[0.3, 0.4, np.sqrt(0.75)], [0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
    om = np.linspace(0, 4e16, 9)
    Ic = oracle.spectrum(s, dirs, om, "cic3d", 0.1e-6, w.dt)
    In = np_oracle.spectrum(s, dirs, om, "cic3d", 0.1e-6, w.dt)
    assert np.max(np.abs(Ic - In)) <= 1e-12 * np.max(In)
