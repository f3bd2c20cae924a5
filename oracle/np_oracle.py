"""Independent numpy FP64 oracle (tiny inputs), written separately from rad_oracle.c.

TEST INFRASTRUCTURE ONLY.  Same definition as the C oracle (Eq. 1 amplitude with
np.cross, Eq. 1 phase, Eq. 12 form factor with the normalised Table 1 shape factor,
Eq. 13 double sum with dt inside the square), evaluated with numpy array operations so
that the two oracles share neither code nor summation order.

Also holds the brute-force pieces used to pin the form-factor formalism itself:
  * `electron_phase_sum`: |sum_k exp(-i omega s_k / c)|^2 for explicit electron offsets
    s_k along n (the configuration form factor of Eq. 8);
  * `sample_offsets`: electron offsets drawn from each Table 1 shape (box, box*box,
    box*box*box, Gaussian) so the ensemble average of Eq. 10 can be estimated by
    Monte Carlo.
"""
from __future__ import annotations

import numpy as np

C = 299792458.0
QE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def shape_g(shape: str, length: float, omega):
    omega = np.asarray(omega, np.float64)
    if shape == "point":
        return np.ones_like(omega)
    if shape == "gauss":
        return np.exp(-(omega * length / C) ** 2)
    x = omega * length / (2.0 * C)
    s = np.sinc(x / np.pi)  # numpy sinc is sin(pi u)/(pi u)
    p = {"cic": 2, "tsc": 4, "qsc": 6}[shape]
    return s ** p


def shape_g3(shape: str, length: float, n, omega):
    """Cubic cell: product over x, y, z of the 1-D factor at omega * |n_c|."""
    n = np.asarray(n, np.float64)
    base = shape[:-2]
    return (shape_g(base, length, np.asarray(omega) * abs(n[0])) * shape_g(base, length, np.asarray(omega) * abs(n[1]))
            * shape_g(base, length, np.asarray(omega) * abs(n[2])))


def form_factor_sq(N, g):
    N = np.asarray(N, np.float64)
    return N + (N * N - N) * g


def amplitude(n, beta, dbeta):
    """Eq. 1 amplitude; n (3,), beta/dbeta (P, 3) -> (P, 3)."""
    n = np.asarray(n, np.float64)
    inner = np.cross(n[None, :] - beta, dbeta)
    outer = np.cross(np.broadcast_to(n, inner.shape), inner)
    D = 1.0 - beta @ n
    return outer / (D * D)[:, None]


def prefactor(dt: float) -> float:
    return (QE * dt) ** 2 / (16.0 * np.pi ** 3 * EPS0 * C)


def spectrum_complex(samples: dict, dirs, omegas, shape: str, shape_len: float,
                     chunk: int = 4096) -> np.ndarray:
    """(n_dir, n_omega, 3) complex128."""
    t = np.asarray(samples["t"], np.float64).reshape(-1)
    r = np.stack([np.asarray(samples[k], np.float64).reshape(-1) for k in ("x", "y", "z")], 1)
    b = np.stack([np.asarray(samples[k], np.float64).reshape(-1) for k in ("bx", "by", "bz")], 1)
    db = np.stack([np.asarray(samples[k], np.float64).reshape(-1) for k in ("dbx", "dby", "dbz")], 1)
    w = np.asarray(samples["w"], np.float64).reshape(-1)
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    omegas = np.asarray(omegas, np.float64).reshape(-1)
    out = np.zeros((dirs.shape[0], omegas.shape[0], 3), np.complex128)
    for d, n in enumerate(dirs):
        g = shape_g3(shape, shape_len, n, omegas) if shape.endswith("3d") else shape_g(shape, shape_len, omegas)
        for s0 in range(0, t.shape[0], chunk):
            sl = slice(s0, s0 + chunk)
            A = amplitude(n, b[sl], db[sl])                   # (P, 3)
            tau = t[sl] - (r[sl] @ n) / C                     # (P,)
            F = np.sqrt(form_factor_sq(w[sl][:, None], g[None, :]))   # (P, K)
            ph = np.exp(1j * tau[:, None] * omegas[None, :])  # (P, K)
            out[d] += np.einsum("pk,pc->kc", F * ph, A)
    return out


def spectrum(samples: dict, dirs, omegas, shape: str, shape_len: float, dt: float) -> np.ndarray:
    S = spectrum_complex(samples, dirs, omegas, shape, shape_len)
    return prefactor(dt) * np.sum(np.abs(S) ** 2, axis=-1)


def sample_offsets(rng: np.random.Generator, shape: str, length: float, size) -> np.ndarray:
    """Electron offsets along n drawn from the normalised Table 1 densities.

    CIC: box of width length; TSC: sum of two such boxes (triangle); QSC: sum of three;
    Gauss: normal with standard deviation length; point: zero.
    """
    if shape == "point":
        return np.zeros(size)
    if shape == "gauss":
        return rng.normal(0.0, length, size)
    k = {"cic": 1, "tsc": 2, "qsc": 3}[shape]
    out = np.zeros(size)
    for _ in range(k):
        out = out + rng.uniform(-0.5 * length, 0.5 * length, size)
    return out


def sample_offsets3(rng: np.random.Generator, shape: str, length: float, size) -> np.ndarray:
    """3-D electron offsets (..., 3) filling a cubic cell: each axis independently drawn from
    the 1-D density of the base shape."""
    base = shape[:-2]
    return np.stack([sample_offsets(rng, base, length, size) for _ in range(3)], axis=-1)


def electron_phase_sum3(offsets: np.ndarray, n, omega: float) -> np.ndarray:
    """Eq. 8 with 3-D offsets (R, N, 3): |sum_k exp(-i omega n.r_k / c)|^2."""
    z = np.exp(-1j * omega * (offsets @ np.asarray(n, np.float64)) / C).sum(axis=-1)
    return np.abs(z) ** 2


def electron_phase_sum(offsets: np.ndarray, omega: float) -> np.ndarray:
    """Eq. 8 for each row of `offsets` (R, N): |sum_k exp(-i omega s_k / c)|^2."""
    z = np.exp(-1j * omega * offsets / C).sum(axis=-1)
    return np.abs(z) ** 2
