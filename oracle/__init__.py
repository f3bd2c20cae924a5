"""FP64 CPU oracle for the macro-particle radiation sum (Eqs. 1, 12, 13 of arXiv:1802.03972).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the bench's CPU-baseline leg
may import this package.  It shares no code with the device path.

Two independent implementations:
  * `rad_oracle.c` (plain C, OpenMP over (direction, frequency) points, libm sin/cos
    per point, Neumaier-compensated sums) wrapped here through ctypes;
  * `np_oracle` (vectorised numpy, used on tiny inputs to cross-check the C one).

Inputs are dicts of flat float64 arrays, one entry per sample (macro-particle at one
step): t, x, y, z [m], bx, by, bz [1], dbx, dby, dbz [1/s], w (weighting N).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "rad_oracle.c")

SHAPE_IDS = {"point": 0, "cic": 1, "tsc": 2, "qsc": 3, "gauss": 4, "cic3d": 5, "tsc3d": 6, "qsc3d": 7}

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math, no fp contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-std=c11", SRC_PATH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_shape_g.restype = ctypes.c_double
        L.oracle_shape_g.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oracle_shape_g3.restype = ctypes.c_double
        L.oracle_shape_g3.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_double]
        L.oracle_form_factor_sq.restype = ctypes.c_double
        L.oracle_form_factor_sq.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_amplitude.restype = None
        L.oracle_amplitude.argtypes = [dp, dp, dp, dp]
        L.oracle_prefactor.restype = ctypes.c_double
        L.oracle_prefactor.argtypes = [ctypes.c_double]
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        common = [ctypes.c_int64] + [dp] * 11 + [ctypes.c_int, dp, ctypes.c_int, dp,
                                                 ctypes.c_int, ctypes.c_double]
        L.oracle_spectrum_complex.restype = ctypes.c_int
        L.oracle_spectrum_complex.argtypes = common + [dp]
        L.oracle_spectrum.restype = ctypes.c_int
        L.oracle_spectrum.argtypes = common + [ctypes.c_double, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(samples: dict, dirs, omegas):
    keys = ("t", "x", "y", "z", "bx", "by", "bz", "dbx", "dby", "dbz", "w")
    arrs = [np.ascontiguousarray(samples[k], dtype=np.float64).reshape(-1) for k in keys]
    n = arrs[0].shape[0]
    for a in arrs:
        if a.shape[0] != n:
            raise ValueError("sample arrays differ in length")
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    omegas = np.ascontiguousarray(omegas, dtype=np.float64).reshape(-1)
    return n, arrs, dirs, omegas


def shape_id(shape) -> int:
    return SHAPE_IDS[shape] if isinstance(shape, str) else int(shape)


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def shape_g(shape, length: float, omega: float) -> float:
    """Normalised Table 1 shape factor |F~(omega)|^2."""
    return float(lib().oracle_shape_g(shape_id(shape), float(length), float(omega)))


def shape_g3(shape, length: float, n, omega: float) -> float:
    """Cubic-cell (3-D) shape factor g(n, omega)."""
    n = np.ascontiguousarray(n, np.float64)
    return float(lib().oracle_shape_g3(shape_id(shape), float(length), _dp(n), float(omega)))


def form_factor_sq(N: float, g: float) -> float:
    """Eq. 12: N + (N^2 - N) g."""
    return float(lib().oracle_form_factor_sq(float(N), float(g)))


def amplitude(n, beta, dbeta) -> np.ndarray:
    """Eq. 1 radiation amplitude for one (direction, particle state)."""
    n = np.ascontiguousarray(n, np.float64)
    b = np.ascontiguousarray(beta, np.float64)
    db = np.ascontiguousarray(dbeta, np.float64)
    out = np.empty(3)
    lib().oracle_amplitude(_dp(n), _dp(b), _dp(db), _dp(out))
    return out


def prefactor(dt: float) -> float:
    return float(lib().oracle_prefactor(float(dt)))


def spectrum_complex(samples: dict, dirs, omegas, shape, shape_len: float) -> np.ndarray:
    """Complex S(n, omega) as a (n_dir, n_omega, 3) complex128 array."""
    n, arrs, dirs, omegas = _prep(samples, dirs, omegas)
    out = np.empty((dirs.shape[0], omegas.shape[0], 3, 2))
    rc = lib().oracle_spectrum_complex(n, *[_dp(a) for a in arrs], dirs.shape[0], _dp(dirs),
                                       omegas.shape[0], _dp(omegas), shape_id(shape),
                                       float(shape_len), _dp(out))
    if rc != 0:
        raise ValueError(f"oracle_spectrum_complex failed ({rc})")
    return out[..., 0] + 1j * out[..., 1]


def spectrum(samples: dict, dirs, omegas, shape, shape_len: float, dt: float) -> np.ndarray:
    """d^2I/(dOmega domega) [J s/sr] as a (n_dir, n_omega) float64 array."""
    n, arrs, dirs, omegas = _prep(samples, dirs, omegas)
    out = np.empty((dirs.shape[0], omegas.shape[0]))
    rc = lib().oracle_spectrum(n, *[_dp(a) for a in arrs], dirs.shape[0], _dp(dirs),
                               omegas.shape[0], _dp(omegas), shape_id(shape), float(shape_len),
                               float(dt), _dp(out))
    if rc != 0:
        raise ValueError(f"oracle_spectrum failed ({rc})")
    return out
