"""The five seeded workloads (sizes, grids, physics draws) used by tests and the bench.

Observation grids: directions n = (tx, ty, sqrt(1 - tx^2 - ty^2)) with tx, ty on an
inclusive linspace of +-half_angle (index d = ix * ny + iy); frequencies are the
uniform grid omega_k = omega_max * k / (n_omega - 1), k = 0..n_omega-1, computed on
the host as omega0 + k * domega with omega0 = 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .betatron import draw_bunch, stack_steps, Bunch

SHAPES = {"point": 0, "cic": 1, "tsc": 2, "qsc": 3, "gauss": 4}


def direction_grid(nx: int, ny: int, half_angle: float) -> np.ndarray:
    tx = np.linspace(-half_angle, half_angle, nx)
    ty = np.linspace(-half_angle, half_angle, ny)
    d = np.empty((nx * ny, 3))
    for ix in range(nx):
        for iy in range(ny):
            k = ix * ny + iy
            d[k, 0] = tx[ix]
            d[k, 1] = ty[iy]
            d[k, 2] = np.sqrt(1.0 - tx[ix] ** 2 - ty[iy] ** 2)
    return d


def omega_grid(omega0: float, domega: float, n: int) -> np.ndarray:
    """omega_k = omega0 + k*domega in float64, one rounding per operation (no fma)."""
    k = np.arange(n, dtype=np.float64)
    return omega0 + k * domega


def block_log_omegas(lo: float, hi: float, n: int, block: int = 16) -> np.ndarray:
    """Log-like frequency list that is uniform inside each aligned block of `block`
    entries: block b starts at s_b = lo * R^b and steps by (s_{b+1} - s_b) / block, so the
    blocks tile [lo, ~hi] with spacings growing geometrically (R = (hi/lo)^(1/blocks))."""
    nb = -(-n // block)
    R = (hi / lo) ** (1.0 / nb)
    out = np.empty(n, np.float64)
    for b in range(nb):
        s0 = lo * R ** b
        st = (lo * R ** (b + 1) - s0) / block
        k = np.arange(min(block, n - b * block), dtype=np.float64)
        out[b * block:b * block + k.size] = s0 + k * st
    return out


@dataclass(frozen=True)
class Workload:
    name: str
    n_particles: int
    n_steps: int
    nx_dir: int
    ny_dir: int
    n_omega: int
    omega_max: float
    shape: str
    shape_len: float
    in_dtype: str  # "f32" | "f64"
    gamma: tuple
    weight: tuple
    t0: float = 0.0
    dt: float = 0.05e-15
    half_angle: float = 0.02
    x0_max: float = 1e-6
    omega_beta: float = 2e13
    seed: int = 0

    @property
    def n_dir(self) -> int:
        return self.nx_dir * self.ny_dir

    @property
    def omega0(self) -> float:
        return 0.0

    @property
    def domega(self) -> float:
        return self.omega_max / (self.n_omega - 1) if self.n_omega > 1 else 0.0

    @property
    def updates(self) -> int:
        return self.n_particles * self.n_steps * self.n_dir * self.n_omega

    @property
    def np_dtype(self):
        return np.float32 if self.in_dtype == "f32" else np.float64

    @property
    def shape_id(self) -> int:
        return SHAPES[self.shape]

    def directions(self) -> np.ndarray:
        return direction_grid(self.nx_dir, self.ny_dir, self.half_angle)

    def omegas(self) -> np.ndarray:
        return omega_grid(self.omega0, self.domega, self.n_omega)

    def times(self, j0: int = 0, j1: int | None = None) -> np.ndarray:
        j1 = self.n_steps if j1 is None else j1
        j = np.arange(j0, j1, dtype=np.float64)
        return self.t0 + j * self.dt

    def bunch(self) -> Bunch:
        rng = np.random.default_rng(self.seed)
        return draw_bunch(rng, self.n_particles, self.gamma, self.weight,
                          x0_max=self.x0_max, omega_beta=self.omega_beta)

    def steps(self, j0: int = 0, j1: int | None = None, bunch: Bunch | None = None,
              workers: int = 1) -> dict:
        """Particle state for steps [j0, j1), arrays (steps, n), already rounded to the
        ingest dtype (float32 configs) and returned as float64 views of those values.
        workers > 1 evaluates groups of steps on a thread pool (every step is a pure
        function of its time, so the arrays do not depend on the worker count)."""
        b = self.bunch() if bunch is None else bunch
        times = self.times(j0, j1)
        if workers > 1 and len(times) > 1:
            from concurrent.futures import ThreadPoolExecutor
            parts = np.array_split(times, min(len(times), 4 * workers))
            with ThreadPoolExecutor(workers) as ex:
                pieces = list(ex.map(lambda ts: stack_steps(b, ts), parts))
            st = {k: np.concatenate([p[k] for p in pieces]) for k in pieces[0]}
        else:
            st = stack_steps(b, times)
        if self.in_dtype == "f32":
            st = {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()}
        return st

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


# Tiny plain-FP64 case: 1024 x 64 steps, 4x4 directions x 64 omega to 5e18, Gauss 0.1 um.
TINY = Workload("tiny_fp64", 1024, 64, 4, 4, 64, 5e18, "gauss", 0.1e-6, "f64",
                gamma=("uniform", 50.0, 150.0), weight=(1e4, 1e5))
# Single-bunch kernel: 65536 x 100 steps, 8x16 directions x 256 omega to 1e19, CIC 0.1 um, fp32 in.
SINGLE = Workload("single_bunch_fp32", 65536, 100, 8, 16, 256, 1e19, "cic", 0.1e-6, "f32",
                  gamma=("lognormal", float(np.log(200.0)), 0.3), weight=(1e3, 1e5))
# Precision stress: 16384 x 10000 steps from t0 = 1 ps, 8x8 x 1024 omega to 1e20, gamma to 1000.
PRECISION = Workload("precision_stress", 16384, 10000, 8, 8, 1024, 1e20, "gauss", 0.1e-6, "f64",
                     gamma=("uniform", 50.0, 1000.0), weight=(1e3, 1e5), t0=1e-12)

CONFIGS = {w.name: w for w in (TINY, SINGLE, PRECISION)}


@dataclass(frozen=True)
class MultiBunch:
    """Several independent bunches, each with its own particle count and (n, omega) grid."""
    name: str
    counts: tuple
    base: Workload
    seeds: tuple = field(default_factory=tuple)

    def bunches(self):
        out = []
        for i, (n, s) in enumerate(zip(self.counts, self.seeds)):
            out.append(self.base.scaled(name=f"{self.name}_b{i}", n_particles=int(n), seed=int(s)))
        return out


def _spawn_seeds(seed: int, k: int) -> tuple:
    ss = np.random.SeedSequence(seed).spawn(k)
    return tuple(int(s.generate_state(1)[0]) for s in ss)


def batched_uneven(seed: int = 0, n_bunches: int = 12, steps: int = 200) -> MultiBunch:
    """12 bunches with log-uniform particle counts in [1e3, 5e5], 8x8 x 256 omega each."""
    rng = np.random.default_rng(seed)
    counts = tuple(int(round(float(np.exp(x)))) for x in rng.uniform(np.log(1e3), np.log(5e5), n_bunches))
    base = SINGLE.scaled(name="batched", n_steps=steps, nx_dir=8, ny_dir=8, n_omega=256)
    return MultiBunch("batched_uneven", counts, base, _spawn_seeds(seed, n_bunches))


def serving_bunches(seed: int = 0, n_bunches: int = 8) -> MultiBunch:
    """8 LWFA-like bunches, counts log-uniform in [1e4, 2e5], gamma ~ U(20, 500), 8x16 x 512."""
    rng = np.random.default_rng(seed + 1)
    counts = tuple(int(round(float(np.exp(x)))) for x in rng.uniform(np.log(1e4), np.log(2e5), n_bunches))
    base = SINGLE.scaled(name="serving", n_steps=1 << 30, nx_dir=8, ny_dir=16, n_omega=512,
                         gamma=("uniform", 20.0, 500.0))
    return MultiBunch("serving", counts, base, _spawn_seeds(seed + 1, n_bunches))


def host_workers() -> int:
    """Threads for input generation: the host cores this process may use, at most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def poisson_trace(rate: float, n_chunks: int, n_bunches: int, seed: int = 0):
    """Arrival times [s] (Poisson process at `rate` per second) and the bunch of each chunk."""
    rng = np.random.default_rng(seed + 2)
    gaps = rng.exponential(1.0 / rate, n_chunks)
    return np.cumsum(gaps), rng.integers(0, n_bunches, n_chunks)


@dataclass(frozen=True)
class Fig3Analogue:
    """Inputs of the synthetic analogue of the paper's Fig. 3 (Sec. 4): ONE macro-particle
    of `electrons` electrons on a betatron trajectory (gamma 100, 2000 steps of 0.05 fs),
    observed on axis and 10 mrad off axis over log-spaced frequencies 1e13 .. 1e19 rad/s,
    with the Gaussian macro-particle shape `sigma`."""
    electrons: float = 1e5
    sigma: float = 0.1e-6
    workload: Workload = TINY.scaled(n_particles=1, n_steps=2000, gamma=("const", 100.0), seed=5)

    def directions(self) -> np.ndarray:
        return np.array([[0.0, 0.0, 1.0], [0.01, 0.0, np.sqrt(1 - 1e-4)]])

    def omegas(self) -> np.ndarray:
        return np.geomspace(1e13, 1e19, 241)

    def trajectory(self, weight: float) -> dict:
        """(steps, 1) arrays of the one macro-particle with weighting `weight`."""
        st = self.workload.steps()
        out = dict(st)
        out["w"] = np.full_like(st["w"], float(weight))
        return out
