"""Seeded synthetic particle trajectories (inputs only; no radiation arithmetic).

The paper demonstrates the method on macro-electrons of a laser-wakefield
simulation (Sec. 4).  Those trajectories are not available, so every input here
is a synthetic stand-in with the same structure: relativistic electrons
(gamma of tens to a thousand) that oscillate transversely (betatron motion)
while streaming along z, sampled at uniform time steps t_j = t0 + j*dt as the
in-situ sum of Eq. 13 requires, each macro-particle carrying a real weighting N.

Betatron orbit used for every bunch (exactly self-consistent, |beta| < 1):
    psi(t)  = omega_b t + phi
    x(t)    = x0 cos psi,            beta_x = -a sin psi,  a = x0 omega_b / c
    y(t)    = y0,                    beta_y = 0
    beta_z  = sqrt(beta^2 - beta_x^2),  beta = sqrt(1 - 1/gamma^2) (constant)
    z(t)    = z0 + (c beta / omega_b) [E(psi | m) - E(phi | m)],  m = a^2 / beta^2
    dbeta_x/dt = -a omega_b cos psi,  dbeta_z/dt = -beta_x dbeta_x/dt / beta_z
E(.|m) is the incomplete elliptic integral of the second kind, so dz/dt = c beta_z
holds exactly (a second-order expansion of z would push |beta| above 1 for the
larger gammas used here).

Also here: a uniform circular orbit (the textbook harmonic-spectrum case used to
pin the oracle) and helpers that build co-located or randomly shifted copies of
one trajectory (coherent / incoherent limits).  Draw order is fixed so every
seed reproduces the same arrays.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ellipeinc

C_LIGHT = 299792458.0  # m/s (exact, SI)

FIELDS = ("x", "y", "z", "bx", "by", "bz", "dbx", "dby", "dbz", "w")


class Bunch:
    """Per-particle constants of a betatron bunch (drawn once, reused every step)."""

    def __init__(self, x0, phi, gamma, weight, y0, z0, omega_beta):
        self.x0 = np.asarray(x0, np.float64)
        self.phi = np.asarray(phi, np.float64)
        self.gamma = np.asarray(gamma, np.float64)
        self.weight = np.asarray(weight, np.float64)
        self.y0 = np.asarray(y0, np.float64)
        self.z0 = np.asarray(z0, np.float64)
        self.omega_beta = float(omega_beta)
        self.beta = np.sqrt(1.0 - 1.0 / self.gamma ** 2)
        self.a = self.x0 * self.omega_beta / C_LIGHT
        self.m = (self.a / self.beta) ** 2
        self.e_phi = ellipeinc(self.phi, self.m)

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    def state(self, t: float) -> dict:
        """r [m], beta [1], dbeta/dt [1/s] and weight at time t, all float64."""
        wb = self.omega_beta
        psi = wb * t + self.phi
        s, c = np.sin(psi), np.cos(psi)
        bx = -self.a * s
        dbx = -self.a * wb * c
        bz = np.sqrt(self.beta ** 2 - bx ** 2)
        dbz = -bx * dbx / bz
        z = self.z0 + (C_LIGHT * self.beta / wb) * (ellipeinc(psi, self.m) - self.e_phi)
        zeros = np.zeros_like(bx)
        return {
            "x": self.x0 * c, "y": self.y0.copy(), "z": z,
            "bx": bx, "by": zeros, "bz": bz,
            "dbx": dbx, "dby": zeros.copy(), "dbz": dbz,
            "w": self.weight.copy(),
        }


def draw_bunch(rng: np.random.Generator, n: int, gamma: tuple, weight: tuple,
               x0_max: float = 1e-6, omega_beta: float = 2e13,
               yz_sigma: float = 1e-6) -> Bunch:
    """Draw n particles.  Order: x0, phi, gamma, weight, y0, z0.

    gamma: ("uniform", lo, hi) | ("lognormal", mu, sigma) | ("const", g)
    weight: (lo, hi) uniform real weighting.
    """
    x0 = rng.uniform(0.0, x0_max, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    kind = gamma[0]
    if kind == "uniform":
        g = rng.uniform(gamma[1], gamma[2], n)
    elif kind == "lognormal":
        g = rng.lognormal(gamma[1], gamma[2], n)
        g = np.maximum(g, 2.0)
    elif kind == "const":
        g = np.full(n, float(gamma[1]))
    else:
        raise ValueError(f"unknown gamma law {gamma!r}")
    w = rng.uniform(weight[0], weight[1], n)
    y0 = rng.normal(0.0, yz_sigma, n)
    z0 = rng.normal(0.0, yz_sigma, n)
    return Bunch(x0, phi, g, w, y0, z0, omega_beta)


def stack_steps(bunch: Bunch, times) -> dict:
    """State at each time in `times`, stacked step-major: arrays of shape (steps, n)."""
    per = [bunch.state(float(t)) for t in times]
    return {k: np.stack([p[k] for p in per]) for k in FIELDS}


def circular_orbit(beta: float, omega0: float, times) -> dict:
    """One electron in uniform circular motion in the x-y plane (radius beta c/omega0).

    r = R (cos w0 t, sin w0 t, 0), beta = b (-sin, cos, 0), dbeta/dt = -b w0 (cos, sin, 0).
    Returned arrays have shape (steps, 1), weight 1.
    """
    t = np.asarray(times, np.float64)
    R = beta * C_LIGHT / omega0
    ps = omega0 * t
    s, c = np.sin(ps), np.cos(ps)
    z = np.zeros_like(t)
    out = {"x": R * c, "y": R * s, "z": z,
           "bx": -beta * s, "by": beta * c, "bz": z.copy(),
           "dbx": -beta * omega0 * c, "dby": -beta * omega0 * s, "dbz": z.copy(),
           "w": np.ones_like(t)}
    return {k: v[:, None] for k, v in out.items()}


def replicate(traj: dict, weights, shifts=None, direction=None) -> dict:
    """Copies of one single-particle trajectory (arrays (steps, 1)) as M macro-particles.

    weights: (M,) weightings.  shifts: optional (M,) displacements [m] along the unit
    vector `direction`, applied to r at every step (same beta, dbeta for all copies).
    """
    weights = np.asarray(weights, np.float64)
    M = weights.shape[0]
    out = {k: np.repeat(traj[k], M, axis=1) for k in FIELDS if k != "w"}
    out["w"] = np.broadcast_to(weights, (traj["x"].shape[0], M)).copy()
    if shifts is not None:
        shifts = np.asarray(shifts, np.float64)
        d = np.asarray(direction, np.float64)
        out["x"] = out["x"] + shifts[None, :] * d[0]
        out["y"] = out["y"] + shifts[None, :] * d[1]
        out["z"] = out["z"] + shifts[None, :] * d[2]
    return out


def flatten(steps: dict, times) -> dict:
    """(steps, n) arrays -> flat per-sample arrays with an explicit time t per sample."""
    times = np.asarray(times, np.float64)
    n = steps["x"].shape[1]
    flat = {k: np.ascontiguousarray(steps[k].reshape(-1)) for k in FIELDS}
    flat["t"] = np.repeat(times, n)
    return flat


def round_to(steps: dict, dtype) -> dict:
    """Round every field to `dtype` (the precision the device path ingests), then widen
    back to float64 so a float64 consumer sees exactly the rounded values."""
    return {k: np.asarray(v, dtype).astype(np.float64) for k, v in steps.items()}
