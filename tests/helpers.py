"""Shared test helpers: device upload of seeded inputs and the parity gate.

The parity gate (oracle.metrics): e_inf and the per-frequency error, both within the
relative tolerance 1e-4 on the spectrum.
"""
from __future__ import annotations

import numpy as np

from oracle.metrics import NULL_FRACTION, TOL, error_report
from workloads import FIELDS, flatten


def e_inf(I, Iref) -> float:
    """max |I - I_ref| / max I_ref over the grid."""
    I = np.asarray(I)
    Iref = np.asarray(Iref)
    m = np.max(np.abs(Iref))
    return float(np.max(np.abs(I - Iref)) / m) if m > 0 else float(np.max(np.abs(I - Iref)))


def to_device(steps: dict, dtype, device=0) -> dict:
    """(steps, n) float64 arrays -> flat step-major CUDA tensors of `dtype`."""
    import torch
    td = torch.float32 if dtype in ("f32", np.float32) else torch.float64
    return {k: torch.as_tensor(np.ascontiguousarray(steps[k]).reshape(-1)).to(device=f"cuda:{device}", dtype=td)
            for k in FIELDS}


def step_slice(dev: dict, j: int, n: int) -> dict:
    return {k: v[j * n:(j + 1) * n] for k, v in dev.items()}


def oracle_samples(steps: dict, times) -> dict:
    return flatten(steps, times)


def in_block_sample(n: int, stride: int = 16, offsets=(0, 7, 15)) -> np.ndarray:
    """Frequency indices for sampled parity: in every block of `stride` frequencies the
    given offsets, plus the last frequency.  A 16-frequency lane is seeded from FP64 at its
    offset 8 and walks to the others (three-term recurrence or complex products): the default
    offsets are the farthest walked backward (0, eight steps), the nearest (7, one) and the
    farthest forward (15, seven)."""
    ks = [np.arange(o, n, stride) for o in offsets]
    return np.unique(np.concatenate(ks + [np.array([n - 1])]))


def assert_parity(I, Iref, what: str = "", tol: float = TOL, ks=None) -> dict:
    """The parity gate: e_inf <= tol and per-frequency error <= tol.  Prints the report."""
    rep = error_report(I, Iref, ks)
    extra = ""
    if "per_frequency_max_by_k_mod_16" in rep:
        extra = ", by k mod 16 " + ", ".join(f"{k}: {v:.1e}" for k, v in rep["per_frequency_max_by_k_mod_16"].items())
    print(f"{what}: e_inf {rep['e_inf']:.3e}, per-frequency {rep['per_frequency_max']:.3e}, "
          f"L2 {rep['l2_rel']:.3e}, per-direction {rep['per_direction_max']:.3e}{extra}", flush=True)
    assert rep["e_inf"] <= tol, (what, rep)
    assert rep["per_frequency_max"] <= tol, (what, rep)
    return rep


def assert_close(I, Iref, what: str = "", tol_inf: float = 1e-6, tol_freq: float = 1e-5) -> dict:
    """Two device results that differ only by FP32 rounding (same kernel arithmetic per
    term, different grouping of the sums): e_inf <= tol_inf and the per-frequency error
    <= tol_freq."""
    rep = error_report(I, Iref)
    print(f"{what}: e_inf {rep['e_inf']:.3e}, per-frequency {rep['per_frequency_max']:.3e}", flush=True)
    assert rep["e_inf"] <= tol_inf, (what, rep)
    assert rep["per_frequency_max"] <= tol_freq, (what, rep)
    return rep


def assert_complex_parity(S, Sref, what: str = "", tol: float = TOL) -> None:
    """Complex spectra (n_dir, n_omega, 3): max |S - S_ref| over the grid against the
    largest |S_ref| component, and per frequency against that frequency's largest."""
    S = np.asarray(S)
    Sref = np.asarray(Sref)
    diff = np.abs(S - Sref)
    mag = np.abs(Sref)
    peak = float(np.max(mag))
    col = np.max(mag, axis=(0, 2))
    live = col >= np.sqrt(NULL_FRACTION) * peak
    g = float(np.max(diff) / peak)
    pf = float(np.max(np.max(diff, axis=(0, 2))[live] / col[live])) if live.any() else 0.0
    print(f"{what}: complex max {g:.3e}, per-frequency {pf:.3e}", flush=True)
    assert g <= tol and pf <= tol, (what, g, pf)
