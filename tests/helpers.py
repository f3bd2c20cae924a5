"""Shared test helpers: device upload of seeded inputs and the parity metric."""
from __future__ import annotations

import numpy as np

from workloads import FIELDS, flatten


def e_inf(I, Iref) -> float:
    """max |I - I_ref| / max I_ref over the grid (the parity metric)."""
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


def error_report(I, Iref) -> dict:
    """e_inf (gate), L2 relative, per-direction peak-normalised max, and per-point relative
    error on bins holding at least 1e-2 of the peak."""
    I = np.asarray(I, np.float64)
    Iref = np.asarray(Iref, np.float64)
    peak = float(np.max(Iref))
    diff = np.abs(I - Iref)
    per_dir = [float(np.max(diff[d]) / max(np.max(Iref[d]), 1e-300)) for d in range(Iref.shape[0])]
    big = Iref >= 1e-2 * peak
    col = np.maximum(np.max(Iref, axis=0), 1e-300)
    return {"e_inf": float(np.max(diff) / peak),
            "per_frequency_max": float(np.max(np.max(diff, axis=0) / col)),
            "per_frequency_max_top_quarter": float(np.max((np.max(diff, axis=0) / col)[-max(1, Iref.shape[1] // 4):])),
            "l2_rel": float(np.linalg.norm(I - Iref) / np.linalg.norm(Iref)),
            "per_direction_max": float(max(per_dir)),
            "per_point_rel_max_bins_ge_1e-2_peak": float(np.max(diff[big] / Iref[big])) if big.any() else 0.0}
