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
