"""Parity metrics between a device spectrum and the oracle's (test infrastructure only,
like the rest of this package: used by tests/, the smoke check and the bench's parity legs).

The gate, at relative tolerance 1e-4 on the spectrum, is two numbers:
  * e_inf = max |I - I_ref| / max I_ref over the grid, and
  * the per-frequency error: for every frequency, max over directions of |I - I_ref|
    divided by that frequency's own oracle peak over directions.
The second is needed because the coherent bins (low omega, F close to N in Eq. 12) sit
about N above the incoherent ones (F close to sqrt N): normalised by the global peak
alone, an error anywhere in the incoherent band -- even a band set to zero -- would be
invisible.  Frequencies whose oracle peak is below NULL_FRACTION of the global peak are
exact nulls (e.g. omega = 0 of a closed orbit); the per-frequency error skips them and
e_inf still covers them.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-4
NULL_FRACTION = 1e-12


def error_report(I, Iref, ks=None) -> dict:
    """e_inf and per_frequency_max (the gate), plus L2 relative, per-direction
    peak-normalised max and per-point relative error on bins of at least 1e-2 of the peak.
    ks: grid indices of the columns, to report the per-frequency error by index mod 16
    (0 is a lane's FP64-seeded frequency, 1..15 come out of the frequency recurrence)."""
    I = np.asarray(I, np.float64)
    Iref = np.asarray(Iref, np.float64)
    if I.ndim == 1:
        I, Iref = I[None, :], Iref[None, :]
    peak = float(np.max(Iref))
    diff = np.abs(I - Iref)
    col = np.max(Iref, axis=0)
    live = col >= NULL_FRACTION * peak
    per_col = np.zeros(col.shape)
    per_col[live] = np.max(diff, axis=0)[live] / col[live]
    row = np.max(Iref, axis=1)
    rlive = row >= NULL_FRACTION * peak
    per_row = np.zeros(row.shape)
    per_row[rlive] = np.max(diff, axis=1)[rlive] / row[rlive]
    big = Iref >= 1e-2 * peak
    nq = max(1, Iref.shape[1] // 4)
    rep = {"e_inf": float(np.max(diff) / peak) if peak > 0 else float(np.max(diff)),
           "per_frequency_max": float(np.max(per_col)) if per_col.size else 0.0,
           "per_frequency_max_top_quarter": float(np.max(per_col[-nq:])),
           "null_columns_skipped": int(np.count_nonzero(~live)),
           "l2_rel": float(np.linalg.norm(I - Iref) / np.linalg.norm(Iref)) if peak > 0 else 0.0,
           "per_direction_max": float(np.max(per_row)) if per_row.size else 0.0,
           "per_point_rel_max_bins_ge_1e-2_peak": float(np.max(diff[big] / Iref[big])) if big.any() else 0.0,
           "abs_max": float(np.max(diff)), "peak": peak}
    if ks is not None:
        ks = np.asarray(ks)
        rep["per_frequency_max_by_k_mod_16"] = {int(m): float(np.max(per_col[ks % 16 == m]))
                                                for m in np.unique(ks % 16)}
    return rep


def passes(rep: dict, tol: float = TOL) -> bool:
    """Both parts of the gate hold."""
    return rep["e_inf"] <= tol and rep["per_frequency_max"] <= tol
