"""Helpers for comparing the HIP path with the FP64 oracle."""
from __future__ import annotations

import numpy as np

# Element-wise bar for float32 outputs against the FP64 oracle:
# |gpu - ref| <= ATOL + RTOL * |ref|.
ATOL = 1e-6
RTOL = 2e-5


def excess(gpu: np.ndarray, ref: np.ndarray, atol=ATOL, rtol=RTOL) -> np.ndarray:
    """How far each element is over the bar (<= 0 means within)."""
    return np.abs(gpu.astype(np.float64) - ref) - (atol + rtol * np.abs(ref))


def compare_outputs(got: dict, ref: dict, idx=None, atol=ATOL, rtol=RTOL):
    """Return (ok, report) for p / nu / d / w of the selected pairs."""
    rep = {}
    ok = True
    for k in ("p", "nu", "d", "w"):
        g = got[k] if idx is None else got[k][idx]
        r = ref[k]
        ex = excess(g, r, atol, rtol)
        bad = ex > 0
        rep[k] = dict(max_abs=float(np.max(np.abs(g - r))) if g.size else 0.0,
                      max_excess=float(ex.max()) if ex.size else 0.0, n_bad=int(bad.sum()), n=int(g.size))
        ok &= not bad.any()
    return ok, rep
