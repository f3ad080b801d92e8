"""Force-error summaries used to report accuracy against a reference sum."""
from __future__ import annotations

import math

import numpy as np


def force_errors(a: np.ndarray, ref: np.ndarray) -> dict:
    """Force-error summaries of `a` against `ref` (rows are particles).

    rms  = sqrt(sum |da|^2 / sum |a_ref|^2)
    max  = max |da| / sqrt(mean |a_ref|^2)
    paper = sum |da| / sum |a_ref| (Sect. 6.1)
    """
    da = np.linalg.norm(a - ref, axis=1)
    ar = np.linalg.norm(ref, axis=1)
    den = float(np.sum(ar * ar))
    rms = math.sqrt(float(np.sum(da * da)) / den) if den > 0 else 0.0
    mx = float(np.max(da)) / math.sqrt(den / len(ar)) if den > 0 else 0.0
    paper = float(np.sum(da)) / float(np.sum(ar)) if np.sum(ar) > 0 else 0.0
    rel = da / np.where(ar > 0, ar, 1.0)
    return dict(rms=rms, max=mx, paper=paper, median_rel=float(np.median(rel)),
                max_rel=float(np.max(rel)))
