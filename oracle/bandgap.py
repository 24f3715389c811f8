"""Band-gap ratio of a computed band structure (Section 6.2).

TEST INFRASTRUCTURE ONLY (see oracle/mfd.py): the product path never imports
this module.

The paper measures a complete gap between two consecutive bands by the
ratio (omega_up - omega_low) / ((omega_up + omega_low) / 2), with omega_low
the highest frequency of the lower band over the sampled Bloch vectors and
omega_up the lowest frequency of the upper one.  The eigenvalue of the
curl-curl problem is lambda = (omega / c)^2, so omega is proportional to
sqrt(lambda) and the ratio does not depend on the units.
"""
from __future__ import annotations

import numpy as np


def gap_ratios(evals) -> np.ndarray:
    """Ratio of every consecutive band pair (j, j + 1), j = 1 .. nbands - 1.
    evals: (nk, nbands), one row per k-point; values below zero (roundoff at
    Gamma) count as zero.  A ratio <= 0 means the two bands overlap."""
    lam = np.asarray(evals, dtype=np.float64)
    omega = np.sqrt(np.clip(lam, 0.0, None))
    low = omega[:, :-1].max(axis=0)
    up = omega[:, 1:].min(axis=0)
    return (up - low) / (0.5 * (up + low))


def gap_ratio(evals):
    """(largest ratio, its lower band, 1-based)."""
    r = gap_ratios(evals)
    j = int(np.argmax(r))
    return float(r[j]), j + 1
