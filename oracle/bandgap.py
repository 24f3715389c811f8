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


def band_table(evals, kpts=None) -> np.ndarray:
    """omega per (k-point, band), NaN where a band has no value.  At k = 0 the
    compensated operator's kernel is the three constant fields (dim H = 3);
    as k -> 0 two of them continue the two lowest (transverse) bands and the
    third, the constant field along the direction of approach, belongs to no
    band.  With ``kpts`` given, a row with k exactly 0 therefore drops its
    third eigenvalue: the bands above it move down by one and the last band
    has no value there."""
    lam = np.asarray(evals, dtype=np.float64)
    omega = np.sqrt(np.clip(lam, 0.0, None))
    if kpts is None:
        return omega
    at_gamma = np.all(np.asarray(kpts, dtype=np.float64).reshape(-1, 3) == 0.0, axis=1)
    out = omega.copy()
    for i in np.flatnonzero(at_gamma):
        out[i] = np.concatenate([omega[i, :2], omega[i, 3:], [np.nan]])[: omega.shape[1]]
    return out


def gap_ratios(evals, kpts=None) -> np.ndarray:
    """Ratio of every consecutive band pair (j, j + 1), j = 1 .. nbands - 1.
    evals: (nk, nbands), one row per k-point; values below zero (roundoff at
    Gamma) count as zero.  A ratio <= 0 means the two bands overlap; NaN
    marks a pair with no values (only k = 0 rows)."""
    omega = band_table(evals, kpts)
    with np.errstate(all="ignore"):
        low = np.nanmax(np.where(np.isnan(omega[:, :-1]), -np.inf, omega[:, :-1]), axis=0)
        up = np.nanmin(np.where(np.isnan(omega[:, 1:]), np.inf, omega[:, 1:]), axis=0)
        r = (up - low) / (0.5 * (up + low))
    return np.where(np.isfinite(r), r, np.nan)


def gap_ratio(evals, kpts=None):
    """(largest ratio, its lower band, 1-based)."""
    r = gap_ratios(evals, kpts)
    j = int(np.nanargmax(r))
    return float(r[j]), j + 1
