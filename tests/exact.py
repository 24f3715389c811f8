"""Closed-form references that hold for the continuum problem (no part of the
oracle or of the library)."""
import numpy as np
from scipy.optimize import brentq


def bragg_omegas(kx, n_roots, eps1=13.0, d1=0.5, eps2=1.0, d2=0.5):
    """Lowest frequencies (units c / L, L = d1 + d2) of the periodic two-layer
    stack at Bloch number kx along the layering: the roots in omega of the
    transfer-matrix dispersion relation
    cos(kx L) = cos(n1 w d1) cos(n2 w d2) - (n1/n2 + n2/n1)/2 sin(n1 w d1) sin(n2 w d2).
    Normal incidence: both polarisations share these frequencies."""
    n1, n2 = np.sqrt(eps1), np.sqrt(eps2)

    def f(w):
        return (np.cos(n1 * w * d1) * np.cos(n2 * w * d2)
                - 0.5 * (n1 / n2 + n2 / n1) * np.sin(n1 * w * d1) * np.sin(n2 * w * d2) - np.cos(kx * (d1 + d2)))
    w = np.linspace(1e-6, 8.0, 80001)
    v = f(w)
    roots = [brentq(f, w[i], w[i + 1]) for i in range(len(w) - 1) if v[i] * v[i + 1] < 0]
    return np.array(roots[:n_roots])
