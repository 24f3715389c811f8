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


def layered_omegas(kx, ky, n_roots, pol, eps1=13.0, d1=0.5, eps2=1.0, d2=0.5):
    """Lowest frequencies of the same two-layer stack (layers normal to x)
    for Bloch number kx across the layers and wavenumber ky along them.
    pol "TE": E along z, tangential to every interface; "TM": H along z, E in
    the x-y plane with a component normal to the interfaces.  With
    q_i = sqrt(eps_i w^2 - ky^2) (imaginary in an evanescent layer):
      TE: cos(kx L) = cos(q1 d1) cos(q2 d2) - (q1/q2 + q2/q1)/2 sin(q1 d1) sin(q2 d2)
      TM: the same with (eps2 q1/(eps1 q2) + eps1 q2/(eps2 q1)) / 2."""
    def f(w):
        q1 = np.sqrt(complex(eps1 * w * w - ky * ky))
        q2 = np.sqrt(complex(eps2 * w * w - ky * ky))
        if pol == "TE":
            c = 0.5 * (q1 / q2 + q2 / q1)
        else:
            c = 0.5 * (eps2 * q1 / (eps1 * q2) + eps1 * q2 / (eps2 * q1))
        v = np.cos(q1 * d1) * np.cos(q2 * d2) - c * np.sin(q1 * d1) * np.sin(q2 * d2) - np.cos(kx * (d1 + d2))
        return v.real
    w = np.linspace(1e-6, 8.0, 80001)
    v = np.array([f(x) for x in w])
    roots = [brentq(f, w[i], w[i + 1]) for i in range(len(w) - 1) if v[i] * v[i + 1] < 0]
    return np.array(roots[:n_roots])


def layered_spectrum(kx, ky, n, eps1=13.0, d1=0.5, eps2=1.0, d2=0.5, L=1.0):
    """The n lowest eigenvalues lambda = omega^2 of the stack at the 3-D Bloch
    vector (kx, ky, 0): every mode is a TE or TM wave of some in-plane
    wavevector (ky + Gy, Gz), G a reciprocal vector along y, z."""
    g = 2.0 * np.pi / L
    w = []
    for Gy in (-2 * g, -g, 0.0, g, 2 * g):
        for Gz in (-2 * g, -g, 0.0, g, 2 * g):
            kp = np.hypot(ky + Gy, Gz)
            for pol in ("TE", "TM"):
                w.extend(layered_omegas(kx, kp, n, pol, eps1, d1, eps2, d2))
    return np.sort(np.array(w) ** 2)[:n]
