"""Shared helpers of the GPU parity tests (inputs only; no method arithmetic)."""
import numpy as np


def rand_eps(rng, N, fill=0.3):
    return 1.0 + 12.0 * (rng.random((N, N, N)) < fill)


def rand_block(rng, nb, N):
    return rng.standard_normal((nb, 3, N, N, N)) + 1j * rng.standard_normal((nb, 3, N, N, N))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())
