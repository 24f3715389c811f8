"""Plain FP64 CPU oracle of the learned warm start: the training target built
from converged blocks, the multilayer perceptron, its gradient, and Adam.

TEST INFRASTRUCTURE ONLY (see oracle/mfd.py): the product path never imports
this module, and it shares no code with the HIP kernels.

The paper has no learned component.  What is computed here is the warm start
of the band solve along a k-path: from the converged blocks X_{j-1}, X_j at
two previous k-points, predict the block at the next one as a combination
Y_j C of the orthonormal basis Y_j of span[X_j, X_{j-1}].

* target (given X_{j+1}): C* = Y_j^H X_{j+1} Q, where Q is the unitary matrix
  closest to aligning X_{j+1} with X_j (orthogonal Procrustes: Q = U V^H for
  X_{j+1}^H X_j = U S V^H).  Q removes the arbitrary phases and in-cluster
  rotations of the eigensolver's output, so C* is a smooth function of k.
* network: x -> h1 = gelu(W1 x + b1) -> h2 = gelu(W2 h1 + b2)
  -> h3 = gelu(W3 h2 + b3) -> y = W4 h3 + b4, gelu(z) = z Phi(z) with the
  exact normal CDF Phi(z) = (1 + erf(z / sqrt 2)) / 2.
* loss: mean squared error over batch and outputs.
* Adam (Kingma and Ba): bias-corrected first and second moments.

Parameters are one flat vector: for each layer W (out x in, row-major) then b.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def layer_shapes(nin, nhidden, nlayers, nout):
    """[(out, in)] of the nlayers hidden layers and the output layer."""
    dims = [nin] + [nhidden] * nlayers + [nout]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(theta, shapes):
    """Views (W, b) per layer of the flat parameter vector."""
    out, off = [], 0
    for o, i in shapes:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(theta, shapes, X):
    """X: (batch, nin).  Returns (Y (batch, nout), cache of pre-activations
    and layer inputs)."""
    layers = unpack(theta, shapes)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a, cache


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def loss_and_grad(theta, shapes, X, T):
    """Mean squared error of the network on (X, T) and its gradient with
    respect to the flat parameters (backpropagation through the layers)."""
    Y, cache = forward(theta, shapes, X)
    B, O = Y.shape
    dA = 2.0 * (Y - T) / (B * O)
    grads = []
    nl = len(shapes)
    layers = unpack(theta, shapes)
    for li in range(nl - 1, -1, -1):
        a_in, z = cache[li]
        dZ = dA if li == nl - 1 else dA * gelu_grad(z)
        W, _ = layers[li]
        grads.append((dZ.T @ a_in, dZ.sum(axis=0)))
        dA = dZ @ W
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in reversed(grads)])
    return mse(Y, T), g


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step count t (1-based).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP64."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def orth_basis(Xb, Xa):
    """Orthonormal basis Y of span[Xb, Xa] (columns in that order) from the
    Cholesky factor of the Gram matrix: Y = [Xb Xa] R^-1."""
    Z = np.concatenate([Xb, Xa], axis=1)
    R = np.linalg.cholesky(Z.conj().T @ Z).conj().T
    return Z @ np.linalg.inv(R), R


def procrustes(Xc, Xb):
    """Unitary Q minimising |Xc Q - Xb|_F."""
    U, _, Vh = np.linalg.svd(Xc.conj().T @ Xb)
    return U @ Vh


def warm_target(Xa, Xb, Xc):
    """C* = Y^H Xc Q for Y = orth[Xb, Xa] (Xa = X_{j-1}, Xb = X_j,
    Xc = X_{j+1}, each n x m).  Returns (C* (2m x m), Y)."""
    Y, _ = orth_basis(Xb, Xa)
    return Y.conj().T @ Xc @ procrustes(Xc, Xb), Y


def c_to_reals(C):
    """2m x m complex -> 4 m^2 reals, (re, im) interleaved, row-major."""
    return np.stack([C.real, C.imag], axis=-1).ravel()


def reals_to_c(r, m):
    r = np.asarray(r).reshape(2 * m, m, 2)
    return r[..., 0] + 1j * r[..., 1]


def features(k_prev, k_next, lam_j, lam_jm1, C_j, L=1.0):
    """Network input for predicting C*_{j+1}: k_{j+1} L / pi, (k_{j+1} - k_j) L / pi,
    the two previous sets of Ritz values over (2 pi / L)^2, and C*_j as reals."""
    s = L / np.pi
    lam_scale = (2.0 * np.pi / L) ** 2
    return np.concatenate([np.asarray(k_next) * s, (np.asarray(k_next) - np.asarray(k_prev)) * s,
                           np.asarray(lam_j) / lam_scale, np.asarray(lam_jm1) / lam_scale, c_to_reals(C_j)])
