"""Pins of the learned warm start's CPU oracle (oracle/mlp.py): finite
differences, closed forms, symmetries and brute force."""
import numpy as np
import pytest

from oracle import mlp


def rand_unitary(rng, m):
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def test_gelu_values_and_symmetry():
    z = np.linspace(-6, 6, 121)
    g = mlp.gelu(z)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # Phi(-z) = 1 - Phi(z)  =>  gelu(-z) = gelu(z) - z
    assert np.allclose(mlp.gelu(-z), g - z, atol=1e-15)
    # far tails: gelu(z) -> z for z >> 0, -> 0 for z << 0
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-13
    assert abs(mlp.gelu(np.array([-8.0]))[0]) < 1e-13
    # z Phi(z) at z = 1 with Phi(1) = 0.8413447460685429 (normal table)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_gelu_grad_finite_difference():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("nlayers", [0, 1, 3])
def test_gradient_central_differences(nlayers):
    rng = np.random.default_rng(3)
    shapes = mlp.layer_shapes(7, 5, nlayers, 4)
    theta = rng.standard_normal(mlp.n_params(shapes)) * 0.5
    X = rng.standard_normal((3, 7))
    T = rng.standard_normal((3, 4))
    _, g = mlp.loss_and_grad(theta, shapes, X, T)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(theta + e, shapes, X, T)[0] - mlp.loss_and_grad(theta - e, shapes, X, T)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_linear_layer_gradient_closed_form():
    """No hidden layer: y = W x + b, L = mean (y - t)^2, dL/dW = 2/(BO) (Y - T)^T X."""
    rng = np.random.default_rng(4)
    shapes = mlp.layer_shapes(6, 0, 0, 3)
    theta = rng.standard_normal(mlp.n_params(shapes))
    X = rng.standard_normal((5, 6))
    T = rng.standard_normal((5, 3))
    W = theta[:18].reshape(3, 6)
    b = theta[18:]
    Y = X @ W.T + b
    loss, g = mlp.loss_and_grad(theta, shapes, X, T)
    assert abs(loss - np.mean((Y - T) ** 2)) < 1e-14
    assert np.allclose(g[:18].reshape(3, 6), 2.0 / 15 * (Y - T).T @ X, rtol=1e-13)
    assert np.allclose(g[18:], 2.0 / 15 * (Y - T).sum(0), rtol=1e-13)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are m = g and
    v = g^2 at every step, so each step moves by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    th = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in (1, 2, 3):
        th_new, m, v = mlp.adam_step(th, g, m, v, t, lr=0.01)
        assert np.allclose(th_new - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        th = th_new


def test_bf16_round_brute_force():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32),
                        np.float32([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.5, 0.0])])
    r = mlp.bf16_round(x)
    for xi, ri in zip(x, r):
        # bracketing bfloat16 values: truncate the low 16 bits, and the next one up in magnitude
        u = np.float32(xi).view(np.uint32)
        lo = np.uint32(u & 0xFFFF0000).view(np.float32)
        hi = np.uint32((u & 0xFFFF0000) + 0x10000).view(np.float32)
        dlo, dhi = abs(float(xi) - float(lo)), abs(float(hi) - float(xi))
        if dlo < dhi:
            want = lo
        elif dhi < dlo:
            want = hi
        else:   # tie: even last mantissa bit of the bfloat16
            want = lo if ((int(u) >> 16) & 1) == 0 else hi
        assert ri == float(want), (xi, ri, want)
    assert mlp.bf16_round(np.float32([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp.bf16_round(np.float32([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def _blocks(rng, n=60, m=4):
    def cplx(*s):
        return rng.standard_normal(s) + 1j * rng.standard_normal(s)
    Xb = np.linalg.qr(cplx(n, m))[0]
    Xa = np.linalg.qr(Xb + 0.1 * cplx(n, m))[0]
    Xc = np.linalg.qr(Xb + 0.1 * cplx(n, m))[0]
    return Xa, Xb, Xc


def test_orth_basis():
    rng = np.random.default_rng(6)
    Xa, Xb, _ = _blocks(rng)
    Y, _ = mlp.orth_basis(Xb, Xa)
    assert np.allclose(Y.conj().T @ Y, np.eye(8), atol=1e-12)
    Z = np.concatenate([Xb, Xa], axis=1)
    assert np.allclose(Y @ (Y.conj().T @ Z), Z, atol=1e-12)       # same span
    assert np.allclose(Y[:, :4] @ (Y[:, :4].conj().T @ Xb), Xb, atol=1e-12)   # Xb first


def test_procrustes_brute_force():
    rng = np.random.default_rng(7)
    _, Xb, Xc = _blocks(rng)
    Q = mlp.procrustes(Xc, Xb)
    assert np.allclose(Q.conj().T @ Q, np.eye(4), atol=1e-12)
    best = np.linalg.norm(Xc @ Q - Xb)
    for _ in range(2000):
        U = rand_unitary(rng, 4)
        assert np.linalg.norm(Xc @ U - Xb) >= best - 1e-12
    # small perturbations of the optimum do not improve it
    for _ in range(200):
        H = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        H = 1e-3 * (H - H.conj().T)
        U = Q @ np.linalg.qr(np.eye(4) + H)[0]
        assert np.linalg.norm(Xc @ U - Xb) >= best - 1e-12


def test_warm_target_gauge_invariance_and_exactness():
    rng = np.random.default_rng(8)
    Xa, Xb, Xc = _blocks(rng)
    C, Y = mlp.warm_target(Xa, Xb, Xc)
    # an eigensolver may return X_{j+1} U for any unitary U: the target is unchanged
    C2, _ = mlp.warm_target(Xa, Xb, Xc @ rand_unitary(rng, 4))
    assert np.allclose(C, C2, atol=1e-12)
    # when X_{j+1} lies in span Y, Y C* reproduces the aligned block exactly
    Xin = Y @ np.linalg.qr(rng.standard_normal((8, 4)) + 1j * rng.standard_normal((8, 4)))[0]
    Cin, _ = mlp.warm_target(Xa, Xb, Xin)
    assert np.allclose(Y @ Cin, Xin @ mlp.procrustes(Xin, Xb), atol=1e-12)
    # no motion: X_{j+1} = X_j gives C* = [I; 0]
    C0, _ = mlp.warm_target(Xa, Xb, Xb)
    assert np.allclose(C0, np.vstack([np.eye(4), np.zeros((4, 4))]), atol=1e-12)


def test_features_layout():
    C = np.arange(8 * 4).reshape(8, 4) + 1j * np.arange(8 * 4).reshape(8, 4) * 2
    f = mlp.features([0.0, 0.0, 0.0], [np.pi, 0.0, 0.0], [4 * np.pi ** 2] * 4, [0.0] * 4, C)
    assert f.shape == (6 + 8 + 64,)
    assert np.allclose(f[:6], [1, 0, 0, 1, 0, 0])
    assert np.allclose(f[6:10], 1.0) and np.allclose(f[10:14], 0.0)
    assert np.allclose(mlp.reals_to_c(f[14:], 4), C)
