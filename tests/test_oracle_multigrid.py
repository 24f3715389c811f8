"""Pins of the multigrid oracle (Section 5.3, Alg 5.2) against what the paper
and the mathematics fix: the scalar operator against the dense Kronecker
assembly (Cor 4.4) and the closed-form symbol, the ILU factors' product
against the operator's stencil, the SAIT sweeps against the exact factor
inverse, the transfers' adjointness and order, the exact coarsest solve, the
V-cycle's contraction towards the FFT inverse, and the distributive form
against the FFT-based preconditioner solve of Alg 5.1."""
import numpy as np
import pytest

from oracle import lobpcg, mfd
from oracle import multigrid as mg

KS = [np.array([0.7, -0.4, 1.3]), np.array([np.pi, np.pi, np.pi])]


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _exact_scalar_inverse(b, N, L, k, sigma):
    """(L_k + sigma)^-1 b through the closed-form symbol sum_i |delta_i|^2."""
    sq = mfd.closed_form_symbol_sq(N, L, k)
    s = sq[2][:, None, None] + sq[1][None, :, None] + sq[0][None, None, :]
    return np.fft.ifftn(np.fft.fftn(b) / (s + sigma))


def test_scalar_operator_is_the_vector_laplacian_block():
    """Cor 4.4: A A' + B'B = diag(L_k, L_k, L_k) with L_k = B B'; the oracle's
    np.roll L_k equals both dense Kronecker-assembled blocks."""
    N, L, k = 4, 1.0, KS[0]
    n = N ** 3
    _, A, B = mfd.dense_operators(N, L, k)
    V = A @ A.conj().T + B.conj().T @ B
    BB = B @ B.conj().T
    Lk = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        Lk[:, j] = mg.scalar_laplacian(e.reshape(N, N, N), k, L / N).reshape(-1)
    scale = np.abs(Lk).max()
    for i in range(3):
        assert np.abs(V[i * n:(i + 1) * n, i * n:(i + 1) * n] - Lk).max() < 1e-12 * scale
    assert np.abs(BB - Lk).max() < 1e-12 * scale


@pytest.mark.parametrize("k", KS + [np.zeros(3)])
def test_stencil_symbol(k):
    """Plane waves are eigenvectors of the stencil with eigenvalue
    sum_i |delta_i(p_i)|^2 + sigma (the closed form, Section 5.2)."""
    N, L, sigma = 8, 1.0, 2.5
    st = mg.stencil(N, L, k, sigma)
    sq = mfd.closed_form_symbol_sq(N, L, k)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    for p in [(1, 2, 3), (0, 0, 0), (5, 7, 4)]:
        u = np.exp(2j * np.pi * (p[0] * x + p[1] * y + p[2] * z) / N)
        lam = sq[0][p[0]] + sq[1][p[1]] + sq[2][p[2]] + sigma
        assert np.allclose(mg.apply_stencil(u, *st), lam * u, rtol=1e-12, atol=1e-10 * abs(lam))


def test_ilu_factor_product():
    """ILU(0) in stencil form: L U reproduces the operator on its 7-point
    pattern; the only other entries are the fill cm_i cp_j / d at -e_i + e_j."""
    N, L, k = 8, 1.0, KS[0]
    a, cm, cp = mg.stencil(N, L, k, 1.3)
    d = mg.ilu_diagonal(a, cm, cp)
    assert abs(d - (a - np.sum(cm * cp) / d)) < 1e-12 * abs(a)
    e = np.zeros((N, N, N), dtype=np.complex128)
    e[4, 4, 4] = 1.0
    Ue = e + sum((cp[i - 1] / d) * mfd._at(e, 1, i) for i in (1, 2, 3))
    LUe = d * Ue + sum(cm[i - 1] * mfd._at(Ue, -1, i) for i in (1, 2, 3))
    Ae = mg.apply_stencil(e, a, cm, cp)
    diff = LUe - Ae
    # (L U - A) u [r] = sum_{i != j} (cm_i cp_j / d) u[r - e_i + e_j]: the
    # column of the impulse at s holds it at r = s + e_i - e_j
    expect = np.zeros_like(diff)
    for i in (1, 2, 3):
        for j in (1, 2, 3):
            if i != j:
                expect += (cm[i - 1] * cp[j - 1] / d) * mfd._at(mfd._at(e, 1, j), -1, i)
    assert np.abs(diff - expect).max() < 1e-12 * abs(a)


def test_sait_sweeps_converge_to_the_factor_inverse():
    """More Jacobi sweeps approach (L U)^-1 r (the circulant factors inverted
    exactly through their symbols), geometrically."""
    rng = np.random.default_rng(1)
    N, L, k = 8, 1.0, KS[0]
    a, cm, cp = mg.stencil(N, L, k, 0.7)
    d = mg.ilu_diagonal(a, cm, cp)
    r = _rand(rng, (N, N, N))
    th = 2 * np.pi * np.arange(N) / N
    # symbols: shift by -e_i -> e^{-i theta}, by +e_i -> e^{+i theta} under numpy's forward FFT
    ph = [np.exp(1j * th)[None, None, :], np.exp(1j * th)[None, :, None], np.exp(1j * th)[:, None, None]]
    Ls = d + sum(cm[i] * np.conj(ph[i]) for i in range(3))
    Us = 1.0 + sum((cp[i] / d) * ph[i] for i in range(3))
    exact = np.fft.ifftn(np.fft.fftn(r) / (Ls * Us))
    errs = [np.abs(mg.sait_apply(r, a, cm, cp, s) - exact).max() for s in (2, 8, 32, 64)]
    assert errs[-1] < 1e-10 * np.abs(exact).max()
    assert errs[0] > errs[1] > errs[2]


def test_transfers():
    rng = np.random.default_rng(2)
    Nc = 4
    u = _rand(rng, (Nc, Nc, Nc))
    f = _rand(rng, (2 * Nc,) * 3)
    # restriction = prolongation^T / 8
    assert abs(np.vdot(f, mg.prolong(u)) / 8.0 - np.vdot(mg.restrict(f), u)) < 1e-12 * np.abs(f).sum()
    assert np.allclose(mg.prolong(np.ones((Nc,) * 3)), 1.0)
    assert np.allclose(mg.restrict(np.ones((2 * Nc,) * 3)), 1.0)
    # second-order interpolation of a smooth periodic function, cell centres
    errs = []
    for Nc in (8, 16, 32):
        xc = (np.arange(Nc) + 0.5) / Nc
        xf = (np.arange(2 * Nc) + 0.5) / (2 * Nc)
        fc = np.cos(2 * np.pi * xc)[None, None, :] * np.ones((Nc, Nc, 1))
        ff = np.cos(2 * np.pi * xf)[None, None, :] * np.ones((2 * Nc, 2 * Nc, 1))
        errs.append(np.abs(mg.prolong(fc) - ff).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


@pytest.mark.parametrize("N", [4, 5])
def test_coarsest_level_is_exact(N):
    """A single-level hierarchy is the direct solve."""
    rng = np.random.default_rng(3)
    L, k, sigma = 1.0, KS[0], 0.4
    assert mg.levels(N) == [N]
    b = _rand(rng, (N, N, N))
    x = mg.mg_solve(b, N, L, k, sigma, cycles=1)
    assert np.abs(x - _exact_scalar_inverse(b, N, L, k, sigma)).max() < 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("k,sigma", [(KS[0], 0.0), (np.zeros(3), np.pi ** 2), (KS[1], 0.0)])
def test_vcycle_contraction(k, sigma):
    """V-cycles (2 pre- and 2 post-smoothing steps, 2 Jacobi sweeps per
    factor) converge to the exact inverse at a rate independent of N (measured
    0.15 at a generic k, 0.1 at Gamma, 0.35 at the zone corner, the same at
    N = 16, 32 and 64)."""
    rng = np.random.default_rng(4)
    L = 1.0
    rates = []
    for N in (16, 32):
        b = _rand(rng, (N, N, N))
        ex = _exact_scalar_inverse(b, N, L, k, sigma)
        hier = mg.hierarchy(N, L, k, sigma)
        x = np.zeros_like(b)
        errs = []
        for _ in range(6):
            x = mg.vcycle(x, b, 0, hier, 2, 2, 2)
            errs.append(np.linalg.norm(x - ex) / np.linalg.norm(ex))
        rates.append((errs[-1] / errs[1]) ** (1.0 / 4))
        assert rates[-1] < 0.4, (N, errs)
    assert abs(rates[1] - rates[0]) < 0.1, rates


@pytest.mark.parametrize("k", [KS[0], np.zeros(3)])
def test_distributive_form_is_the_fft_inverse(k):
    """With the scalar solves converged, the distributive solve of Section 5.3
    is (P + c)^-1, the FFT solve of Alg 5.1; with two V-cycles it is close."""
    rng = np.random.default_rng(5)
    N, L = 16, 1.0
    g = mfd.gamma_rule(N, L, k)
    c = mfd.shift_rule(L, k)
    r = _rand(rng, (3, N, N, N))
    ref = mfd.precond_solve(r, N, L, k, g, 2, c)
    x = mg.precond_solve_mg(r, N, L, k, g, c, cycles=14)
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()
    x2 = mg.precond_solve_mg(r, N, L, k, g, c, cycles=2)
    assert np.linalg.norm(x2 - ref) < 0.05 * np.linalg.norm(ref)


def test_mg_preconditioned_lobpcg_reaches_dense_bands():
    """LOBPCG preconditioned by two V-cycles of the distributive solve reaches
    the lowest eigenvalues of the dense compensated matrix (random eps)."""
    rng = np.random.default_rng(6)
    N, L, m = 6, 1.0, 6
    k = np.array([0.5, 0.1, 0.2]) * np.pi
    eps = 1.0 + 12.0 * (rng.random((N, N, N)) < 0.3)
    mu = mfd.mu_from_eps(eps)
    g = mfd.gamma_rule(N, L, k)
    n = 3 * N ** 3
    A = lambda X: mfd.apply_op(X.T.reshape(-1, 3, N, N, N), mu, k, L / N, g).reshape(-1, n).T
    T = lambda R: mg.precond_solve_mg(R.T.reshape(-1, 3, N, N, N), N, L, k, g, 0.0).reshape(-1, n).T
    X0 = _rand(rng, (n, m + 2))
    th, X, info = lobpcg.lobpcg(A, T, X0, 1e-10, maxiter=300, nconv=m)
    ev = np.linalg.eigvalsh(mfd.dense_matrix(eps, L, k, g))[:m]
    assert np.allclose(th[:m], ev, rtol=1e-10), (th[:m], ev)
