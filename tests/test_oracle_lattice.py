"""Pins of the general-lattice oracle (Section 2's coordinate change and
Section 4.2's D^_i = sum_j b_ji K_j + i L_i) against constructions and
closed forms it does not itself use."""
import numpy as np
import pytest

from oracle import lattice as lat
from oracle import lobpcg, mfd

RNG = np.random.default_rng(20250319)
K_GEN = np.array([0.4, -0.9, 1.3])
# a triclinic cell: A is not symmetric, so a transposed b changes the spectrum
TRICLINIC = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.4], [-0.3, 0.2, 1.2]])


def _field(N, rng=RNG):
    return rng.standard_normal((3, N, N, N)) + 1j * rng.standard_normal((3, N, N, N))


@pytest.mark.parametrize("A", [lat.bcc_primitive(), lat.fcc_primitive(), TRICLINIC])
def test_stencil_matches_kronecker_assembly(A):
    """The np.roll operator against the dense matrix built from eq. (blocks)
    by Kronecker products, on random eps and a generic k (N = 4)."""
    N = 4
    eps = 1.0 + 3.0 * RNG.random((N, N, N))
    mu = mfd.mu_from_eps(eps)
    g = 3.7
    M = lat.dense_matrix(eps, A, K_GEN, g)
    v = _field(N)
    w = lat.apply_op(v, mu, K_GEN, A, g)
    assert np.abs(M @ v.reshape(-1) - w.reshape(-1)).max() <= 1e-13 * np.abs(w).max()
    assert np.abs(M - M.conj().T).max() <= 1e-13 * np.abs(M).max()
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > -1e-10 * ev.max()          # positive semidefinite


def test_orders_match_kronecker_assembly():
    N = 8
    eps = 1.0 + RNG.random((N, N, N))
    mu = mfd.mu_from_eps(eps)
    A = lat.bcc_primitive(1.4)
    v = _field(N)
    for order in (4, 6, 8):
        D = lat.dense_blocks(N, A, K_GEN, order)
        for i in (1, 2, 3):
            want = (D[i - 1] @ v[0].reshape(-1)).reshape(N, N, N)
            got = lat.Dh(v[0], i, K_GEN, lat.b_matrix(A), N, order)
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    w = lat.apply_op(v, mu, K_GEN, A, 2.0, order=4)
    assert np.isfinite(w).all()


def test_cubic_lattice_is_the_cubic_operator():
    """A = L I gives b = I / L and reduces D^_i to the D_i of eq. (discre)."""
    N, L = 6, 1.3
    eps = 1.0 + RNG.random((N, N, N))
    mu = mfd.mu_from_eps(eps)
    v = _field(N)
    for order in (2, 4):
        a = lat.apply_op(v, mu, K_GEN, L * np.eye(3), 5.0, order)
        b = mfd.apply_op(v, mu, K_GEN, L / N, 5.0, order)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_discrete_de_rham_on_a_general_lattice():
    """curl grad = 0 and div curl = 0 still hold (Section 4.2: the K^_i are
    combinations of commuting K_j)."""
    N = 6
    A = lat.fcc_primitive(0.8)
    b = lat.b_matrix(A)
    phi = RNG.standard_normal((N, N, N)) + 1j * RNG.standard_normal((N, N, N))
    v = _field(N)
    g = lat.grad(phi, K_GEN, b, N)
    c = lat.curl(v, K_GEN, b, N)
    assert np.abs(lat.curl(g, K_GEN, b, N)).max() <= 1e-12 * np.abs(g).max() * N
    assert np.abs(lat.div(c, K_GEN, b, N)).max() <= 1e-12 * np.abs(c).max() * N


def test_homogeneous_closed_form_against_dense_eigh():
    N = 4
    A = lat.bcc_primitive()
    g = 6.0
    ev = np.linalg.eigvalsh(lat.dense_matrix(np.ones((N, N, N)), A, K_GEN, g))
    _, full = lat.closed_form_spectrum(N, A, K_GEN, g)
    assert np.abs(np.sort(ev) - full).max() <= 1e-12 * full.max()


def test_preconditioner_inverts_the_homogeneous_operator():
    N, c = 4, 0.7
    A = lat.fcc_primitive()
    g = 4.0
    r = _field(N)
    t = lat.precond_solve(r, N, A, K_GEN, g, shift=c)
    M = lat.dense_matrix(np.ones((N, N, N)), A, K_GEN, g, shift=c)
    assert np.abs(M @ t.reshape(-1) - r.reshape(-1)).max() <= 1e-12 * np.abs(r).max()


def test_symbols_tend_to_the_reciprocal_lattice_vectors():
    """delta^(p) -> i (k + G(p)), G(p) = 2 pi b^T p, for |p| << N."""
    N = 256
    A = lat.bcc_primitive()
    d = lat.symbols(N, A, K_GEN)
    b = lat.b_matrix(A)
    for p in ((1, 0, 0), (0, 2, -1), (-1, 1, 1)):
        G = 2 * np.pi * np.array(p, dtype=float) @ b
        got = d[:, p[2] % N, p[1] % N, p[0] % N]
        assert np.abs(got - 1j * (K_GEN + G)).max() <= 0.1 * np.linalg.norm(K_GEN + G)


@pytest.mark.parametrize("name, A", [("bcc", lat.bcc_primitive()), ("fcc", lat.fcc_primitive()),
                                     ("triclinic", TRICLINIC)])
def test_free_photons_converge_at_second_order(name, A):
    """eps = 1: the lowest 12 physical eigenvalues approach the free-photon
    spectrum |k + G|^2 of the reciprocal lattice, the error falling by about 4
    per halving of h.  For the triclinic cell the transposed lattice matrix
    (b_ij in place of b_ji) stays 7-10% off at every N."""
    for k in (np.zeros(3), K_GEN):
        ref = lat.free_photon_omega2(A, k, 12)
        err = []
        for N in (16, 32, 64):
            phys, _ = lat.closed_form_spectrum(N, A, k, 10.0)
            err.append(np.abs(phys[:12] - ref).max() / ref.max())
        assert err[2] < 1e-2
        assert err[1] / err[2] > 3.5
        if name == "fcc":
            assert err[0] / err[1] > 3.5
        if name == "triclinic":
            phys, _ = lat.closed_form_spectrum(64, A.T, k, 10.0)
            assert np.abs(phys[:12] - ref).max() / ref.max() > 0.05


def test_lobpcg_on_a_lattice_matches_dense_filtered_spectrum():
    """The FP64 LOBPCG oracle (lattice=A) against dense eigh of the lattice
    matrix, with Alg 4.1's filter applied to the dense eigenvectors."""
    N, m = 6, 6
    A = lat.bcc_primitive()
    eps = np.ones((N, N, N))
    eps[: N // 2, : N // 2, :] = 8.0
    k = np.array([0.9, 0.4, -0.3])
    Lc = lat.cell_length(A)
    g = mfd.gamma_rule(N, Lc, k)
    lam, X, info = lobpcg.solve_bands(eps, 1.0, k, m, tol=1e-10, lattice=A)
    assert info["converged"]
    M = lat.dense_matrix(eps, A, k, g)
    ev, V = np.linalg.eigh(M)
    mu = mfd.mu_from_eps(eps)
    ref = []
    for j in range(len(ev)):
        x = V[:, j].reshape(3, N, N, N)
        if abs(lat.lambda_re(x, mu, k, A) - ev[j]) <= 1e-8 * abs(ev[j]) + 1e-10:
            ref.append(ev[j])
        if len(ref) == m:
            break
    assert np.abs(lam - np.array(ref)).max() <= 1e-8 * max(ref)


def test_singular_lattice_is_rejected():
    with pytest.raises(ValueError):
        lat.b_matrix(np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 0.0, 1.0]]))
