"""Plain FP64 CPU oracle of the kernel-compensated MFD operator on a general
(non-cubic) lattice.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path.

Section 2 maps a primitive cell spanned by the lattice vectors a_1, a_2, a_3
(the columns of A) onto the unit cube by x = A y, so that the derivative along
Cartesian axis i becomes sum_j b_ji d/dy_j with b = A^-1 (eq.
(coordinate_change)).  Section 4.2 ("Matrix representation on general
lattices") discretises this by replacing every D_i of eq.
(discrete_2nd_block) by

    D^_i = K^_i + i L_i,    K^_i = sum_j b_ji K_j,

with K_j the difference along grid axis j (eq. (blocks), grid step h = 1/N
of the unit cube) and L_i the unchanged averaging alpha_i D_0 along axis i.
The Bloch shift alpha is the Cartesian wave vector k.  Everything else (M_0
on the edges from the cell permittivity, the compensated matrix
A M_0 A' + gamma B'B, Alg 4.1) is as in the cubic case; ``oracle.mfd`` with
A = L I is the special case b = I / L.

Conventions are those of ``oracle.mfd``: arrays ``[z][y][x]`` with x fastest,
vector fields ``[3][z][y][x]``, paper axis i = 1, 2, 3 = numpy axis 3 - i.

Parity status: pinned by tests/test_oracle_lattice.py (dense Kronecker
assembly, the cubic special case, exact discrete symbols, the discrete de Rham
identities, and convergence to the free-photon spectrum |k + G|^2 of the
reciprocal lattice).
"""
from __future__ import annotations

import numpy as np

from . import mfd


def b_matrix(A) -> np.ndarray:
    """b = A^-1 (eq. (coordinate_change)); A holds the lattice vectors as columns."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape != (3, 3) or abs(np.linalg.det(A)) < 1e-12:
        raise ValueError("A must be a non-singular 3 x 3 matrix")
    return np.linalg.inv(A)


def cell_length(A) -> float:
    """Length scale of the cell, |det A|^(1/3): the side of the cube of equal
    volume.  It takes the place of L in the penalty and shift rules."""
    return float(abs(np.linalg.det(np.asarray(A, dtype=np.float64))) ** (1.0 / 3.0))


def K(u, j, N, order=2):
    """K_j u: the order-2K difference along grid axis j (eq. (blocks), with
    the stencil of Section 4.2.1) on the unit cube, h = 1/N:
        (K_j u)[r] = N sum_s c_s (u[r+s] - u[r+1-s])."""
    c, _ = mfd.STENCIL[order]
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(c) + 1):
        out += (c[s - 1] * N) * (mfd._at(u, s, j) - mfd._at(u, 1 - s, j))
    return out


def Kt(u, j, N, order=2):
    """K_j' u (transpose of K_j): N sum_s c_s (u[r-s] - u[r-1+s])."""
    c, _ = mfd.STENCIL[order]
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(c) + 1):
        out += (c[s - 1] * N) * (mfd._at(u, -s, j) - mfd._at(u, s - 1, j))
    return out


def Lavg(u, i, alpha, order=2):
    """L_i u = alpha_i D_0 along axis i: alpha_i sum_s d_s (u[r+s] + u[r+1-s])."""
    _, d = mfd.STENCIL[order]
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(d) + 1):
        out += (alpha[i - 1] * d[s - 1]) * (mfd._at(u, s, i) + mfd._at(u, 1 - s, i))
    return out


def Lavg_t(u, i, alpha, order=2):
    """L_i' u: alpha_i sum_s d_s (u[r-s] + u[r-1+s])."""
    _, d = mfd.STENCIL[order]
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(d) + 1):
        out += (alpha[i - 1] * d[s - 1]) * (mfd._at(u, -s, i) + mfd._at(u, s - 1, i))
    return out


def Dh(u, i, alpha, b, N, order=2):
    """D^_i u = sum_j b_ji K_j u + i L_i u (Section 4.2, general lattices)."""
    out = 1j * Lavg(u, i, alpha, order)
    for j in (1, 2, 3):
        if b[j - 1, i - 1] != 0.0:
            out += b[j - 1, i - 1] * K(u, j, N, order)
    return out


def Dh_t(u, i, alpha, b, N, order=2):
    """D^_i' u, the conjugate transpose: sum_j b_ji K_j' u - i L_i' u (b real)."""
    out = -1j * Lavg_t(u, i, alpha, order)
    for j in (1, 2, 3):
        if b[j - 1, i - 1] != 0.0:
            out += b[j - 1, i - 1] * Kt(u, j, N, order)
    return out


def curl(u, alpha, b, N, order=2):
    """A = [[0, -D^_3, D^_2], [D^_3, 0, -D^_1], [-D^_2, D^_1, 0]] (eq. (unified_mat))."""
    D = lambda f, i: Dh(f, i, alpha, b, N, order)
    return np.stack([-D(u[1], 3) + D(u[2], 2), D(u[0], 3) - D(u[2], 1), -D(u[0], 2) + D(u[1], 1)])


def curl_adj(v, alpha, b, N, order=2):
    """A', block (i, j) = (block (j, i) of A)'."""
    Dt = lambda f, i: Dh_t(f, i, alpha, b, N, order)
    return np.stack([Dt(v[1], 3) - Dt(v[2], 2), -Dt(v[0], 3) + Dt(v[2], 1), Dt(v[0], 2) - Dt(v[1], 1)])


def div(v, alpha, b, N, order=2):
    """B = [D^_1 D^_2 D^_3]."""
    return sum(Dh(v[i - 1], i, alpha, b, N, order) for i in (1, 2, 3))


def div_adj(q, alpha, b, N, order=2):
    """B' = [D^_1'; D^_2'; D^_3']."""
    return np.stack([Dh_t(q, i, alpha, b, N, order) for i in (1, 2, 3)])


def grad(phi, alpha, b, N, order=2):
    """grad = [D^_1; D^_2; D^_3]."""
    return np.stack([Dh(phi, i, alpha, b, N, order) for i in (1, 2, 3)])


def apply_op(v, mu, alpha, A, gamma, order=2, shift=0.0):
    """(A M_0 A' + gamma B'B + shift I) v on the lattice of A (eq. (Ker_comp)
    with the D^_i of Section 4.2), one band at a time; v (..., 3, N, N, N)."""
    v = np.asarray(v, dtype=np.complex128)
    if v.ndim > 4:
        return np.stack([apply_op(x, mu, alpha, A, gamma, order, shift) for x in v])
    b = b_matrix(A)
    N = v.shape[-1]
    e = mu * curl_adj(v, alpha, b, N, order)
    w = curl(e, alpha, b, N, order) + gamma * div_adj(div(v, alpha, b, N, order), alpha, b, N, order)
    return w + shift * v if shift else w


def lambda_re(x, mu, alpha, A, order=2) -> float:
    """Alg 4.1, step 2, on the lattice of A: |M_0^(1/2) A' x|^2 / |x|^2."""
    x = np.asarray(x, dtype=np.complex128)
    e = curl_adj(x, alpha, b_matrix(A), x.shape[-1], order)
    return float(np.sum(mu * np.abs(e) ** 2) / np.sum(np.abs(x) ** 2))


# ---------------------------------------------------------------------------
# Dense assembly (tiny N), by Kronecker products
# ---------------------------------------------------------------------------

def dense_blocks(N, A, alpha, order=2):
    """Dense D^_1, D^_2, D^_3 (N^3 x N^3): K_j of eq. (blocks) on the unit cube
    (h = 1/N), combined as sum_j b_ji K_j, plus i alpha_i D_0 along axis i."""
    b = b_matrix(A)
    v1, v0 = mfd.circ_generators(N, order)
    D1, D0 = mfd.circ(v1) * N, mfd.circ(v0)
    I = np.eye(N)
    kron3 = lambda p, q, r: np.kron(p, np.kron(q, r))
    Kd = [kron3(I, I, D1), kron3(I, D1, I), kron3(D1, I, I)]
    Ld = [kron3(I, I, D0), kron3(I, D0, I), kron3(D0, I, I)]
    return [sum(b[j, i] * Kd[j] for j in range(3)) + 1j * alpha[i] * Ld[i] for i in range(3)]


def dense_matrix(eps, A, alpha, gamma, order=2, shift=0.0):
    """Dense A M_0 A' + gamma B'B (+ shift I) on the lattice of A."""
    N = eps.shape[0]
    D1, D2, D3 = dense_blocks(N, A, alpha, order)
    Z = np.zeros_like(D1)
    Am = np.block([[Z, -D3, D2], [D3, Z, -D1], [-D2, D1, Z]])
    Bm = np.hstack([D1, D2, D3])
    m0 = mfd.mu_from_eps(eps).reshape(-1)
    return (Am * m0[None, :]) @ Am.conj().T + gamma * (Bm.conj().T @ Bm) + shift * np.eye(Am.shape[0])


# ---------------------------------------------------------------------------
# FFT preconditioner and the homogeneous spectrum
# ---------------------------------------------------------------------------

def symbols(N, A, alpha, order=2):
    """Symbols of D^_1, D^_2, D^_3 at every frequency p = (p_x, p_y, p_z):
    delta^_i(p) = sum_j b_ji kappa(p_j) + i alpha_i lambda(p_i), where kappa and
    lambda are the eigenvalues (eq. (diag_of_circ)) of N Circ(v_1) and Circ(v_0)
    under the forward transform exp(-2 pi i p r / N).  Returns (3, N, N, N)
    indexed [i][p_z][p_y][p_x]."""
    b = b_matrix(A)
    v1, v0 = mfd.circ_generators(N, order)
    kap = N * np.fft.ifft(v1 * N)
    lam = N * np.fft.ifft(v0)
    one = np.ones((N, N, N))
    kx, ky, kz = kap[None, None, :] * one, kap[None, :, None] * one, kap[:, None, None] * one
    lx, ly, lz = lam[None, None, :] * one, lam[None, :, None] * one, lam[:, None, None] * one
    kj, li = (kx, ky, kz), (lx, ly, lz)
    return np.stack([sum(b[j, i] * kj[j] for j in range(3)) + 1j * alpha[i] * li[i] for i in range(3)])


def precond_matrices(N, A, alpha, gamma, order=2, shift=0.0):
    """3 x 3 symbol of A A' + gamma B'B + shift I at every frequency, from the
    symbols of A and B as in the cubic case.  Shape (N, N, N, 3, 3)."""
    d1, d2, d3 = symbols(N, A, alpha, order)
    z = np.zeros((N, N, N), dtype=np.complex128)
    Ah = np.stack([np.stack([z, -d3, d2], -1), np.stack([d3, z, -d1], -1),
                   np.stack([-d2, d1, z], -1)], -2)
    Bh = np.stack([d1, d2, d3], -1)[..., None, :]
    P = Ah @ np.conj(np.swapaxes(Ah, -1, -2)) + gamma * (np.conj(np.swapaxes(Bh, -1, -2)) @ Bh)
    return P + shift * np.eye(3)


def precond_solve(r, N, A, alpha, gamma, order=2, shift=0.0, Pinv=None):
    """T = (P + shift I)^-1 r via Alg 5.1 with the symbols above."""
    if Pinv is None:
        Pinv = np.linalg.inv(precond_matrices(N, A, alpha, gamma, order, shift))
    return mfd.precond_solve(r, N, 1.0, alpha, gamma, order, shift, Pinv=Pinv)


def closed_form_spectrum(N, A, alpha, gamma, order=2):
    """Spectrum for eps = 1: every operator is a polynomial in the grid shifts,
    so the 3-D DFT diagonalises them all and the 3 x 3 symbol is
    s I + (gamma - 1) conj(delta^) delta^^T with s = |delta^|^2.  Its eigenvalues
    are s, s (physical, delta^^T x = 0) and gamma s.  Returns (physical, full),
    sorted."""
    s = np.sum(np.abs(symbols(N, A, alpha, order)) ** 2, axis=0).reshape(-1)
    return np.sort(np.concatenate([s, s])), np.sort(np.concatenate([s, s, gamma * s]))


def free_photon_omega2(A, k, count, gmax=6):
    """Continuum free-photon spectrum of the lattice (eps = 1): the plane waves
    exp(i (k + G) . x) with G = 2 pi b^T m, m integer (the reciprocal lattice of
    the columns of A), each with two transverse polarisations and
    omega^2 = |k + G|^2.  Returns the lowest ``count`` values, sorted."""
    b = b_matrix(A)
    r = np.arange(-gmax, gmax + 1)
    m = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    G = 2 * np.pi * m @ b
    w2 = np.sum((np.asarray(k, dtype=np.float64)[None, :] + G) ** 2, axis=1)
    return np.sort(np.concatenate([w2, w2]))[:count]


def bcc_primitive(a=1.0) -> np.ndarray:
    """Primitive vectors of the body-centred cubic lattice of cube side a, as
    columns: a/2 (-1, 1, 1), a/2 (1, -1, 1), a/2 (1, 1, -1)."""
    return 0.5 * a * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])


def fcc_primitive(a=1.0) -> np.ndarray:
    """Primitive vectors of the face-centred cubic lattice of cube side a, as
    columns: a/2 (0, 1, 1), a/2 (1, 0, 1), a/2 (1, 1, 0)."""
    return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
