"""Plain FP64 CPU oracle of the kernel-compensated MFD Maxwell operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link this module; only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, table or constant with the HIP path.

Every function follows the paper (arXiv 2503.19379) directly and cites the
passage it writes out.  Conventions (the paper leaves them implicit):

* grid functions are arrays ``[z][y][x]`` with x the fastest index, which is
  what the Kronecker order K_1 = I (x) I (x) D_1/h of eq. (blocks) implies;
  paper axis i = 1, 2, 3 (x, y, z) is numpy axis 3 - i of an (N, N, N) array;
* a vector field is an array ``[3][z][y][x]`` ordered (v_1, v_2, v_3), as in
  eq. (discrete_2nd_block);
* the Bloch shift alpha of Section 4.1.2 is the wave vector k (Cartesian, in
  units of 1/L);
* the unknown lives on faces F_h and M_0 (from eps^-1) on edges E_h
  (eqs. (DoFs_grid), (original_FD_formulation)).

Parity status: every function here is pinned by tests/test_oracle_*.py
(closed forms, dense assembly, exact identities, the paper's Tables iso1-iso4).
"""
from __future__ import annotations

import numpy as np

# Table FD_1D (Section 4.1.3): order-2K one-dimensional stencils
# (c_1..c_K) for the derivative and (d_1..d_K) for the midpoint value.
# The table prints c_1 = 25/64 for K = 3; the consistency condition
# sum_s (2s-1) c_s = 1 (exactness on linear functions) holds only for 75/64,
# which is the value used here.
STENCIL = {
    2: ((1.0,), (0.5,)),
    4: ((9.0 / 8.0, -1.0 / 24.0), (9.0 / 16.0, -1.0 / 16.0)),
    6: ((75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0),
        (75.0 / 128.0, -25.0 / 256.0, 3.0 / 256.0)),
    8: ((1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0),
        (1225.0 / 2048.0, -245.0 / 2048.0, 49.0 / 2048.0, -5.0 / 2048.0)),
}


def _axis(i: int, ndim: int) -> int:
    """numpy axis of paper axis i (1 = x, 2 = y, 3 = z) for a [...][z][y][x] array."""
    return ndim - i


def _at(u: np.ndarray, s: int, i: int) -> np.ndarray:
    """u[r + s] along paper axis i, periodic (Section 4.1.1: evaluation at x
    equals evaluation at x + e_n)."""
    return np.roll(u, -s, axis=_axis(i, u.ndim))


def D(u: np.ndarray, i: int, alpha, h: float, order: int = 2) -> np.ndarray:
    """D_i u = (K_i + i L_i) u  (eqs. (discre), (blocks)).

    K_i applies Circ(v_1^(k))/h and L_i applies alpha_i Circ(v_0^(k)) along
    axis i, with v_1^(k) = (-c_1, c_1, c_2, .., c_k, 0, .., -c_k, .., -c_2) and
    v_0^(k) = (d_1, d_1, d_2, .., d_k, 0, .., d_k, .., d_2) (Section 4.2.1).
    Row r of Circ(a) holds a shifted right by r (eq. (circ_def)), so
    (Circ(a) u)[r] = sum_t a[t] u[r + t], i.e.
        (D_i u)[r] = (1/h) sum_s c_s (u[r+s] - u[r+1-s])
                     + i alpha_i sum_s d_s (u[r+s] + u[r+1-s]).
    """
    c, d = STENCIL[order]
    a = complex(alpha[i - 1])
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(c) + 1):
        fwd = _at(u, s, i)
        bwd = _at(u, 1 - s, i)
        out += (c[s - 1] / h) * (fwd - bwd) + 1j * a * d[s - 1] * (fwd + bwd)
    return out


def Dt(u: np.ndarray, i: int, alpha, h: float, order: int = 2) -> np.ndarray:
    """D_i' u, the conjugate transpose of D_i (Section 3: ' is the conjugate
    transpose).  Circ(a)^T has (Circ(a)^T u)[r] = sum_t a[t] u[r - t], so
        (D_i' u)[r] = (1/h) sum_s c_s (u[r-s] - u[r-1+s])
                      - i alpha_i sum_s d_s (u[r-s] + u[r-1+s])."""
    c, d = STENCIL[order]
    a = complex(alpha[i - 1])
    out = np.zeros(u.shape, dtype=np.complex128)
    for s in range(1, len(c) + 1):
        bwd = _at(u, -s, i)
        fwd = _at(u, s - 1, i)
        out += (c[s - 1] / h) * (bwd - fwd) - 1j * a * d[s - 1] * (bwd + fwd)
    return out


# ---------------------------------------------------------------------------
# Block operators of eq. (discrete_2nd_block) and their adjoints (Section 4.3)
# ---------------------------------------------------------------------------

def grad(phi, alpha, h, order=2):
    """grad_alpha = [D_1; D_2; D_3] : N_h -> E_h  (eq. (discrete_2nd_block))."""
    return np.stack([D(phi, i, alpha, h, order) for i in (1, 2, 3)])


def curl(u, alpha, h, order=2):
    """A = curl_alpha = [[0, -D_3, D_2], [D_3, 0, -D_1], [-D_2, D_1, 0]] : E_h -> F_h."""
    return np.stack([
        -D(u[1], 3, alpha, h, order) + D(u[2], 2, alpha, h, order),
        D(u[0], 3, alpha, h, order) - D(u[2], 1, alpha, h, order),
        -D(u[0], 2, alpha, h, order) + D(u[1], 1, alpha, h, order),
    ])


def curl_adj(v, alpha, h, order=2):
    """A' = curl_alpha' : F_h -> E_h, the block conjugate transpose of curl:
    block (i, j) of A' is (block (j, i) of A)'."""
    return np.stack([
        Dt(v[1], 3, alpha, h, order) - Dt(v[2], 2, alpha, h, order),
        -Dt(v[0], 3, alpha, h, order) + Dt(v[2], 1, alpha, h, order),
        Dt(v[0], 2, alpha, h, order) - Dt(v[1], 1, alpha, h, order),
    ])


def div(v, alpha, h, order=2):
    """B = div_alpha = [D_1 D_2 D_3] : F_h -> C_h."""
    return D(v[0], 1, alpha, h, order) + D(v[1], 2, alpha, h, order) + D(v[2], 3, alpha, h, order)


def div_adj(q, alpha, h, order=2):
    """B' = [D_1'; D_2'; D_3'] : C_h -> F_h."""
    return np.stack([Dt(q, i, alpha, h, order) for i in (1, 2, 3)])


def mu_from_eps(eps: np.ndarray) -> np.ndarray:
    """Diagonal of M_0 on the edges from a cell-centred permittivity grid
    (Section 4.4).  An edge is shared by four cells; its entry is the
    harmonic average of eps^-1 over them, 4 / (sum of the four eps), which is
    eps^-1 where the four cells agree.

    Edge e_1[c, b, a] sits at ((a+1/2)h, bh, ch) and touches the cells
    (a, b or b-1, c or c-1); likewise for e_2 (x and z neighbours) and e_3
    (x and y neighbours).  Returns mu with shape (3, N, N, N)."""
    eps = np.asarray(eps, dtype=np.float64)

    def back(u, i):  # u[r - 1] along paper axis i
        return _at(u, -1, i)

    mu = np.empty((3,) + eps.shape)
    mu[0] = 4.0 / (eps + back(eps, 2) + back(eps, 3) + back(back(eps, 2), 3))
    mu[1] = 4.0 / (eps + back(eps, 1) + back(eps, 3) + back(back(eps, 1), 3))
    mu[2] = 4.0 / (eps + back(eps, 1) + back(eps, 2) + back(back(eps, 1), 2))
    return mu


def gamma_rule(N: int, L: float, k, literal: bool = False) -> float:
    """Penalty number of eq. (pnt_number), gamma = 2 max{1/h, |alpha|^-2}.

    1/h carries a length, so the rule depends on units.  The paper computes
    with lattice constant 2 pi (Section 6.1); in those units h = 2 pi / N and
    |alpha| becomes L |k| / (2 pi), giving gamma = 2 max{N / (2 pi),
    (2 pi / (L |k|))^2}.  Near Gamma the |k|^-2 term grows without bound and
    FP64 rounding of gamma B'B x then dominates the residual of a converged
    band; |k| is therefore clamped below at K_BALL = pi / (2 L) (inside that
    ball the one compensation mode gamma |k|^2 may fall among the wanted bands
    and is removed by Alg 4.1).  ``literal=True`` applies the formula in the
    units of L with no clamp: 2 max{N / L, |k|^-2}."""
    kn = float(np.linalg.norm(np.asarray(k, dtype=np.float64)))
    if literal:
        a, b = N / L, (kn ** -2 if kn > 0 else 0.0)
    else:
        kc = max(kn, k_ball(L))
        a, b = N / (2 * np.pi), (2 * np.pi / (L * kc)) ** 2
    return 2.0 * max(a, b)


def k_ball(L: float) -> float:
    """Radius pi / (2 L) of the neighbourhood of Gamma where the shift of
    Remark 5.1 is used and the penalty rule is clamped."""
    return np.pi / (2.0 * L)


def shift_rule(L: float, k) -> float:
    """Shift c of Remark 5.1.  A A' + gamma B'B is singular at alpha = 0 and its
    smallest eigenvalue is |k|^2 near it; the shifted problem is solved (and c
    subtracted) for |k| < pi / (2 L), with c = (pi / L)^2.  The eigenpairs do not
    depend on c."""
    return (np.pi / L) ** 2 if float(np.linalg.norm(k)) < k_ball(L) else 0.0


def apply_op(v, mu, alpha, h, gamma, order=2, shift=0.0):
    """(A M_0 A' + gamma B'B + shift I) v for v of shape (..., 3, N, N, N)
    (eq. (Ker_comp); the shift of Remark 5.1).  Written as the composition of
    the block operators above, one band at a time."""
    v = np.asarray(v, dtype=np.complex128)
    if v.ndim > 4:
        return np.stack([apply_op(x, mu, alpha, h, gamma, order, shift) for x in v])
    e = mu * curl_adj(v, alpha, h, order)
    w = curl(e, alpha, h, order) + gamma * div_adj(div(v, alpha, h, order), alpha, h, order)
    if shift:
        w = w + shift * v
    return w


def lambda_re(x, mu, alpha, h, order=2) -> float:
    """Alg 4.1, step 2: |M_0^(1/2) A' x|^2 / |x|^2."""
    e = curl_adj(np.asarray(x, dtype=np.complex128), alpha, h, order)
    return float(np.sum(mu * np.abs(e) ** 2) / np.sum(np.abs(x) ** 2))


# ---------------------------------------------------------------------------
# Dense assembly (tiny N): an independent construction by Kronecker products
# ---------------------------------------------------------------------------

def circ(a) -> np.ndarray:
    """Circ(a) of eq. (circ_def): row r is a shifted right r times."""
    a = np.asarray(a)
    N = a.shape[0]
    idx = (np.arange(N)[None, :] - np.arange(N)[:, None]) % N
    return a[idx]


def circ_generators(N: int, order: int = 2):
    """Generating vectors v_1^(k), v_0^(k) of D_1^(k), D_0^(k) (Section 4.2.1)."""
    c, d = STENCIL[order]
    K = len(c)
    if N < 2 * K:
        raise ValueError("grid too small for the stencil")
    v1 = np.zeros(N)
    v0 = np.zeros(N)
    v1[0] = -c[0]
    v0[0] = d[0]
    for s in range(1, K + 1):
        v1[s] += c[s - 1]
        v0[s] += d[s - 1]
    for s in range(2, K + 1):
        v1[N - s + 1] -= c[s - 1]
        v0[N - s + 1] += d[s - 1]
    return v1, v0


def dense_blocks(N, L, alpha, order=2):
    """Dense D_1, D_2, D_3 (N^3 x N^3) from eqs. (discre), (blocks):
    K_1 = I (x) I (x) D_1/h, K_2 = I (x) D_1/h (x) I, K_3 = D_1/h (x) I (x) I,
    and the same with alpha_i D_0 for L_i."""
    h = L / N
    v1, v0 = circ_generators(N, order)
    D1, D0 = circ(v1), circ(v0)
    I = np.eye(N)
    kron3 = lambda a, b, c: np.kron(a, np.kron(b, c))
    K = [kron3(I, I, D1 / h), kron3(I, D1 / h, I), kron3(D1 / h, I, I)]
    Lm = [kron3(I, I, alpha[0] * D0), kron3(I, alpha[1] * D0, I), kron3(alpha[2] * D0, I, I)]
    return [K[i] + 1j * Lm[i] for i in range(3)]


def dense_operators(N, L, alpha, order=2):
    """Dense (grad, curl, div) of eq. (discrete_2nd_block)."""
    D1, D2, D3 = dense_blocks(N, L, alpha, order)
    Z = np.zeros_like(D1)
    G = np.vstack([D1, D2, D3])
    A = np.block([[Z, -D3, D2], [D3, Z, -D1], [-D2, D1, Z]])
    B = np.hstack([D1, D2, D3])
    return G, A, B


def dense_matrix(eps, L, alpha, gamma, order=2, shift=0.0, parts=False):
    """Dense compensated matrix A M_0 A' + gamma B'B (+ shift I), eq. (Ker_comp).
    With ``parts=True`` also returns (A M_0 A', B'B)."""
    N = eps.shape[0]
    _, A, B = dense_operators(N, L, alpha, order)
    m0 = mu_from_eps(eps).reshape(-1)
    AMA = (A * m0[None, :]) @ A.conj().T
    BB = B.conj().T @ B
    M = AMA + gamma * BB + shift * np.eye(A.shape[0])
    return (M, AMA, BB) if parts else M


# ---------------------------------------------------------------------------
# FFT preconditioner (Section 5.1 eq. (penalised_marix), Section 5.2 Alg 5.1)
# ---------------------------------------------------------------------------

def symbols(N, L, alpha, order=2):
    """Eigenvalues of D_1, D_2, D_3 under the Fourier basis (eq. (diag_of_circ)):
    xi_p = sum_t a[t] w^(p t), w = exp(2 pi i / N), for the generating vector
    a = v_1^(k)/h + i alpha_i v_0^(k).  Returns delta with shape (3, N):
    delta[i-1][p] is the symbol of D_i at frequency p along axis i.  This
    matches the forward transform u_hat(p) = sum_r u[r] exp(-2 pi i p r / N)
    (numpy.fft.fft)."""
    h = L / N
    v1, v0 = circ_generators(N, order)
    out = np.empty((3, N), dtype=np.complex128)
    for i in range(3):
        a = v1 / h + 1j * alpha[i] * v0
        out[i] = N * np.fft.ifft(a)
    return out


def precond_matrices(N, L, alpha, gamma, order=2, shift=0.0):
    """The 3 x 3 symbol of P + shift I = A A' + gamma B'B + shift I at every
    frequency (eq. (penalised_marix)), built from the symbols of A and B:
    A_hat = [[0, -d3, d2], [d3, 0, -d1], [-d2, d1, 0]], B_hat = [d1 d2 d3].
    Returns an array (N, N, N, 3, 3) indexed [p_z][p_y][p_x]."""
    dl = symbols(N, L, alpha, order)
    d1 = dl[0][None, None, :] * np.ones((N, N, N))
    d2 = dl[1][None, :, None] * np.ones((N, N, N))
    d3 = dl[2][:, None, None] * np.ones((N, N, N))
    z = np.zeros((N, N, N), dtype=np.complex128)
    Ah = np.stack([np.stack([z, -d3, d2], -1), np.stack([d3, z, -d1], -1),
                   np.stack([-d2, d1, z], -1)], -2)
    Bh = np.stack([d1, d2, d3], -1)[..., None, :]          # 1 x 3
    P = Ah @ np.conj(np.swapaxes(Ah, -1, -2)) + gamma * (np.conj(np.swapaxes(Bh, -1, -2)) @ Bh)
    return P + shift * np.eye(3)


# Threads of the FFTs in precond_solve.  Only a performance setting (the
# transform computed is the same); the CPU baseline of the benchmark sets it
# to the host's core count.
FFT_WORKERS = 1


def precond_solve(r, N, L, alpha, gamma, order=2, shift=0.0, Pinv=None):
    """T = (P + shift I)^-1 r via Alg 5.1: forward FFT along each axis, solve
    with the (here 3 x 3 block) diagonal, inverse FFT along each axis.
    r has shape (..., 3, N, N, N).  ``Pinv`` may carry precomputed inverses."""
    import scipy.fft as sfft
    if Pinv is None:
        Pinv = np.linalg.inv(precond_matrices(N, L, alpha, gamma, order, shift))
    rh = sfft.fftn(np.asarray(r, dtype=np.complex128), axes=(-3, -2, -1), workers=FFT_WORKERS)
    rh = np.moveaxis(rh, -4, -1)[..., None]                 # (..., z, y, x, 3, 1)
    th = (Pinv @ rh)[..., 0]
    th = np.moveaxis(th, -1, -4)
    return sfft.ifftn(th, axes=(-3, -2, -1), workers=FFT_WORKERS)


# ---------------------------------------------------------------------------
# Homogeneous medium: exact discrete spectrum
# ---------------------------------------------------------------------------

def closed_form_symbol_sq(N, L, alpha, order=2):
    """|delta_i(p)|^2 written out with sines and cosines.  With theta = 2 pi p / N,
    the symbol of D_i is sum_s c_s (e^{i s th} - e^{i (1-s) th})/h
    + i alpha sum_s d_s (e^{i s th} + e^{i (1-s) th})
    = e^{i th / 2} [ (2i/h) sum_s c_s sin((2s-1) th / 2)
                     + 2 i alpha sum_s d_s cos((2s-1) th / 2) ],
    so |delta|^2 = [ (2/h) sum_s c_s sin(.) + 2 alpha sum_s d_s cos(.) ]^2.
    Returns shape (3, N)."""
    c, d = STENCIL[order]
    h = L / N
    th = 2 * np.pi * np.arange(N) / N
    out = np.empty((3, N))
    for i in range(3):
        t = np.zeros(N)
        for s in range(1, len(c) + 1):
            t += (2.0 / h) * c[s - 1] * np.sin((2 * s - 1) * th / 2)
            t += 2.0 * alpha[i] * d[s - 1] * np.cos((2 * s - 1) * th / 2)
        out[i] = t ** 2
    return out


def closed_form_spectrum(N, L, alpha, gamma, order=2):
    """Spectrum of the compensated matrix for eps = 1.  Then M_0 = I and, by
    Cor 4.4, A A' + B'B = diag(L, L, L); under the 3-D Fourier transform this is
    s(p) I with s = sum_i |delta_i|^2, and gamma B'B - B'B is the rank-one
    (gamma - 1) conj(delta) delta^T.  Eigenvalues per frequency: s, s (the
    physical pair, delta^T x = 0) and gamma s (the compensation mode).
    Returns (physical sorted, full sorted)."""
    sq = closed_form_symbol_sq(N, L, alpha, order)
    s = (sq[2][:, None, None] + sq[1][None, :, None] + sq[0][None, None, :]).reshape(-1)
    phys = np.sort(np.concatenate([s, s]))
    full = np.sort(np.concatenate([s, s, gamma * s]))
    return phys, full
