"""Plain FP64 CPU oracle of the multigrid preconditioner solve (Section 5.3).

TEST INFRASTRUCTURE ONLY (see oracle/mfd.py): the product path never imports
this module.

Section 5.3 solves the preconditioner system (P + c) x = f, P = A A' + gamma B'B
(eq. (penalised_marix), with the shift of Remark 5.1), by the multigrid method
of Alg 5.2 after a distributive reformulation.  Written out:

* With p = B x the system is the block system with matrix
  [[A A' + (gamma+1) B'B, -B'], [-B, I]]; the paper right-multiplies it by
  L_0 = [[I, B'], [gamma B, (gamma+1) L_k]].  Since B A = 0 (div curl = 0) and
  A A' + B'B = diag(L_k, L_k, L_k) with L_k = B B' (Cor 4.4), the product is
  block lower triangular with Laplacians on its diagonal.  Including the shift
  c (the paper's product is printed garbled, with "(gamma-1) B + c"), the exact
  solution of (P + c) x = f is
      y = (L_k + c)^-1 f          (one scalar solve per component of f),
      q = -(gamma L_k + c)^-1 (gamma - 1) B y,
      x = y + B' q.
  precond_solve_mg() does exactly this with each scalar solve replaced by
  multigrid V-cycles.
* Alg 5.2 (a V-cycle on the level hierarchy): pre-smoothing n1 times,
  residual, restriction, the same cycle on the coarser level from a zero
  guess, prolongation of its result as a correction (the listing omits the
  prolongation; it is read in), post-smoothing n2 times; on the coarsest level
  an exact solve.
* Smoother: x <- x + (L U)^-1 (b - A x), L U an incomplete LU factorisation of
  A.  On the periodic grid the operator is a constant 7-point stencil, and its
  ILU(0) in lexicographic order tends, away from the start of the ordering, to
  constant factors: L with the lower couplings of A and a diagonal d, U = I +
  (upper couplings)/d, where d solves d = a - sum_e c-_e c+_e / d (a the centre
  coefficient, c-_e and c+_e the couplings to the neighbours -e and +e).  These
  stencil factors are used at every point.
* SAIT (Section 5.3): each triangular factor is inverted approximately by
  Jacobi's iteration, so that no triangular solve is needed.  Here a fixed
  number of Jacobi sweeps is applied to the vector (the sweeps are the
  approximate inverse applied without forming it, so the dropping threshold of
  SAIT, which only sparsifies the formed inverse, has no counterpart).
* Hierarchy: rediscretisation of L_k + sigma on grids N, N/2, ... (same Bloch
  vector, h doubled), halving while N is even and above 4; the coarsest grid
  is solved directly (dense).  Transfers: cell-centred trilinear prolongation
  (weights 3/4, 1/4 per axis) and its adjoint divided by 8 as restriction.
"""
from __future__ import annotations

import numpy as np

from . import mfd


# ---------------------------------------------------------------------------
# The scalar operator L_k = B B' = sum_i D_i D_i' (Cor 4.4) and its stencil
# ---------------------------------------------------------------------------

def scalar_laplacian(u, alpha, h):
    """L_k u = div_alpha div_alpha' u = sum_i D_i (D_i' u) on an (N, N, N) grid
    function (Cor 4.4), second order."""
    u = np.asarray(u, dtype=np.complex128)
    return sum(mfd.D(mfd.Dt(u, i, alpha, h), i, alpha, h) for i in (1, 2, 3))


def stencil(N, L, alpha, sigma):
    """The constant 7-point stencil of L_k + sigma on the periodic N^3 grid,
    read off by applying the operator to a unit impulse at the origin:
    returns (a, cm, cp) with a the centre coefficient and, for paper axis
    i = 1, 2, 3 (index i - 1), cm[i-1] the coupling of a point to its
    neighbour at -e_i and cp[i-1] to its neighbour at +e_i."""
    h = L / N
    e = np.zeros((N, N, N), dtype=np.complex128)
    e[0, 0, 0] = 1.0
    col = scalar_laplacian(e, alpha, h) + sigma * e   # column of the origin
    a = col[0, 0, 0]
    # (A e_0)[r] = A[r][0]: the entry at r = +e_i is the coupling of point +e_i
    # to its neighbour at -e_i (cm), the entry at r = -e_i that to +e_i (cp)
    cm = np.array([col[0, 0, 1], col[0, 1, 0], col[1, 0, 0]])
    cp = np.array([col[0, 0, -1], col[0, -1, 0], col[-1, 0, 0]])
    return a, cm, cp


def apply_stencil(u, a, cm, cp):
    """(L_k + sigma) u from its stencil (periodic)."""
    out = a * u
    for i in (1, 2, 3):
        out = out + cm[i - 1] * mfd._at(u, -1, i) + cp[i - 1] * mfd._at(u, 1, i)
    return out


# ---------------------------------------------------------------------------
# ILU-SAIT smoother (Alg 5.2's smoothing step, Section 5.3's smoother)
# ---------------------------------------------------------------------------

def ilu_diagonal(a, cm, cp):
    """Diagonal d of the constant ILU(0) factors: the root of
    d^2 - a d + sum_e cm_e cp_e = 0 that tends to a as the couplings vanish."""
    s = np.sum(cm * cp)
    return 0.5 * (a + np.sqrt(a * a - 4.0 * s))


def sait_apply(r, a, cm, cp, sweeps):
    """z ~ (L U)^-1 r: `sweeps` Jacobi sweeps on L z1 = r (L: diagonal d,
    lower couplings cm at -e_i), then on U z = z1 (U: unit diagonal, upper
    couplings cp / d at +e_i); each starts from the diagonal solve."""
    d = ilu_diagonal(a, cm, cp)
    z1 = r / d
    for _ in range(sweeps):
        z1 = (r - sum(cm[i - 1] * mfd._at(z1, -1, i) for i in (1, 2, 3))) / d
    z = z1.copy()
    for _ in range(sweeps):
        z = z1 - sum((cp[i - 1] / d) * mfd._at(z, 1, i) for i in (1, 2, 3))
    return z


def smooth(x, b, st, steps, sweeps):
    """Alg 5.2's smoothing: x <- x - (L U)^-1 (A x - b), `steps` times."""
    a, cm, cp = st
    for _ in range(steps):
        x = x + sait_apply(b - apply_stencil(x, a, cm, cp), a, cm, cp, sweeps)
    return x


# ---------------------------------------------------------------------------
# Grid transfers (cell-centred)
# ---------------------------------------------------------------------------

def _prolong_axis(u, ax):
    """Coarse -> fine along one numpy axis: fine 2I takes 3/4 of coarse I and
    1/4 of coarse I-1, fine 2I+1 3/4 of I and 1/4 of I+1 (periodic)."""
    lo = 0.75 * u + 0.25 * np.roll(u, 1, axis=ax)
    hi = 0.75 * u + 0.25 * np.roll(u, -1, axis=ax)
    shape = list(u.shape)
    shape[ax] *= 2
    out = np.empty(shape, dtype=u.dtype)
    idx = [slice(None)] * u.ndim
    idx[ax] = slice(0, None, 2)
    out[tuple(idx)] = lo
    idx[ax] = slice(1, None, 2)
    out[tuple(idx)] = hi
    return out


def prolong(u):
    """Trilinear cell-centred interpolation, (N/2)^3 -> N^3."""
    for ax in (0, 1, 2):
        u = _prolong_axis(u, ax)
    return u


def _restrict_axis(u, ax):
    """Adjoint of _prolong_axis along one axis (unscaled)."""
    idx = [slice(None)] * u.ndim
    idx[ax] = slice(0, None, 2)
    ev = u[tuple(idx)]
    idx[ax] = slice(1, None, 2)
    od = u[tuple(idx)]
    # coarse I receives 3/4 from fine 2I and 2I+1, 1/4 from fine 2I+2 and 2I-1
    return 0.75 * (ev + od) + 0.25 * (np.roll(ev, -1, axis=ax) + np.roll(od, 1, axis=ax))


def restrict(u):
    """Full weighting: the adjoint of prolong() divided by 8."""
    for ax in (0, 1, 2):
        u = _restrict_axis(u, ax)
    return u / 8.0


# ---------------------------------------------------------------------------
# V-cycle (Alg 5.2) and the scalar solve
# ---------------------------------------------------------------------------

def levels(N):
    """Grid sizes of the hierarchy: N, N/2, ... while even and above 4."""
    out = [N]
    while out[-1] % 2 == 0 and out[-1] > 4:
        out.append(out[-1] // 2)
    return out


def coarse_matrix(N, L, alpha, sigma):
    """Dense L_k + sigma on the coarsest grid (columns = impulse responses)."""
    n = N ** 3
    a, cm, cp = stencil(N, L, alpha, sigma)
    M = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = apply_stencil(e.reshape(N, N, N), a, cm, cp).reshape(-1)
    return M


def vcycle(x, b, lev, hier, n1, n2, sweeps):
    """MG(x, b, A_l, n1, n2) of Alg 5.2 on level `lev` of `hier` (a list of
    dicts with the stencil, and the dense inverse on the last level)."""
    H = hier[lev]
    if lev == len(hier) - 1:
        return (H["inv"] @ b.reshape(-1)).reshape(b.shape)
    x = smooth(x, b, H["st"], n1, sweeps)
    r = b - apply_stencil(x, *H["st"])
    ec = vcycle(np.zeros_like(restrict(r)), restrict(r), lev + 1, hier, n1, n2, sweeps)
    x = x + prolong(ec)
    return smooth(x, b, H["st"], n2, sweeps)


def hierarchy(N, L, alpha, sigma):
    hier = []
    for n in levels(N):
        H = {"N": n, "st": stencil(n, L, alpha, sigma)}
        hier.append(H)
    hier[-1]["inv"] = np.linalg.inv(coarse_matrix(hier[-1]["N"], L, alpha, sigma))
    return hier


def mg_solve(b, N, L, alpha, sigma, cycles=2, n1=2, n2=2, sweeps=2, hier=None):
    """(L_k + sigma)^-1 b approximated by `cycles` V-cycles from a zero guess."""
    if hier is None:
        hier = hierarchy(N, L, alpha, sigma)
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    for _ in range(cycles):
        x = vcycle(x, b, 0, hier, n1, n2, sweeps)
    return x


# ---------------------------------------------------------------------------
# The preconditioner solve (Section 5.3's distributive form)
# ---------------------------------------------------------------------------

def precond_solve_mg(r, N, L, alpha, gamma, shift=0.0, cycles=2, n1=2, n2=2, sweeps=2):
    """x ~ (P + shift I)^-1 r for fields r of shape (..., 3, N, N, N):
    y = (L_k + c)^-1 r (per component), q = -(gamma L_k + c)^-1 (gamma-1) B y,
    x = y + B' q, each scalar inverse replaced by multigrid V-cycles (the
    second as (L_k + c/gamma)^-1 / gamma)."""
    r = np.asarray(r, dtype=np.complex128)
    if r.ndim > 4:
        return np.stack([precond_solve_mg(x, N, L, alpha, gamma, shift, cycles, n1, n2, sweeps) for x in r])
    h = L / N
    hy = hierarchy(N, L, alpha, shift)
    hq = hierarchy(N, L, alpha, shift / gamma)
    y = np.stack([mg_solve(r[i], N, L, alpha, shift, cycles, n1, n2, sweeps, hier=hy) for i in range(3)])
    g = -(gamma - 1.0) / gamma * mfd.div(y, alpha, h)
    q = mg_solve(g, N, L, alpha, shift / gamma, cycles, n1, n2, sweeps, hier=hq)
    return y + mfd.div_adj(q, alpha, h)
