"""Plain FP64 CPU oracle of the band solve: block LOBPCG with the FFT
preconditioner (Section 5) wrapped in the recompute check of Alg 4.1.

TEST INFRASTRUCTURE ONLY (see oracle/mfd.py): the product path never imports
this module.

The paper cites LOBPCG (Knyazev) without fixing a variant (Section 5.1).  This
is the textbook method, with the choices the paper leaves open written down:
block size m, no guard vectors; basis [X, W, P] with W the preconditioned
residuals of the unconverged columns and P the W/P part of the previous
update ("soft locking" of converged columns); Rayleigh-Ritz in the span of the
basis, orthonormalised by a scaled Gram eigendecomposition with near-null
directions dropped, and P restarted (left out for one step) when the Gram
matrix of [X, W, P] is ill-conditioned.  The variant changes iteration
counts, not the result.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import lattice as lat
from . import mfd


def _ritz(X, AX):
    """Rayleigh-Ritz on span(X) (generalised form, X need not be orthonormal).
    Returns (theta, X V, AX V, V)."""
    G = X.conj().T @ X
    H = X.conj().T @ AX
    H = 0.5 * (H + H.conj().T)
    G = 0.5 * (G + G.conj().T)
    th, V = sla.eigh(H, G)
    return th, X @ V, AX @ V, V


def lobpcg(apply_A, apply_T, X0, tol, maxiter=500, drop=1e-10, restart=1e-8, lock=True, nconv=None):
    """Smallest m eigenpairs of the Hermitian positive definite operator
    ``apply_A`` ((n, j) -> (n, j)), preconditioned by ``apply_T``.

    Convergence of column i: |A x_i - th_i x_i| <= tol |th_i| |x_i|; the
    iteration stops when the lowest ``nconv`` columns (default all) converge.
    Returns (theta, X, info) with info = dict(iters, res, converged)."""
    X = np.array(X0, dtype=np.complex128)
    m = X.shape[1]
    X, _ = np.linalg.qr(X)
    AX = apply_A(X)
    th, X, AX, _ = _ritz(X, AX)
    P = AP = None
    res = np.full(m, np.inf)
    it = 0
    for it in range(1, maxiter + 1):
        R = AX - X * th[None, :]
        res = np.linalg.norm(R, axis=0) / (np.abs(th) * np.linalg.norm(X, axis=0))
        active = res > tol
        if not active[:nconv if nconv else m].any():
            it -= 1
            break
        if not lock:
            active[:] = True
        W = apply_T(R[:, active])
        AW = apply_A(W)
        S = [X, W]
        AS = [AX, AW]
        if P is not None:
            S.append(P[:, active])
            AS.append(AP[:, active])
        while True:
            Sm = np.hstack(S)
            ASm = np.hstack(AS)
            G = Sm.conj().T @ Sm
            H = Sm.conj().T @ ASm
            G = 0.5 * (G + G.conj().T)
            H = 0.5 * (H + H.conj().T)
            dsc = 1.0 / np.sqrt(np.real(np.diag(G)))
            Gs = G * dsc[:, None] * dsc[None, :]
            Hs = H * dsc[:, None] * dsc[None, :]
            g, V = np.linalg.eigh(Gs)
            # An ill-conditioned basis (P nearly inside span[X, W]) limits the
            # attainable residual; drop P for this step (restart the
            # conjugate direction) when that happens.
            if len(S) == 3 and g.min() < restart * g.max():
                S, AS = S[:2], AS[:2]
                continue
            break
        keep = g > drop * g.max()
        U = V[:, keep] / np.sqrt(g[keep])[None, :]
        mu, Y = np.linalg.eigh(U.conj().T @ Hs @ U)
        C = dsc[:, None] * (U @ Y[:, :m])
        Xn = Sm @ C
        AXn = ASm @ C
        P = Sm[:, m:] @ C[m:]
        AP = ASm[:, m:] @ C[m:]
        # re-impose orthonormality of X (and keep column j of P paired with
        # column j of X, which the next soft-locking selection relies on)
        th, X, AX, V = _ritz(Xn, AXn)
        P = P @ V
        AP = AP @ V
    # final residual from a fresh operator application
    AX = apply_A(X)
    nrm = np.linalg.norm(X, axis=0)
    X = X / nrm[None, :]
    AX = AX / nrm[None, :]
    th = np.real(np.sum(X.conj() * AX, axis=0))
    order = np.argsort(th)
    th, X, AX = th[order], X[:, order], AX[:, order]
    res = np.linalg.norm(AX - X * th[None, :], axis=0) / np.abs(th)
    return th, X, dict(iters=it, res=res, converged=bool(np.all(res[:nconv if nconv else m] <= tol)))


def spurious_flags(lam, lam_re, scale, rel=1e-4, abs_tol=1e-10):
    """Alg 4.1, step 3, in floating point: lambda - lambda_re = gamma |Bx|^2/|x|^2
    >= 0 exactly, so a band is physical when that gap is at round-off level and
    spurious when it is a visible fraction of lambda."""
    lam = np.asarray(lam)
    return (lam - np.asarray(lam_re)) > rel * np.abs(lam) + abs_tol * scale


def solve_bands(eps, L, k, m, tol=1e-10, order=2, gamma=None, X0=None, seed=0,
                maxiter=500, max_doublings=4, check=True, guard=2, mu=None, lattice=None):
    """Lowest m physical eigenpairs of A M_0 A' + gamma B'B at Bloch vector k
    (eq. (Ker_comp)), following Alg 4.1: compute the lowest eigenpairs, recompute
    lambda_re = |M_0^(1/2) A'x|^2 / |x|^2, and treat a band with lambda_re !=
    lambda as spurious.  Spurious bands are discarded (the block carries
    ``guard`` extra columns for them); if fewer than m physical bands remain
    among the m + guard, gamma is doubled and the solve repeated.

    eps: cell permittivity (N, N, N); k: Cartesian Bloch vector (1/L units).
    mu: M_0 on the edges (3, N, N, N) in place of the one eps gives
    (Section 6.2 sets it per edge for its cubic lattices); eps then only
    fixes N.
    lattice: 3 x 3 matrix whose columns are the lattice vectors (Section 2's
    coordinate change, Section 4.2's D^_i; ``oracle.lattice``); L is then
    ignored and |det A|^(1/3) takes its place in the penalty and shift rules.
    X0: (m + guard, 3, N, N, N) start block (default: seeded complex Gaussian).
    Convergence: |A x - lambda x| <= tol (|lambda| + c) |x|, c the shift of
    ``mfd.shift_rule``.
    Returns (lam (m,), X (m, 3, N, N, N), info)."""
    eps = np.asarray(eps, dtype=np.float64)
    N = eps.shape[0]
    n = 3 * N ** 3
    if lattice is not None:
        L = lat.cell_length(lattice)
    h = L / N
    k = np.asarray(k, dtype=np.float64)
    mb = m + guard
    mu = mfd.mu_from_eps(eps) if mu is None else np.asarray(mu, dtype=np.float64)
    g = mfd.gamma_rule(N, L, k) if gamma is None else float(gamma)
    c = mfd.shift_rule(L, k)
    if X0 is None:
        rng = np.random.default_rng(seed)
        X0 = rng.standard_normal((mb, 3, N, N, N)) + 1j * rng.standard_normal((mb, 3, N, N, N))
    X = np.asarray(X0, dtype=np.complex128).reshape(mb, n).T
    doublings = 0
    total_iters = 0
    nreq = m
    while True:
        if lattice is None:
            Pinv = np.linalg.inv(mfd.precond_matrices(N, L, k, g, order, c))
        else:
            Pinv = np.linalg.inv(lat.precond_matrices(N, lattice, k, g, order, c))

        def apply_A(Y, g=g):
            V = Y.T.reshape(-1, 3, N, N, N)
            if lattice is not None:
                return lat.apply_op(V, mu, k, lattice, g, order, c).reshape(-1, n).T
            return mfd.apply_op(V, mu, k, h, g, order, c).reshape(-1, n).T

        def apply_T(R, g=g, Pinv=Pinv):
            V = R.T.reshape(-1, 3, N, N, N)
            return mfd.precond_solve(V, N, L, k, g, order, c, Pinv=Pinv).reshape(-1, n).T

        th, X, info = lobpcg(apply_A, apply_T, X, tol, maxiter, nconv=nreq)
        total_iters += info["iters"]
        lam = th - c
        Xb = X.T.reshape(mb, 3, N, N, N)
        if lattice is None:
            lam_re = np.array([mfd.lambda_re(x, mu, k, h, order) for x in Xb])
        else:
            lam_re = np.array([lat.lambda_re(x, mu, k, lattice, order) for x in Xb])
        spur = spurious_flags(lam, lam_re, (2 * np.pi / L) ** 2) if check else np.zeros(mb, bool)
        phys = np.flatnonzero(~spur)
        if len(phys) >= m:
            need = phys[m - 1] + 1
            if need > nreq and info["iters"] < maxiter:
                nreq = need                  # discarded bands: converge one band further
                continue
            sel = phys[:m]
            info.update(gamma=g, doublings=doublings, lam_re=lam_re[sel], spurious=spur[sel],
                        discarded=int(spur[:need].sum()), total_iters=total_iters, shift=c,
                        res=info["res"][sel], converged=bool(info["res"][sel].max() <= tol))
            return lam[sel], Xb[sel], info
        if doublings >= max_doublings:
            sel = np.arange(m)
            info.update(gamma=g, doublings=doublings, lam_re=lam_re[sel], spurious=spur[sel],
                        discarded=0, total_iters=total_iters, shift=c, res=info["res"][sel])
            return lam[sel], Xb[sel], info
        g *= 2.0
        doublings += 1
        nreq = m
        # A spurious column is an exact compensation eigenvector of the new
        # matrix too (eigenvalue doubled) and would stay locked at zero
        # residual: replace it by fresh noise.
        rng = np.random.default_rng(seed + 7919 * doublings)
        ns = int(spur.sum())
        X = X.copy()
        X[:, spur] = rng.standard_normal((n, ns)) + 1j * rng.standard_normal((n, ns))
