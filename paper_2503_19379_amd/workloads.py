"""Seeded synthetic inputs: permittivity voxel grids, Brillouin-zone k-paths
and random start blocks.

This module holds none of the method's arithmetic (no operator, symbol,
penalty or solver): it only draws inputs, and it is the one module that both
the HIP path's callers and the CPU oracle's callers share.  It imports numpy
only.

Geometry follows the paper's lattices where the paper gives them (simple cubic
cell [0, L]^3, Section 6 eq. (translation_vecs); Brillouin-zone points of the
simple cubic lattice, Section 6) and the synthetic workloads otherwise:
a dielectric sphere, the conventional cubic cell of a diamond lattice of
spheres, and thresholded Gaussian random fields.
"""
from __future__ import annotations

import numpy as np

EPS_HIGH = 13.0
EPS_LOW = 1.0


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def eps_homogeneous(N: int, value: float = 1.0) -> np.ndarray:
    return np.full((N, N, N), float(value))


def eps_spheres(N: int, centers, r: float, L: float = 1.0, eps_in: float = EPS_HIGH,
                eps_out: float = EPS_LOW, sub: int = 4) -> np.ndarray:
    """Cell permittivity of periodic dielectric spheres of radius r, each cell
    the arithmetic mean over sub^3 cell-centred sub-samples (voxel average).
    Arrays are [z][y][x]."""
    h = L / N
    base = np.arange(N, dtype=np.float64)
    cen = np.asarray(centers, dtype=np.float64)
    frac = np.zeros((N, N, N))
    for oz in range(sub):
        z = (base + (oz + 0.5) / sub) * h
        for oy in range(sub):
            y = (base + (oy + 0.5) / sub) * h
            for ox in range(sub):
                x = (base + (ox + 0.5) / sub) * h
                inside = np.zeros((N, N, N), dtype=bool)
                for c in cen:
                    dx = _min_image(x - c[0], L) ** 2
                    dy = _min_image(y - c[1], L) ** 2
                    dz = _min_image(z - c[2], L) ** 2
                    inside |= (dz[:, None, None] + dy[None, :, None] + dx[None, None, :]) <= r * r
                frac += inside
    frac /= sub ** 3
    return eps_out + (eps_in - eps_out) * frac


def eps_sphere(N: int, r: float = 0.25, L: float = 1.0, sub: int = 4) -> np.ndarray:
    """One sphere of radius r at the cell centre, eps 13 inside, 1 outside."""
    return eps_spheres(N, [(0.5 * L, 0.5 * L, 0.5 * L)], r, L, sub=sub)


DIAMOND_SITES = np.array([
    (0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0),
    (0.25, 0.25, 0.25), (0.25, 0.75, 0.75), (0.75, 0.25, 0.75), (0.75, 0.75, 0.25),
])


def eps_diamond(N: int, r: float = 0.13, L: float = 1.0, sub: int = 4) -> np.ndarray:
    """Conventional cubic cell of a diamond lattice: spheres of radius r at the
    eight sites (fcc sites and the same shifted by (1/4, 1/4, 1/4))."""
    return eps_spheres(N, DIAMOND_SITES * L, r, L, sub=sub)


def eps_random_field(N: int, seed: int, corr: float = 0.15, fill: float = 0.30,
                     L: float = 1.0) -> np.ndarray:
    """Gaussian random field with correlation length ``corr`` (covariance
    exp(-r^2 / (2 corr^2))), thresholded so that the top ``fill`` fraction of
    cells get eps = 13 and the rest eps = 1."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    q = 2 * np.pi * np.fft.fftfreq(N, d=L / N)
    q2 = q[:, None, None] ** 2 + q[None, :, None] ** 2 + q[None, None, :] ** 2
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * np.exp(-q2 * corr * corr / 4.0)))
    thr = np.quantile(field, 1.0 - fill)
    return np.where(field > thr, EPS_HIGH, EPS_LOW)


def sc_points(L: float = 1.0) -> dict:
    """Symmetry points of the simple cubic Brillouin zone (Section 6): the
    paper's L(pi/l, 0, 0) and N(pi/l, pi/l, pi/l) are the usual X and R."""
    p = np.pi / L
    return {"G": (0.0, 0.0, 0.0), "X": (p, 0.0, 0.0), "M": (p, p, 0.0), "R": (p, p, p)}


def kpath(labels: str, n: int, L: float = 1.0) -> np.ndarray:
    """n k-points uniform in arc length along the polyline through the named
    simple cubic points (e.g. "GXMGR"), both ends included.  Shape (n, 3)."""
    pts = sc_points(L)
    P = np.array([pts[c] for c in labels], dtype=np.float64)
    seg = np.linalg.norm(np.diff(P, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.linspace(0.0, cum[-1], n)
    out = np.empty((n, 3))
    for j, t in enumerate(s):
        i = min(np.searchsorted(cum, t, side="right") - 1, len(seg) - 1)
        f = (t - cum[i]) / seg[i]
        out[j] = P[i] + f * (P[i + 1] - P[i])
    out[np.abs(out) < 1e-15] = 0.0
    return out


def bcc_points(l: float = 1.0) -> dict:
    """Symmetry points of the BCC Brillouin zone (Section 6, lattice constant
    l): H'(0, 0, 2 pi/l) is "h", Gamma "G", P, N and H."""
    p = np.pi / l
    return {"h": (0.0, 0.0, 2 * p), "G": (0.0, 0.0, 0.0), "P": (p, p, p), "N": (p, 0.0, p),
            "H": (0.0, 2 * p, 0.0)}


def fcc_points(l: float = 1.0) -> dict:
    """Symmetry points of the FCC Brillouin zone (Section 6, lattice constant
    l): X, U, L, Gamma ("G"), W, K.  The paper prints U as (pi/2l, 0, pi/2l),
    which is not on the zone boundary; U here is the usual (pi/2l, 2 pi/l,
    pi/2l), the end of the X-U edge."""
    p = np.pi / l
    return {"X": (0.0, 2 * p, 0.0), "U": (0.5 * p, 2 * p, 0.5 * p), "L": (p, p, p), "G": (0.0, 0.0, 0.0),
            "W": (p, 2 * p, 0.0), "K": (1.5 * p, 1.5 * p, 0.0)}


def lattice_vectors(kind: str, l: float = 1.0) -> np.ndarray:
    """Primitive vectors of eq. (translation_vecs) as the columns of a 3 x 3
    matrix: "sc", "fcc" or "bcc" with lattice constant l."""
    h = 0.5 * l
    cols = {"sc": [(l, 0, 0), (0, l, 0), (0, 0, l)],
            "fcc": [(0, h, h), (h, 0, h), (h, h, 0)],
            "bcc": [(-h, h, h), (h, -h, h), (h, h, -h)]}[kind]
    return np.array(cols, dtype=np.float64).T


def kpath_vertices(labels: str, n: int, L: float = 1.0, points: dict | None = None) -> np.ndarray:
    """About n k-points along the polyline through the named points (simple
    cubic ones unless ``points`` is given), each segment sampled in
    proportion to its length with its end points included (band extrema sit
    at the symmetry points).  Shape (n', 3)."""
    pts = sc_points(L) if points is None else points
    P = np.array([pts[c] for c in labels], dtype=np.float64)
    seg = np.linalg.norm(np.diff(P, axis=0), axis=1)
    out = []
    for i, sl in enumerate(seg):
        m = max(1, int(round((n - 1) * sl / seg.sum())))
        for j in range(m):
            out.append(P[i] + (j / m) * (P[i + 1] - P[i]))
    out.append(P[-1])
    out = np.array(out)
    out[np.abs(out) < 1e-15] = 0.0
    return out


def mu_sc_sphere_cylinders(N: int, L: float = 1.0, r_sphere: float = 0.345, r_cyl: float = 0.11,
                           eps_in: float = EPS_HIGH, eps_out: float = EPS_LOW) -> np.ndarray:
    """M_0 on the edges for the simple cubic cell of Section 6.2 with a
    curved interface: material inside the sphere of radius r_sphere L about
    the cell centre and inside the three cylinders of radius r_cyl L along
    the axes through the centre.  An edge takes eps_in^-1 when its midpoint
    is in the material, else eps_out^-1 (the paper's rule for these cells).
    Edge e_1[z, y, x] sits at ((x + 1/2) h, y h, z h), e_2 at
    (x h, (y + 1/2) h, z h), e_3 at (x h, y h, (z + 1/2) h).  Shape
    (3, N, N, N)."""
    h = L / N
    c = 0.5 * L
    i = np.arange(N) * h
    half = i + 0.5 * h
    mu = np.empty((3, N, N, N))
    for comp in range(3):
        ax = [i, i, i]
        ax[comp] = half   # x, y, z coordinate arrays of this component's edges
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        dx, dy, dz = X - c, Y - c, Z - c
        inside = ((dx * dx + dy * dy + dz * dz <= (r_sphere * L) ** 2)
                  | (dy * dy + dz * dz <= (r_cyl * L) ** 2)
                  | (dx * dx + dz * dz <= (r_cyl * L) ** 2)
                  | (dx * dx + dy * dy <= (r_cyl * L) ** 2))
        mu[comp] = np.where(inside, 1.0 / eps_in, 1.0 / eps_out)
    return mu


def mu_bcc_gyroid(N: int, l: float = 1.0, t: float = 1.1, eps_in: float = 16.0,
                  eps_out: float = 1.0) -> np.ndarray:
    """M_0 on the edges of the unit-cube grid of the BCC primitive cell for
    the single gyroid of Section 6.3: material where
    g = sin(2 pi x/l) cos(2 pi y/l) + sin(2 pi y/l) cos(2 pi z/l) + sin(2 pi z/l) cos(2 pi x/l) > t,
    eps_in / eps_out = 16.  g is invariant under the BCC translations, so it
    is periodic on the cell.  Edge e_1[z, y, x] sits at y = ((x + 1/2), y, z) / N
    in cell coordinates (e_2, e_3 likewise), mapped to Cartesian by the BCC
    vectors; an edge takes eps_in^-1 when its midpoint is in the material.
    Shape (3, N, N, N)."""
    A = lattice_vectors("bcc", l)
    i = np.arange(N) / N
    half = i + 0.5 / N
    mu = np.empty((3, N, N, N))
    w = 2 * np.pi / l
    for comp in range(3):
        ax = [i, i, i]
        ax[comp] = half
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        cx = A[0, 0] * X + A[0, 1] * Y + A[0, 2] * Z
        cy = A[1, 0] * X + A[1, 1] * Y + A[1, 2] * Z
        cz = A[2, 0] * X + A[2, 1] * Y + A[2, 2] * Z
        g = (np.sin(w * cx) * np.cos(w * cy) + np.sin(w * cy) * np.cos(w * cz)
             + np.sin(w * cz) * np.cos(w * cx))
        mu[comp] = np.where(g > t, 1.0 / eps_in, 1.0 / eps_out)
    return mu


def mu_fcc_diamond(N: int, l: float = 1.0, r: float = 0.12, b: float = 0.11, eps_in: float = 13.0,
                   eps_out: float = 1.0) -> np.ndarray:
    """M_0 on the edges of the unit-cube grid of the FCC primitive cell for the
    sp3 diamond structure of Section 6.3: dielectric spheres of radius r l at
    the two basis sites 0 and (l/4)(1, 1, 1) of every lattice point, joined
    along the four nearest-neighbour bonds by prolate spheroids whose foci
    are the two sphere centres.  The paper's minor axis b l is read as the
    spheroid's minor radius (semi-minor axis), so the semi-major axis is
    sqrt((sqrt(3) l/8)^2 + (b l)^2); with b l as the full minor axis the cell
    has half the gap the paper reports.  eps_in / eps_out = 13.  An edge
    takes eps_in^-1 when its midpoint (mapped to Cartesian by the FCC
    vectors) is in the material.  Shape (3, N, N, N)."""
    A = lattice_vectors("fcc", l)
    q = 0.25 * l
    bonds = q * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    semi = np.sqrt((0.5 * np.linalg.norm(bonds[0])) ** 2 + (b * l) ** 2)
    n = np.arange(-1, 2)
    T = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3) @ A.T   # 27 lattice images
    sites = np.concatenate([T, T + bonds[0]])
    i = np.arange(N) / N
    half = i + 0.5 / N
    mu = np.empty((3, N, N, N))
    for comp in range(3):
        ax = [i, i, i]
        ax[comp] = half
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) @ A.T
        inside = np.zeros(P.shape[0], dtype=bool)
        for c0 in range(0, P.shape[0], 1 << 16):
            p = P[c0:c0 + (1 << 16)]
            ins = np.zeros(p.shape[0], dtype=bool)
            for s_ in sites:
                ins |= np.sum((p - s_) ** 2, axis=1) <= (r * l) ** 2
            for t in T:
                d0 = np.sqrt(np.sum((p - t) ** 2, axis=1))
                for bd in bonds:
                    ins |= d0 + np.sqrt(np.sum((p - t - bd) ** 2, axis=1)) <= 2 * semi
            inside[c0:c0 + (1 << 16)] = ins
        mu[comp] = np.where(inside.reshape(N, N, N), 1.0 / eps_in, 1.0 / eps_out)
    return mu


def start_block(m: int, N: int, seed: int) -> np.ndarray:
    """Seeded complex Gaussian start block, shape (m, 3, N, N, N), complex128
    (real and imaginary parts independent standard normals)."""
    rng = np.random.default_rng(seed)
    shp = (m, 3, N, N, N)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


# Synthetic workloads (shapes, seeds, paths).  Units: L = 1.
CONFIGS = {
    # homogeneous unit cube, dense check
    "homog_n8": dict(N=8, eps="homogeneous", kpts=[(0.3 * np.pi, 0.2 * np.pi, 0.1 * np.pi)],
                     nbands=8, precision="fp64"),
    # simple cubic lattice of one sphere, FP64
    "sphere_n32": dict(N=32, eps="sphere", path="GXMGR", nk=20, nbands=10, tol=1e-8,
                       precision="fp64"),
    # diamond conventional cell, mixed precision
    "diamond_n64": dict(N=64, eps="diamond", path="GXMGR", nk=64, nbands=16, tol=1e-8,
                        precision="mixed"),
    # 32 random-field crystals of uneven grids
    "random_batch": dict(Ns=(24, 32, 48, 64), ncrys=32, eps="random", path="GXMGR", nk=8,
                         nbands=12, tol=1e-8, precision="mixed"),
    # simple cubic sphere + three cylinders (Section 6.2), M_0 on edges, band gap
    # at the paper's grid N = 150
    "sc_sphere_cyl": dict(N=150, mu="sc_sphere_cyl", path="GXMGRXMR", nk=40, nbands=10, tol=1e-5,
                          precision="mixed", gap_ratio_paper=0.14019, N_paper=150),
    # BCC single gyroid (Section 6.3, Table time_comp_bc): first 10 bands at
    # k = (pi, pi, pi)/l, N = 100 and 120, relative residual 1e-5; the band
    # structure and gap at the paper's grid N = 150
    "bcc_gyroid": dict(Ns=(100, 120), N_path=150, lattice="bcc", mu="bcc_gyroid", k=(np.pi, np.pi, np.pi),
                       nbands=10, tol=1e-5, precision="mixed", path="hGPNH", nk=40, gap_ratio_paper=0.31745,
                       N_paper=150),
    # FCC sp3 diamond of spheres and spheroids (Section 6.3): band gap
    "fcc_diamond": dict(lattice="fcc", mu="fcc_diamond", path="XULGXWK", nk=40, nbands=10, tol=1e-5,
                        precision="mixed", gap_ratio_paper=0.31182, N_paper=150),
    # diamond at N = 96, learned warm start
    "diamond_n96": dict(N=96, eps="diamond", path="GXMGRX", nk=100, nbands=20, tol=1e-8,
                        precision="mixed"),
}


def crystal_eps(name: str, N: int, seed: int = 0) -> np.ndarray:
    if name == "homogeneous":
        return eps_homogeneous(N)
    if name == "sphere":
        return eps_sphere(N)
    if name == "diamond":
        return eps_diamond(N)
    if name == "random":
        return eps_random_field(N, seed)
    raise ValueError(name)


def random_batch_crystals(ncrys: int = 32, Ns=(24, 32, 48, 64)):
    """(N, eps) for crystal c = 0..ncrys-1: N = Ns[c mod len(Ns)], seed c."""
    return [(Ns[c % len(Ns)], eps_random_field(Ns[c % len(Ns)], c)) for c in range(ncrys)]
