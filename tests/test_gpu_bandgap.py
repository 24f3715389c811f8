"""Contexts built from M_0 on the edges, physics against an exact dispersion
relation, and the band-gap driver of Section 6.2, through the C ABI."""
import numpy as np
import pytest
from oracle import bandgap, lobpcg as olob, mfd
from paper_2503_19379_amd import workloads
from tests.exact import bragg_omegas, layered_spectrum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("kx", [np.pi, 0.5 * np.pi])
def test_bragg_stack_exact_dispersion(B, kx):
    """eps 13 for x < 1/2, 1 above (interfaces on cell faces), Bloch vector
    along x: each frequency of the one-dimensional stack appears twice (two
    polarisations).  N = 64, FP64; second-order error about 1e-3 in lambda."""
    N = 64
    eps = np.ones((N, N, N))
    eps[:, :, : N // 2] = 13.0
    ctx = B.mfd_build(N, 1.0, 2, eps)
    ev, st, status = B.mfd_bands(ctx, [(kx, 0.0, 0.0)], 4, 1e-10, B.default_opts(precision=0, streams=1))
    assert status == 0, st
    lam = bragg_omegas(kx, 2) ** 2
    assert np.allclose(ev[0], np.repeat(lam, 2), rtol=2e-3), (ev[0], lam)
    assert abs(ev[0][0] - ev[0][1]) <= 1e-9 * ev[0][0] and abs(ev[0][2] - ev[0][3]) <= 1e-9 * ev[0][2]


def test_layered_stack_oblique_exact_dispersion(B):
    """The same stack with a wavevector along the layers, k = (0, pi/2, 0):
    a TE wave (E tangential to the interfaces), a TM wave (E with a component
    normal to them) and the first folded ones, against the exact transfer-
    matrix relations.  N = 64, FP64."""
    N = 64
    eps = np.ones((N, N, N))
    eps[:, :, : N // 2] = 13.0
    ctx = B.mfd_build(N, 1.0, 2, eps)
    k = (0.0, 0.5 * np.pi, 0.0)
    ev, st, status = B.mfd_bands(ctx, [k], 4, 1e-10, B.default_opts(precision=0, streams=1))
    assert status == 0, st
    lam = layered_spectrum(k[0], k[1], 4)
    assert np.allclose(ev[0], lam, rtol=3e-3), (ev[0], lam)


def test_build_mu_matches_oracle(B):
    """The Section 6.2 sphere + cylinders cell with M_0 set per edge, N = 20,
    FP64, at M: the oracle's LOBPCG on the same M_0."""
    N, m = 20, 6
    k = np.array([np.pi, np.pi, 0.0])
    mu = workloads.mu_sc_sphere_cylinders(N)
    ctx = B.mfd_build_mu(N, 1.0, 2, mu)
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-10, B.default_opts(precision=0, streams=1))
    assert status == 0, st
    lam, _, _ = olob.solve_bands(np.ones((N, N, N)), 1.0, k, m, tol=1e-10, mu=mu)
    assert np.allclose(ev[0], lam, rtol=1e-8), (ev[0], lam)


def test_build_mu_equals_build_eps(B):
    """mfd_build_mu fed the M_0 that mfd_build forms from eps gives the same
    operator."""
    N = 16
    rng = np.random.default_rng(9)
    eps = 1.0 + 12.0 * (rng.random((N, N, N)) < 0.3)
    k = np.array([0.4, -0.2, 0.7])
    a = B.mfd_build(N, 1.0, 2, eps)
    b = B.mfd_build_mu(N, 1.0, 2, mfd.mu_from_eps(eps))
    X = torch.from_numpy(rng.standard_normal((2, 3, N, N, N)) + 1j * rng.standard_normal((2, 3, N, N, N))).cuda()
    Ya, Yb = torch.empty_like(X), torch.empty_like(X)
    B.mfd_op_apply(a, k, X, Ya)
    B.mfd_op_apply(b, k, X, Yb)
    torch.cuda.synchronize()
    assert torch.equal(Ya, Yb)


def test_band_gap_driver(B):
    """The sphere + cylinders cell at N = 64, mixed precision, the paper's
    LOBPCG tolerance 1e-5, 10 bands along Gamma-X-M-Gamma-R-X-M-R with every
    symmetry point included: every k-point converges, the library's gap ratio
    is the oracle's for the same band structure, and with the static zero
    mode at Gamma skipped the gap opens between bands 5 and 6 at the paper's
    0.14019 (N = 150) within 0.004.  Taken as returned (third zero band
    counted at Gamma) bands 5 and 6 overlap."""
    cfg = workloads.CONFIGS["sc_sphere_cyl"]
    N = 64
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"])
    ctx = B.mfd_build_mu(N, 1.0, 2, workloads.mu_sc_sphere_cylinders(N))
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"],
                                 B.default_opts(precision=1, warm_start=1, guard=2, streams=8, max_iter=500))
    assert status == 0, st
    assert all(s["max_rel_resid"] <= cfg["tol"] for s in st)
    r, below = B.mfd_gap_ratio(ev, kp)
    ro, bo = bandgap.gap_ratio(ev, kp)
    assert r == pytest.approx(ro, rel=1e-12) and below == bo
    r0, _ = B.mfd_gap_ratio(ev)
    print(f"N = {N}: largest gap ratio {r:.5f} above band {below}, {r0:.5f} with the static mode counted "
          f"(the paper prints {cfg['gap_ratio_paper']} at N = {cfg['N_paper']})")
    assert below == 5 and abs(r - cfg["gap_ratio_paper"]) < 0.004
    assert r0 < 0


def test_gamma_row_minus_the_static_mode_is_the_physical_spectrum(B):
    """eps = 1 at k = 0: the solver's three zero bands are the two transverse
    zeros of the closed-form physical spectrum plus one static mode; without
    the third, the row is the physical spectrum."""
    N, m = 12, 9
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    ev, st, status = B.mfd_bands(ctx, [np.zeros(3)], m, 1e-10, B.default_opts(precision=0, streams=1))
    assert status == 0, st
    assert np.abs(ev[0][:3]).max() < 1e-9
    phys, _ = mfd.closed_form_spectrum(N, 1.0, np.zeros(3), st[0]["gamma"])
    row = np.concatenate([ev[0][:2], ev[0][3:]])
    assert np.allclose(row, phys[: m - 1], rtol=1e-9, atol=1e-9), (row, phys[: m - 1])


def test_bcc_gyroid_band_gap(B):
    """Section 6.3's single gyroid on the BCC lattice (eps 16 in 1, M_0 per
    edge) at N = 64, 10 bands on H'-Gamma-P-N-H with every symmetry point,
    tol 1e-5, mixed precision: the gap opens between bands 2 and 3 and its
    ratio approaches the paper's 0.31745 (N = 150) from below as N grows
    (0.3122 at N = 100, 0.3150 at N = 120)."""
    cfg = workloads.CONFIGS["bcc_gyroid"]
    N = 64
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.bcc_points())
    ctx = B.mfd_build_lattice_mu(N, workloads.lattice_vectors("bcc"), 2, workloads.mu_bcc_gyroid(N))
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"],
                                 B.default_opts(precision=1, warm_start=1, guard=2, streams=8, max_iter=500))
    assert status == 0, st
    assert all(s["max_rel_resid"] <= cfg["tol"] for s in st)
    r, below = B.mfd_gap_ratio(ev, kp)
    ro, bo = bandgap.gap_ratio(ev, kp)
    assert r == pytest.approx(ro, rel=1e-12) and below == bo
    print(f"N = {N}: gyroid gap ratio {r:.5f} above band {below} (the paper prints {cfg['gap_ratio_paper']} "
          f"at N = {cfg['N_paper']})")
    assert below == 2 and 0.28 < r < cfg["gap_ratio_paper"]


def test_fcc_diamond_band_gap(B):
    """Section 6.3's FCC sp3 diamond (spheres r = 0.12 l joined by spheroids
    of minor radius 0.11 l, eps 13 in 1, M_0 per edge) at N = 64, 10 bands
    on X-U-L-Gamma-X-W-K with every symmetry point, tol 1e-5, mixed
    precision: the gap opens between bands 2 and 3 at 0.309, close to the
    paper's 0.31182 (N = 150); 0.31098 at N = 100."""
    cfg = workloads.CONFIGS["fcc_diamond"]
    N = 64
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.fcc_points())
    ctx = B.mfd_build_lattice_mu(N, workloads.lattice_vectors("fcc"), 2, workloads.mu_fcc_diamond(N))
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"],
                                 B.default_opts(precision=1, warm_start=1, guard=2, streams=8, max_iter=500))
    assert status == 0, st
    assert all(s["max_rel_resid"] <= cfg["tol"] for s in st)
    r, below = B.mfd_gap_ratio(ev, kp)
    ro, bo = bandgap.gap_ratio(ev, kp)
    assert r == pytest.approx(ro, rel=1e-12) and below == bo
    print(f"N = {N}: FCC diamond gap ratio {r:.5f} above band {below} (the paper prints "
          f"{cfg['gap_ratio_paper']} at N = {cfg['N_paper']})")
    assert below == 2 and abs(r - cfg["gap_ratio_paper"]) < 0.005


def test_paper_gap_ratios_at_n150(B):
    """The paper's own grid, N = 150, for both of its printed band-gap ratios
    (Section 6.2's cubic cell, Section 6.3's BCC gyroid), 10 bands, tol 1e-5,
    mixed precision, 5 segments: every k-point converges and the ratios match
    the printed 0.14019 (bands 5-6) and 0.31745 (bands 2-3) to their last
    printed digit.  The FFT preconditioner runs its x-y plane pass as
    separate x and y passes at this N."""
    opts = B.default_opts(precision=1, warm_start=1, guard=2, streams=5, max_iter=500)
    cfg = workloads.CONFIGS["sc_sphere_cyl"]
    N = 150
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"])
    ctx = B.mfd_build_mu(N, 1.0, 2, workloads.mu_sc_sphere_cylinders(N))
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], opts)
    ctx.close()
    assert status == 0 and all(s["max_rel_resid"] <= cfg["tol"] for s in st), st
    r, below = B.mfd_gap_ratio(ev, kp)
    print(f"cubic cell, N = 150: gap ratio {r:.6f} above band {below} (paper {cfg['gap_ratio_paper']})")
    assert below == 5 and abs(r - cfg["gap_ratio_paper"]) < 5e-6
    cfg = workloads.CONFIGS["bcc_gyroid"]
    kp = workloads.kpath_vertices(cfg["path"], cfg["nk"], points=workloads.bcc_points())
    ctx = B.mfd_build_lattice_mu(N, workloads.lattice_vectors("bcc"), 2, workloads.mu_bcc_gyroid(N))
    ev, st, status = B.mfd_bands(ctx, kp, cfg["nbands"], cfg["tol"], opts)
    ctx.close()
    assert status == 0 and all(s["max_rel_resid"] <= cfg["tol"] for s in st), st
    r, below = B.mfd_gap_ratio(ev, kp)
    print(f"BCC gyroid, N = 150: gap ratio {r:.6f} above band {below} (paper {cfg['gap_ratio_paper']})")
    assert below == 2 and abs(r - cfg["gap_ratio_paper"]) < 5e-6
