"""General lattices (Section 2's coordinate change, Section 4.2's
D^_i = sum_j b_ji K_j + i L_i) on the GPU: operator, preconditioner and
Alg 4.1's recompute against the FP64 lattice oracle, and the band solve
against the exact discrete spectrum of a homogeneous cell, the oracle's
LOBPCG and the free-photon spectrum |k + G|^2."""
import numpy as np
import pytest

from oracle import lattice as lat
from oracle import lobpcg as olob
from oracle import mfd
from tests.gpu_util import rand_block, rand_eps, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TRICLINIC = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.4], [-0.3, 0.2, 1.2]])
LATTICES = {"bcc": lat.bcc_primitive(), "fcc": lat.fcc_primitive(1.3), "triclinic": TRICLINIC}
KS = [np.array([0.7, -0.4, 1.3]), np.zeros(3)]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


def _ctx(B, name, N, eps, order=2):
    A = LATTICES[name]
    return A, B.mfd_build_lattice(N, A, order, eps)


@pytest.mark.parametrize("name", sorted(LATTICES))
@pytest.mark.parametrize("N,ki,order", [(10, 0, 2), (12, 1, 2), (20, 0, 2), (16, 0, 4)])
def test_op_precond_lambda_fp64(B, name, N, ki, order):
    rng = np.random.default_rng(N * 7 + ki + order)
    k = KS[ki]
    eps = rand_eps(rng, N)
    X = rand_block(rng, 3, N)
    A, ctx = _ctx(B, name, N, eps, order)
    g, c = B.mfd_gamma_shift(ctx, k)
    Lc = lat.cell_length(A)
    assert g == pytest.approx(mfd.gamma_rule(N, Lc, k), rel=1e-14)
    assert c == pytest.approx(mfd.shift_rule(Lc, k), rel=1e-14, abs=0)
    mu = mfd.mu_from_eps(eps)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd)
    torch.cuda.synchronize()
    assert rel_err(Yd.cpu().numpy(), lat.apply_op(X, mu, k, A, g, order, c)) < 1e-13
    Td = torch.empty_like(Xd)
    B.mfd_precond_solve(ctx, k, Xd, Td)
    torch.cuda.synchronize()
    assert rel_err(Td.cpu().numpy(), lat.precond_solve(X, N, A, k, g, order, c)) < 1e-12
    lre = B.mfd_lambda_re(ctx, k, Xd)
    for b in range(3):
        assert abs(lre[b] - lat.lambda_re(X[b], mu, k, A, order)) <= 1e-12 * abs(lre[b])


@pytest.mark.parametrize("name", ["bcc", "triclinic"])
def test_op_fp32_storage(B, name):
    """FP32 fields: FP32 arithmetic (C64) and FP64 arithmetic (C64_F64)."""
    rng = np.random.default_rng(3)
    N, k = 16, np.array([0.3, 0.2, -0.9]) * np.pi
    eps = rand_eps(rng, N)
    X = rand_block(rng, 2, N).astype(np.complex64)
    A, ctx = _ctx(B, name, N, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    ref = lat.apply_op(X.astype(np.complex128), mfd.mu_from_eps(eps), k, A, g, 2, c)
    Xd = torch.from_numpy(X).cuda()
    for fp64 in (False, True):
        Yd = torch.empty_like(Xd)
        B.mfd_op_apply(ctx, k, Xd, Yd, fp64_arith=fp64)
        torch.cuda.synchronize()
        assert rel_err(Yd.cpu().numpy(), ref) < (1e-7 if fp64 else 3e-6)
    Td = torch.empty_like(Xd)
    B.mfd_precond_solve(ctx, k, Xd, Td)
    torch.cuda.synchronize()
    assert rel_err(Td.cpu().numpy(), lat.precond_solve(X.astype(np.complex128), N, A, k, g, 2, c)) < 3e-6


@pytest.mark.parametrize("name", sorted(LATTICES))
def test_precond_inverts_op_homogeneous(B, name):
    """For eps = 1 the FFT solve is the operator's exact inverse: the
    lattice symbols of the z-pass against the two-pass stencil."""
    rng = np.random.default_rng(11)
    N, k = 16, np.array([0.5, 0.1, 0.2]) * np.pi
    _, ctx = _ctx(B, name, N, np.ones((N, N, N)))
    X = torch.from_numpy(rand_block(rng, 2, N)).cuda()
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)
    B.mfd_op_apply(ctx, k, X, Y)
    B.mfd_precond_solve(ctx, k, Y, Z)
    torch.cuda.synchronize()
    assert rel_err(Z.cpu().numpy(), X.cpu().numpy()) < 1e-12


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["bcc", "fcc"])
def test_bands_homogeneous_closed_form(B, name, precision):
    """eps = 1: the band solve returns the exact discrete spectrum
    (closed form of the lattice symbols), and at N = 24 it lies within
    the second-order discretisation error of |k + G|^2."""
    N, m = 24, 10
    k = np.array([0.9, -0.3, 1.7])
    A, ctx = _ctx(B, name, N, np.ones((N, N, N)))
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-8 if precision else 1e-10,
                                 B.default_opts(precision=precision, streams=1))
    assert status == 0, st
    phys, _ = lat.closed_form_spectrum(N, A, k, st[0]["gamma"])
    assert np.allclose(ev[0], phys[:m], rtol=1e-7 if precision else 1e-10), (ev[0], phys[:m])
    free = lat.free_photon_omega2(A, k, m)      # discretisation error 4.9% (BCC), 0.5% (FCC)
    assert np.abs(ev[0] - free).max() <= 0.06 * free.max(), (ev[0], free)


@pytest.mark.parametrize("precision", [0, 1])
def test_bands_random_fcc_vs_oracle(B, precision):
    """A random two-material FCC cell at N = 12: GPU bands against the FP64
    LOBPCG oracle on the same lattice, two k-points on one call."""
    N, m = 12, 6
    rng = np.random.default_rng(5)
    eps = rand_eps(rng, N)
    A, ctx = _ctx(B, "fcc", N, eps)
    kp = np.array([[0.6, 0.2, -0.4], [2.0, 1.0, 0.5]])
    ev, st, status = B.mfd_bands(ctx, kp, m, 1e-8 if precision else 1e-10,
                                 B.default_opts(precision=precision, streams=1))
    assert status == 0, st
    for i, k in enumerate(kp):
        lam, _, info = olob.solve_bands(eps, 1.0, k, m, tol=1e-10, lattice=A)
        assert info["converged"]
        assert np.allclose(ev[i], lam, rtol=1e-7 if precision else 1e-10), (i, ev[i], lam)
        assert st[i]["max_rel_resid"] <= (1e-8 if precision else 1e-10)


def test_cubic_cell_through_the_lattice_path_matches_the_cubic_context(B):
    """A = L I through mfd_build_lattice (the z-marching lattice kernel and
    the lattice FFT symbols) against mfd_build (the fused cubic stencil and
    its closed-form symbols): two independent kernels, one operator."""
    rng = np.random.default_rng(21)
    N, L = 24, 1.3
    k = np.array([0.8, -0.3, 1.9])
    eps = rand_eps(rng, N)
    cl = B.mfd_build_lattice(N, L * np.eye(3), 2, eps)
    cc = B.mfd_build(N, L, 2, eps)
    assert B.mfd_gamma_shift(cl, k) == pytest.approx(B.mfd_gamma_shift(cc, k), rel=1e-14)
    X = torch.from_numpy(rand_block(rng, 4, N)).cuda()
    Ya, Yb, Ta, Tb = (torch.empty_like(X) for _ in range(4))
    B.mfd_op_apply(cl, k, X, Ya)
    B.mfd_op_apply(cc, k, X, Yb)
    B.mfd_precond_solve(cl, k, X, Ta)
    B.mfd_precond_solve(cc, k, X, Tb)
    torch.cuda.synchronize()
    assert rel_err(Ya.cpu().numpy(), Yb.cpu().numpy()) < 1e-13
    assert rel_err(Ta.cpu().numpy(), Tb.cpu().numpy()) < 1e-13
    ea, sa, _ = B.mfd_bands(cl, [k], 6, 1e-10, B.default_opts(precision=0, streams=1))
    eb, sb, _ = B.mfd_bands(cc, [k], 6, 1e-10, B.default_opts(precision=0, streams=1))
    assert np.allclose(ea, eb, rtol=1e-9)


def test_fused_lattice_kernel_ragged_tiles_and_uneven_chunks(B):
    """N = 100 (16 x 10 tiles leave a ragged edge of 4 columns; N = 12 above
    has ragged rows), 5 FP32-stored bands with FP64 arithmetic: 7 x 10 tiles
    x 5 bands call for 6 z chunks of 16 or 17 planes.  Against the oracle on
    the same FP32 inputs; the only difference is the final rounding to
    FP32."""
    rng = np.random.default_rng(22)
    N, k = 100, np.array([1.1, 0.4, -0.7])
    A = LATTICES["bcc"]
    eps = rand_eps(rng, N)
    ctx = B.mfd_build_lattice(N, A, 2, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    X = rand_block(rng, 5, N).astype(np.complex64)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd, fp64_arith=True)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    mu = mfd.mu_from_eps(eps)
    for b in range(5):
        ref = lat.apply_op(X[b].astype(np.complex128), mu, k, A, g, 2, c)
        assert rel_err(Y[b], ref) < 1e-7, b
