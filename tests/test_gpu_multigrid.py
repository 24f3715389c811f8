"""GPU parity of the multigrid preconditioner solve (Section 5.3, Alg 5.2)
against the oracle's multigrid (oracle/multigrid.py, same cycles, smoothing
steps and sweeps), element by element, through the C ABI; and band solves
preconditioned by it against the FFT-preconditioned ones and the oracle."""
import numpy as np
import pytest

from oracle import lobpcg as olob
from oracle import mfd
from oracle import multigrid as omg
from paper_2503_19379_amd import workloads
from tests.gpu_util import rand_block, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


KS = [np.array([0.7, -0.4, 1.3]), np.zeros(3), np.array([np.pi, np.pi, np.pi])]


@pytest.mark.parametrize("N,ki", [(16, 0), (16, 1), (16, 2), (24, 0), (20, 1), (32, 0)])
def test_precond_mg_fp64_matches_oracle(B, N, ki):
    """Hierarchies 16-8-4, 24-12-6-3, 20-10-5 and 32-16-8-4; generic k, Gamma
    (shifted) and the zone corner; two fields; in place and out of place."""
    rng = np.random.default_rng(700 + N + ki)
    L, k = 1.0, KS[ki]
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    g, c = B.mfd_gamma_shift(ctx, k)
    R = rand_block(rng, 2, N)
    Rd = torch.from_numpy(R).cuda()
    Td = torch.empty_like(Rd)
    B.mfd_precond_solve_mg(ctx, k, Rd, Td, cycles=2, smooth=2, sweeps=2)
    torch.cuda.synchronize()
    ref = omg.precond_solve_mg(R, N, L, k, g, c, cycles=2, n1=2, n2=2, sweeps=2)
    assert rel_err(Td.cpu().numpy(), ref) < 1e-12
    B.mfd_precond_solve_mg(ctx, k, Rd, Rd, cycles=2, smooth=2, sweeps=2)
    torch.cuda.synchronize()
    assert rel_err(Rd.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("cycles,smooth,sweeps", [(1, 1, 0), (3, 1, 3)])
def test_precond_mg_other_settings(B, cycles, smooth, sweeps):
    rng = np.random.default_rng(710 + cycles)
    N, L, k = 16, 1.0, KS[0]
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    g, c = B.mfd_gamma_shift(ctx, k)
    R = rand_block(rng, 1, N)
    Rd = torch.from_numpy(R).cuda()
    Td = torch.empty_like(Rd)
    B.mfd_precond_solve_mg(ctx, k, Rd, Td, cycles=cycles, smooth=smooth, sweeps=sweeps)
    torch.cuda.synchronize()
    ref = omg.precond_solve_mg(R, N, L, k, g, c, cycles=cycles, n1=smooth, n2=smooth, sweeps=sweeps)
    assert rel_err(Td.cpu().numpy(), ref) < 1e-12


def test_precond_mg_fp32_storage(B):
    rng = np.random.default_rng(720)
    N, L, k = 32, 1.0, KS[0]
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    g, c = B.mfd_gamma_shift(ctx, k)
    R = rand_block(rng, 2, N).astype(np.complex64)
    Rd = torch.from_numpy(R).cuda()
    Td = torch.empty_like(Rd)
    B.mfd_precond_solve_mg(ctx, k, Rd, Td)
    torch.cuda.synchronize()
    ref = omg.precond_solve_mg(R.astype(np.complex128), N, L, k, g, c)
    assert rel_err(Td.cpu().numpy(), ref) < 5e-6


def test_precond_mg_converges_to_fft_solve(B):
    """Enough V-cycles give (P + c)^-1 R, the FFT solve of Alg 5.1."""
    rng = np.random.default_rng(730)
    N, L, k = 32, 1.0, KS[0]
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    R = torch.from_numpy(rand_block(rng, 2, N)).cuda()
    T1 = torch.empty_like(R)
    T2 = torch.empty_like(R)
    B.mfd_precond_solve_mg(ctx, k, R, T1, cycles=16)
    B.mfd_precond_solve(ctx, k, R, T2)
    torch.cuda.synchronize()
    assert rel_err(T1.cpu().numpy(), T2.cpu().numpy()) < 1e-10


def test_precond_mg_unsupported(B):
    assert B.mfd_mg_supported(64) and B.mfd_mg_supported(96) and B.mfd_mg_supported(24)
    assert not B.mfd_mg_supported(100) and not B.mfd_mg_supported(120)
    N = 100
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    R = torch.zeros((1, 3, N, N, N), dtype=torch.complex64, device="cuda")
    with pytest.raises(B.MfdError):
        B.mfd_precond_solve_mg(ctx, [0.1, 0.2, 0.3], R, R)
    with pytest.raises(B.MfdError):
        B.mfd_bands(ctx, [[0.1, 0.2, 0.3]], 4, 1e-8, B.default_opts(precond=1))


@pytest.mark.parametrize("precision", [0, 1])
def test_bands_with_multigrid_match_oracle(B, precision):
    """Sphere N = 16, three k-points: LOBPCG preconditioned by the multigrid
    solve returns the oracle's bands (1e-10 FP64, 1e-7 mixed)."""
    N, m = 16, 6
    eps = workloads.eps_sphere(N)
    kp = workloads.kpath("GXMGR", 5)[[1, 2, 4]]
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    ev, st, status = B.mfd_bands(ctx, kp, m, tol, B.default_opts(precision=precision, precond=1, streams=1))
    assert status == 0, st
    for i, k in enumerate(kp):
        lam, _, _ = olob.solve_bands(eps, 1.0, k, m, tol=1e-10)
        assert np.allclose(ev[i], lam, rtol=1e-7 if precision else 1e-10), (i, ev[i], lam)
