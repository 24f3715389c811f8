"""GPU parity of the operator, the FFT preconditioner and Alg 4.1's
recompute against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import mfd
from tests.gpu_util import rand_block, rand_eps, rel_err

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


@pytest.mark.parametrize("N", [8, 12, 20, 24, 32, 64, 96, 100, 128])
@pytest.mark.parametrize("ki", [0, 1, 2])
def test_op_apply_fp64(B, N, ki):
    """Every lane layout of the stencil: whole rows packed 8, 5, 3, 2 and 2 to
    a wave (N = 8, 12, 20, 24, 32), one row (64), and rows cut into segments
    with halo lanes: 2 x 48 (96), 2 x 50 (100) and 43 + 43 + 42 (128)."""
    rng = np.random.default_rng(100 + N + ki)
    L = 1.0
    k = KS[ki]
    eps = rand_eps(rng, N)
    nb = 3 if N <= 32 else 2 if N <= 64 else 1
    X = rand_block(rng, nb, N)
    ctx = B.mfd_build(N, L, 2, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    assert np.isclose(g, mfd.gamma_rule(N, L, k)) and np.isclose(c, mfd.shift_rule(L, k))
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd)
    torch.cuda.synchronize()
    ref = mfd.apply_op(X, mfd.mu_from_eps(eps), k, L / N, g, 2, c)
    assert rel_err(Yd.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("N", [16, 48, 96, 100, 120, 128, 150])
def test_op_apply_fp32(B, N):
    """Rows packed 4 to a wave (16), a 48-lane row (48), and segmented rows
    (96, 100, 120: two segments, 128 and 150: three)."""
    rng = np.random.default_rng(7 + N)
    L, k = 1.0, np.array([0.3, 0.2, -0.9]) * np.pi
    eps = rand_eps(rng, N)
    X = rand_block(rng, 2 if N <= 48 else 1, N)
    ctx = B.mfd_build(N, L, 2, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    Xd = torch.from_numpy(X.astype(np.complex64)).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd)
    torch.cuda.synchronize()
    ref = mfd.apply_op(X.astype(np.complex64).astype(np.complex128), mfd.mu_from_eps(eps), k, L / N, g, 2, c)
    assert rel_err(Yd.cpu().numpy(), ref) < 2e-6


@pytest.mark.parametrize("N", [16, 24, 32, 48, 64, 96, 100])
@pytest.mark.parametrize("ki", [0, 1])
def test_op_apply_fp32_storage_fp64_arith(B, N, ki):
    """MFD_C64_F64, the operator the mixed-precision solver applies to its
    FP32-stored blocks: FP64 arithmetic on FP32 inputs, so the only error is
    the FP32 rounding of the output (2^-24 per component)."""
    rng = np.random.default_rng(400 + N + ki)
    L, k = 1.0, KS[ki]
    eps = rand_eps(rng, N)
    X = rand_block(rng, 2 if N <= 64 else 1, N).astype(np.complex64)
    ctx = B.mfd_build(N, L, 2, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd, fp64_arith=True)
    torch.cuda.synchronize()
    ref = mfd.apply_op(X.astype(np.complex128), mfd.mu_from_eps(eps), k, L / N, g, 2, c)
    got = Yd.cpu().numpy().astype(np.complex128)
    assert rel_err(got, ref) < 1e-7
    # element-wise: the FP32 rounding of each output component, plus the FP64
    # level of the operator (1e-12 of the largest entry, as in the FP64 test)
    assert np.all(np.abs(got - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-12 * np.max(np.abs(ref)))


@pytest.mark.parametrize("nb,dtype", [(11, "f64"), (11, "f64s32"), (16, "f32")])
def test_op_apply_n64_uneven_z_chunks(B, nb, dtype):
    """N = 64 stencil on wider blocks: 11 fields make 352 waves per z chunk,
    so the default target of 2048 waves cuts z into 6 chunks of 10 or 11
    planes (uneven); 16 fields in FP32 are the benchmark's full block.
    Against the FP64 oracle, element-wise as in the tests above."""
    N = 64
    rng = np.random.default_rng(900 + nb)
    L, k = 1.0, np.array([0.7, -0.4, 1.3])
    eps = rand_eps(rng, N)
    X = rand_block(rng, nb, N)
    if dtype != "f64":
        X = X.astype(np.complex64)
    ctx = B.mfd_build(N, L, 2, eps)
    g, c = B.mfd_gamma_shift(ctx, k)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    B.mfd_op_apply(ctx, k, Xd, Yd, fp64_arith=(dtype == "f64s32"))
    torch.cuda.synchronize()
    ref = mfd.apply_op(X.astype(np.complex128), mfd.mu_from_eps(eps), k, L / N, g, 2, c)
    got = Yd.cpu().numpy().astype(np.complex128)
    if dtype == "f64":
        assert rel_err(got, ref) < 1e-13
    elif dtype == "f64s32":
        assert np.all(np.abs(got - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-12 * np.max(np.abs(ref)))
    else:
        assert rel_err(got, ref) < 2e-6


@pytest.mark.parametrize("N", [8, 12, 20, 24, 32, 48, 64, 100, 150])
@pytest.mark.parametrize("ki", [0, 1])
def test_precond_fp64(B, N, ki):
    """N = 100 and 150: FP64 planes larger than LDS, transformed as separate
    x and y passes."""
    rng = np.random.default_rng(200 + N + ki)
    L = 1.0
    k = KS[ki]
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    g, c = B.mfd_gamma_shift(ctx, k)
    R = rand_block(rng, 2, N)
    Rd = torch.from_numpy(R).cuda()
    Td = torch.empty_like(Rd)
    B.mfd_precond_solve(ctx, k, Rd, Td)
    torch.cuda.synchronize()
    ref = mfd.precond_solve(R, N, L, k, g, 2, c)
    assert rel_err(Td.cpu().numpy(), ref) < 1e-12
    # in place
    B.mfd_precond_solve(ctx, k, Rd, Rd)
    torch.cuda.synchronize()
    assert rel_err(Rd.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("N", [16, 96])
def test_precond_fp32(B, N):
    rng = np.random.default_rng(300 + N)
    L, k = 1.0, np.array([0.5, -0.25, 0.1]) * np.pi
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    g, c = B.mfd_gamma_shift(ctx, k)
    R = rand_block(rng, 1, N).astype(np.complex64)
    Rd = torch.from_numpy(R).cuda()
    Td = torch.empty_like(Rd)
    B.mfd_precond_solve(ctx, k, Rd, Td)
    torch.cuda.synchronize()
    ref = mfd.precond_solve(R.astype(np.complex128), N, L, k, g, 2, c)
    assert rel_err(Td.cpu().numpy(), ref) < 5e-6


@pytest.mark.parametrize("N,xrun", [(64, 4), (64, 8), (64, 16), (64, -1), (32, -1), (16, -1), (100, 0), (120, 0),
                                    (150, 0)])
def test_precond_fp32_solver_instances(B, N, xrun):
    """Element-wise FP32 parity of the instances the solves run: N = 64 with
    each z-pass x run the autotuner may pick, the register-resident passes
    (plan -1) at N = 16, 32, 64, the radix-5 and radix-3 plans of N = 100
    and 120 (band-gap workloads), and N = 150 (split x and y passes, z runs of
    10 x), on a two-field block at a generic k and at
    k = 0 (shifted)."""
    rng = np.random.default_rng(400 + N + xrun)
    L = 1.0
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    if xrun:
        B.mfd_set_tuning(ctx, dict(gram_workgroups=256, update_workgroups=512, stencil_workgroups=2048,
                                   fft_x_run=xrun, update_rows=0))
    for k in (np.array([0.5, -0.25, 0.1]) * np.pi, np.zeros(3)):
        g, c = B.mfd_gamma_shift(ctx, k)
        R = rand_block(rng, 2, N).astype(np.complex64)
        Rd = torch.from_numpy(R).cuda()
        Td = torch.empty_like(Rd)
        B.mfd_precond_solve(ctx, k, Rd, Td)
        torch.cuda.synchronize()
        got = Td.cpu().numpy()
        ref = mfd.precond_solve(R.astype(np.complex128), N, L, k, g, 2, c)
        # element-wise, against the block's largest entry: FP32 FFTs of
        # length N err by about log2 N unit roundoffs
        assert rel_err(got, ref) < 5e-6, (N, xrun, k)


def test_precond_inverts_operator_homogeneous(B):
    """eps = 1: P = the compensated operator, so precond(op(x)) = x."""
    N, L = 32, 1.0
    k = np.array([0.3, 0.2, 0.1]) * np.pi
    rng = np.random.default_rng(5)
    ctx = B.mfd_build(N, L, 2, np.ones((N, N, N)))
    X = torch.from_numpy(rand_block(rng, 2, N)).cuda()
    Y = torch.empty_like(X)
    B.mfd_op_apply(ctx, k, X, Y)
    B.mfd_precond_solve(ctx, k, Y, Y)
    torch.cuda.synchronize()
    assert rel_err(Y.cpu().numpy(), X.cpu().numpy()) < 1e-11


def test_lambda_re(B):
    N, L = 16, 1.0
    k = np.array([0.4, 0.1, -0.3]) * np.pi
    rng = np.random.default_rng(9)
    eps = rand_eps(rng, N)
    X = rand_block(rng, 3, N)
    ctx = B.mfd_build(N, L, 2, eps)
    got = B.mfd_lambda_re(ctx, k, torch.from_numpy(X).cuda())
    mu = mfd.mu_from_eps(eps)
    ref = [mfd.lambda_re(x, mu, k, L / N) for x in X]
    assert np.allclose(got, ref, rtol=1e-12)


def test_invalid_arguments(B):
    N = 8
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    X = torch.zeros((1, 3, N, N, N), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.MfdError):
        B.mfd_op_apply(ctx, [0.1, 0.2, np.nan], X, torch.zeros_like(X))
    with pytest.raises(B.MfdError):
        B.mfd_op_apply(ctx, [0.1, 0.2, 0.3], X, X)          # aliasing
    with pytest.raises(B.MfdError):
        B.mfd_build(N, 1.0, 2, -np.ones((N, N, N)))
    with pytest.raises(B.MfdError):
        B.mfd_build(7, 1.0, 2, np.ones((7, 7, 7)))
