"""mfd_lambda_re_static (no device allocation, static scratch) against
mfd_lambda_re, the entry point it mirrors, through the C ABI: two calls in a
row on one GPU, the second with a smaller input (fewer fields on a smaller
grid), each checked against the allocating call and the oracle."""
import numpy as np
import pytest

from oracle import mfd
from tests.gpu_util import rand_block, rand_eps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


def _case(B, N, nb, seed, k):
    rng = np.random.default_rng(seed)
    eps = rand_eps(rng, N)
    X = rand_block(rng, nb, N)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    Xd = torch.from_numpy(X).cuda()
    out = torch.full((nb,), float("nan"), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.mfd_lambda_re_static(ctx, k, Xd, out, stream=s.cuda_stream)
    s.synchronize()
    got = out.cpu().numpy()
    ref = B.mfd_lambda_re(ctx, k, Xd)
    mu = mfd.mu_from_eps(eps)
    orc = [mfd.lambda_re(x, mu, k, 1.0 / N) for x in X]
    return got, ref, orc


def test_static_matches_allocating_call_twice(B):
    k1 = np.array([0.4, 0.1, -0.3]) * np.pi
    got, ref, orc = _case(B, 24, 7, 11, k1)
    # same kernels, same launch shape, same summation order: identical values
    assert np.array_equal(got, ref), (got, ref)
    assert np.allclose(got, orc, rtol=1e-12)
    # a second call with a smaller input: the array keeps the first call's
    # partial sums, which the second call must not pick up
    k2 = np.zeros(3)
    got2, ref2, orc2 = _case(B, 12, 3, 12, k2)
    assert np.array_equal(got2, ref2), (got2, ref2)
    assert np.allclose(got2, orc2, rtol=1e-12)


def test_static_rejects_sizes_beyond_its_array(B):
    N = 8
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    X = torch.zeros((65, 3, N, N, N), dtype=torch.complex128, device="cuda")
    out = torch.zeros(65, dtype=torch.float64, device="cuda")
    with pytest.raises(B.MfdError):
        B.mfd_lambda_re_static(ctx, [0.1, 0.2, 0.3], X, out)
