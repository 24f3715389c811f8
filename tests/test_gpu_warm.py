"""The learned warm start on the GPU: the network's forward, gradient and Adam
kernels and the training target against the FP64 oracle (oracle/mlp.py), and
the band solve with warm_start = 2."""
import numpy as np
import pytest

from oracle import lobpcg as olob
from oracle import mlp as omlp
from paper_2503_19379_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


# the production shapes for mb = 8 columns (6 bands + 2 guard) and mb = 22
# (20 bands + 2 guard, a full replay buffer), and a ragged small one
SHAPES = [(6 + 16 + 256, 256, 3, 256, 5), (6 + 44 + 1936, 256, 3, 1936, 64), (37, 20, 2, 19, 3)]


def _net(B, nin, nh, nl, nout, bmax, bf16, seed=0):
    rng = np.random.default_rng(seed)
    shapes = omlp.layer_shapes(nin, nh, nl, nout)
    theta = (rng.standard_normal(omlp.n_params(shapes)) * 0.1).astype(np.float32)
    net = B.Mlp(nin, nh, nl, nout, bmax, bf16=bf16)
    assert net.nparams == theta.size
    net.set_params(theta)
    X = rng.standard_normal((bmax, nin)).astype(np.float32)
    T = rng.standard_normal((bmax, nout)).astype(np.float32)
    return net, shapes, theta, X, T


def _weights_bf16(theta, shapes):
    """Round the W parts (not the biases) to bfloat16, as the kernels read them."""
    t = theta.astype(np.float64).copy()
    off = 0
    for o, i in shapes:
        t[off:off + o * i] = omlp.bf16_round(theta[off:off + o * i])
        off += o * i + o
    return t


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_forward_and_gradient(B, shape, bf16):
    nin, nh, nl, nout, bmax = shape
    net, shapes, theta, X, T = _net(B, nin, nh, nl, nout, bmax, bf16)
    ref_theta = _weights_bf16(theta, shapes) if bf16 else theta.astype(np.float64)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    Yd = torch.empty(bmax, nout, dtype=torch.float32, device="cuda")
    net.forward(Xd, Yd)
    Yref, _ = omlp.forward(ref_theta, shapes, X.astype(np.float64))
    assert np.max(np.abs(Yd.cpu().numpy() - Yref)) <= 1e-5 * np.max(np.abs(Yref))
    g = torch.empty(net.nparams, dtype=torch.float32, device="cuda")
    loss = net.loss_grad(Xd, Td, g)
    lref, gref = omlp.loss_and_grad(ref_theta, shapes, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lref) <= 1e-5 * lref
    gg = g.cpu().numpy()
    assert np.max(np.abs(gg - gref)) <= 1e-4 * np.max(np.abs(gref)), np.max(np.abs(gg - gref))


def test_mlp_adam_step(B):
    nin, nh, nl, nout, bmax = SHAPES[-1]   # the ragged small shape
    net, shapes, theta, X, T = _net(B, nin, nh, nl, nout, bmax, False, seed=2)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in (1, 2, 3):
        net.loss_grad(Xd, Td)
        net.adam_step(1e-2)
        _, g = omlp.loss_and_grad(th, shapes, X.astype(np.float64), T.astype(np.float64))
        th, m, v = omlp.adam_step(th, g, m, v, t, lr=1e-2)
        # |step| <= lr per parameter; FP32 gradients change it by far less than lr / 100
        assert np.max(np.abs(net.get_params() - th)) <= 1e-4, t


def test_mlp_training_reduces_loss(B):
    """Fits a fixed regression with the bfloat16 forward/backward and Adam."""
    rng = np.random.default_rng(3)
    nin, nout, bmax = 40, 30, 16
    net = B.Mlp(nin, 64, 3, nout, bmax, bf16=True, seed=5)
    X = torch.from_numpy(rng.standard_normal((bmax, nin)).astype(np.float32)).cuda()
    W = rng.standard_normal((nout, nin)) / np.sqrt(nin)
    T = torch.tanh(X @ torch.from_numpy(np.ascontiguousarray(W.T).astype(np.float32)).cuda())
    l0 = net.loss_grad(X, T)
    for _ in range(300):
        net.loss_grad(X, T)
        net.adam_step(3e-3)
    assert net.loss_grad(X, T) < 0.05 * l0


def _blocks(rng, n, mb, step=0.1):
    def cplx(*s):
        return rng.standard_normal(s) + 1j * rng.standard_normal(s)
    Xb = np.linalg.qr(cplx(n, mb))[0]
    Xa = np.linalg.qr(Xb + step * cplx(n, mb))[0]
    Xc = np.linalg.qr(Xb + step * cplx(n, mb))[0]
    return Xa, Xb, Xc


@pytest.mark.parametrize("n,mb", [(700, 5), (3000, 21)])
def test_warm_target_vs_oracle(B, n, mb):
    rng = np.random.default_rng(n)
    Xa, Xb, Xc = _blocks(rng, n, mb)
    dev = lambda X: torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    C = torch.empty(2 * mb, mb, dtype=torch.complex128, device="cuda")
    Ri = torch.empty(2 * mb, 2 * mb, dtype=torch.complex128, device="cuda")
    B.mfd_warm_target(dev(Xa), dev(Xb), dev(Xc), C, Ri)
    Cref, _ = omlp.warm_target(Xa, Xb, Xc)
    assert np.max(np.abs(C.cpu().numpy() - Cref)) <= 1e-10
    _, R2 = omlp.orth_basis(Xc @ omlp.procrustes(Xc, Xb), Xb)
    assert np.max(np.abs(Ri.cpu().numpy() - np.linalg.inv(R2))) <= 1e-9 * np.max(np.abs(np.linalg.inv(R2)))


def test_warm_target_dependent_blocks(B):
    rng = np.random.default_rng(9)
    Xa, Xb, Xc = _blocks(rng, 500, 4)
    dev = lambda X: torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    C = torch.empty(8, 4, dtype=torch.complex128, device="cuda")
    with pytest.raises(B.MfdError) as e:
        B.mfd_warm_target(dev(Xb), dev(Xb), dev(Xc), C)
    assert e.value.status == -4


@pytest.mark.parametrize("mb,L", [(8, 1.0), (22, 1.7)])
def test_warm_features_vs_oracle(B, mb, L):
    """The network's input row built on the device equals the oracle's
    features() (FP32 rounding of the FP64 values)."""
    rng = np.random.default_rng(mb)
    k_prev, k_next = rng.standard_normal(3), rng.standard_normal(3)
    lam_j, lam_jm1 = rng.random(mb) * 40, rng.random(mb) * 40
    C = rng.standard_normal((2 * mb, mb)) + 1j * rng.standard_normal((2 * mb, mb))
    row = torch.empty(6 + 2 * mb + 4 * mb * mb, dtype=torch.float32, device="cuda")
    B.mfd_warm_features(L, k_prev, k_next, lam_j, lam_jm1, torch.from_numpy(C).cuda(), row)
    ref = omlp.features(k_prev, k_next, lam_j, lam_jm1, C, L=L)
    assert ref.shape == row.shape
    assert np.array_equal(row.cpu().numpy(), ref.astype(np.float32))


def _path_run(B, ctx, kp, m, tol, **kw):
    ev, st, status = B.mfd_bands(ctx, kp, m, tol, B.default_opts(streams=1, **kw))
    assert status == 0, st
    return ev, st


def test_learned_warm_start_bands(B):
    """warm_start = 2 returns the same bands as the previous-k start; no
    proposal before the 4th training pair (the first history triple holds the
    constant fields of Gamma, whose blocks are dependent, so pairs start one
    solve later); some proposals pass the Ritz-sum test; the bands match the
    oracle at sampled k-points."""
    N, m = 16, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 40)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    # 1e-9: at 1e-10 a k-point 0.05 from Gamma (a compensation mode inside the
    # band window there) sits at the FP64 limit for some start blocks
    e1, s1 = _path_run(B, ctx, kp, m, 1e-9, warm_start=1)
    e2, s2 = _path_run(B, ctx, kp, m, 1e-9, warm_start=2)
    assert np.allclose(e1, e2, rtol=1e-8, atol=1e-9)
    fb = [s["used_fallback"] for s in s2]
    assert fb[0] == 0 and all(f == 1 for f in fb[1:8]), fb
    used = [i for i, f in enumerate(fb) if i > 0 and f == 0]
    assert len(used) >= 5, fb
    for i in (used[0], used[-1]):
        lam, _, _ = olob.solve_bands(eps, 1.0, kp[i], m, tol=1e-10)
        assert np.allclose(e2[i], lam, rtol=1e-8), (i, e2[i], lam)


def test_learned_warm_start_gain(B):
    """Once the network proposes (k-points 8 on), the learned start needs fewer
    LOBPCG iterations than the previous-k start, in FP64 and in mixed
    precision; the untrained network (learn_steps = 0, which proposes the
    previous step's combination unchanged) is reported beside it."""
    N, m = 16, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 40)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    for prec in (0, 1):
        _, s1 = _path_run(B, ctx, kp, m, 1e-8, warm_start=1, precision=prec)
        _, s2 = _path_run(B, ctx, kp, m, 1e-8, warm_start=2, precision=prec)
        _, s0 = _path_run(B, ctx, kp, m, 1e-8, warm_start=2, precision=prec, learn_steps=0)
        it1 = sum(s["iters"] for s in s1[7:])
        it2 = sum(s["iters"] for s in s2[7:])
        it0 = sum(s["iters"] for s in s0[7:])
        print(f"precision {prec}: iterations over k-points 8..40: previous-k {it1}, learned {it2}, "
              f"untrained {it0}")
        assert it2 < it1
