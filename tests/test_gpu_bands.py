"""GPU band solve (LOBPCG + FFT preconditioner + Alg 4.1) against the oracle:
closed form (eps = 1), dense eigendecomposition (tiny grids) and the oracle's
LOBPCG."""
import functools

import numpy as np
import pytest

from oracle import lobpcg as olob
from oracle import mfd
from paper_2503_19379_amd import workloads
from tests.gpu_util import rand_eps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_19379_amd import binding
    binding.lib()
    return binding


def test_homog_n8_closed_form(B):
    cfg = workloads.CONFIGS["homog_n8"]
    N, k, m = cfg["N"], np.array(cfg["kpts"][0]), cfg["nbands"]
    ctx = B.mfd_build(N, 1.0, 2, workloads.crystal_eps(cfg["eps"], N))
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-10)
    assert status == 0, st
    g = mfd.gamma_rule(N, 1.0, k)
    phys, _ = mfd.closed_form_spectrum(N, 1.0, k, g)
    assert np.allclose(ev[0], phys[:m], rtol=1e-10), (ev, phys[:m])
    assert st[0]["gamma_doublings"] == 0 and st[0]["max_rel_resid"] <= 1e-10


def test_homog_n8_literal_gamma_alg41(B):
    """With gamma = 16 a compensation eigenvalue sits third; Alg 4.1 flags it."""
    N, k, m = 8, np.array([0.3, 0.2, 0.1]) * np.pi, 8
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    B.mfd_set_gamma(ctx, 16.0)
    phys, _ = mfd.closed_form_spectrum(N, 1.0, k, 16.0)
    # as printed (no spare columns): flag, double gamma, solve again
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-10, B.default_opts(guard=0))
    assert status == 0
    assert np.allclose(ev[0], phys[:m], rtol=1e-10)
    assert st[0]["gamma_doublings"] == 1 and st[0]["gamma"] == 32.0
    # with spare columns the flagged band is discarded
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-10, B.default_opts(guard=2))
    assert status == 0
    assert np.allclose(ev[0], phys[:m], rtol=1e-10)
    assert st[0]["gamma_doublings"] == 0 and st[0]["discarded"] == 1


@pytest.mark.parametrize("k", [np.array([0.5, 0.1, 0.2]) * np.pi, np.zeros(3), np.array([np.pi, np.pi, 0.0])])
def test_random_eps_n8_dense(B, k):
    rng = np.random.default_rng(1)
    N, m = 8, 8
    eps = rand_eps(rng, N)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-10)
    assert status == 0, st
    g = st[0]["gamma"]
    ref = np.linalg.eigvalsh(mfd.dense_matrix(eps, 1.0, k, g))[:m]
    if np.linalg.norm(k) == 0:
        assert np.all(np.abs(ev[0][:3]) < 1e-8)
        assert np.allclose(ev[0][3:], ref[3:], rtol=1e-10)
    else:
        assert np.allclose(ev[0], ref, rtol=1e-10)


def test_sphere_n16_vs_oracle(B):
    N, m = 16, 6
    eps = workloads.eps_sphere(N)
    kp = workloads.kpath("GXMGR", 5)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    ev, st, status = B.mfd_bands(ctx, kp, m, 1e-10)
    assert status == 0, st
    for i, k in enumerate(kp):
        lam, _, info = olob.solve_bands(eps, 1.0, k, m, tol=1e-10)
        if np.linalg.norm(k) == 0:
            assert np.all(np.abs(ev[i][:3]) < 1e-8)
            assert np.allclose(ev[i][3:], lam[3:], rtol=1e-10)
        else:
            assert np.allclose(ev[i], lam, rtol=1e-10), (i, ev[i], lam)


def test_stream_segments_match_single_stream(B):
    """Cutting the k-path into concurrently solved segments changes only the
    start blocks, not the converged eigenvalues."""
    N, m = 16, 6
    eps = workloads.eps_sphere(N)
    kp = workloads.kpath("GXMGR", 8)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, 1e-10, B.default_opts(streams=1))
    e4, s4, st4 = B.mfd_bands(ctx, kp, m, 1e-10, B.default_opts(streams=4))
    assert st1 == 0 and st4 == 0
    assert np.allclose(e1, e4, rtol=1e-9, atol=1e-9)


def test_batch_uneven_grids(B):
    """Several random-field crystals of different N in one batch call agree
    with solving each crystal alone."""
    Ns = (8, 12, 16, 24)
    crystals = [(N, workloads.eps_random_field(N, c)) for c, N in enumerate(Ns)]
    kp = workloads.kpath("GXMGR", 3)
    ctxs = [B.mfd_build(N, 1.0, 2, eps) for N, eps in crystals]
    evs, sts, status = B.mfd_bands_batch(ctxs, [kp] * len(ctxs), 5, 1e-10, B.default_opts(streams=3))
    assert status == 0
    for c, (N, eps) in enumerate(crystals):
        one = B.mfd_build(N, 1.0, 2, eps)
        e1, s1, st1 = B.mfd_bands(one, kp, 5, 1e-10, B.default_opts(streams=1))
        assert st1 == 0
        assert np.allclose(evs[c], e1, rtol=1e-9, atol=1e-9), (N, evs[c], e1)
    # and one crystal against the oracle
    N, eps = crystals[1]
    lam, _, info = olob.solve_bands(eps, 1.0, kp[1], 5, tol=1e-10)
    assert np.allclose(evs[1][1], lam, rtol=1e-10)


@pytest.mark.parametrize("N,kidx", [(16, (0, 2, 5, 7)), (24, (3,))])
def test_mixed_precision_vs_oracle(B, N, kidx):
    """FP32 corrections (preconditioner, stencil on W, W/P/AW/AP storage) with
    FP64 X, AX, Gram sums, Rayleigh-Ritz and residual refresh: eigenvalues
    within 1e-7 relative of the FP64 oracle, residuals verified with the FP64
    operator."""
    m = 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 8)[list(kidx)]
    ctx = B.mfd_build(N, 1.0, 2, eps)
    ev, st, status = B.mfd_bands(ctx, kp, m, 1e-8, B.default_opts(precision=1, streams=2))
    assert status == 0, st
    for i, k in enumerate(kp):
        assert st[i]["max_rel_resid"] <= 1e-8
        lam, _, info = olob.solve_bands(eps, 1.0, k, m, tol=1e-10)
        assert np.allclose(ev[i], lam, rtol=1e-7, atol=1e-9), (k, ev[i], lam)


def test_mixed_precision_fp64_fallback(B):
    """A stall window of 2 iterations forces the switch from FP32-stored
    directions to FP64 mid-solve (the path taken when a clustered spectrum
    stalls the mixed iteration); the bands still match the FP64 oracle."""
    N, m = 16, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 8)[[2, 5]]
    ctx = B.mfd_build(N, 1.0, 2, eps)
    ev, st, status = B.mfd_bands(ctx, kp, m, 1e-8, B.default_opts(precision=1, streams=1, stall_window=2))
    assert status == 0, st
    assert all(s["fp64_fallback"] == 1 for s in st), st
    for i, k in enumerate(kp):
        assert st[i]["max_rel_resid"] <= 1e-8
        lam, _, _ = olob.solve_bands(eps, 1.0, k, m, tol=1e-10)
        assert np.allclose(ev[i], lam, rtol=1e-7, atol=1e-9), (k, ev[i], lam)
    _, st0, _ = B.mfd_bands(ctx, kp, m, 1e-8, B.default_opts(precision=1, streams=1, stall_window=0))
    assert all(s["fp64_fallback"] == 0 for s in st0)


def test_large_grid_fp64_preconditioner_staged(B):
    """N = 100: the FP64 plane FFT does not fit in LDS, so FP64 iterations
    apply the preconditioner to an FP32 copy of W.  Homogeneous eps: the bands
    are the oracle's closed-form spectrum."""
    N, m = 100, 4
    k = np.array([0.3, 0.2, 0.1]) * np.pi
    ctx = B.mfd_build(N, 1.0, 2, np.ones((N, N, N)))
    ev, st, status = B.mfd_bands(ctx, [k], m, 1e-9, B.default_opts(precision=0, streams=1, max_iter=300))
    assert status == 0, st
    assert st[0]["max_rel_resid"] <= 1e-9, st
    phys, _ = mfd.closed_form_spectrum(N, 1.0, k, mfd.gamma_rule(N, 1.0, k))
    assert np.allclose(ev[0], phys[:m], rtol=1e-10), (ev, phys[:m])


def test_large_grid_mixed_fallback_to_staged_fp64(B):
    """N = 100, diamond: a stall window of 2 sends the mixed solve to FP64,
    whose preconditioner is staged through FP32 on this grid; the result
    reaches 1e-8 (fresh FP64 operator) and agrees with the FP64 solve."""
    N, m = 100, 4
    k = workloads.kpath("GXMGR", 8)[2]
    ctx = B.mfd_build(N, 1.0, 2, workloads.eps_diamond(N))
    ev1, st1, status = B.mfd_bands(ctx, [k], m, 1e-8, B.default_opts(precision=1, streams=1, max_iter=400,
                                                                      stall_window=2))
    assert status == 0, st1
    assert st1[0]["fp64_fallback"] == 1 and st1[0]["max_rel_resid"] <= 1e-8, st1
    ev0, st0, status = B.mfd_bands(ctx, [k], m, 1e-8, B.default_opts(precision=0, streams=1, max_iter=400))
    assert status == 0, st0
    assert np.allclose(ev1[0], ev0[0], rtol=1e-7), (ev1, ev0)


def test_autotune_changes_launch_shapes_not_results(B):
    """The autotuner picks each launch shape from its candidates; the bands
    agree with the built-in shapes'."""
    N, m = 24, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 6)
    c0 = B.mfd_build(N, 1.0, 2, eps)
    e0, s0, st0 = B.mfd_bands(c0, kp, m, 1e-9, B.default_opts(autotune=0, streams=2))
    assert st0 == 0 and B.mfd_tuning(c0)[0] is False
    c1 = B.mfd_build(N, 1.0, 2, eps)
    e1, s1, st1 = B.mfd_bands(c1, kp, m, 1e-9, B.default_opts(autotune=1, streams=2))
    assert st1 == 0
    tuned, t = B.mfd_tuning(c1)
    assert tuned
    assert t["gram_workgroups"] in (128, 256, 512, 1024)
    assert t["update_workgroups"] in (256, 512, 1024, 2048)
    assert t["stencil_workgroups"] in (512, 1024, 2048, 4096)
    assert t["fft_x_run"] in (4, 8)   # N = 24: no register-resident plan
    assert t["update_rows"] in (0, 16, 32)
    assert np.allclose(e0, e1, rtol=1e-8, atol=1e-9)


@functools.lru_cache(maxsize=None)
def _oracle_bands_n10(m):
    k = workloads.kpath("GXMGR", 8)[3]
    lam, _, _ = olob.solve_bands(workloads.eps_diamond(10), 1.0, k, m, tol=1e-10)
    return lam


@pytest.mark.parametrize("form", [0, 16, 32])
@pytest.mark.parametrize("precision", [0, 1])
def test_update_forms_agree(B, form, precision):
    """The three forms of the block update (one wave per 16-row strip, 16- or
    32-row workgroup blocks) give the same bands, all within the oracle's;
    mb = 18 exercises the two-tile column blocks, a ragged last strip
    (n = 3 * 10^3 = 3000 rows) the row masks."""
    N, m = 10, 16
    eps = workloads.eps_diamond(N)
    k = workloads.kpath("GXMGR", 8)[3]
    ctx = B.mfd_build(N, 1.0, 2, eps)
    B.mfd_set_tuning(ctx, dict(gram_workgroups=256, update_workgroups=256, stencil_workgroups=2048,
                               fft_x_run=0, update_rows=form))
    assert B.mfd_tuning(ctx) == (True, dict(gram_workgroups=256, update_workgroups=256,
                                            stencil_workgroups=2048, fft_x_run=0, update_rows=form))
    tol = 1e-8 if precision else 1e-10
    ev, st, status = B.mfd_bands(ctx, [k], m, tol, B.default_opts(precision=precision, streams=1))
    assert status == 0, st
    lam = _oracle_bands_n10(m)
    assert np.allclose(ev[0], lam, rtol=1e-7 if precision else 1e-10), (form, ev[0], lam)
    with pytest.raises(B.MfdError):
        B.mfd_set_tuning(ctx, dict(gram_workgroups=256, update_workgroups=256, stencil_workgroups=2048,
                                   fft_x_run=0, update_rows=8))
    B.mfd_set_tuning(ctx, None)
    assert B.mfd_tuning(ctx)[0] is False


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_block_vs_oracle(B, precision):
    """20 bands with 2 guard columns (the largest block, 22 columns: a
    66-column basis, five 16-column Gram blocks, six tail bands in the
    update) on a random two-material crystal against the oracle."""
    assert B.max_block() == 22
    N, m = 12, 20
    rng = np.random.default_rng(12)
    eps = rand_eps(rng, N)
    k = np.array([0.6, -0.2, 0.3]) * np.pi
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    ev, st, status = B.mfd_bands(ctx, [k], m, tol, B.default_opts(precision=precision, guard=2, streams=1))
    assert status == 0, st
    lam, _, info = olob.solve_bands(eps, 1.0, k, m, tol=1e-10)
    assert np.allclose(ev[0], lam, rtol=1e-7 if precision else 1e-10), (ev[0], lam)
    with pytest.raises(B.MfdError):
        B.mfd_bands(ctx, [k], m, tol, B.default_opts(guard=3, streams=1))


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_chunks_match_host_stepped(B, precision):
    """Iterations replayed from captured graphs (opts.graph = 1) give the same
    bands as the host-stepped loop, with fewer host synchronisations per
    iteration."""
    N, m = 16, 8
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 6)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    e0, s0, st0 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(precision=precision, streams=2, graph=0))
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(precision=precision, streams=2, graph=1))
    assert st0 == 0 and st1 == 0, (s0, s1)
    assert all(s["max_rel_resid"] <= tol for s in s1)
    assert np.allclose(e0, e1, rtol=1e-7 if precision else 1e-9, atol=1e-9), (e0, e1)
    per0 = sum(s["host_syncs"] for s in s0) / sum(s["iters"] for s in s0)
    per1 = sum(s["host_syncs"] for s in s1) / sum(s["iters"] for s in s1)
    assert per1 < 0.6 * per0, (per0, per1)


def test_graph_batch_matches_single(B):
    """The multi-crystal batch with graph chunks equals each crystal alone."""
    Ns = (8, 12, 16)
    crystals = [(N, workloads.eps_random_field(N, c)) for c, N in enumerate(Ns)]
    kp = workloads.kpath("GXMGR", 4)
    ctxs = [B.mfd_build(N, 1.0, 2, eps) for N, eps in crystals]
    evs, sts, status = B.mfd_bands_batch(ctxs, [kp] * len(ctxs), 5, 1e-9,
                                         B.default_opts(precision=1, streams=3, graph=1))
    assert status == 0
    for c, (N, eps) in enumerate(crystals):
        one = B.mfd_build(N, 1.0, 2, eps)
        e1, s1, st1 = B.mfd_bands(one, kp, 5, 1e-9, B.default_opts(precision=1, streams=1, graph=0))
        assert st1 == 0
        assert np.allclose(evs[c], e1, rtol=1e-7, atol=1e-9), (N, evs[c], e1)


@pytest.mark.parametrize("precision", [0, 1])
def test_plane_wave_cold_start(B, precision):
    """cold_start = 1 (segments start from the lowest transverse plane waves
    at their first k-point, Gamma's three constant fields among them) changes
    only the start blocks: the diamond N = 16 path in 4 segments returns the
    random-start bands, and a k-point matches the oracle."""
    N, m = 16, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 12)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    opts = dict(precision=precision, streams=4, guard=2)
    e0, s0, st0 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(cold_start=0, **opts))
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(cold_start=1, **opts))
    assert st0 == 0 and st1 == 0, (s0, s1)
    assert all(s["max_rel_resid"] <= tol for s in s1)
    assert np.allclose(e0, e1, rtol=1e-7 if precision else 1e-9, atol=1e-9)
    lam, _, _ = olob.solve_bands(eps, 1.0, kp[3], m, tol=1e-10)
    assert np.allclose(e1[3], lam, rtol=1e-7 if precision else 1e-9), (e1[3], lam)


def test_plane_wave_cold_start_on_a_lattice(B):
    """The same on a BCC cell (reciprocal vectors 2 pi A^-T m): random and
    plane-wave starts give the same bands."""
    N, m = 12, 6
    A = workloads.lattice_vectors("bcc")
    rng = np.random.default_rng(5)
    ctx = B.mfd_build_lattice(N, A, 2, rand_eps(rng, N))
    kp = workloads.kpath_vertices("hGPNH", 8, points=workloads.bcc_points())
    e0, s0, st0 = B.mfd_bands(ctx, kp, m, 1e-9, B.default_opts(cold_start=0, streams=2))
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, 1e-9, B.default_opts(cold_start=1, streams=2))
    assert st0 == 0 and st1 == 0, (s0, s1)
    assert np.allclose(e0, e1, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_balanced_segments(B, precision):
    """opts.balance = 1 (a stream whose segment is done takes the second half
    of the k-points ahead of the busiest other one, with a cold start) changes
    only where segments start: the diamond N = 16 path on 3 streams returns
    the fixed-segment bands, every k-point is solved, a k-point matches the
    oracle, and warm_start 2 with balance is refused."""
    N, m = 16, 6
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 16)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    opts = dict(precision=precision, streams=3, guard=2, cold_start=1)
    e0, s0, st0 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(balance=0, **opts))
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(balance=1, **opts))
    assert st0 == 0 and st1 == 0, (s0, s1)
    assert all(s["iters"] > 0 and s["max_rel_resid"] <= tol for s in s1)
    rt = 1e-7 if precision else 1e-9
    assert np.allclose(e0, e1, rtol=rt, atol=1e-9)
    lam, _, _ = olob.solve_bands(eps, 1.0, kp[11], m, tol=1e-10)
    assert np.allclose(e1[11], lam, rtol=rt), (e1[11], lam)
    with pytest.raises(RuntimeError):
        B.mfd_bands(ctx, kp[:4], m, tol, B.default_opts(balance=1, warm_start=2, **opts))


@pytest.mark.parametrize("precision", [0, 1])
def test_hard_lock_matches_soft(B, precision):
    """opts.hard_lock = 1 (once at most 8 bands iterate, the converged ones
    are locked and the iteration runs on the rest, its search directions made
    orthogonal to the locked vectors) returns the soft-locking bands: diamond
    N = 16, 10 bands + 2 guard on a 10-point path, every k-point converged, and
    a k-point matches the oracle."""
    N, m = 16, 10
    eps = workloads.eps_diamond(N)
    kp = workloads.kpath("GXMGR", 10)
    ctx = B.mfd_build(N, 1.0, 2, eps)
    tol = 1e-8 if precision else 1e-10
    opts = dict(precision=precision, streams=2, guard=2, cold_start=1)
    e0, s0, st0 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(hard_lock=0, **opts))
    e1, s1, st1 = B.mfd_bands(ctx, kp, m, tol, B.default_opts(hard_lock=1, **opts))
    assert st0 == 0 and st1 == 0, (s0, s1)
    assert all(s["max_rel_resid"] <= tol for s in s1)
    rt = 1e-7 if precision else 1e-9
    assert np.allclose(e0, e1, rtol=rt, atol=1e-9)
    lam, _, _ = olob.solve_bands(eps, 1.0, kp[6], m, tol=1e-10)
    assert np.allclose(e1[6], lam, rtol=rt), (e1[6], lam)


@pytest.mark.parametrize("hard", [0, 1])
def test_repeated_solves_bit_identical(B, hard):
    """With the launch shapes fixed (autotune off), the same band solve on
    concurrent segments gives the same iteration counts and the same
    eigenvalue bits when repeated: every sum runs in a fixed order and no
    segment reads another's buffers (diamond N = 16, 10 bands + 2 guard,
    10 k-points on 3 segments, mixed precision)."""
    N, m = 16, 10
    ctx = B.mfd_build(N, 1.0, 2, workloads.eps_diamond(N))
    kp = workloads.kpath("GXMGR", 10)
    o = B.default_opts(precision=1, streams=3, guard=2, cold_start=1, hard_lock=hard, autotune=0)
    runs = [B.mfd_bands(ctx, kp, m, 1e-8, o) for _ in range(3)]
    for ev, st, status in runs:
        assert status == 0
    its0 = [s["iters"] for s in runs[0][1]]
    for ev, st, _ in runs[1:]:
        assert [s["iters"] for s in st] == its0
        assert np.array_equal(ev, runs[0][0])
