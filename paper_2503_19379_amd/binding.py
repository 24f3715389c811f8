"""Thin ctypes binding of the mfdkc C ABI (include/mfdkc.h).

Argument marshalling only: every call goes straight to libmfdkc.so, built
in-tree by ``paper_2503_19379_amd.build``.  Device buffers are torch tensors
(complex128 for MFD_C128, complex64 for MFD_C64) of shape (nb, 3, N, N, N);
streams are the current torch stream unless one is passed.  There is no CPU
fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfdkc.so")

MFD_C64 = 1
MFD_C128 = 2
MFD_C64_F64 = 3   # FP32 storage, FP64 arithmetic (mfd_op_apply)
STATUS = {0: "MFD_OK", -1: "MFD_EINVAL", -2: "MFD_ENOMEM", -3: "MFD_EDEVICE", -4: "MFD_ENOTCONV",
          -5: "MFD_ESPURIOUS", -6: "MFD_EUNSUPPORTED"}


class MfdError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


class mfd_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("precision", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("max_gamma_doublings", ctypes.c_int), ("guard", ctypes.c_int),
                ("streams", ctypes.c_int), ("x0", ctypes.c_void_p), ("stall_window", ctypes.c_int),
                ("learn_steps", ctypes.c_int), ("learn_rate", ctypes.c_float), ("autotune", ctypes.c_int),
                ("precond", ctypes.c_int), ("mg_cycles", ctypes.c_int), ("mg_smooth", ctypes.c_int),
                ("mg_sweeps", ctypes.c_int), ("graph", ctypes.c_int), ("cold_start", ctypes.c_int),
                ("balance", ctypes.c_int), ("hard_lock", ctypes.c_int)]


class mfd_kstats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("gamma_doublings", ctypes.c_int), ("gamma", ctypes.c_double),
                ("max_rel_resid", ctypes.c_double), ("spurious", ctypes.c_int), ("discarded", ctypes.c_int),
                ("used_fallback", ctypes.c_int), ("fp64_fallback", ctypes.c_int), ("ms", ctypes.c_float),
                ("rejected_steps", ctypes.c_int), ("host_syncs", ctypes.c_int), ("segment_start", ctypes.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_19379_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.mfd_build.argtypes = [i, d, i, dp, vp, ctypes.POINTER(vp)]
        L.mfd_build_mu.argtypes = [i, d, i, dp, vp, ctypes.POINTER(vp)]
        L.mfd_build_lattice.argtypes = [i, dp, i, dp, vp, ctypes.POINTER(vp)]
        L.mfd_build_lattice_mu.argtypes = [i, dp, i, dp, vp, ctypes.POINTER(vp)]
        L.mfd_gap_ratio.argtypes = [i, i, dp, dp, dp, ctypes.POINTER(i)]
        L.mfd_supported_n.argtypes = [i]
        L.mfd_max_block.argtypes = []
        L.mfd_lambda_re_static.argtypes = [vp, dp, i, vp, vp, vp]
        L.mfd_precond_solve_mg.argtypes = [vp, dp, i, i, i, i, i, vp, vp, vp]
        L.mfd_mg_supported.argtypes = [i]
        L.mfd_set_gamma.argtypes = [vp, d]
        L.mfd_gamma_shift.argtypes = [vp, dp, dp, dp]
        L.mfd_op_apply.argtypes = [vp, dp, i, i, vp, vp, vp]
        L.mfd_precond_solve.argtypes = [vp, dp, i, i, vp, vp, vp]
        L.mfd_lambda_re.argtypes = [vp, dp, i, vp, dp, vp]
        L.mfd_bands.argtypes = [vp, i, dp, i, d, ctypes.POINTER(mfd_opts), dp, vp,
                                ctypes.POINTER(mfd_kstats), vp]
        L.mfd_bands_batch.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(dp), i, d,
                                      ctypes.POINTER(mfd_opts), ctypes.POINTER(dp),
                                      ctypes.POINTER(ctypes.POINTER(mfd_kstats)), vp]
        L.mfd_default_opts.argtypes = [ctypes.POINTER(mfd_opts)]
        L.mfd_default_opts.restype = None
        L.mfd_profile.argtypes = [vp, i]
        L.mfd_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), dp]
        L.mfd_destroy.argtypes = [vp]
        L.mfd_destroy.restype = None
        L.mfd_strerror.argtypes = [i]
        L.mfd_strerror.restype = ctypes.c_char_p
        L.mfd_last_error.restype = ctypes.c_char_p
        fp = ctypes.POINTER(ctypes.c_float)
        L.mfd_mlp_create.argtypes = [i, i, i, i, i, i, ctypes.c_ulonglong, ctypes.POINTER(vp)]
        L.mfd_mlp_num_params.argtypes = [vp]
        L.mfd_mlp_num_params.restype = ctypes.c_longlong
        L.mfd_mlp_set_params.argtypes = [vp, fp]
        L.mfd_mlp_get_params.argtypes = [vp, fp]
        L.mfd_mlp_forward.argtypes = [vp, i, vp, vp, vp]
        L.mfd_mlp_loss_grad.argtypes = [vp, i, vp, vp, dp, vp, vp]
        L.mfd_mlp_adam_step.argtypes = [vp, ctypes.c_float, vp]
        L.mfd_mlp_destroy.argtypes = [vp]
        L.mfd_mlp_destroy.restype = None
        L.mfd_warm_target.argtypes = [ctypes.c_longlong, i, vp, vp, vp, vp, vp, vp]
        L.mfd_warm_features.argtypes = [ctypes.c_double, i, dp, dp, dp, dp, vp, vp, vp]
        L.mfd_tuning.argtypes = [vp, ctypes.POINTER(i)]
        L.mfd_set_tuning.argtypes = [vp, ctypes.POINTER(i)]
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise MfdError(status, lib().mfd_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _k(k):
    a = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(3))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dtype(t):
    import torch
    if t.dtype == torch.complex128:
        return MFD_C128
    if t.dtype == torch.complex64:
        return MFD_C64
    raise TypeError("fields must be complex64 or complex128")


def _dev(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns an mfd_ctx handle (freed by close() or garbage collection)."""

    def __init__(self, handle, N, L):
        self.handle = handle
        self.N = N
        self.L = L

    def close(self):
        if self.handle:
            lib().mfd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfd_supported_n(N: int) -> bool:
    return bool(lib().mfd_supported_n(int(N)))


def mfd_build(N: int, L: float, order: int, eps, stream=None) -> Context:
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    if eps.shape != (N, N, N):
        raise ValueError("eps must have shape (N, N, N)")
    h = ctypes.c_void_p()
    _check(lib().mfd_build(int(N), float(L), int(order), eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           _stream(stream), ctypes.byref(h)))
    return Context(h, N, L)


def mfd_build_mu(N: int, L: float, order: int, mu, stream=None) -> Context:
    """A context from M_0 on the edges: mu of shape (3, N, N, N)."""
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    if mu.shape != (3, N, N, N):
        raise ValueError("mu must have shape (3, N, N, N)")
    h = ctypes.c_void_p()
    _check(lib().mfd_build_mu(int(N), float(L), int(order), mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              _stream(stream), ctypes.byref(h)))
    return Context(h, N, L)


def mfd_build_lattice(N: int, lattice, order: int, eps, stream=None) -> Context:
    """A context on a general lattice: ``lattice`` is the 3 x 3 matrix whose
    columns are the primitive vectors, eps of shape (N, N, N) on the unit-cube
    grid of y = lattice^-1 x."""
    A = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64))
    if A.shape != (3, 3):
        raise ValueError("lattice must be 3 x 3")
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    if eps.shape != (N, N, N):
        raise ValueError("eps must have shape (N, N, N)")
    h = ctypes.c_void_p()
    dptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().mfd_build_lattice(int(N), dptr(A), int(order), dptr(eps), _stream(stream), ctypes.byref(h)))
    return Context(h, N, float(abs(np.linalg.det(A))) ** (1.0 / 3.0))


def mfd_build_lattice_mu(N: int, lattice, order: int, mu, stream=None) -> Context:
    """A context on a general lattice from M_0 on the edges: mu of shape
    (3, N, N, N) on the unit-cube grid of y = lattice^-1 x."""
    A = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64))
    if A.shape != (3, 3):
        raise ValueError("lattice must be 3 x 3")
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    if mu.shape != (3, N, N, N):
        raise ValueError("mu must have shape (3, N, N, N)")
    h = ctypes.c_void_p()
    dptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().mfd_build_lattice_mu(int(N), dptr(A), int(order), dptr(mu), _stream(stream), ctypes.byref(h)))
    return Context(h, N, float(abs(np.linalg.det(A))) ** (1.0 / 3.0))


def mfd_gap_ratio(evals, kpts=None):
    """(ratio, below) of the band structure evals (nk x nbands): the largest
    gap ratio over consecutive band pairs and its lower band (1-based).
    kpts (nk x 3): the k-points of evals; a k = 0 row then skips the static
    third zero band."""
    ev = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
    if ev.ndim != 2:
        raise ValueError("evals must be nk x nbands")
    kp = None
    if kpts is not None:
        kp = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64).reshape(-1, 3))
        if kp.shape[0] != ev.shape[0]:
            raise ValueError("kpts must have one row per row of evals")
    dptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    r = ctypes.c_double()
    b = ctypes.c_int()
    _check(lib().mfd_gap_ratio(int(ev.shape[0]), int(ev.shape[1]), dptr(kp), dptr(ev), ctypes.byref(r),
                               ctypes.byref(b)))
    return r.value, b.value


def mfd_set_gamma(ctx: Context, gamma: float):
    _check(lib().mfd_set_gamma(ctx.handle, float(gamma)))


def mfd_gamma_shift(ctx: Context, k):
    ka, kp = _k(k)
    g, c = ctypes.c_double(), ctypes.c_double()
    _check(lib().mfd_gamma_shift(ctx.handle, kp, ctypes.byref(g), ctypes.byref(c)))
    return g.value, c.value


def mfd_op_apply(ctx: Context, k, X, Y, stream=None, fp64_arith: bool = False):
    """Y <- op(k) X (device tensors of shape (nb, 3, N, N, N)).  fp64_arith
    with complex64 tensors: FP32 storage, FP64 arithmetic (MFD_C64_F64)."""
    ka, kp = _k(k)
    if X.dtype != Y.dtype or X.shape != Y.shape:
        raise ValueError("X and Y must match in dtype and shape")
    dt = _dtype(X)
    if fp64_arith:
        if dt != MFD_C64:
            raise ValueError("fp64_arith applies to complex64 tensors")
        dt = MFD_C64_F64
    _check(lib().mfd_op_apply(ctx.handle, kp, int(X.shape[0]), dt, _dev(X), _dev(Y), _stream(stream)))
    return Y


def mfd_precond_solve(ctx: Context, k, R, T, stream=None):
    """T <- (P + c I)^-1 R (device tensors; T may be R)."""
    ka, kp = _k(k)
    if R.dtype != T.dtype or R.shape != T.shape:
        raise ValueError("R and T must match in dtype and shape")
    _check(lib().mfd_precond_solve(ctx.handle, kp, int(R.shape[0]), _dtype(R), _dev(R), _dev(T), _stream(stream)))
    return T


def mfd_precond_solve_mg(ctx: Context, k, R, T, cycles=2, smooth=2, sweeps=2, stream=None):
    """T <- multigrid approximation of (P + c I)^-1 R (device tensors; T may be R)."""
    ka, kp = _k(k)
    if R.dtype != T.dtype or R.shape != T.shape:
        raise ValueError("R and T must match in dtype and shape")
    _check(lib().mfd_precond_solve_mg(ctx.handle, kp, int(R.shape[0]), _dtype(R), int(cycles), int(smooth),
                                      int(sweeps), _dev(R), _dev(T), _stream(stream)))
    return T


def mfd_mg_supported(N: int) -> bool:
    return bool(lib().mfd_mg_supported(int(N)))


def mfd_lambda_re(ctx: Context, k, X, stream=None):
    ka, kp = _k(k)
    nb = int(X.shape[0])
    out = np.zeros(nb)
    _check(lib().mfd_lambda_re(ctx.handle, kp, nb, _dev(X), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               _stream(stream)))
    return out


def mfd_lambda_re_static(ctx: Context, k, X, out, stream=None):
    """out (device float64 tensor, nb entries) <- lambda_re of the nb fields of
    X, with no device allocation (mfd_lambda_re_static)."""
    import torch
    ka, kp = _k(k)
    nb = int(X.shape[0])
    if out.dtype != torch.float64 or out.numel() < nb:
        raise ValueError("out must be a float64 device tensor with nb entries")
    _check(lib().mfd_lambda_re_static(ctx.handle, kp, nb, _dev(X), _dev(out), _stream(stream)))
    return out


PROFILE_CATEGORIES = ("stencil", "precond", "gram", "rr", "update", "other")


def mfd_profile(ctx: Context, enable: bool):
    _check(lib().mfd_profile(ctx.handle, int(bool(enable))))


def mfd_profile_read(ctx: Context) -> dict:
    ms = (ctypes.c_double * 6)()
    cnt = (ctypes.c_longlong * 6)()
    by = (ctypes.c_double * 6)()
    _check(lib().mfd_profile_read(ctx.handle, ms, cnt, by))
    return {PROFILE_CATEGORIES[i]: dict(ms=ms[i], count=cnt[i], bytes=by[i]) for i in range(6)}


def max_block() -> int:
    """Largest nbands + guard a band solve accepts."""
    return int(lib().mfd_max_block())


def default_opts(**kw) -> mfd_opts:
    o = mfd_opts()
    lib().mfd_default_opts(ctypes.byref(o))
    for key, v in kw.items():
        if key == "x0":
            v = ctypes.c_void_p(v.data_ptr()) if v is not None else None
        setattr(o, key, v)
    return o


def mfd_bands(ctx: Context, kpts, nbands: int, tol: float, opts: mfd_opts | None = None, evecs=None,
              stream=None, raise_on=(-1, -2, -3, -6)):
    """Returns (evals (nk, nbands), stats list, status).  evecs: optional device
    complex128 tensor (nk, nbands, 3, N, N, N)."""
    kp = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64).reshape(-1, 3))
    nk = kp.shape[0]
    ev = np.zeros((nk, nbands))
    st = (mfd_kstats * nk)()
    o = opts if opts is not None else default_opts()
    status = lib().mfd_bands(ctx.handle, nk, kp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(nbands),
                             float(tol), ctypes.byref(o), ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             _dev(evecs) if evecs is not None else None, st, _stream(stream))
    if status in raise_on:
        _check(status)
    stats = _stats_list(st)
    return ev, stats, status


def _stats_list(st):
    return [dict(iters=s.iters, gamma_doublings=s.gamma_doublings, gamma=s.gamma,
                 max_rel_resid=s.max_rel_resid, spurious=s.spurious, discarded=s.discarded,
                 used_fallback=s.used_fallback, fp64_fallback=s.fp64_fallback, ms=s.ms,
                 rejected_steps=s.rejected_steps, host_syncs=s.host_syncs, segment_start=s.segment_start)
            for s in st]


def mfd_bands_batch(ctxs, kpts_list, nbands: int, tol: float, opts: mfd_opts | None = None, stream=None,
                    raise_on=(-1, -2, -3, -6)):
    """Many crystals (uneven grids allowed) in one call.  Returns
    (list of evals (nk_c, nbands), list of stats lists, status)."""
    nc = len(ctxs)
    ks = [np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, 3)) for k in kpts_list]
    evs = [np.zeros((k.shape[0], nbands)) for k in ks]
    sts = [(mfd_kstats * k.shape[0])() for k in ks]
    dp = ctypes.POINTER(ctypes.c_double)
    h = (ctypes.c_void_p * nc)(*[c.handle for c in ctxs])
    nk = (ctypes.c_int * nc)(*[k.shape[0] for k in ks])
    kp = (dp * nc)(*[k.ctypes.data_as(dp) for k in ks])
    ep = (dp * nc)(*[e.ctypes.data_as(dp) for e in evs])
    sp = (ctypes.POINTER(mfd_kstats) * nc)(*[ctypes.cast(s, ctypes.POINTER(mfd_kstats)) for s in sts])
    o = opts if opts is not None else default_opts()
    status = lib().mfd_bands_batch(nc, h, nk, kp, int(nbands), float(tol), ctypes.byref(o), ep, sp,
                                   _stream(stream))
    if status in raise_on:
        _check(status)
    return evs, [_stats_list(s) for s in sts], status


class Mlp:
    """The warm start's network (mfd_mlp_*): device FP32 batches in and out."""

    def __init__(self, nin, nhidden, nlayers, nout, max_batch, bf16=True, seed=0):
        h = ctypes.c_void_p()
        _check(lib().mfd_mlp_create(nin, nhidden, nlayers, nout, max_batch, int(bf16), seed, ctypes.byref(h)))
        self.handle = h
        self.nparams = int(lib().mfd_mlp_num_params(h))

    def set_params(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        assert a.size == self.nparams
        _check(lib().mfd_mlp_set_params(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        a = np.empty(self.nparams, dtype=np.float32)
        _check(lib().mfd_mlp_get_params(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    def forward(self, X, Y, stream=None):
        _check(lib().mfd_mlp_forward(self.handle, X.shape[0], _dev(X), _dev(Y), _stream(stream)))

    def loss_grad(self, X, T, grad=None, stream=None):
        loss = ctypes.c_double()
        _check(lib().mfd_mlp_loss_grad(self.handle, X.shape[0], _dev(X), _dev(T), ctypes.byref(loss),
                                       _dev(grad) if grad is not None else None, _stream(stream)))
        return loss.value

    def adam_step(self, lr, stream=None):
        _check(lib().mfd_mlp_adam_step(self.handle, float(lr), _stream(stream)))

    def close(self):
        if self.handle:
            lib().mfd_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfd_warm_target(Xa, Xb, Xc, C, Rinv=None, stream=None):
    """C (2mb x mb c128) and Rinv (2mb x 2mb) from three device blocks of mb
    columns (tensors (mb, n) c128: row q is column q of the block)."""
    mb, n = Xa.shape
    _check(lib().mfd_warm_target(n, mb, _dev(Xa), _dev(Xb), _dev(Xc), _dev(C),
                                 _dev(Rinv) if Rinv is not None else None, _stream(stream)))


def mfd_warm_features(L, k_prev, k_next, lam_j, lam_jm1, C, row, stream=None):
    """The network's input row (device f32 tensor of 6 + 2mb + 4mb^2) from
    host k-points and Ritz values and the device target C (2mb x mb c128)."""
    mb = C.shape[1]
    arr = lambda v, n: (ctypes.c_double * n)(*[float(x) for x in v])
    _check(lib().mfd_warm_features(float(L), mb, arr(k_prev, 3), arr(k_next, 3), arr(lam_j, mb),
                                   arr(lam_jm1, mb), _dev(C), _dev(row), _stream(stream)))


def mfd_tuning(ctx: Context):
    """(tuned, dict of the launch shapes the autotuner chose for ctx)."""
    out = (ctypes.c_int * 5)()
    r = lib().mfd_tuning(ctx.handle, out)
    if r < 0:
        _check(r)
    return bool(r), dict(gram_workgroups=out[0], update_workgroups=out[1], stencil_workgroups=out[2],
                         fft_x_run=out[3], update_rows=out[4])


_TUNING_KEYS = ("gram_workgroups", "update_workgroups", "stencil_workgroups", "fft_x_run", "update_rows")


def mfd_set_tuning(ctx: Context, shapes):
    """Pin the launch shapes (a dict with mfd_tuning's keys) for every later
    solve on ctx; None clears the pin."""
    if shapes is None:
        _check(lib().mfd_set_tuning(ctx.handle, None))
        return
    arr = (ctypes.c_int * 5)(*[int(shapes[k]) for k in _TUNING_KEYS])
    _check(lib().mfd_set_tuning(ctx.handle, arr))
