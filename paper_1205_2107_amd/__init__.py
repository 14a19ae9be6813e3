"""MI355X-native MRRR solver for the real symmetric tridiagonal eigenproblem.

Thin PyTorch binding of the C ABI in ``include/mrrr.h``: torch supplies device
memory and the stream; every step of the solver runs in the HIP kernels of
``libmrrr.so`` (gfx950, FP64).  Nothing here computes eigen-arithmetic.

    w, Z = eigh_tridiagonal(d, e)                      # all eigenpairs
    w, Z = eigh_tridiagonal(d, e, select="i", il=1, iu=100)
    w, Z = eigh_tridiagonal(d, e, select="v", vl=-1.0, vu=1.0)
    w, Z, zoff = eigh_tridiagonal_batched(d, e, sizes)  # packed problems
    w, Z = MRRRFunction.apply(d, e)                    # differentiable
    Y = backtransform(V, tau, Z)                       # Stage 5: Y = Q Z
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import MrrrError, MrrrInfo, MrrrRange, MrrrTuning  # noqa: F401

__all__ = ["eigh_tridiagonal", "eigh_tridiagonal_batched", "autotune_batched", "eigh_tridiagonal_backward",
           "eigh_tridiagonal_backward_batched", "MRRRFunction", "get_tuning", "set_tuning", "profile",
           "profile_read", "release", "workspace_size", "get_limits", "set_limits", "probe_division",
           "backtransform", "tridiagonalize", "cholesky", "sygst", "trsm_lt", "eigh_generalized",
           "eigh_tridiagonal_f32", "eigh_dense"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_dev(x, device=None):
    torch = _torch()
    if not torch.is_tensor(x):
        x = torch.as_tensor(x, dtype=torch.float64)
    if device is None:
        device = x.device if x.is_cuda else torch.device("cuda")
    return x.to(device=device, dtype=torch.float64).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _range(select, il, iu, vl, vu, n):
    rng = MrrrRange()
    if select == "a":
        rng.kind = _lib.MRRR_ALL
        m = n
    elif select == "i":
        rng.kind = _lib.MRRR_INDEX
        rng.il, rng.iu = int(il), int(iu)
        m = max(0, int(iu) - int(il) + 1)
    elif select == "v":
        rng.kind = _lib.MRRR_VALUE
        rng.vl, rng.vu = float(vl), float(vu)
        m = n
    else:
        raise ValueError("select must be 'a', 'i' or 'v'")
    return rng, m


def workspace_size(n, select="a", il=None, iu=None, vl=None, vu=None):
    """Bytes of caller workspace mrrr_step_ws suggests for this problem size."""
    rng, _ = _range(select, il, iu, vl, vu, int(n))
    return int(_lib.load().mrrr_workspace_size(int(n), rng))


def eigh_tridiagonal(d, e, select="a", il=None, iu=None, vl=None, vu=None, eigvals_only=False,
                     stream=None, return_info=False, work=None):
    """Eigenpairs of the symmetric tridiagonal matrix (diagonal d, off-diagonal e).

    select: "a" all, "i" indices il..iu (1-based, inclusive), "v" values in (vl, vu].
    work: optional device tensor used as the solver's whole workspace
    (mrrr_step_ws; nothing is allocated by the library; see workspace_size).
    Returns w (ascending, float64, on the GPU) and Z (n x m column-major view:
    a tensor of shape (n, m) whose columns are the eigenvectors), plus the info
    dict when return_info is set.
    """
    torch = _torch()
    lib = _lib.load()
    d = _as_dev(d)
    n = d.numel()
    e = _as_dev(e, d.device) if n > 1 else torch.zeros(1, dtype=torch.float64, device=d.device)
    rng, m = _range(select, il, iu, vl, vu, n)
    w = torch.empty(max(m, 1), dtype=torch.float64, device=d.device)
    Zbuf = None if eigvals_only else torch.empty((max(m, 1), max(n, 1)), dtype=torch.float64, device=d.device)
    info = MrrrInfo()
    if work is None:
        rc = lib.mrrr_step(n, _ptr(d), _ptr(e), rng, _ptr(w), _ptr(Zbuf), max(n, 1), ctypes.byref(info),
                           _stream_ptr(stream))
        _lib.check(rc)
    else:
        info_dev = torch.zeros(ctypes.sizeof(MrrrInfo) // 8, dtype=torch.int64, device=d.device)
        rc = lib.mrrr_step_ws(n, _ptr(d), _ptr(e), rng, _ptr(w), _ptr(Zbuf), max(n, 1), _ptr(work),
                              work.numel() * work.element_size(), _ptr(info_dev), _stream_ptr(stream))
        _lib.check(rc)
        host = info_dev.cpu().numpy()  # kept alive across the copy
        ctypes.memmove(ctypes.addressof(info), host.ctypes.data, ctypes.sizeof(MrrrInfo))
    mm = int(info.m) if n > 0 else 0
    w = w[:mm]
    Z = None if Zbuf is None else Zbuf[:mm, :n].t()
    out = (w, Z)
    if return_info:
        out = out + (info.as_dict(),)
    return out


def eigh_tridiagonal_f32(d, e, select="a", il=None, iu=None, vl=None, vu=None, eigvals_only=False,
                         stream=None, return_info=False):
    """eigh_tridiagonal for FP32 data with FP64 arithmetic inside
    (mrrr_step_f32): d and e are taken as float32, w and Z are float32 with
    orthogonality and residuals at the FP32 rounding level."""
    torch = _torch()
    lib = _lib.load()

    def f32(x, device=None):
        if not torch.is_tensor(x):
            x = torch.as_tensor(np.asarray(x, dtype=np.float32))
        if device is None:
            device = x.device if x.is_cuda else torch.device("cuda")
        return x.to(device=device, dtype=torch.float32).contiguous()

    d = f32(d)
    n = d.numel()
    e = f32(e, d.device) if n > 1 else torch.zeros(1, dtype=torch.float32, device=d.device)
    rng, m = _range(select, il, iu, vl, vu, n)
    w = torch.empty(max(m, 1), dtype=torch.float32, device=d.device)
    Zbuf = None if eigvals_only else torch.empty((max(m, 1), max(n, 1)), dtype=torch.float32, device=d.device)
    info = MrrrInfo()
    _lib.check(lib.mrrr_step_f32(n, _ptr(d), _ptr(e), rng, _ptr(w), _ptr(Zbuf), max(n, 1), ctypes.byref(info),
                                 _stream_ptr(stream)))
    mm = int(info.m) if n > 0 else 0
    w = w[:mm]
    Z = None if Zbuf is None else Zbuf[:mm, :n].t()
    out = (w, Z)
    if return_info:
        out = out + (info.as_dict(),)
    return out


def eigh_tridiagonal_batched(d, e, sizes, eigvals_only=False, stream=None, return_info=False):
    """All eigenpairs of len(sizes) independent tridiagonals packed back to back:
    problem b owns d[off_b : off_b + n_b] and e[off_b : off_b + n_b - 1] (e has one
    unused entry per problem).  Returns (w, Z, zoff): w packed like d, Z a flat
    buffer with problem b's n_b x n_b column-major block at zoff[b]."""
    torch = _torch()
    lib = _lib.load()
    d = _as_dev(d)
    e = _as_dev(e, d.device)
    sizes = [int(x) for x in sizes]
    B = len(sizes)
    n_arr = (ctypes.c_int64 * max(B, 1))(*sizes)
    offs = [0] * B
    zoffs = [0] * B
    acc = zacc = 0
    for b, nb in enumerate(sizes):
        offs[b] = acc
        zoffs[b] = zacc
        acc += nb
        zacc += nb * nb
    off_arr = (ctypes.c_int64 * max(B, 1))(*offs)
    zoff_arr = (ctypes.c_int64 * max(B, 1))(*zoffs)
    w = torch.empty(max(acc, 1), dtype=torch.float64, device=d.device)
    Z = None if eigvals_only else torch.empty(max(zacc, 1), dtype=torch.float64, device=d.device)
    infos = (MrrrInfo * max(B, 1))()
    rc = lib.mrrr_step_batched(B, n_arr, off_arr, _ptr(d), _ptr(e), _ptr(w), _ptr(Z), zoff_arr, infos,
                               _stream_ptr(stream))
    _lib.check(rc)
    out = (w[:acc], Z, zoffs)
    if return_info:
        out = out + ([infos[b].as_dict() for b in range(B)],)
    return out


def autotune_batched(d, e, sizes, stream=None):
    """Pick launch shapes for batches shaped like this one (mrrr_autotune_batched):
    a coordinate search timing about ten solves of the batch; the choice is cached
    for later eigh_tridiagonal_batched calls with the same size histogram.
    Returns the chosen tuning as a dict."""
    torch = _torch()
    lib = _lib.load()
    d = _as_dev(d)
    e = _as_dev(e, d.device)
    sizes = [int(x) for x in sizes]
    B = len(sizes)
    n_arr = (ctypes.c_int64 * max(B, 1))(*sizes)
    offs, zoffs = [0] * B, [0] * B
    acc = zacc = 0
    for b, nb in enumerate(sizes):
        offs[b], zoffs[b] = acc, zacc
        acc += nb
        zacc += nb * nb
    off_arr = (ctypes.c_int64 * max(B, 1))(*offs)
    zoff_arr = (ctypes.c_int64 * max(B, 1))(*zoffs)
    w = torch.empty(max(acc, 1), dtype=torch.float64, device=d.device)
    Z = torch.empty(max(zacc, 1), dtype=torch.float64, device=d.device)
    t = MrrrTuning()
    rc = lib.mrrr_autotune_batched(B, n_arr, off_arr, _ptr(d), _ptr(e), _ptr(w), _ptr(Z), zoff_arr, ctypes.byref(t),
                                   _stream_ptr(stream))
    _lib.check(rc)
    return {"grid_density": t.grid_density, "refine_wave_slots": t.refine_wave_slots,
            "vec_wave_slots": t.vec_wave_slots, "vec_ckpt_min_run": t.vec_ckpt_min_run}


def _colmajor(X, n):
    """Square n x n tensor -> buffer whose column j is contiguous (ld = n)."""
    X = X.to(dtype=_torch().float64)
    return X.t().contiguous()  # row j of the result is column j of X


def eigh_tridiagonal_backward(w, Z, gw=None, gZ=None, stream=None):
    """(grad_d, grad_e) of a loss with cotangents gw (eigenvalues) and gZ
    (eigenvectors, n x n) for the full decomposition (w, Z)."""
    torch = _torch()
    lib = _lib.load()
    w = _as_dev(w)
    n = w.numel()
    V = _colmajor(Z.to(w.device), n)
    G = _colmajor(gZ.to(w.device), n) if gZ is not None else None
    gwt = _as_dev(gw, w.device) if gw is not None else None
    gd = torch.empty(max(n, 1), dtype=torch.float64, device=w.device)
    ge = torch.empty(max(n, 1), dtype=torch.float64, device=w.device)
    ld = max(n, 1)
    rc = lib.mrrr_step_backward(n, _ptr(w), _ptr(V), ld, _ptr(gwt), _ptr(G), ld, _ptr(gd), _ptr(ge),
                                _stream_ptr(stream))
    _lib.check(rc)
    return gd[:n], ge[:max(n - 1, 0)]


def eigh_tridiagonal_backward_batched(w, Z, sizes, gw=None, gZ=None, stream=None):
    """Backward for the packed layout of eigh_tridiagonal_batched."""
    torch = _torch()
    lib = _lib.load()
    sizes = [int(x) for x in sizes]
    B = len(sizes)
    offs, zoffs = [], []
    acc = zacc = 0
    for nb in sizes:
        offs.append(acc)
        zoffs.append(zacc)
        acc += nb
        zacc += nb * nb
    n_arr = (ctypes.c_int64 * max(B, 1))(*sizes)
    off_arr = (ctypes.c_int64 * max(B, 1))(*offs)
    zoff_arr = (ctypes.c_int64 * max(B, 1))(*zoffs)
    gd = torch.empty(max(acc, 1), dtype=torch.float64, device=w.device)
    ge = torch.empty(max(acc, 1), dtype=torch.float64, device=w.device)
    rc = lib.mrrr_step_backward_batched(B, n_arr, off_arr, zoff_arr, _ptr(w), _ptr(Z), _ptr(gw), _ptr(gZ),
                                        _ptr(gd), _ptr(ge), _stream_ptr(stream))
    _lib.check(rc)
    return gd[:acc], ge[:acc]


def _make_function():
    torch = _torch()

    class MRRRFunction(torch.autograd.Function):
        """(d, e) -> (w, Z) by the GPU MRRR solver; backward by the GPU adjoint
        kernels.  Requires distinct eigenvalues for the eigenvector term.

        MRRRFunction.apply(d, e, recompute): with recompute set, only d, e and
        w are kept for the backward (O(n) memory instead of the n x n
        eigenvectors), which solves again for Z; the solver is deterministic,
        so the recomputed Z and the gradients equal those of the saved Z bit
        for bit."""

        @staticmethod
        def forward(ctx, d, e, recompute=False):
            w, Z = eigh_tridiagonal(d, e)
            ctx.recompute = bool(recompute)
            if ctx.recompute:
                ctx.save_for_backward(d, e, w)
            else:
                ctx.save_for_backward(w, Z)
            return w, Z

        @staticmethod
        def backward(ctx, gw, gZ):
            if ctx.recompute:
                d, e, w = ctx.saved_tensors
                _, Z = eigh_tridiagonal(d.detach(), e.detach())
            else:
                w, Z = ctx.saved_tensors
            gd, ge = eigh_tridiagonal_backward(w, Z, gw, gZ)
            return gd, ge, None

    return MRRRFunction


class _Lazy:
    _fn = None

    def __getattr__(self, name):
        if _Lazy._fn is None:
            _Lazy._fn = _make_function()
        return getattr(_Lazy._fn, name)


MRRRFunction = _Lazy()


def get_tuning():
    t = MrrrTuning()
    _lib.check(_lib.load().mrrr_get_tuning(ctypes.byref(t)))
    return {"grid_density": t.grid_density, "refine_wave_slots": t.refine_wave_slots,
            "vec_wave_slots": t.vec_wave_slots, "vec_ckpt_min_run": t.vec_ckpt_min_run,
            "vec_ckpt_min_n": t.vec_ckpt_min_n}


def set_tuning(grid_density=None, refine_wave_slots=None, vec_wave_slots=None, vec_ckpt_min_run=None,
               vec_ckpt_min_n=None):
    t = MrrrTuning()
    lib = _lib.load()
    _lib.check(lib.mrrr_get_tuning(ctypes.byref(t)))
    if grid_density is not None:
        t.grid_density = int(grid_density)
    if refine_wave_slots is not None:
        t.refine_wave_slots = int(refine_wave_slots)
    if vec_wave_slots is not None:
        t.vec_wave_slots = int(vec_wave_slots)
    if vec_ckpt_min_run is not None:
        t.vec_ckpt_min_run = int(vec_ckpt_min_run)
    if vec_ckpt_min_n is not None:
        t.vec_ckpt_min_n = int(vec_ckpt_min_n)
    if lib.mrrr_set_tuning(ctypes.byref(t)) != 0:
        raise ValueError("tuning value out of range")


def get_limits():
    t = _lib.MrrrLimits()
    _lib.check(_lib.load().mrrr_get_limits(ctypes.byref(t)))
    return {"max_depth": t.max_depth, "child_growth_limit": t.child_growth_limit}


def set_limits(max_depth=None, child_growth_limit=None):
    """Lower the representation tree's depth limit or set a hard limit on the
    element growth of child representations (tests of the status paths)."""
    lib = _lib.load()
    t = _lib.MrrrLimits()
    _lib.check(lib.mrrr_get_limits(ctypes.byref(t)))
    if max_depth is not None:
        t.max_depth = int(max_depth)
    if child_growth_limit is not None:
        t.child_growth_limit = float(child_growth_limit)
    if lib.mrrr_set_limits(ctypes.byref(t)) != 0:
        raise ValueError("limit out of range")


def profile(enable=True):
    """Turn the library's per-kernel event timing on or off (and reset it)."""
    lib = _lib.load()
    _lib.check(lib.mrrr_profile_reset())
    _lib.check(lib.mrrr_profile_enable(1 if enable else 0))


def profile_read():
    """{kernel: {launches, ms, work (flops), bytes}} accumulated since profile()."""
    lib = _lib.load()
    out = {}
    for k, name in enumerate(_lib.KERNELS):
        t = _lib.MrrrKernelTime()
        _lib.check(lib.mrrr_profile_read(k, ctypes.byref(t)))
        out[name] = {"launches": int(t.launches), "ms": float(t.ms), "work": float(t.work), "bytes": float(t.bytes)}
    return out


def release():
    _lib.check(_lib.load().mrrr_release())


def backtransform(V, tau, Z, stream=None):
    """Stage 5 back-transformation: Y = Q Z for the n - 1 Householder
    reflectors of a lower tridiagonal reduction (V n x n holding v_i[i+2:] in
    V[i+2:, i], tau of length n - 1), on the GPU.  Z (n x m) is overwritten
    when it is a column-major float64 device tensor (e.g. the eigenvectors
    eigh_tridiagonal returns); otherwise a column-major copy is transformed.
    Returns the transformed tensor."""
    torch = _torch()
    Zd = Z if torch.is_tensor(Z) else torch.as_tensor(np.asarray(Z), dtype=torch.float64)
    if Zd.dim() != 2:
        raise ValueError("Z must be 2-D")
    n, m = Zd.shape
    dev = Zd.device if Zd.is_cuda else torch.device("cuda")
    if not (Zd.is_cuda and Zd.dtype == torch.float64 and (Zd.numel() == 0 or
                                                           (Zd.stride(0) == 1 and Zd.stride(1) >= max(1, n)))):
        Zd = Zd.to(device=dev, dtype=torch.float64).t().contiguous().t()
    Vt = V if torch.is_tensor(V) else torch.as_tensor(np.asarray(V), dtype=torch.float64)
    if Vt.dim() != 2 or Vt.shape[0] != n or (n > 1 and Vt.shape[1] < n - 1):
        raise ValueError("V must be n x (n - 1) or larger")
    if not (Vt.is_cuda and Vt.dtype == torch.float64 and (Vt.numel() == 0 or
                                                           (Vt.stride(0) == 1 and Vt.stride(1) >= max(1, n)))):
        Vt = Vt.to(device=dev, dtype=torch.float64).t().contiguous().t()
    t = _as_dev(tau, dev)
    if n > 1 and t.numel() < n - 1:
        raise ValueError("tau must hold n - 1 entries")
    ldv = max(1, n, Vt.stride(1) if Vt.numel() > 0 else 1)
    ldz = max(1, n, Zd.stride(1) if Zd.numel() > 0 else 1)
    with torch.cuda.device(dev):
        _lib.check(_lib.load().mrrr_backtransform(n, m, _ptr(Vt), ldv, _ptr(t), _ptr(Zd), ldz,
                                                   _stream_ptr(stream)))
    return Zd


def tridiagonalize(A, stream=None):
    """Stage 3 reduction T = Q^T M Q of the real symmetric M (its lower
    triangle read), on the GPU.  A (n x n) is overwritten when it is a
    column-major float64 device tensor; otherwise a column-major copy is
    reduced.  Returns (d, e, tau, V): T's diagonal and off-diagonal, the
    reflector scalars, and the reduced matrix V holding v_i[i+2:] in
    V[i+2:, i] (the input of backtransform; its strict upper triangle is
    neither read nor written)."""
    torch = _torch()
    Ad = A if torch.is_tensor(A) else torch.as_tensor(np.asarray(A), dtype=torch.float64)
    if Ad.dim() != 2 or Ad.shape[0] != Ad.shape[1]:
        raise ValueError("A must be square")
    n = Ad.shape[0]
    dev = Ad.device if Ad.is_cuda else torch.device("cuda")
    if not (Ad.is_cuda and Ad.dtype == torch.float64 and (Ad.numel() == 0 or
                                                           (Ad.stride(0) == 1 and Ad.stride(1) >= max(1, n)))):
        Ad = Ad.to(device=dev, dtype=torch.float64).t().contiguous().t()
    d = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 0), dtype=torch.float64, device=dev)
    tau = torch.empty(max(n - 1, 0), dtype=torch.float64, device=dev)
    lda = max(1, n, Ad.stride(1) if Ad.numel() > 0 else 1)
    with torch.cuda.device(dev):
        _lib.check(_lib.load().mrrr_tridiagonalize(n, _ptr(Ad), lda, _ptr(d), _ptr(e), _ptr(tau),
                                                    _stream_ptr(stream)))
    return d, e, tau, Ad


def _dense_colmajor(X, dev, square=False):
    """X itself when it is a column-major float64 tensor on dev, else a
    column-major copy there"""
    torch = _torch()
    Xt = X if torch.is_tensor(X) else torch.as_tensor(np.asarray(X), dtype=torch.float64)
    if Xt.dim() != 2 or (square and Xt.shape[0] != Xt.shape[1]):
        raise ValueError("a square matrix is required" if square else "a matrix is required")
    n = Xt.shape[0]
    if not (Xt.is_cuda and Xt.device == dev and Xt.dtype == torch.float64 and
            (Xt.numel() == 0 or (Xt.stride(0) == 1 and Xt.stride(1) >= max(1, n)))):
        Xt = Xt.to(device=dev, dtype=torch.float64).t().contiguous().t()
    return Xt


def _ld(X):
    return max(1, X.shape[0], X.stride(1) if X.numel() > 0 else 1)


def _dev_of(X):
    torch = _torch()
    return X.device if torch.is_tensor(X) and X.is_cuda else torch.device("cuda")


def cholesky(B, stream=None):
    """B = L L^T on the GPU (lower triangle of B read; L written over it when
    B is a column-major float64 device tensor, else into a copy).  Returns L
    (its strict upper triangle is whatever B held there); raises when B is
    not positive definite."""
    dev = _dev_of(B)
    Bd = _dense_colmajor(B, dev, square=True)
    info = ctypes.c_int64(0)
    with _torch().cuda.device(dev):
        _lib.check(_lib.load().mrrr_cholesky(Bd.shape[0], _ptr(Bd), _ld(Bd), ctypes.byref(info),
                                              _stream_ptr(stream)))
    if info.value:
        raise ValueError(f"matrix not positive definite (pivot of column {info.value})")
    return Bd


def sygst(A, L, stream=None):
    """M = L^{-1} A L^{-T} on the GPU (lower triangle of A read; M written over
    A when it is a column-major float64 device tensor, else into a copy)."""
    dev = _dev_of(A)
    Ad = _dense_colmajor(A, dev, square=True)
    Ld = _dense_colmajor(L, dev, square=True)
    if Ld.shape != Ad.shape:
        raise ValueError("A and L must have one order")
    with _torch().cuda.device(dev):
        _lib.check(_lib.load().mrrr_sygst(Ad.shape[0], _ptr(Ad), _ld(Ad), _ptr(Ld), _ld(Ld), _stream_ptr(stream)))
    return Ad


def trsm_lt(L, Y, stream=None):
    """Y <- L^{-T} Y on the GPU (in place on a column-major float64 device
    tensor, else on a copy); returns the result."""
    dev = _dev_of(Y)
    Yd = _dense_colmajor(Y, dev)
    Ld = _dense_colmajor(L, dev, square=True)
    if Ld.shape[0] != Yd.shape[0]:
        raise ValueError("L and Y must have the same number of rows")
    with _torch().cuda.device(dev):
        _lib.check(_lib.load().mrrr_trsm_lt(Yd.shape[0], Yd.shape[1], _ptr(Ld), _ld(Ld), _ptr(Yd), _ld(Yd),
                                             _stream_ptr(stream)))
    return Yd


def eigh_dense(A, select="a", il=None, iu=None, vl=None, vu=None, stream=None):
    """Eigenpairs of the dense symmetric A (lower triangle read) through the
    library's driver mrrr_syevr: reduction to tridiagonal form, the MRRR
    tridiagonal eigensolver for the selected eigenpairs (select as for
    eigh_tridiagonal), back-transformation of those vectors only, all on the
    GPU.  A is overwritten when it is a column-major float64 device tensor.
    Returns (w ascending, Z column-major, one column per eigenvalue)."""
    torch = _torch()
    dev = _dev_of(A)
    Ad = _dense_colmajor(A, dev, square=True)
    n = Ad.shape[0]
    rng, m = _range(select, il, iu, vl, vu, n)
    w = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    Z = torch.empty((max(m, 1), max(n, 1)), dtype=torch.float64, device=dev)
    info = MrrrInfo()
    with torch.cuda.device(dev):
        _lib.check(_lib.load().mrrr_syevr(n, _ptr(Ad), _ld(Ad), rng, _ptr(w), _ptr(Z), max(n, 1), ctypes.byref(info),
                                           _stream_ptr(stream)))
    mm = int(info.m) if n > 0 else 0
    return w[:mm], Z[:mm, :n].t()


def eigh_generalized(A, B, select="a", il=None, iu=None, vl=None, vu=None, stream=None):
    """Eigenpairs of A x = lambda B x (A symmetric, B symmetric positive
    definite, lower triangles read) through the library's driver mrrr_sygvr,
    every stage on the GPU: Cholesky factorization, reduction to standard
    form, reduction to tridiagonal form, the MRRR tridiagonal eigensolver for
    the selected eigenpairs (select as for eigh_tridiagonal), and both
    back-transformations of those vectors.  A and B are overwritten when they
    are column-major float64 device tensors.  Returns (w ascending, X
    column-major with X^T B X = I); raises when B is not positive definite."""
    torch = _torch()
    dev = _dev_of(A)
    Ad = _dense_colmajor(A, dev, square=True)
    Bd = _dense_colmajor(B, dev, square=True)
    if Bd.shape != Ad.shape:
        raise ValueError("A and B must have one order")
    n = Ad.shape[0]
    rng, m = _range(select, il, iu, vl, vu, n)
    w = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    X = torch.empty((max(m, 1), max(n, 1)), dtype=torch.float64, device=dev)
    bad = ctypes.c_int64(0)
    info = MrrrInfo()
    with torch.cuda.device(dev):
        _lib.check(_lib.load().mrrr_sygvr(n, _ptr(Ad), _ld(Ad), _ptr(Bd), _ld(Bd), rng, _ptr(w), _ptr(X), max(n, 1),
                                           ctypes.byref(bad), ctypes.byref(info), _stream_ptr(stream)))
    if bad.value:
        raise ValueError(f"B not positive definite (pivot of column {bad.value})")
    mm = int(info.m) if n > 0 else 0
    return w[:mm], X[:mm, :n].t()


def probe_division(a, b, stream=None):
    """The kernels' reciprocal and quotient forms on device operands a, b (same
    length): returns (v_rcp_f64(b), one Newton step, two steps, a / b) as
    device tensors, computed by the library's probe kernel."""
    torch = _torch()
    a = _as_dev(a)
    b = _as_dev(b, a.device)
    if a.shape != b.shape or a.dim() != 1:
        raise ValueError("a and b must be 1-D of one length")
    n = a.numel()
    out = torch.empty(4 * n, dtype=torch.float64, device=a.device)
    with torch.cuda.device(a.device):
        _lib.check(_lib.load().mrrr_probe_division(n, _ptr(a), _ptr(b), _ptr(out), _stream_ptr(stream)))
    return out[:n], out[n:2 * n], out[2 * n:3 * n], out[3 * n:]
