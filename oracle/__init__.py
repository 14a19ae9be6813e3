"""CPU oracle for the MRRR tridiagonal eigensolver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_1205_2107_amd``)
never touches it, and it shares no code with the GPU library.

* ``mrrr``           -- plain single-threaded FP64 MRRR in C (``mrrr_oracle.c``),
                        following Sec. 3.1.1 of arXiv:1205.2107 step by step.
* ``bisect_T``       -- j-th eigenvalue by plain Sturm bisection on T (textbook
                        definition; used for sampled checks at large n).
* ``count_T``        -- Sturm count on T.
* ``dense_adjoint``  -- (grad_w, grad_Z) -> (grad_d, grad_e) by the dense formula
                        (see ``adjoint.py``).
* ``apply_q``        -- Stage 5 back-transformation Y = Q Z, one Householder
                        reflector at a time (see ``backtransform.py``).
* ``tridiagonalize`` -- Stage 3 reduction T = Q^T M Q, one Householder
                        reflector at a time (see ``tridiagonalize.py``).
* ``ghep``           -- the generalized problem A x = lambda B x through all
                        six stages (see ``ghep.py``).
* ``mrrr_fp32``      -- FP32 data solved in FP64 (the mixed-precision use of
                        Sec. 2.3): the inputs widened exactly, ``mrrr``, the
                        results rounded to FP32.
"""
import ctypes
import os
import subprocess

import numpy as np

from .adjoint import dense_adjoint  # noqa: F401
from .backtransform import apply_q  # noqa: F401
from .tridiagonalize import tridiagonalize  # noqa: F401
from . import ghep  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrrr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STAT_NAMES = ("nodes", "max_depth", "sturm_steps", "twisted", "fallbacks", "child_tries",
              "singletons", "clusters")
RANGE_ALL, RANGE_INDEX, RANGE_VALUE = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
                           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        I64 = ctypes.c_int64
        lib.oracle_mrrr.restype = ctypes.c_int
        lib.oracle_mrrr.argtypes = [I64, P, P, ctypes.c_int, I64, I64, ctypes.c_double, ctypes.c_double,
                                    P, P, I64, ctypes.POINTER(I64), ctypes.POINTER(I64)]
        lib.oracle_bisect_T.restype = ctypes.c_int
        lib.oracle_bisect_T.argtypes = [I64, P, P, I64, P, P]
        lib.oracle_count_T.restype = I64
        lib.oracle_count_T.argtypes = [I64, P, P, ctypes.c_double]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    pass


def mrrr(d, e, kind=RANGE_ALL, il=0, iu=0, vl=0.0, vu=0.0, vectors=True, return_stats=False):
    """Eigenpairs of the symmetric tridiagonal matrix with diagonal d and
    off-diagonal e.  Returns (w, Z, status) -- or (w, Z, status, stats) -- with w
    ascending and Z column-major n x m (None when vectors=False)."""
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    e = np.ascontiguousarray(e, dtype=np.float64) if n > 1 else np.zeros(1)
    if n > 1 and e.shape[0] < n - 1:
        raise ValueError("e must have n-1 entries")
    e_full = np.zeros(max(n, 1))
    e_full[: max(n - 1, 0)] = e[: max(n - 1, 0)]
    w = np.zeros(max(n, 1))
    Z = np.zeros((max(n, 1), max(n, 1)), order="F") if vectors else None
    m = ctypes.c_int64(0)
    stats = (ctypes.c_int64 * 8)()
    zp = _ptr(Z) if vectors else ctypes.POINTER(ctypes.c_double)()
    st = lib.oracle_mrrr(n, _ptr(d), _ptr(e_full), kind, il, iu, vl, vu, _ptr(w), zp, max(n, 1),
                         ctypes.byref(m), stats)
    if st < 0:
        raise OracleError(f"oracle_mrrr: argument {-st} invalid")
    mm = m.value
    w = w[:mm].copy()
    if vectors:
        Z = np.asfortranarray(Z[:n, :mm])
    out = (w, Z, st)
    if return_stats:
        out = out + (dict(zip(STAT_NAMES, list(stats))),)
    return out


def mrrr_fp32(d, e, **kw):
    """(w, Z, status) of the FP32 tridiagonal (d, e): widened exactly to FP64,
    solved by ``mrrr``, w and Z rounded to FP32."""
    d64 = np.asarray(d, dtype=np.float32).astype(np.float64)
    e64 = np.asarray(e, dtype=np.float32).astype(np.float64)
    w, Z, st = mrrr(d64, e64, **kw)[:3]
    return w.astype(np.float32), (None if Z is None else Z.astype(np.float32)), st


def bisect_T(d, e, j):
    """Bracket [lo, hi] of the j-th (1-based) eigenvalue of T by plain bisection on T."""
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    e_full = np.zeros(max(n, 1))
    e_full[: n - 1] = np.asarray(e, dtype=np.float64)[: n - 1]
    lo = ctypes.c_double(0)
    hi = ctypes.c_double(0)
    if lib.oracle_bisect_T(n, _ptr(d), _ptr(e_full), j, ctypes.byref(lo), ctypes.byref(hi)) != 0:
        raise OracleError("bad index")
    return lo.value, hi.value


def count_T(d, e, tau):
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    e_full = np.zeros(max(n, 1))
    e_full[: n - 1] = np.asarray(e, dtype=np.float64)[: n - 1]
    return int(lib.oracle_count_T(n, _ptr(d), _ptr(e_full), float(tau)))


def splitmix64(seed, counter):
    return int(_load().oracle_splitmix64(seed, counter))
