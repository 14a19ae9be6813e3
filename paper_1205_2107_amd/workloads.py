"""Seeded synthetic tridiagonal workloads.

This module only draws inputs; it holds none of the eigensolver's arithmetic.
Every generator is deterministic in its seed (numpy PCG64 ``default_rng``; d is
drawn before e).  Matrix types follow the paper's experiments (Sec. 2.3, Fig. 3:
the "1-2-1" and "Wilkinson" matrices) plus random and prescribed-spectrum types.

* ``random_uniform``   d_i, e_i ~ U(-1, 1)
* ``toeplitz``         constant diagonal a and off-diagonal b ("1-2-1" is a=2, b=-1)
* ``wilkinson``        the paper's Wilkinson matrix: e = 1, d = (m, ..., 1, 0, 1, ..., m)
* ``glued_wilkinson``  W_{2m+1}^+ blocks (d_i = |m - i|, e = 1) joined by glue
                       g * U(0.5, 1.5); the last block is truncated to fit n
* ``from_spectrum``    the Lanczos tridiagonal of diag(lam) from a uniformly random
                       unit start vector (distribution of the Householder form of
                       Q diag(lam) Q^T, Q Haar), built by an O(n^2) Givens method
* ``geometric``        spectrum 10^(-8 (n - i)/(n - 1)), i = 1..n  (kappa = 1e8)
* ``separated``        spectrum sort(U(-1,1)) + 1e-3 * i (gaps >= 1e-3)
* ``batched_mix``      sizes log-uniform in [32, 2048]; 60% random, 20% 1-2-1,
                       20% glued Wilkinson
* ``reflectors``       n - 1 Householder reflectors in the storage of a lower
                       tridiagonal reduction (input of the back-transformation):
                       v_i has a unit entry at row i + 1, zeros above, entries
                       U(-1, 1) / sqrt(n - i - 1) below; tau_i = 2 / (v_i^T v_i)
* ``dense_symmetric``  dense symmetric M (input of the reduction to tridiagonal
                       form): lower triangle U(-1, 1), mirrored above (numpy);
                       ``dense_symmetric_device`` draws the same kind of matrix
                       on a torch device with torch's seeded generator
* ``dense_spd``        symmetric positive definite B = G G^T / n + I with G
                       having U(-1, 1) entries (spectrum within [1, 7/3]);
                       ``dense_spd_device`` the same on a torch device
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "rkpw.c")
_LIB = os.path.join(_HERE, "_rkpw.so")

SEEDS = {"c1": 1000, "c2_random": 2001, "c2_toeplitz": 2002, "c2_geometric": 2003, "c3": 3001,
         "c4": 4001, "c5": 5001, "c5_fd": 5101}


def build(force=True):
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-shared", "-fPIC", "-o", tmp,
                           _SRC, "-lm"])
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
        lib.workload_rkpw.restype = ctypes.c_int
        lib.workload_rkpw.argtypes = [ctypes.c_int64, P, P, P, P]
        _lib = lib
    return _lib


def random_uniform(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, n)
    e = rng.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


def toeplitz(n, a=2.0, b=-1.0):
    return np.full(n, float(a)), np.full(max(n - 1, 0), float(b))


def wilkinson(n):
    """Paper's Wilkinson matrix (Sec. 2.3): unit off-diagonals, diagonal
    (m, m-1, ..., 1, 0, 1, ..., m) with m = (n - 1)/2; n must be odd."""
    if n % 2 != 1:
        raise ValueError("the Wilkinson matrix is defined for odd n")
    m = (n - 1) // 2
    return np.abs(np.arange(n, dtype=np.float64) - m), np.ones(n - 1)


def glued_wilkinson(n, seed, m=10, glue=1e-10):
    rng = np.random.default_rng(seed)
    bs = 2 * m + 1
    d = np.abs(np.arange(n) % bs - m).astype(np.float64)
    e = np.ones(max(n - 1, 0))
    joints = np.arange(bs - 1, n - 1, bs)
    e[joints] = glue * rng.uniform(0.5, 1.5, joints.shape[0])
    return d, e


def from_spectrum(lam, seed):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    n = lam.shape[0]
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n)
    om = np.ascontiguousarray(g / np.linalg.norm(g))
    d = np.zeros(n)
    e = np.zeros(max(n, 1))
    P = ctypes.POINTER(ctypes.c_double)
    rc = _load().workload_rkpw(n, lam.ctypes.data_as(P), om.ctypes.data_as(P), d.ctypes.data_as(P),
                               e.ctypes.data_as(P))
    if rc != 0:
        raise MemoryError("workload_rkpw")
    return d, e[: max(n - 1, 0)].copy()


def geometric_spectrum(n, kappa=1e8):
    i = np.arange(1, n + 1, dtype=np.float64)
    return 10.0 ** (-np.log10(kappa) * (n - i) / max(n - 1, 1))


def geometric(n, seed, kappa=1e8):
    return from_spectrum(geometric_spectrum(n, kappa), seed)


def separated_spectrum(n, seed, spacing=1e-3):
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(-1.0, 1.0, n)) + spacing * np.arange(1, n + 1)


def separated(n, seed, spacing=1e-3):
    lam = separated_spectrum(n, seed, spacing)
    return from_spectrum(lam, seed + 1)


def batched_mix(count, seed, nmin=32, nmax=2048):
    """List of (d, e, kind) for the batched workload."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), count))).astype(np.int64)
    kinds = rng.choice(3, size=count, p=[0.6, 0.2, 0.2])
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for nb, k, s in zip(sizes, kinds, seeds):
        nb = int(nb)
        if k == 0:
            d, e = random_uniform(nb, int(s))
            out.append((d, e, "random"))
        elif k == 1:
            d, e = toeplitz(nb)
            out.append((d, e, "toeplitz"))
        else:
            d, e = glued_wilkinson(nb, int(s))
            out.append((d, e, "glued_wilkinson"))
    return out


def pack(problems):
    """Pack a list of (d, e, ...) into ragged buffers: d and e of total length
    sum(n_b) (e padded with one zero per problem), offsets int64[batch + 1]."""
    ns = np.array([p[0].shape[0] for p in problems], dtype=np.int64)
    off = np.zeros(ns.shape[0] + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    d = np.zeros(int(off[-1]))
    e = np.zeros(int(off[-1]))
    for k, p in enumerate(problems):
        o = int(off[k])
        nb = int(ns[k])
        d[o:o + nb] = p[0]
        e[o:o + nb - 1] = p[1][: nb - 1]
    return d, e, ns, off


def reflectors(n, seed, fill=0.0):
    """(V, tau) for n - 1 Householder reflectors H_i = I - tau_i v_i v_i^T,
    i = 0 .. n - 2, stored as a lower tridiagonal reduction stores them: V is
    n x n with v_i[i + 2:] in V[i + 2:, i]; v_i[i + 1] = 1 and v_i[:i + 1] = 0
    are implicit.  Every other entry of V (on and above the first
    subdiagonal, and the last column) is set to ``fill`` (NaN in tests that
    check it is never read).  tau_i = 2 / (v_i^T v_i), so each H_i is an exact
    reflection up to the rounding of tau_i."""
    rng = np.random.default_rng(seed)
    V = np.full((n, n), fill, dtype=np.float64)
    tau = np.zeros(max(n - 1, 0))
    for i in range(n - 1):
        k = n - i - 2
        below = rng.uniform(-1.0, 1.0, k) / np.sqrt(max(k + 1, 1))
        V[i + 2:, i] = below
        tau[i] = 2.0 / (1.0 + float(below @ below))
    return V, tau


def dense_symmetric(n, seed):
    """n x n symmetric matrix, column-major: entries on and below the diagonal
    U(-1, 1), mirrored above."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (n, n))
    return np.asfortranarray(np.tril(X) + np.tril(X, -1).T)


def dense_symmetric_device(n, seed, device):
    """(lower, full) on a torch device: ``lower`` is column-major with U(-1, 1)
    entries everywhere (only its lower triangle defines the matrix; the strict
    upper triangle holds unrelated values, which a reduction must not read),
    ``full`` the symmetric matrix its lower triangle defines."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    X = torch.rand((n, n), generator=g, device=device, dtype=torch.float64)
    X.mul_(2.0).sub_(1.0)
    lower = X.t().contiguous().t()
    full = torch.tril(X)
    full += torch.tril(X, -1).t()
    return lower, full.t().contiguous().t()


def dense_spd(n, seed):
    """n x n symmetric positive definite matrix, column-major: G G^T / n + I
    with G U(-1, 1)."""
    rng = np.random.default_rng(seed)
    G = rng.uniform(-1.0, 1.0, (n, n))
    S = G @ G.T / max(n, 1) + np.eye(n)
    return np.asfortranarray(0.5 * (S + S.T))


def dense_spd_device(n, seed, device):
    """the same kind of matrix as ``dense_spd`` drawn on a torch device with
    torch's seeded generator (column-major, symmetric)"""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    G = torch.rand((n, n), generator=g, device=device, dtype=torch.float64)
    G.mul_(2.0).sub_(1.0)
    S = G @ G.t()
    del G
    S.div_(max(n, 1))
    S.diagonal().add_(1.0)
    S = 0.5 * (S + S.t())
    return S.t().contiguous().t()
