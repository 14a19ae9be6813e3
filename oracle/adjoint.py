"""Dense adjoint of the tridiagonal eigendecomposition -- TEST INFRASTRUCTURE ONLY.

For T = V diag(w) V^T with simple eigenvalues, first-order perturbation theory
gives  d w_k = v_k^T dT v_k  and  d v_k = sum_{i != k} v_i (v_i^T dT v_k) / (w_k - w_i).
Hence a loss L(w, V) with cotangents gw = dL/dw and gV = dL/dV has

    dL/dT = V (diag(gw) + F o (V^T gV)) V^T,   F_ik = 1 / (w_k - w_i) (i != k), F_kk = 0,

and because T is tridiagonal with d on the diagonal and e on both off-diagonals,
    grad_d_i = (dL/dT)_{i,i},   grad_e_i = (dL/dT)_{i,i+1} + (dL/dT)_{i+1,i}.
The eigenvector sign convention (largest-magnitude entry positive) is locally
constant, so it contributes nothing.  Plain numpy FP64, written out as the
definition; no blocking or fusion.
"""
import numpy as np


def dense_adjoint(w, V, gw=None, gV=None):
    w = np.asarray(w, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n = w.shape[0]
    M = np.zeros((n, n))
    if gw is not None:
        M += np.diag(np.asarray(gw, dtype=np.float64))
    if gV is not None:
        C = V.T @ np.asarray(gV, dtype=np.float64)
        diff = w[None, :] - w[:, None]          # diff[i, k] = w_k - w_i
        F = np.zeros((n, n))
        off = ~np.eye(n, dtype=bool)
        F[off] = 1.0 / diff[off]
        M += F * C
    A = V @ M @ V.T
    gd = np.diag(A).copy()
    ge = np.diag(A, 1) + np.diag(A, -1)
    return gd, ge
