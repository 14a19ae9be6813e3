"""Reduction to tridiagonal form T = Q^T M Q -- TEST INFRASTRUCTURE ONLY.

Stage 3 of the eigensolver pipeline (Sec. 1.2, stage list: reduction to
tridiagonal form; Sec. 2.2 names the direct reduction the pipeline uses and
the band-reduction alternative).  M is real symmetric, only its lower
triangle is read.  Column i = 0 .. n-2 in turn: the Householder reflector
H_i = I - tau_i v_i v_i^T with v_i[:i+1] = 0, v_i[i+1] = 1 maps the
column's entries below the diagonal, x = A[i+1:, i], onto beta e_1, and the
trailing matrix becomes H_i A H_i.  Written out as that definition: one
reflector at a time, no blocking, plain numpy FP64.

The reflector of x = (alpha, x_2..):  beta = -sign(alpha) ||x||  (alpha = +0
or -0 counts as positive), tau = (beta - alpha) / beta,
v[1:] = x[1:] / (alpha - beta); when x[1:] is zero, H = I (tau = 0,
beta = alpha).  ||x|| is formed after scaling x by a power of two near its
largest entry (exact), so no square over- or underflows.  The two-sided
update H A H of the trailing matrix is the rank-two form
A - v w^T - w v^T with y = tau A v, w = y - (tau/2)(v^T y) v.

Output in the storage a lower reduction leaves: d (n), e (n-1) with e_i =
beta_i, tau (n-1; the last is 0, its reflector has no entries to zero),
and V with v_i[i+2:] in V[i+2:, i], d on its diagonal and e on its first
subdiagonal; the entries above the diagonal are those of M.
"""
import numpy as np


def householder(x):
    """(beta, tau, v_tail) of the reflector mapping x onto beta e_1 (v[0] = 1)."""
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    tail = x[1:]
    if tail.size == 0 or not np.any(tail != 0.0):
        return alpha, 0.0, np.zeros(tail.size)
    big = max(abs(alpha), float(np.abs(tail).max()))
    _, ex = np.frexp(big)
    s_alpha = np.ldexp(alpha, -ex)
    s_tail = np.ldexp(tail, -ex)
    norm = float(np.ldexp(np.sqrt(s_alpha * s_alpha + np.dot(s_tail, s_tail)), ex))
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    v_tail = tail * (1.0 / (alpha - beta))
    return beta, tau, v_tail


def tridiagonalize(M):
    """(d, e, tau, V) of the lower Householder reduction of the symmetric M."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    A = np.tril(M) + np.tril(M, -1).T          # the symmetric matrix the lower triangle defines
    V = np.array(M, dtype=np.float64, copy=True, order="F")
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    tau = np.zeros(max(n - 1, 0))
    for i in range(n - 1):
        beta, t, v_tail = householder(A[i + 1:, i])
        e[i] = beta
        tau[i] = t
        V[i + 2:, i] = v_tail
        v = np.empty(n - i - 1)
        v[0] = 1.0
        v[1:] = v_tail
        T22 = A[i + 1:, i + 1:]
        y = t * (T22 @ v)
        w = y - (0.5 * t * (v @ y)) * v
        A[i + 1:, i + 1:] = T22 - np.outer(v, w) - np.outer(w, v)
        A[i + 1:, i] = 0.0
        A[i, i + 1:] = 0.0
        A[i + 1, i] = A[i, i + 1] = beta
    if n:
        d[:] = np.diag(A)
        V[np.arange(n), np.arange(n)] = d
        V[np.arange(1, n), np.arange(n - 1)] = e
    return d, e, tau, V
