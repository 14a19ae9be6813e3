"""Back-transformation y = Q z -- TEST INFRASTRUCTURE ONLY.

Stage 5 of the eigensolver pipeline (Sec. 1.2, stage list: the first
back-transformation): after the reduction T = Q^T M Q of Stage 3, the
eigenvectors of M are Y = Q Z for the tridiagonal eigenvectors Z.  Here Q is
the product of n - 1 Householder reflectors as a lower tridiagonal reduction
leaves them,

    Q = H_0 H_1 ... H_{n-2},   H_i = I - tau_i v_i v_i^T,
    v_i[:i + 1] = 0,  v_i[i + 1] = 1,  v_i[i + 2:] = V[i + 2:, i],

so Q Z applies H_{n-2} first and H_0 last.  Written out as that definition:
one reflector at a time, no blocking, plain numpy FP64.  Entries of V on or
above the first subdiagonal are never read.
"""
import numpy as np


def apply_q(V, tau, Z):
    """Y = Q Z for the reflectors (V, tau); Z is n x m, returned as a new array."""
    V = np.asarray(V, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    Y = np.array(Z, dtype=np.float64, copy=True)
    n = Y.shape[0]
    for i in range(n - 2, -1, -1):
        v = np.empty(n - i - 1)
        v[0] = 1.0
        v[1:] = V[i + 2:, i]
        rows = Y[i + 1:, :]
        rows -= tau[i] * np.outer(v, v @ rows)
    return Y
