"""Dense generalized eigenproblem A x = lambda B x -- TEST INFRASTRUCTURE ONLY.

The stage list of Sec. 1.2 for A symmetric and B symmetric positive
definite, each stage written out as its definition:
  1. Cholesky factorization B = L L^T (numpy's cholesky, a library
     primitive);
  2. reduction to the standard problem M = L^{-1} A L^{-T} (two triangular
     solves, scipy's solve_triangular);
  3. reduction to tridiagonal form T = Q^T M Q (``tridiagonalize``);
  4. the tridiagonal eigenproblem (the C oracle ``mrrr``);
  5. first back-transformation Y = Q Z (``apply_q``);
  6. second back-transformation X = L^{-T} Y (solve_triangular).
Only the lower triangles of A and B are read.
"""
import numpy as np
from scipy.linalg import solve_triangular

from .backtransform import apply_q
from .tridiagonalize import tridiagonalize


def cholesky(B):
    """L with B = L L^T from the lower triangle of B."""
    B = np.asarray(B, dtype=np.float64)
    S = np.tril(B) + np.tril(B, -1).T
    return np.linalg.cholesky(S)


def standard_form(A, L):
    """M = L^{-1} A L^{-T} for the symmetric A given by its lower triangle."""
    A = np.asarray(A, dtype=np.float64)
    S = np.tril(A) + np.tril(A, -1).T
    X = solve_triangular(L, S, lower=True)
    return solve_triangular(L, X.T, lower=True)


def back_transform_b(L, Y):
    """X = L^{-T} Y."""
    return solve_triangular(L.T, Y, lower=False)


def eigh_generalized(A, B, mrrr):
    """(w, X) of A x = lambda B x through the six stages; ``mrrr`` is the
    tridiagonal eigensolver (d, e) -> (w, Z, status)."""
    L = cholesky(B)
    M = standard_form(A, L)
    d, e, tau, V = tridiagonalize(M)
    w, Z, st = mrrr(d, e)
    if st != 0:
        raise RuntimeError(f"tridiagonal eigensolver status {st}")
    Y = apply_q(V, tau, Z)
    return w, back_transform_b(L, Y)
