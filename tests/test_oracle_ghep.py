"""Pins of the generalized-eigenproblem oracle (oracle/ghep.py) against
LAPACK's own generalized solver (scipy.linalg.eigh(A, B): dsygvd), the
defining identities A X = B X diag(w) and X^T B X = I, and a closed form
(B = c I scales the spectrum of A by 1/c)."""
import numpy as np
import pytest

import oracle
from oracle import ghep
from paper_1205_2107_amd import workloads as W

scipy_linalg = pytest.importorskip("scipy.linalg")

EPS = np.finfo(np.float64).eps


def spd(n, seed):
    return W.dense_spd(n, seed)


@pytest.mark.parametrize("n", [1, 2, 5, 40, 130])
def test_against_lapack_sygvd(n):
    A = W.dense_symmetric(n, 500 + n)
    B = spd(n, 600 + n)
    w, X = ghep.eigh_generalized(A, B, oracle.mrrr)
    wr = scipy_linalg.eigh(A, B, eigvals_only=True)
    normA = np.abs(np.linalg.eigvalsh(A)).max()
    kappa = np.linalg.cond(B)
    assert np.abs(w - wr).max() <= 20 * n * EPS * normA * kappa
    R = A @ X - (B @ X) * w[None, :]
    assert np.abs(R).max() <= 20 * n * EPS * normA * kappa * np.abs(X).max()
    assert np.abs(X.T @ B @ X - np.eye(n)).max() <= 20 * n * EPS * kappa


def test_scaled_identity_b():
    # B = 4 I: the eigenvalues are those of A over 4 and X^T X = I / 4
    n = 60
    A = W.dense_symmetric(n, 11)
    w, X = ghep.eigh_generalized(A, 4.0 * np.eye(n), oracle.mrrr)
    assert np.abs(w - np.linalg.eigvalsh(A) / 4.0).max() <= 20 * n * EPS
    assert np.abs(X.T @ X - np.eye(n) / 4.0).max() <= 20 * n * EPS


def test_stages():
    n = 50
    A = W.dense_symmetric(n, 12)
    B = spd(n, 13)
    L = ghep.cholesky(B)
    assert np.abs(L @ L.T - B).max() <= 20 * n * EPS * np.abs(B).max()
    assert np.array_equal(L, np.tril(L))
    M = ghep.standard_form(A, L)
    assert np.abs(L @ M @ L.T - A).max() <= 50 * n * EPS * np.abs(A).max() * np.linalg.cond(B)
    Y = np.random.default_rng(1).standard_normal((n, 7))
    X = ghep.back_transform_b(L, Y)
    assert np.abs(L.T @ X - Y).max() <= 20 * n * EPS * np.abs(Y).max() * np.linalg.cond(L)
    # only the lower triangles are read
    U = A.copy()
    U[np.triu_indices(n, 1)] = np.nan
    assert np.array_equal(ghep.standard_form(U, L), M)
