"""Pins of the reduction oracle (oracle/tridiagonalize.py) against what does
not depend on it: LAPACK's own lower reduction (dsytrd uses the same
reflector convention, so d, e, tau and the reflectors agree up to rounding),
the eigenvalues of M (LAPACK's eigvalsh), M = Q T Q^T with Q from the pinned
back-transformation oracle, a closed form (the all-ones matrix), and the
special cases that leave the matrix as it is."""
import numpy as np
import pytest

from oracle.backtransform import apply_q
from oracle.tridiagonalize import householder, tridiagonalize

scipy_lapack = pytest.importorskip("scipy.linalg.lapack")

EPS = np.finfo(np.float64).eps


def sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, (n, n))
    return 0.5 * (A + A.T)


def tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("n", [2, 3, 4, 17, 64, 65, 150, 301])
def test_against_lapack_dsytrd(n):
    M = sym(n, 300 + n)
    d, e, tau, V = tridiagonalize(M)
    c, d2, e2, tau2, info = scipy_lapack.dsytrd(M, lower=1)
    assert info == 0
    norm = np.abs(np.linalg.eigvalsh(M)).max()
    bar = 100 * n * EPS * norm
    assert np.abs(d - d2).max() <= bar
    assert np.abs(e - e2).max() <= bar
    assert np.abs(tau - tau2).max() <= bar
    low = np.tril(np.ones((n, n), dtype=bool), -2)
    if low.any():
        assert np.abs(V[low] - c[low]).max() <= bar
    assert np.array_equal(np.diag(V), d)
    assert np.array_equal(np.diag(V, -1), e)


@pytest.mark.parametrize("n", [5, 40, 129])
def test_reduction_identity_and_spectrum(n):
    M = sym(n, 400 + n)
    d, e, tau, V = tridiagonalize(M)
    Q = apply_q(V, tau, np.eye(n))
    T = tri(d, e)
    norm = np.abs(np.linalg.eigvalsh(M)).max()
    assert np.abs(Q @ T @ Q.T - M).max() <= 20 * n * EPS * norm
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 20 * n * EPS
    assert np.abs(np.linalg.eigvalsh(T) - np.linalg.eigvalsh(M)).max() <= 2 * n * EPS * norm
    assert tau[-1] == 0.0


@pytest.mark.parametrize("n", [3, 10, 101])
def test_all_ones_closed_form(n):
    # J = 1 1^T: the first reflector maps (1, .., 1) onto -sqrt(n-1) e_1, after
    # which the trailing matrix is (n-1) e_1 e_1^T, so
    # T = [[1, -sqrt(n-1)], [-sqrt(n-1), n-1]] (+) 0 (the later reflectors act
    # on rounding noise, so their tau is not fixed)
    d, e, tau, V = tridiagonalize(np.ones((n, n)))
    r = np.sqrt(n - 1.0)
    d_ref = np.zeros(n)
    d_ref[0], d_ref[1] = 1.0, n - 1.0
    e_ref = np.zeros(n - 1)
    e_ref[0] = -r
    assert np.abs(d - d_ref).max() <= 8 * n * EPS
    assert np.abs(e - e_ref).max() <= 8 * n * EPS
    assert abs(tau[0] - (1.0 + 1.0 / r)) <= 8 * EPS
    assert np.abs(V[2:, 0] - 1.0 / (1.0 + r)).max() <= 8 * EPS


def test_tridiagonal_and_diagonal_inputs_are_left_alone():
    rng = np.random.default_rng(5)
    n = 30
    dd, ee = rng.standard_normal(n), rng.standard_normal(n - 1)
    d, e, tau, V = tridiagonalize(tri(dd, ee))
    assert np.array_equal(d, dd) and np.array_equal(e, ee) and not tau.any()
    d, e, tau, V = tridiagonalize(np.diag(dd))
    assert np.array_equal(d, dd) and not e.any() and not tau.any()


def test_only_the_lower_triangle_is_read():
    M = sym(50, 9)
    U = M.copy()
    U[np.triu_indices(50, 1)] = np.nan
    a, b = tridiagonalize(M), tridiagonalize(U)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_householder_reflector():
    rng = np.random.default_rng(3)
    for alpha_sign in (1.0, -1.0, 0.0):
        x = rng.standard_normal(12)
        x[0] = alpha_sign * abs(x[0])
        beta, tau, vt = householder(x)
        v = np.concatenate(([1.0], vt))
        H = np.eye(12) - tau * np.outer(v, v)
        target = np.zeros(12)
        target[0] = beta
        assert np.abs(H @ x - target).max() <= 8 * EPS * np.linalg.norm(x)
        assert abs(abs(beta) - np.linalg.norm(x)) <= 4 * EPS * np.linalg.norm(x)
        assert (beta < 0) == (x[0] >= 0)
        assert abs(tau * (v @ v) - 2.0) <= 8 * EPS
    # power-of-two scaling is exact: tiny and huge vectors give the same
    # reflector and beta scaled by the same power
    x = rng.standard_normal(9)
    ref = householder(x)
    for s in (2.0 ** -1000, 2.0 ** 1000):
        b, t, vt = householder(x * s)
        assert b == ref[0] * s and t == ref[1] and np.array_equal(vt, ref[2])
    # a zero tail: H = I
    b, t, vt = householder(np.array([3.0, 0.0, 0.0]))
    assert (b, t) == (3.0, 0.0) and not vt.any()


def test_trivial_orders():
    d, e, tau, V = tridiagonalize(np.array([[2.5]]))
    assert d.tolist() == [2.5] and e.size == 0 and tau.size == 0
    d, e, tau, V = tridiagonalize(np.array([[1.0, 2.0], [2.0, 3.0]]))
    assert d.tolist() == [1.0, 3.0] and e.tolist() == [2.0] and tau.tolist() == [0.0]
