"""Pins of the back-transformation oracle (oracle/backtransform.py) against
what does not depend on it: LAPACK's own tridiagonal reduction (dsytrd, lower)
must satisfy M = Q T Q^T with the oracle's Q, and LAPACK's reflector
application (dormqr on the reflectors below the first subdiagonal, the way a
lower back-transformation is built from it) must agree with the oracle."""
import numpy as np
import pytest

from oracle.backtransform import apply_q
from paper_1205_2107_amd import workloads as W

scipy_lapack = pytest.importorskip("scipy.linalg.lapack")

EPS = np.finfo(np.float64).eps


def sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, (n, n))
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n", [2, 3, 7, 40, 129])
def test_reduction_identity(n):
    # dsytrd (lower) reduces M to T = Q^T M Q and stores Q's reflectors;
    # the oracle's Q must rebuild M from T
    M = sym(n, 100 + n)
    c, d, e, tau, info = scipy_lapack.dsytrd(M, lower=1)
    assert info == 0
    Q = apply_q(c, tau, np.eye(n))
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(Q @ T @ Q.T - M).max() <= 20 * n * EPS * np.abs(M).max()
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 20 * n * EPS


@pytest.mark.parametrize("n,m", [(5, 3), (64, 64), (150, 17)])
def test_against_lapack_dormqr(n, m):
    # a lower reduction's Q is diag(1, Q') with Q' the product of the
    # reflectors stored from row 1 on, in the QR storage dormqr applies
    M = sym(n, 200 + n)
    c, d, e, tau, info = scipy_lapack.dsytrd(M, lower=1)
    rng = np.random.default_rng(n + m)
    Z = rng.standard_normal((n, m))
    Y = apply_q(c, tau, Z)
    ref = Z.copy()
    if n > 1:
        out = scipy_lapack.dormqr("L", "N", np.asfortranarray(c[1:, :n - 1]), tau,
                                  np.asfortranarray(Z[1:, :]), lwork=max(1, 64 * m))
        ref[1:, :] = out[0]
        assert out[-1] == 0
    assert np.abs(Y - ref).max() <= 20 * n * EPS * np.abs(Z).max()


def test_unreferenced_entries_and_synthetic_reflectors():
    # NaN on and above the first subdiagonal is never read; the synthetic
    # reflectors give an orthogonal Q (each H_i an exact reflection up to tau's rounding)
    n = 90
    V, tau = W.reflectors(n, 7, fill=np.nan)
    V0, tau0 = W.reflectors(n, 7, fill=0.0)
    assert np.array_equal(tau, tau0)
    Q = apply_q(V, tau, np.eye(n))
    assert np.isfinite(Q).all()
    assert np.array_equal(Q, apply_q(V0, tau0, np.eye(n)))
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 20 * n * EPS
    # each H_i maps v_i to -v_i
    i = 10
    v = np.zeros(n)
    v[i + 1] = 1.0
    v[i + 2:] = V[i + 2:, i]
    H = np.eye(n) - tau[i] * np.outer(v, v)
    assert np.abs(H @ v + v).max() <= 8 * EPS


def test_trivial_orders():
    for n in (0, 1):
        Z = np.arange(float(n * 3)).reshape(n, 3)
        assert np.array_equal(apply_q(np.zeros((n, n)), np.zeros(0), Z), Z)
