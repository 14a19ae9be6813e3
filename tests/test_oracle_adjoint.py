"""Pins of the dense adjoint (oracle/adjoint.py) against central finite
differences, the Hellmann-Feynman closed form and exact invariances."""
import numpy as np
import pytest

import oracle
from common import dense, jacobi_eigh, sign_normalize
from paper_1205_2107_amd import workloads as W


def loss_eigh(d, e, c, G, solver):
    w, V = solver(dense(d, e))
    V = sign_normalize(V)
    return float(c @ w + np.sum(G * V))


def fd_grad(d, e, c, G, solver, h=1e-6):
    gd = np.zeros_like(d)
    ge = np.zeros_like(e)
    for i in range(len(d)):
        dp = d.copy(); dp[i] += h
        dm = d.copy(); dm[i] -= h
        gd[i] = (loss_eigh(dp, e, c, G, solver) - loss_eigh(dm, e, c, G, solver)) / (2 * h)
    for i in range(len(e)):
        ep = e.copy(); ep[i] += h
        em = e.copy(); em[i] -= h
        ge[i] = (loss_eigh(d, ep, c, G, solver) - loss_eigh(d, em, c, G, solver)) / (2 * h)
    return gd, ge


@pytest.mark.parametrize("n,solver", [(8, "jacobi"), (16, "jacobi"), (32, "lapack"), (64, "lapack")])
def test_fd(n, solver):
    rng = np.random.default_rng(W.SEEDS["c5_fd"] + n)
    d, e = W.separated(n, W.SEEDS["c5_fd"] + n)
    c = rng.standard_normal(n)
    G = rng.standard_normal((n, n))
    f = jacobi_eigh if solver == "jacobi" else np.linalg.eigh
    w, V, st = oracle.mrrr(d, e)
    gd, ge = oracle.dense_adjoint(w, V, c, G)
    fgd, fge = fd_grad(d, e, c, G, f)
    g = np.concatenate([gd, ge])
    fg = np.concatenate([fgd, fge])
    assert np.abs(g - fg).max() <= 1e-6 * np.abs(fg).max()


def test_hellmann_feynman_toeplitz():
    n = 40
    d, e = W.toeplitz(n)
    k = np.arange(1, n + 1)
    j = np.arange(1, n + 1)[:, None]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * np.pi / (n + 1))
    c = np.random.default_rng(0).standard_normal(n)
    w, Z, st = oracle.mrrr(d, e)
    gd, ge = oracle.dense_adjoint(w, Z, c, None)
    # d lambda_k / d d_i = v_k(i)^2, d lambda_k / d e_i = 2 v_k(i) v_k(i+1)
    hd = (V ** 2) @ c
    he = (2 * V[:-1] * V[1:]) @ c
    assert np.abs(gd - hd).max() <= 1e-12
    assert np.abs(ge - he).max() <= 1e-12


def test_invariances():
    n = 80
    d, e = W.separated(n, 77)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(n)
    G = rng.standard_normal((n, n))
    w, V, st = oracle.mrrr(d, e)
    # shift T -> T + t I moves every eigenvalue by t and no vector: sum(gd) = sum(c)
    gd, ge = oracle.dense_adjoint(w, V, c, G)
    assert abs(gd.sum() - c.sum()) <= 1e-9 * np.abs(c).sum()
    # scaling T -> s T scales eigenvalues and keeps vectors: Euler identity
    lhs = d @ gd + e @ ge
    assert abs(lhs - c @ w) <= 1e-9 * (np.abs(c) @ np.abs(w) + 1)
