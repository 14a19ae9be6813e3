"""The norm of the twisted solve's vector from the derivative of gamma.

The eigenvector kernels take ||z||^2 (z_r = 1) of the twisted factorization
of L D L^T - lam I (Sec. 3.1.1: one step of inverse iteration with a twisted
factorization) not from the solved vector but from derivatives carried along
the two transforms:

    d s_{i+1} = (L+_i)^2 d s_i - 1,   d s_1 = -1     (stationary, top-down)
    d p_i     = (U-_i)^2 d p_{i+1} - 1, d p_n = -1   (progressive, bottom-up)
    ||z||^2   = -(d s_r + d p_r + 1) = -d gamma_r / d lam.

These tests pin that identity on small matrices against three things that
do not use it: the vector from the twisted solve, a central difference of
gamma_r(lam), and the dense formula gamma_r^2 e_r^T (L D L^T - lam I)^{-2} e_r.
Plain float64 NumPy; neither the oracle nor the kernels are involved.
"""
import numpy as np


def ldl_from_tridiagonal(d, e, sigma):
    """L D L^T = T - sigma I (unit lower bidiagonal L, diagonal D)."""
    n = d.size
    D = np.empty(n)
    L = np.zeros(max(n - 1, 0))
    D[0] = d[0] - sigma
    for i in range(n - 1):
        L[i] = e[i] / D[i]
        D[i + 1] = d[i + 1] - sigma - L[i] * e[i]
    return D, L


def twisted(D, L, lam):
    """Transforms, twist index, derivatives and the solved vector.

    s_i: stationary transform (D+_i = D_i + s_i, L+_i = L_i D_i / D+_i);
    p_i: progressive transform (p_i = D_i (p_{i+1} / (L_i^2 D_i + p_{i+1})) - lam,
    U-_i = L_i D_i / (L_i^2 D_i + p_{i+1})); gamma_k = s_k + p_k + lam."""
    n = D.size
    LD = L * D[:-1]
    LLD = L * LD
    s = np.empty(n)
    ds = np.empty(n)
    Lp = np.empty(n - 1)
    s[0], ds[0] = -lam, -1.0
    for i in range(n - 1):
        dp = D[i] + s[i]
        Lp[i] = LD[i] / dp
        s[i + 1] = s[i] * LLD[i] / dp - lam
        ds[i + 1] = Lp[i] ** 2 * ds[i] - 1.0
    p = np.empty(n)
    dpv = np.empty(n)
    Um = np.empty(n - 1)
    p[n - 1], dpv[n - 1] = D[n - 1] - lam, -1.0
    for i in range(n - 2, -1, -1):
        den = LLD[i] + p[i + 1]
        Um[i] = LD[i] / den
        p[i] = p[i + 1] * D[i] / den - lam
        dpv[i] = Um[i] ** 2 * dpv[i + 1] - 1.0
    gamma = s + p + lam
    r = int(np.argmin(np.abs(gamma)))
    z = np.empty(n)
    z[r] = 1.0
    for i in range(r - 1, -1, -1):
        z[i] = -Lp[i] * z[i + 1]
    for i in range(r, n - 1):
        z[i + 1] = -Um[i] * z[i]
    return gamma, r, ds, dpv, z


def cases():
    rng = np.random.default_rng(20261202)
    for n, kind in [(40, "random"), (97, "random"), (64, "toeplitz"), (120, "graded")]:
        if kind == "random":
            d = rng.uniform(-1, 1, n)
            e = rng.uniform(-1, 1, n - 1)
        elif kind == "toeplitz":
            d = np.full(n, 2.0)
            e = np.full(n - 1, -1.0)
        else:
            d = np.geomspace(1.0, 1e-6, n)
            e = 0.3 * np.sqrt(d[:-1] * d[1:])
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        w = np.linalg.eigvalsh(T)
        sigma = w[0] - 1e-3 * (w[-1] - w[0])  # definite shift below the spectrum
        D, L = ldl_from_tridiagonal(d, e, sigma)
        A = np.diag(D) + np.diag(L * D[:-1], 1) + np.diag(L * D[:-1], -1) + np.diag(np.r_[0.0, L ** 2 * D[:-1]])
        for j in (0, n // 3, n - 1):
            mu = w[j] - sigma
            gap = np.min(np.abs(np.delete(w, j) - w[j]))
            for rel in (1e-3, 1e-7):  # a shift near the eigenvalue, as in the Rayleigh-quotient rounds
                yield A, D, L, mu + rel * gap, gap


def test_norm_from_derivatives_equals_sum_of_squares():
    for A, D, L, lam, _ in cases():
        gamma, r, ds, dp, z = twisted(D, L, lam)
        nrm_direct = float(np.sum(z * z))
        nrm_deriv = -(ds[r] + dp[r] + 1.0)
        assert np.isclose(nrm_deriv, nrm_direct, rtol=1e-11), (nrm_deriv, nrm_direct)


def test_norm_is_minus_the_derivative_of_gamma():
    for A, D, L, lam, gap in cases():
        gamma, r, ds, dp, z = twisted(D, L, lam)
        # gamma_r(lam) is smooth on the scale of the eigenvalue gap
        h = 1e-5 * gap
        gp = twisted(D, L, lam + h)[0][r]
        gm = twisted(D, L, lam - h)[0][r]
        fd = -(gp - gm) / (2.0 * h)
        assert np.isclose(fd, np.sum(z * z), rtol=1e-5), (fd, np.sum(z * z))


def test_norm_matches_the_dense_resolvent():
    for A, D, L, lam, gap in cases():
        gamma, r, ds, dp, z = twisted(D, L, lam)
        n = D.size
        er = np.zeros(n)
        er[r] = 1.0
        x = np.linalg.solve(A - lam * np.eye(n), er)
        # z = gamma_r (A - lam)^{-1} e_r, so ||z||^2 = gamma_r^2 ||(A - lam)^{-1} e_r||^2;
        # the dense solve with lam this close to an eigenvalue loses about
        # eps ||A|| / |lam - lambda_j| relative accuracy
        tol = 1e-9 + 1e-14 * np.abs(A).sum(axis=1).max() / abs(gamma[r])
        dense = gamma[r] ** 2 * float(x @ x)
        assert np.isclose(-(ds[r] + dp[r] + 1.0), dense, rtol=tol), (-(ds[r] + dp[r] + 1.0), dense, tol)
        # and the solved vector is that resolvent column, scaled
        assert np.allclose(z, gamma[r] * x, rtol=tol, atol=tol * np.max(np.abs(z)))
