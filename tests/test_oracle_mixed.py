"""Pins of the FP32-data oracle (oracle.mrrr_fp32: FP64 solve of the exactly
widened inputs, results rounded to FP32) against the Toeplitz closed form
rounded to FP32 and the FP32 rounding bounds of its vectors."""
import numpy as np

import oracle

EPS32 = np.finfo(np.float32).eps


def test_toeplitz_closed_form_rounded():
    # 1-2-1: lambda_k = 2 - 2 cos(k pi / (n + 1)); the FP32 result is the FP64
    # value (within 2 n eps64 of the exact one) rounded, so within one FP32
    # ulp of the exact value rounded
    n = 300
    d = np.full(n, 2.0, dtype=np.float32)
    e = np.full(n - 1, -1.0, dtype=np.float32)
    w, Z, st = oracle.mrrr_fp32(d, e)
    assert st == 0 and w.dtype == np.float32 and Z.dtype == np.float32
    k = np.arange(1, n + 1)
    exact = (2.0 - 2.0 * np.cos(k * np.pi / (n + 1))).astype(np.float32)
    ulps = np.abs(w.astype(np.float64) - exact.astype(np.float64)) / np.spacing(np.abs(exact))
    assert ulps.max() <= 1.0
    # sine eigenvectors, to FP32 rounding
    j = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * np.pi / (n + 1))
    Zd = Z.astype(np.float64)
    S *= np.sign((S * Zd).sum(axis=0))  # the largest entries come in pairs of equal magnitude: compare sign-blind
    assert np.abs(Zd - S).max() <= 4 * EPS32


def test_rounded_vectors_are_orthogonal_to_fp32_rounding():
    rng = np.random.default_rng(3)
    n = 400
    d = rng.uniform(-1, 1, n).astype(np.float32)
    e = rng.uniform(-1, 1, n - 1).astype(np.float32)
    w, Z, st = oracle.mrrr_fp32(d, e)
    Zd = Z.astype(np.float64)
    # each entry rounded by at most eps32 / 2 relative: |z_i^T z_j| <= eps32
    # plus the FP64 solve's O(n eps64)
    assert np.abs(Zd.T @ Zd - np.eye(n)).max() <= 2 * EPS32
