"""The stored oracle eigenvalues of the full-size matrices (tests/golden/,
written by tests/golden/make_eigenvalues.py from the oracle alone) are pinned
here to what does not depend on the oracle: the generator still produces the
matrix each file was written for (SHA-256 of its bytes), the closed form of the
1-2-1 spectrum, the prescribed geometric spectrum, the trace invariants, and a
Sturm certificate on T itself (counts with plain LDL^T pivots of T - tau I)."""
import functools
import hashlib
import json
import os

import numpy as np
import pytest

from common import EPS, norm1, sturm_counts_T
from paper_1205_2107_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def manifest():
    with open(os.path.join(GOLDEN, "eigvals_manifest.json")) as f:
        return json.load(f)


def load(name):
    return np.load(os.path.join(GOLDEN, f"eigvals_{name}.npy"), allow_pickle=False)


@functools.lru_cache(maxsize=None)
def make(expr):
    return eval(expr, {}, {k: getattr(W, k) for k in dir(W) if not k.startswith("_")})


NAMES = sorted(manifest())


@pytest.mark.parametrize("name", NAMES)
def test_golden_inputs_unchanged(name):
    m = manifest()[name]
    d, e = make(m["expr"])
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(d, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(e, dtype="<f8").tobytes())
    assert h.hexdigest() == m["input_sha256"], "the generator no longer produces this matrix"
    w = load(name)
    assert w.shape == (m["n"],) and np.all(np.diff(w) >= 0)


def test_golden_toeplitz_closed_form():
    w = load("c2_toeplitz_n20000")
    n = w.shape[0]
    k = np.arange(1, n + 1)
    lam = 4.0 * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    d, e = W.toeplitz(n)
    assert np.abs(w - lam).max() <= 2 * n * EPS * norm1(d, e)


def test_golden_geometric_prescribed_spectrum():
    w = load("c2_geometric_n20000")
    n = w.shape[0]
    d, e = make(manifest()["c2_geometric_n20000"]["expr"])
    assert np.abs(w - W.geometric_spectrum(n)).max() <= 2 * n * EPS * norm1(d, e)


@pytest.mark.parametrize("name", NAMES)
def test_golden_trace_invariants(name):
    d, e = make(manifest()[name]["expr"])
    w = load(name)
    n = d.shape[0]
    tn = norm1(d, e)
    assert abs(w.sum() - d.sum()) <= n * n * EPS * tn
    assert abs((w ** 2).sum() - (d ** 2).sum() - 2 * (e ** 2).sum()) <= n * n * EPS * tn ** 2


@pytest.mark.parametrize("name", ["c2_random_n20000", "glued1_n20000", "c2_geometric_n20000",
                                  "c3_glued_n60000"])
def test_golden_sturm_certificate(name):
    # cnt_T(w_j - t) <= j - 1 and cnt_T(w_j + t) >= j with t = 2 n eps ||T||_1:
    # every stored value is within t of the j-th eigenvalue of T (counts on T
    # are exact for a matrix within a few eps ||T|| of T)
    if name not in manifest():
        pytest.skip("file not written")
    d, e = make(manifest()[name]["expr"])
    w = load(name)
    n = d.shape[0]
    t = 2 * n * EPS * norm1(d, e)
    j = np.arange(1, n + 1)
    if n > 20000:
        j = j[::7]
    assert np.all(sturm_counts_T(d, e, w[j - 1] - t) <= j - 1)
    assert np.all(sturm_counts_T(d, e, w[j - 1] + t) >= j)
