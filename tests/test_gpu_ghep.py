"""GPU tests of the generalized eigenproblem A x = lambda B x: the Cholesky
factorization (mrrr_cholesky), the reduction to standard form (mrrr_sygst)
and the second back-transformation (mrrr_trsm_lt) against the oracle's
stages (oracle/ghep.py), and the whole pipeline on the GPU against the
oracle's pipeline and LAPACK's dsygvd.

Tolerances.  Each stage is backward stable; with B's condition number kappa
(below 7/3 for these inputs) the forward errors are bounded by c n eps kappa
times the norms involved: Cholesky factors to 20 n eps ||B||, the standard
form to 50 n eps ||A|| kappa, the solves to 20 n eps kappa ||Y||, the
generalized eigenvalues to 20 n eps ||A|| kappa, A X - B X diag(w) and
X^T B X - I to 20 n eps (||A|| kappa ||X|| and kappa).
"""
import numpy as np
import pytest

import oracle
from oracle import ghep
from paper_1205_2107_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def M():
    import paper_1205_2107_amd as pkg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return pkg


def dev_lower(A):
    """column-major device copy with NaN in the strict upper triangle"""
    n = A.shape[0]
    X = np.array(A, order="F")
    X[np.triu_indices(n, 1)] = np.nan
    return torch.tensor(X.T, device="cuda").t()


# one block, a block plus one, several blocks with a ragged last one
@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 130, 300])
def test_cholesky_vs_oracle(M, n):
    B = W.dense_spd(n, 1000 + n)
    Ld = M.cholesky(dev_lower(B))
    Lg = Ld.cpu().numpy()
    assert np.isnan(Lg[np.triu_indices(n, 1)]).all()  # upper triangle not referenced
    Lg = np.tril(np.nan_to_num(Lg, nan=0.0))
    L0 = ghep.cholesky(B)
    assert np.abs(Lg - L0).max() <= 20 * n * EPS * np.abs(B).max()
    assert np.abs(Lg @ Lg.T - B).max() <= 20 * n * EPS * np.abs(B).max()


def test_cholesky_not_positive_definite(M):
    n = 150
    B = W.dense_spd(n, 1200)
    bad = B.copy()
    bad[0, 0] = -1.0
    with pytest.raises(ValueError, match="column 1"):
        M.cholesky(dev_lower(bad))
    # a negative eigenvalue that only shows in the third block of columns
    bad = B.copy()
    bad[140, 140] = -50.0
    with pytest.raises(ValueError, match="not positive definite"):
        M.cholesky(dev_lower(bad))
    # the library stays usable
    Lg = np.tril(np.nan_to_num(M.cholesky(dev_lower(B)).cpu().numpy(), nan=0.0))
    assert np.abs(Lg @ Lg.T - B).max() <= 20 * n * EPS * np.abs(B).max()


@pytest.mark.parametrize("n", [1, 3, 64, 65, 130, 300])
def test_standard_form_vs_oracle(M, n):
    A = W.dense_symmetric(n, 1300 + n)
    B = W.dense_spd(n, 1400 + n)
    L0 = ghep.cholesky(B)
    Md = M.sygst(dev_lower(A), torch.tensor(L0.T, device="cuda").t()).cpu().numpy()
    M0 = ghep.standard_form(A, L0)
    kappa = np.linalg.cond(B)
    assert np.abs(Md - M0).max() <= 50 * n * EPS * np.abs(A).max() * kappa


@pytest.mark.parametrize("n,m", [(1, 3), (64, 64), (65, 10), (130, 200), (300, 77)])
def test_trsm_lt_vs_oracle(M, n, m):
    B = W.dense_spd(n, 1500 + n)
    L0 = ghep.cholesky(B)
    Y = np.random.default_rng(n + m).standard_normal((n, m))
    Xd = M.trsm_lt(torch.tensor(L0.T, device="cuda").t(), Y).cpu().numpy()
    X0 = ghep.back_transform_b(L0, Y)
    kappa = np.linalg.cond(L0)
    assert np.abs(Xd - X0).max() <= 20 * n * EPS * kappa * np.abs(X0).max()


def generalized_checks(A, B, w, X, wref):
    n = A.shape[0]
    normA = np.abs(np.linalg.eigvalsh(A)).max()
    kappa = np.linalg.cond(B)
    assert np.abs(w - wref).max() <= 20 * n * EPS * normA * kappa
    R = A @ X - (B @ X) * w[None, :]
    res = np.abs(R).max() / (n * EPS * normA * kappa * np.abs(X).max())
    borth = np.abs(X.T @ B @ X - np.eye(n)).max() / (n * EPS * kappa)
    return res, borth


@pytest.mark.parametrize("n", [2, 65, 200, 500])
def test_generalized_pipeline_vs_oracle(M, n):
    scipy_linalg = pytest.importorskip("scipy.linalg")
    A = W.dense_symmetric(n, 1600 + n)
    B = W.dense_spd(n, 1700 + n)
    w, X = M.eigh_generalized(dev_lower(A), dev_lower(B))
    w, X = w.cpu().numpy(), X.cpu().numpy()
    wo, Xo = ghep.eigh_generalized(A, B, oracle.mrrr)
    wl = scipy_linalg.eigh(A, B, eigvals_only=True)
    res, borth = generalized_checks(A, B, w, X, wl)
    reso, borto = generalized_checks(A, B, wo, Xo, wl)
    print(f"n={n}: GPU residual {res:.2f}, B-orthogonality {borth:.2f}; oracle {reso:.2f}, {borto:.2f}")
    assert res <= 20.0 and borth <= 20.0
    kappa = np.linalg.cond(B)
    assert np.abs(w - wo).max() <= 20 * n * EPS * np.abs(np.linalg.eigvalsh(A)).max() * kappa


def test_generalized_full_size_sampled(M):
    # order 20000 (the paper's generalized-problem size): every stage on the
    # GPU; sampled eigenpairs checked against A x = lambda B x and
    # B-orthogonality
    n = 20000
    lower, full = W.dense_symmetric_device(n, 1800, "cuda")
    Bf = W.dense_spd_device(n, 1900, "cuda")
    Bw = Bf.clone()
    w, X = M.eigh_generalized(lower, Bw)
    assert torch.isfinite(w).all()
    assert bool((w[1:] >= w[:-1]).all())
    cols = torch.tensor([0, 1, 4321, 10000, 19998, 19999], device="cuda")
    Xs = X[:, cols]
    ws = w[cols]
    R = full @ Xs - (Bf @ Xs) * ws[None, :]
    normA = float(full.abs().sum(dim=0).max())
    res = float(R.abs().max()) / (n * EPS * normA * float(Xs.abs().max()))
    G = Xs.t() @ (Bf @ Xs) - torch.eye(len(cols), dtype=torch.float64, device="cuda")
    borth = float(G.abs().max()) / (n * EPS)
    print(f"n={n}: sampled residual {res:.3f} n eps ||A||_1 max|x|, B-orthogonality {borth:.3f} n eps")
    assert res <= 20.0 and borth <= 20.0 * 3.0  # the spectrum of G G^T / n + I lies in [1, 7/3]
    del lower, full, Bf, Bw, X
    torch.cuda.empty_cache()


def test_drivers_equal_the_stages(M):
    # mrrr_syev and mrrr_sygv run the same kernels in the same order as the
    # stage-by-stage calls: identical bits
    n = 170
    A = W.dense_symmetric(n, 2100)
    B = W.dense_spd(n, 2101)
    w1, Z1 = M.eigh_dense(dev_lower(A))
    d, e, tau, V = M.tridiagonalize(dev_lower(A))
    w2, Z2 = M.eigh_tridiagonal(d, e)
    Y2 = M.backtransform(V, tau, Z2)
    assert torch.equal(w1, w2) and torch.equal(Z1, Y2)
    wg1, X1 = M.eigh_generalized(dev_lower(A), dev_lower(B))
    L = M.cholesky(dev_lower(B))
    Ms = M.sygst(dev_lower(A), L)
    d, e, tau, V = M.tridiagonalize(Ms)
    wg2, Zg = M.eigh_tridiagonal(d, e)
    X2 = M.trsm_lt(L, M.backtransform(V, tau, Zg))
    assert torch.equal(wg1, wg2) and torch.equal(X1, X2)
    bad = B.copy()
    bad[100, 100] = -5.0
    with pytest.raises(ValueError, match="not positive definite"):
        M.eigh_generalized(dev_lower(A), dev_lower(bad))
    # trivial orders
    w0, Z0 = M.eigh_dense(torch.zeros((0, 0), dtype=torch.float64, device="cuda"))
    assert w0.numel() == 0
    w1, X1 = M.eigh_generalized(np.array([[3.0]]), np.array([[4.0]]))
    assert abs(float(w1[0]) - 0.75) <= 4 * EPS and abs(float(X1[0, 0]) - 0.5) <= 4 * EPS


def test_leading_dimensions_and_nonfinite_input(M):
    # leading dimensions above n (views into taller buffers) give the same
    # bits; a NaN in A reaches the tridiagonal solver, which reports it
    n = 90
    A = W.dense_symmetric(n, 2200)
    B = W.dense_spd(n, 2201)

    def tall(X, extra):
        big = torch.full((n + extra, n), float("nan"), dtype=torch.float64, device="cuda").t().contiguous().t()
        big[:n, :] = torch.tensor(X, device="cuda")
        return big[:n, :]

    w1, X1 = M.eigh_generalized(dev_lower(A), dev_lower(B))
    Av, Bv = tall(A, 7), tall(B, 13)
    assert Av.stride(1) == n + 7 and Bv.stride(1) == n + 13
    w2, X2 = M.eigh_generalized(Av, Bv)
    assert torch.equal(w1, w2) and torch.equal(X1, X2)
    bad = A.copy()
    bad[50, 20] = np.nan
    with pytest.raises(Exception):
        M.eigh_generalized(dev_lower(bad), dev_lower(B))
    with pytest.raises(Exception):
        M.eigh_dense(dev_lower(bad))
    # the library stays usable
    w3, X3 = M.eigh_generalized(dev_lower(A), dev_lower(B))
    assert torch.equal(w1, w3)


def test_dense_drivers_on_subsets(M):
    # index and value ranges: only the selected eigenvectors are computed and
    # back-transformed; they are eigenpairs of the dense (generalized) problem
    n = 300
    A = W.dense_symmetric(n, 2300)
    B = W.dense_spd(n, 2301)
    wl = np.linalg.eigvalsh(A)
    norm1 = np.abs(A).sum(axis=0).max()
    w, Z = M.eigh_dense(dev_lower(A), select="i", il=50, iu=120)
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    assert w.shape == (71,) and Z.shape == (n, 71)
    assert np.abs(w - wl[49:120]).max() <= 2 * n * EPS * norm1
    assert np.linalg.norm(A @ Z - Z * w[None, :], axis=0).max() <= 10 * n * EPS * norm1
    assert np.abs(Z.T @ Z - np.eye(71)).max() <= 30 * n * EPS
    vl, vu = float(wl[199]) + 1e-9, float(wl[260]) + 1e-9
    w, Z = M.eigh_dense(dev_lower(A), select="v", vl=vl, vu=vu)
    assert w.shape == (61,) and Z.shape == (n, 61)
    assert np.abs(w.cpu().numpy() - wl[200:261]).max() <= 2 * n * EPS * norm1
    scipy_linalg = pytest.importorskip("scipy.linalg")
    wg = scipy_linalg.eigh(A, B, eigvals_only=True)
    w, X = M.eigh_generalized(dev_lower(A), dev_lower(B), select="i", il=1, iu=40)
    w, X = w.cpu().numpy(), X.cpu().numpy()
    kappa = np.linalg.cond(B)
    normA = np.abs(wl).max()
    assert np.abs(w - wg[:40]).max() <= 20 * n * EPS * normA * kappa
    R = A @ X - (B @ X) * w[None, :]
    assert np.abs(R).max() <= 20 * n * EPS * normA * kappa * np.abs(X).max()
    assert np.abs(X.T @ B @ X - np.eye(40)).max() <= 20 * n * EPS * kappa
