"""GPU tests of the Stage 5 back-transformation Y = Q Z (mrrr_backtransform,
blocked compact-WY form on FP64 matrix cores) against the oracle's
one-reflector-at-a-time definition (oracle/backtransform.py), and of the
pipeline it completes: LAPACK's lower tridiagonal reduction of a dense
symmetric matrix, the GPU eigensolver on its tridiagonal, then the GPU
back-transformation, checked by the dense matrix's own residual and
orthogonality.

Tolerance: a product of Householder reflections applied in floating point has
columnwise backward error ||dy|| <= c n eps ||z|| (the classical bound for
sequences of reflections); both sides meet it, so their difference is held to
||y_gpu - y_oracle||_2 <= 10 n eps ||z||_2 per column.
"""
import numpy as np
import pytest

from oracle.backtransform import apply_q
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


def colerr(Y, R, Z):
    n = Z.shape[0]
    den = 10.0 * max(n, 1) * EPS * np.maximum(np.linalg.norm(Z, axis=0), np.finfo(float).tiny)
    return float((np.linalg.norm(Y - R, axis=0) / den).max()) if Z.size else 0.0


# orders spanning one block, a block plus one reflector, several blocks with a
# ragged last block, two full blocks as one pair with no rows below it (129),
# a pair and a lone first block (193), two pairs (257); column counts below,
# at and above the 64-column tile
@pytest.mark.parametrize("n,m", [(2, 3), (3, 1), (64, 64), (65, 65), (66, 10), (129, 70), (130, 200), (193, 64),
                                 (257, 129), (300, 300), (1000, 257)])
def test_backtransform_vs_oracle(M, n, m):
    V, tau = W.reflectors(n, 9000 + n, fill=np.nan)  # unreferenced entries are NaN
    rng = np.random.default_rng(n * 7 + m)
    Z = rng.standard_normal((n, m))
    ref = apply_q(V, tau, Z)
    Y = M.backtransform(V, tau, Z).cpu().numpy()
    assert np.isfinite(Y).all()
    assert colerr(Y, ref, Z) <= 1.0


def test_backtransform_in_place_on_eigenvectors(M):
    # the eigenvector tensor of eigh_tridiagonal is column-major: transformed in place
    n = 500
    d, e = W.random_uniform(n, 9101)
    w, Z = M.eigh_tridiagonal(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda"))
    Z0 = Z.cpu().numpy()
    V, tau = W.reflectors(n, 9102)
    Y = M.backtransform(V, tau, Z)
    assert Y.data_ptr() == Z.data_ptr()
    assert colerr(Y.cpu().numpy(), apply_q(V, tau, Z0), Z0) <= 1.0


@pytest.mark.parametrize("n", [150, 400])
def test_dense_pipeline_with_lapack_reduction(M, n):
    # M = Q T Q^T from LAPACK's dsytrd; eigenvectors of T on the GPU; Y = Q Z on
    # the GPU must be the eigenvectors of the dense matrix
    lapack = pytest.importorskip("scipy.linalg.lapack")
    rng = np.random.default_rng(9200 + n)
    A = rng.uniform(-1.0, 1.0, (n, n))
    A = 0.5 * (A + A.T)
    c, d, e, tau, info = lapack.dsytrd(A, lower=1)
    assert info == 0
    w, Z = M.eigh_tridiagonal(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda"))
    Zn = Z.cpu().numpy()  # before the in-place back-transformation
    Y = M.backtransform(c, tau, Z).cpu().numpy()
    wn = w.cpu().numpy()
    norm1 = np.abs(A).sum(axis=0).max()
    res = np.linalg.norm(A @ Y - Y * wn[None, :], axis=0).max() / (n * EPS * norm1)
    # orthogonality: the tridiagonal eigenvectors meet 10 n eps; the
    # back-transformation moves each column by at most 10 n eps (its parity
    # bar), which enters Y^T Y twice
    orth_z = np.abs(Zn.T @ Zn - np.eye(n)).max() / (n * EPS)
    orth = np.abs(Y.T @ Y - np.eye(n)).max() / (n * EPS)
    print(f"n={n}: residual {res:.2f} n eps ||M||_1, orthogonality {orth:.2f} n eps (tridiagonal {orth_z:.2f})")
    assert res <= 10.0 and orth_z <= 10.0 and orth <= orth_z + 20.0, (res, orth_z, orth)
    assert np.abs(wn - np.linalg.eigvalsh(A)).max() <= 2 * n * EPS * norm1


def test_full_size_sampled_columns(M):
    # n = m = 20000 (the eigenvectors of the order-20000 1-2-1 matrix): every
    # column keeps its norm; sampled columns against the oracle
    n = 20000
    d, e = W.toeplitz(n)
    w, Z = M.eigh_tridiagonal(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda"))
    cols = np.array([0, 1, 4999, 10000, 19998, 19999])
    Zs = Z[:, cols].cpu().numpy()
    V, tau = W.reflectors(n, 9300)
    Vd = torch.tensor(V.T, device="cuda").t()  # column-major on the device
    del V
    norms0 = torch.linalg.vector_norm(Z, dim=0)
    Y = M.backtransform(Vd, tau, Z)
    norms1 = torch.linalg.vector_norm(Y, dim=0)
    assert float((norms1 - norms0).abs().max()) <= 10 * n * EPS
    Vh = Vd.t().cpu().numpy().T
    ref = apply_q(Vh, tau, Zs)
    assert colerr(Y[:, cols].cpu().numpy(), ref, Zs) <= 1.0
    del Vd, Y, Z
    torch.cuda.empty_cache()


def test_trivial_sizes(M):
    Z = torch.ones((1, 4), dtype=torch.float64, device="cuda").t().contiguous().t()
    assert torch.equal(M.backtransform(np.zeros((1, 1)), np.zeros(0), Z), torch.ones((1, 4), dtype=torch.float64,
                                                                                     device="cuda"))
    Z = torch.zeros((5, 0), dtype=torch.float64, device="cuda")
    V, tau = W.reflectors(5, 1)
    assert M.backtransform(V, tau, Z).shape == (5, 0)
