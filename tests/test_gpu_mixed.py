"""GPU tests of the FP32 interface with FP64 arithmetic inside
(mrrr_step_f32): against the oracle's FP32-data solve (oracle.mrrr_fp32:
widen exactly, FP64 MRRR, round), with the bars FP32 rounding sets --
eigenvalues within one FP32 ulp of the oracle's FP64 value plus the FP64
bound 2 n eps64 ||T||, residual and orthogonality O(eps32) independent of n
(each rounded entry moves by at most eps32 / 2 relative; the relaxed
classification threshold keeps the FP64 vectors' own error below eps32 / 4).
"""
import numpy as np
import pytest

import oracle
from paper_1205_2107_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


@pytest.fixture(scope="module")
def M():
    import paper_1205_2107_amd as pkg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return pkg


def f32(d, e):
    return np.asarray(d, dtype=np.float32), np.asarray(e, dtype=np.float32)


def check(d, e, w, Z, wo64):
    n = d.size
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = np.abs(d64).max() + 2 * (np.abs(e64).max() if n > 1 else 0.0)
    wd = w.astype(np.float64)
    bar = np.spacing(np.abs(wo64).astype(np.float32)).astype(np.float64) + 2 * n * EPS64 * tn
    assert (np.abs(wd - wo64) <= bar).all()
    if Z is None:
        return 0.0, 0.0
    Zd = Z.astype(np.float64)
    TZ = d64[:, None] * Zd
    if n > 1:
        TZ[:-1] += e64[:, None] * Zd[1:]
        TZ[1:] += e64[:, None] * Zd[:-1]
    res = np.linalg.norm(TZ - Zd * wd[None, :], axis=0).max() / (EPS32 * tn)
    orth = np.abs(Zd.T @ Zd - np.eye(Zd.shape[1])).max() / EPS32
    return res, orth


@pytest.mark.parametrize("kind,n", [("random", 1), ("random", 2), ("random", 50), ("random", 500),
                                    ("random", 3000), ("toeplitz", 1000), ("glued", 2000), ("geometric", 1500)])
def test_fp32_interface_vs_oracle(M, kind, n):
    if kind == "random":
        d, e = W.random_uniform(n, 8100 + n)
    elif kind == "toeplitz":
        d, e = W.toeplitz(n)
    elif kind == "glued":
        d, e = W.glued_wilkinson(n, 3)
    else:
        d, e = W.geometric(n, 8200)
    d, e = f32(d, e)
    w, Z, info = M.eigh_tridiagonal_f32(d, e, return_info=True)
    assert w.dtype == torch.float32 and Z.dtype == torch.float32
    wo, Zo, st = oracle.mrrr(d.astype(np.float64), e.astype(np.float64))
    assert st == 0 and info["status"] == 0
    res, orth = check(d, e, w.cpu().numpy(), Z.cpu().numpy(), wo)
    print(f"{kind} n={n}: residual {res:.2f} eps32 ||T||, orthogonality {orth:.2f} eps32, nodes {info['nodes']}")
    assert res <= 4.0 and orth <= 4.0


def test_relaxed_threshold_shortens_the_tree(M):
    # glued Wilkinson blocks: the FP64 threshold makes clusters of the
    # blocks' near-equal eigenvalues; FP32 results need fewer of them
    d, e = f32(*W.glued_wilkinson(3000, 4))
    _, _, i64 = M.eigh_tridiagonal(d.astype(np.float64), e.astype(np.float64), return_info=True)
    w, Z, i32 = M.eigh_tridiagonal_f32(d, e, return_info=True)
    print(f"nodes: FP64 interface {i64['nodes']}, FP32 interface {i32['nodes']}; "
          f"depth {i64['max_depth']} / {i32['max_depth']}")
    assert i32["nodes"] <= i64["nodes"]
    wo, _, _ = oracle.mrrr(d.astype(np.float64), e.astype(np.float64))
    res, orth = check(d, e, w.cpu().numpy(), Z.cpu().numpy(), wo)
    assert res <= 4.0 and orth <= 4.0


def test_fp32_subsets(M):
    d, e = f32(*W.random_uniform(700, 8300))
    wo, _, _ = oracle.mrrr(d.astype(np.float64), e.astype(np.float64))
    w, Z = M.eigh_tridiagonal_f32(d, e, select="i", il=100, iu=180)
    assert w.shape[0] == 81 and Z.shape == (700, 81)
    res, orth = check(d, e, w.cpu().numpy(), Z.cpu().numpy(), wo[99:180])
    assert res <= 4.0 and orth <= 4.0
    vl, vu = float(wo[299]) + 1e-9, float(wo[350]) + 1e-9
    w, Z = M.eigh_tridiagonal_f32(d, e, select="v", vl=vl, vu=vu)
    assert w.shape[0] == 51
    res, orth = check(d, e, w.cpu().numpy(), Z.cpu().numpy(), wo[300:351])
    assert res <= 4.0 and orth <= 4.0
    w, _ = M.eigh_tridiagonal_f32(d, e, eigvals_only=True)
    check(d, e, w.cpu().numpy(), None, wo)


def test_fp32_nonfinite_input_reports(M):
    d, e = f32(*W.random_uniform(64, 8400))
    d[10] = np.nan
    with pytest.raises(Exception, match="non-finite|inf|NaN|4"):
        M.eigh_tridiagonal_f32(d, e)
    d, e = f32(*W.random_uniform(64, 8400))
    w, Z = M.eigh_tridiagonal_f32(d, e)
    assert torch.isfinite(w).all() and torch.isfinite(Z).all()
