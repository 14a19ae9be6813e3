"""GPU tests of the boundary: the caller-workspace entry point (mrrr_step_ws)
and the status codes the tree limits force (no representation, depth limit,
workspace capacity).  Every call goes through the C ABI; results are compared
with the library-workspace entry point bit for bit and with the oracle's bars.
"""
import numpy as np
import pytest

import oracle
from common import eig_tol, orth_ratio, residual_ratio
from paper_1205_2107_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1205_2107_amd as pkg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return pkg


def solve(M, d, e, **kw):
    w, Z, info = M.eigh_tridiagonal(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda"),
                                    return_info=True, **kw)
    return w.cpu().numpy(), (None if Z is None else Z.cpu().numpy()), info


MATS = [("random700", lambda: W.random_uniform(700, 21)), ("toeplitz600", lambda: W.toeplitz(600)),
        ("glued500", lambda: W.glued_wilkinson(500, 23)), ("geometric650", lambda: W.geometric(650, 24))]


@pytest.mark.parametrize("case", MATS, ids=lambda c: c[0])
def test_caller_workspace_equals_library_workspace(M, case):
    name, gen = case
    d, e = gen()
    n = d.shape[0]
    w0, Z0, i0 = solve(M, d, e)
    work = torch.empty(M.workspace_size(n), dtype=torch.uint8, device="cuda")
    w1, Z1, i1 = solve(M, d, e, work=work)
    assert i1["status"] == 0 and i1["m"] == n
    assert np.array_equal(w0, w1) and np.array_equal(Z0, Z1)
    assert 0 < i1["workspace_bytes"] <= work.numel()
    # a subset through the same workspace
    w2, Z2, i2 = solve(M, d, e, select="i", il=n // 3, iu=n // 2, work=work)
    w3, Z3, _ = solve(M, d, e, select="i", il=n // 3, iu=n // 2)
    assert np.array_equal(w2, w3) and np.array_equal(Z2, Z3)


def test_shrinking_workspace_is_exact_or_reports_capacity(M):
    # halving the workspace: every call either returns the library-workspace
    # result bit for bit (the eigenvector phase then runs in more launches)
    # or stops with the capacity status -- never another outcome
    d, e = W.glued_wilkinson(2100, 31)
    n = d.shape[0]
    w0, Z0, _ = solve(M, d, e)
    size = M.workspace_size(n)
    ok = 0
    codes = []
    while size >= 4096:
        work = torch.empty(size, dtype=torch.uint8, device="cuda")
        try:
            w1, Z1, info = solve(M, d, e, work=work)
            assert np.array_equal(w0, w1) and np.array_equal(Z0, Z1), size
            ok += 1
        except M.MrrrError as ex:
            codes.append(ex.code)
        size //= 2
        del work
    assert ok >= 2
    assert codes and set(codes) == {3}


def test_forced_depth_status(M):
    # the 1-2-1 matrix's tree of order 20000 is a chain of 16 clusters: with
    # depth 3 allowed, the clustered eigenvalues of the deepest node are
    # computed from it as singletons and the call reports the depth status
    d, e = W.toeplitz(20000)
    old = M.get_limits()
    try:
        M.set_limits(max_depth=3)
        with pytest.raises(M.MrrrError) as ex:
            solve(M, d, e)
        assert ex.value.code == 2
    finally:
        M.set_limits(**old)
    w, Z, info = solve(M, d, e)
    assert info["status"] == 0 and info["max_depth"] > 3


def test_forced_no_representation_status(M):
    # a growth limit no candidate can meet: clusters get no child and the
    # call reports the missing representation
    d, e = W.glued_wilkinson(420, 5)
    old = M.get_limits()
    try:
        M.set_limits(child_growth_limit=1e-300)
        with pytest.raises(M.MrrrError) as ex:
            solve(M, d, e)
        assert ex.value.code == 1
    finally:
        M.set_limits(**old)
    w, Z, info = solve(M, d, e)
    wo, Zo, st = oracle.mrrr(d, e)
    assert info["status"] == 0 and np.abs(w - wo).max() <= eig_tol(d, e)
    assert residual_ratio(d, e, w, Z) <= 10 and orth_ratio(Z) <= 10
