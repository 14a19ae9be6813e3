"""The allocation-free entry point (mrrr_step_noalloc, workspace in a fixed
device array of the library) against the existing caller-workspace entry point
mrrr_step_ws, through the C ABI: two calls in a row, the second on a smaller
input, each bit-identical to mrrr_step_ws on the same input and within the
oracle's bars."""
import ctypes

import numpy as np
import pytest

import oracle
from common import eig_tol, orth_ratio, residual_ratio
from paper_1205_2107_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def call(lib, fn, d, e, work=None):
    n = d.shape[0]
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e, device="cuda")
    w = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    Z = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    info = torch.zeros(18, dtype=torch.int64, device="cuda")
    rng = lib_range()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if fn == "noalloc":
        rc = lib.mrrr_step_noalloc(n, _ptr(dt), _ptr(et), rng, _ptr(w), _ptr(Z), n, _ptr(info), stream)
    else:
        rc = lib.mrrr_step_ws(n, _ptr(dt), _ptr(et), rng, _ptr(w), _ptr(Z), n, _ptr(work),
                              work.numel(), _ptr(info), stream)
    torch.cuda.synchronize()
    return rc, w.cpu().numpy(), Z.cpu().numpy().T.copy(), info.cpu().numpy()


def lib_range():
    from paper_1205_2107_amd import _lib
    r = _lib.MrrrRange()
    r.kind = _lib.MRRR_ALL
    return r


def test_noalloc_matches_workspace_entry_point_twice():
    from paper_1205_2107_amd import _lib
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    lib = _lib.load()
    inputs = [W.glued_wilkinson(1000, 41), W.random_uniform(700, 42)]  # second call smaller
    for d, e in inputs:
        n = d.shape[0]
        print(f"noalloc call n={n}", flush=True)
        rc, w, Z, info = call(lib, "noalloc", d, e)
        assert rc == 0, lib.mrrr_last_error()
        assert info[0] == n and info[1] & 0xFFFFFFFF == 0  # m, status
        work = torch.empty(lib.mrrr_workspace_size(n, lib_range()), dtype=torch.uint8, device="cuda")
        rc2, w2, Z2, _ = call(lib, "ws", d, e, work)
        assert rc2 == 0
        assert np.array_equal(w, w2) and np.array_equal(Z, Z2)
        wo, Zo, st = oracle.mrrr(d, e)
        assert np.abs(w - wo).max() <= eig_tol(d, e)
        assert residual_ratio(d, e, w, Z) <= 10 and orth_ratio(Z) <= 10


def test_noalloc_rejects_orders_beyond_its_limit():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(256)
    rc = lib.mrrr_step_noalloc(1025, fake, fake, lib_range(), fake, fake, 1025, None, None)
    assert rc == -1
    assert b"allocation-free limit" in lib.mrrr_last_error()
