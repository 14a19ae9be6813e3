"""The C-ABI library loads on the CPU host and exports every entry point that
include/mrrr.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mrrr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mrrr_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mrrr_step", "mrrr_step_batched", "mrrr_step_backward", "mrrr_step_backward_batched",
                     "mrrr_status_string", "mrrr_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1205_2107_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmrrr.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) <= set(declared_functions())


def test_host_side_argument_checks():
    """negative return codes are decided on the host before any device work"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    r = _lib.MrrrRange()
    r.kind = _lib.MRRR_ALL
    assert lib.mrrr_step(-1, None, None, r, None, None, 1, None, None) == -1
    assert lib.mrrr_step(5, None, None, r, None, None, 5, None, None) == -2
    r.kind = 7
    fake = ctypes.c_void_p(16)
    assert lib.mrrr_step(5, fake, fake, r, fake, None, 5, None, None) == -4
    r.kind = _lib.MRRR_INDEX
    r.il, r.iu = 3, 2
    assert lib.mrrr_step(5, fake, fake, r, fake, None, 5, None, None) == -4
    r.kind = _lib.MRRR_ALL
    assert lib.mrrr_step(5, fake, fake, r, fake, fake, 4, None, None) == -7
    assert lib.mrrr_step(0, None, None, r, None, None, 1, None, None) == 0
    assert lib.mrrr_status_string(4).decode() == "non-finite entry in d or e"
    assert lib.mrrr_step_backward(-1, None, None, 1, None, None, 1, None, None, None) == -1


def test_batched_host_side_argument_checks():
    """the batched entry point rejects bad sizes and offsets on the host, before
    any device work, and leaves a message for the calling thread"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    I64 = ctypes.c_int64
    ns = (I64 * 3)(4, 0, 5)
    off = (I64 * 3)(0, 4, 4)
    assert lib.mrrr_step_batched(-1, None, None, None, None, None, None, None, None, None) == -1
    assert lib.mrrr_step_batched(0, None, None, None, None, None, None, None, None, None) == 0
    assert lib.mrrr_step_batched(3, None, off, fake, fake, fake, None, None, None, None) == -2
    assert lib.mrrr_step_batched(3, ns, None, fake, fake, fake, None, None, None, None) == -3
    assert lib.mrrr_step_batched(3, ns, off, None, fake, fake, None, None, None, None) == -4
    assert lib.mrrr_step_batched(3, ns, off, fake, fake, None, None, None, None, None) == -6
    assert lib.mrrr_step_batched(3, ns, off, fake, fake, fake, fake, None, None, None) == -8
    assert lib.mrrr_step_batched(3, ns, off, fake, fake, fake, None, None, None, None) == -2
    assert b"n_host[1]" in lib.mrrr_last_error()
    ns[1] = 2
    off[2] = -6
    assert lib.mrrr_step_batched(3, ns, off, fake, fake, fake, None, None, None, None) == -3
    assert b"off_host[2]" in lib.mrrr_last_error()


def test_tuning_roundtrip():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    t = _lib.MrrrTuning()
    assert lib.mrrr_get_tuning(ctypes.byref(t)) == 0
    old = t.grid_density
    t.grid_density = 99
    assert lib.mrrr_set_tuning(ctypes.byref(t)) == -1
    t.grid_density = old
    assert lib.mrrr_set_tuning(ctypes.byref(t)) == 0
    for bad in (-2, (1 << 30) + 1):
        t.vec_ckpt_min_run = bad
        assert lib.mrrr_set_tuning(ctypes.byref(t)) == -1
    for ok in (-1, 1, 0):
        t.vec_ckpt_min_run = ok
        assert lib.mrrr_set_tuning(ctypes.byref(t)) == 0
    for bad in (-1, 1, 63, (1 << 30) + 1):
        t.vec_ckpt_min_n = bad
        assert lib.mrrr_set_tuning(ctypes.byref(t)) == -1
    for ok in (64, 4096, 0):
        t.vec_ckpt_min_n = ok
        assert lib.mrrr_set_tuning(ctypes.byref(t)) == 0


def test_workspace_size_is_host_only_and_monotone():
    """mrrr_workspace_size needs no device: 0 for invalid arguments, growing
    with the order, smaller for a narrow index range than for all pairs"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    r = _lib.MrrrRange()
    r.kind = _lib.MRRR_ALL
    assert lib.mrrr_workspace_size(-1, r) == 0
    sizes = [lib.mrrr_workspace_size(n, r) for n in (1, 10, 100, 1000, 20000)]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] < 64 << 30
    r.kind = _lib.MRRR_INDEX
    r.il, r.iu = 5, 4
    assert lib.mrrr_workspace_size(100, r) == 0
    r.il, r.iu = 1, 10
    sub = lib.mrrr_workspace_size(20000, r)
    assert 0 < sub < sizes[-1]
    r.kind = 9
    assert lib.mrrr_workspace_size(10, r) == 0


def test_workspace_entry_point_argument_checks():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    r = _lib.MrrrRange()
    r.kind = _lib.MRRR_ALL
    fake = ctypes.c_void_p(256)
    assert lib.mrrr_step_ws(-1, None, None, r, None, None, 1, None, 0, None, None) == -1
    assert lib.mrrr_step_ws(5, fake, fake, r, fake, fake, 4, fake, 1 << 20, None, None) == -7
    assert lib.mrrr_step_ws(5, fake, fake, r, fake, fake, 5, fake, 16, None, None) == -9
    assert lib.mrrr_step_ws(0, None, None, r, None, None, 1, fake, 1 << 20, None, None) == 0


def test_limits_round_trip_and_validation():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    old = _lib.MrrrLimits()
    assert lib.mrrr_get_limits(ctypes.byref(old)) == 0
    assert old.max_depth == 64 and old.child_growth_limit == 0.0
    bad = _lib.MrrrLimits()
    for md, gl in [(0, 0.0), (65, 0.0), (10, -1.0), (10, float("nan")), (10, float("inf"))]:
        bad.max_depth, bad.child_growth_limit = md, gl
        assert lib.mrrr_set_limits(ctypes.byref(bad)) == -1
    new = _lib.MrrrLimits()
    new.max_depth, new.child_growth_limit = 3, 1.5
    try:
        assert lib.mrrr_set_limits(ctypes.byref(new)) == 0
        got = _lib.MrrrLimits()
        lib.mrrr_get_limits(ctypes.byref(got))
        assert got.max_depth == 3 and got.child_growth_limit == 1.5
    finally:
        lib.mrrr_set_limits(ctypes.byref(old))


def test_division_probe_argument_checks():
    """the arithmetic probe rejects bad sizes and null operands on the host"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    assert lib.mrrr_probe_division(-1, None, None, None, None) == -1
    assert lib.mrrr_probe_division((1 << 31) + 1, None, None, None, None) == -1
    assert lib.mrrr_probe_division(4, None, None, None, None) == -2
    assert lib.mrrr_probe_division(0, None, None, None, None) == 0


def test_backtransform_argument_checks():
    """the back-transformation rejects bad sizes, pointers and leading
    dimensions on the host; trivial sizes return at once"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    assert lib.mrrr_backtransform(-1, 1, fake, 1, fake, fake, 1, None) == -1
    assert lib.mrrr_backtransform(4, -1, fake, 4, fake, fake, 4, None) == -2
    assert lib.mrrr_backtransform(4, 2, None, 4, fake, fake, 4, None) == -3
    assert lib.mrrr_backtransform(4, 2, fake, 3, fake, fake, 4, None) == -4
    assert lib.mrrr_backtransform(4, 2, fake, 4, None, fake, 4, None) == -5
    assert lib.mrrr_backtransform(4, 2, fake, 4, fake, None, 4, None) == -6
    assert lib.mrrr_backtransform(4, 2, fake, 4, fake, fake, 3, None) == -7
    assert lib.mrrr_backtransform(1, 5, None, 1, None, fake, 1, None) == 0
    assert lib.mrrr_backtransform(6, 0, fake, 6, fake, None, 6, None) == 0


def test_tridiagonalize_argument_checks():
    """the reduction rejects bad sizes, pointers and leading dimensions on the
    host; n = 0 returns at once"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    assert lib.mrrr_tridiagonalize(-1, fake, 1, fake, fake, fake, None) == -1
    assert lib.mrrr_tridiagonalize((1 << 18) + 1, fake, (1 << 18) + 1, fake, fake, fake, None) == -1
    assert lib.mrrr_tridiagonalize(4, None, 4, fake, fake, fake, None) == -2
    assert lib.mrrr_tridiagonalize(4, fake, 3, fake, fake, fake, None) == -3
    assert lib.mrrr_tridiagonalize(4, fake, 4, None, fake, fake, None) == -4
    assert lib.mrrr_tridiagonalize(4, fake, 4, fake, None, fake, None) == -5
    assert lib.mrrr_tridiagonalize(4, fake, 4, fake, fake, None, None) == -6
    assert lib.mrrr_tridiagonalize(0, None, 1, None, None, None, None) == 0


def test_generalized_stage_argument_checks():
    """Cholesky, reduction to standard form and the L^T solve reject bad
    sizes, pointers and leading dimensions on the host"""
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    info = ctypes.c_int64(7)
    assert lib.mrrr_cholesky(-1, fake, 1, ctypes.byref(info), None) == -1
    assert lib.mrrr_cholesky(4, None, 4, ctypes.byref(info), None) == -2
    assert lib.mrrr_cholesky(4, fake, 3, ctypes.byref(info), None) == -3
    assert lib.mrrr_cholesky(4, fake, 4, None, None) == -4
    assert lib.mrrr_cholesky(0, None, 1, ctypes.byref(info), None) == 0 and info.value == 0
    assert lib.mrrr_sygst(-1, fake, 1, fake, 1, None) == -1
    assert lib.mrrr_sygst(4, None, 4, fake, 4, None) == -2
    assert lib.mrrr_sygst(4, fake, 3, fake, 4, None) == -3
    assert lib.mrrr_sygst(4, fake, 4, None, 4, None) == -4
    assert lib.mrrr_sygst(4, fake, 4, fake, 3, None) == -5
    assert lib.mrrr_sygst(0, None, 1, None, 1, None) == 0
    assert lib.mrrr_trsm_lt(-1, 1, fake, 1, fake, 1, None) == -1
    assert lib.mrrr_trsm_lt(4, -1, fake, 4, fake, 4, None) == -2
    assert lib.mrrr_trsm_lt(4, 2, None, 4, fake, 4, None) == -3
    assert lib.mrrr_trsm_lt(4, 2, fake, 3, fake, 4, None) == -4
    assert lib.mrrr_trsm_lt(4, 2, fake, 4, None, 4, None) == -5
    assert lib.mrrr_trsm_lt(4, 2, fake, 4, fake, 3, None) == -6
    assert lib.mrrr_trsm_lt(4, 0, fake, 4, None, 4, None) == 0


def test_binding_helpers_are_not_shadowed():
    """every module-level name of the binding is defined once (a later
    definition would silently replace an earlier helper)"""
    import ast
    src = open(os.path.join(ROOT, "paper_1205_2107_amd", "__init__.py")).read()
    names = [n.name for n in ast.parse(src).body if isinstance(n, (ast.FunctionDef, ast.ClassDef))]
    dup = sorted({x for x in names if names.count(x) > 1})
    assert not dup, dup


def test_dense_driver_argument_checks():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    bad = ctypes.c_int64(3)
    assert lib.mrrr_syev(-1, fake, 1, fake, fake, 1, None, None) == -1
    assert lib.mrrr_syev(4, None, 4, fake, fake, 4, None, None) == -2
    assert lib.mrrr_syev(4, fake, 3, fake, fake, 4, None, None) == -3
    assert lib.mrrr_syev(4, fake, 4, None, fake, 4, None, None) == -4
    assert lib.mrrr_syev(4, fake, 4, fake, None, 4, None, None) == -5
    assert lib.mrrr_syev(4, fake, 4, fake, fake, 3, None, None) == -6
    assert lib.mrrr_syev(0, None, 1, None, None, 1, None, None) == 0
    assert lib.mrrr_sygv(4, fake, 4, None, 4, fake, fake, 4, ctypes.byref(bad), None, None) == -4
    assert lib.mrrr_sygv(4, fake, 4, fake, 3, fake, fake, 4, ctypes.byref(bad), None, None) == -5
    assert lib.mrrr_sygv(4, fake, 4, fake, 4, fake, fake, 4, None, None, None) == -9
    assert lib.mrrr_sygv(0, None, 1, None, 1, None, None, 1, ctypes.byref(bad), None, None) == 0 and bad.value == 0


def test_subset_driver_argument_checks():
    from paper_1205_2107_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    bad = ctypes.c_int64(0)
    rng = _lib.MrrrRange()
    rng.kind = 7
    assert lib.mrrr_syevr(4, fake, 4, rng, fake, fake, 4, None, None) == -4
    rng.kind = _lib.MRRR_ALL
    assert lib.mrrr_syevr(4, fake, 4, rng, None, fake, 4, None, None) == -5
    assert lib.mrrr_syevr(4, fake, 4, rng, fake, fake, 3, None, None) == -7
    rng.kind = 9
    assert lib.mrrr_sygvr(4, fake, 4, fake, 4, rng, fake, fake, 4, ctypes.byref(bad), None, None) == -6
    rng.kind = _lib.MRRR_ALL
    assert lib.mrrr_sygvr(4, fake, 4, fake, 4, rng, fake, fake, 4, None, None, None) == -10
