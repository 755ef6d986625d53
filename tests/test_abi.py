"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every entry point that include/lqscan.h declares, and argument errors are
returned synchronously."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqscan.h")
LIB = os.path.join(ROOT, "paper_2409_20027_amd", "liblqscan.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lq_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2409_20027_amd import build
        build.build(force=True)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "lq_scan_solve" in names and "lq_rollout" in names and "lq_build_elements" in names
    for name in names:
        assert hasattr(lib, name), name


def test_plan_create_rejects_bad_arguments(lib):
    plan = ctypes.c_void_p()
    arr = ctypes.c_int32 * 1
    f = lib.lq_plan_create
    f.restype = ctypes.c_int
    assert f(0, arr(2), arr(1), arr(4), 0, 0, 0, ctypes.byref(plan)) == -1          # batch 0
    assert f(1, arr(2), arr(1), arr(0), 0, 0, 0, ctypes.byref(plan)) == -1          # T = 0
    assert f(1, arr(16), arr(1), arr(4), 0, 0, 0, ctypes.byref(plan)) == -7         # n too large
    assert f(1, arr(4), arr(5), arr(4), 0, 0, 0, ctypes.byref(plan)) == -7          # m too large
    assert f(1, arr(4), arr(1), arr(4), 7, 0, 0, ctypes.byref(plan)) == -1          # precision
    assert f(1, arr(4), arr(1), arr(4), 0, 0, -3, ctypes.byref(plan)) == -1         # seg_len
    # the status word (-code) | (k << 8) holds stages below 2^23: longer horizons are refused
    # (for n <= 15 this also keeps the (T + 1) n^2 stage offsets within 32 bits), and
    # T = INT32_MAX does not wrap
    assert f(1, arr(15), arr(1), arr(10_000_000), 0, 0, 0, ctypes.byref(plan)) == -7
    assert f(1, arr(1), arr(1), arr(1 << 23), 0, 0, 0, ctypes.byref(plan)) == -7
    assert f(1, arr(1), arr(1), arr(2**31 - 1), 0, 0, 0, ctypes.byref(plan)) == -7


def test_plan_create_tuned_rejects_bad_arguments(lib, tmp_path):
    """lq_plan_create_tuned: argument errors, an unreadable cache file and a
    cache entry without a segment length are refused before any device call."""
    plan = ctypes.c_void_p()
    arr = ctypes.c_int32 * 1
    f = lib.lq_plan_create_tuned
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                  ctypes.c_char_p, ctypes.c_void_p]
    assert f(0, arr(2), arr(1), arr(4), 0, None, ctypes.byref(plan)) == -1                 # batch 0
    assert f(1, arr(2), arr(1), arr(4), 7, None, ctypes.byref(plan)) == -1                 # precision
    missing = str(tmp_path / "missing.json").encode()
    assert f(1, arr(2), arr(1), arr(4), 0, missing, ctypes.byref(plan)) == -1              # unreadable
    bad = tmp_path / "bad.json"
    bad.write_text('{"n2_m1_T4_B1_fp64": {"ms": {"0": 1.0}}}')
    assert f(1, arr(2), arr(1), arr(4), 0, str(bad).encode(), ctypes.byref(plan)) == -1    # no "L"
    bad.write_text('{"n2_m1_T4_B1_fp64": {"L": "x"}}')
    assert f(1, arr(2), arr(1), arr(4), 0, str(bad).encode(), ctypes.byref(plan)) == -1    # unreadable "L"


def test_version(lib):
    lib.lq_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.lq_version()


# entry point -> number of arguments (all pointers or int32 here); each is
# called with a null plan (or null buffers) and must return LQ_ERR_ARG (-1)
# before any device work
NULL_PLAN_CALLS = {"lq_build_elements": 5, "lq_scan_solve": 7, "lq_rollout": 9, "lq_rollout_cv": 9, "lq_solve": 10,
                   "lq_solve_static": 9, "lq_adjoint": 12,
                   "lq_solve_ckpt": 12, "lq_adjoint_ckpt": 13, "nmpc_init": 5, "newton_step": 6, "nmpc_admm_update": 5, "nmpc_shift": 6,
                   "lq_plan_phase_times": 3}


@pytest.mark.parametrize("name", sorted(NULL_PLAN_CALLS))
def test_null_plan_is_an_argument_error(lib, name):
    f = getattr(lib, name)
    f.restype = ctypes.c_int
    assert f(*([None] * NULL_PLAN_CALLS[name])) == -1


def test_size_queries_of_a_null_plan(lib):
    for name in ("lq_plan_workspace_bytes", "lq_plan_elements_bytes", "nmpc_workspace_bytes", "lq_plan_static_bytes"):
        f = getattr(lib, name)
        f.restype = ctypes.c_size_t
        f.argtypes = [ctypes.c_void_p]
        assert f(None) == 0
    lib.lq_plan_checkpoint_bytes.restype = ctypes.c_size_t
    lib.lq_plan_checkpoint_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    assert lib.lq_plan_checkpoint_bytes(None, 1) == 0
    lib.lq_plan_adjoint_ckpt_workspace_bytes.restype = ctypes.c_size_t
    lib.lq_plan_adjoint_ckpt_workspace_bytes.argtypes = [ctypes.c_void_p]
    assert lib.lq_plan_adjoint_ckpt_workspace_bytes(None) == 0
    lib.lq_plan_seg_len.restype = ctypes.c_int32
    assert lib.lq_plan_seg_len(None) == 0
    lib.lq_plan_set_timing.restype = ctypes.c_int
    lib.lq_plan_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32]
    assert lib.lq_plan_set_timing(None, 1, 4) == -1


def test_selftests_reject_bad_arguments(lib):
    """Sizes outside a tile, a homogeneous block without room for its last
    row, missing buffers and an unknown precision are refused before launch."""
    inv = lib.lq_selftest_tile_inverse
    inv.restype = ctypes.c_int
    inv.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                    ctypes.c_void_p]
    fake = ctypes.c_void_p(256)   # never dereferenced: every call below fails its checks first
    assert inv(fake, fake, 0, 0, fake, None) == -1
    assert inv(fake, fake, 17, 0, fake, None) == -1
    assert inv(fake, fake, 1, 1, fake, None) == -1
    assert inv(fake, fake, 4, 0, None, None) == -1
    assert inv(None, fake, 4, 0, fake, None) == -1
    mm = lib.lq_selftest_tile_mm
    mm.restype = ctypes.c_int
    mm.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32] * 3 + [ctypes.c_void_p]
    assert mm(fake, fake, fake, fake, 0, 0, 7, None) == -1
    assert mm(None, fake, fake, fake, 0, 0, 0, None) == -1
