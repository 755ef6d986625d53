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
    assert f(1, arr(15), arr(1), arr(10_000_000), 0, 0, 0, ctypes.byref(plan)) == -7  # (T + 1) n^2 >= 2^31


def test_version(lib):
    lib.lq_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.lq_version()
