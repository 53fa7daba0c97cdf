"""The C-ABI library without a GPU: it loads, exports every function that
include/foa.h declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "foa.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(foa_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def F():
    from paper_1805_05821_amd import foa

    return foa


def test_header_declares_the_calls():
    names = _declared()
    for must in ("foa_init", "foa_push_snapshot", "foa_truncate", "foa_modes", "foa_indicators",
                 "foa_batch_init", "foa_batch_push"):
        assert must in names


def test_library_exports_every_declared_symbol(F):
    lib = ctypes.CDLL(F.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(F.EXPORTED) == sorted(_declared())


def test_workspace_bytes(F):
    a = F.foa_workspace_bytes(1000, 50, F.FOA_PREC_F64)
    b = F.foa_workspace_bytes(1000, 50, F.FOA_PREC_F32)
    c = F.foa_workspace_bytes(100000, 50, F.FOA_PREC_F32)
    d = F.foa_workspace_bytes(100000, 50, F.FOA_PREC_F64)
    assert a > 0 and b > 0
    # V alone: ceil(n/64)*64 rows x n_max columns; only V and the FP64 row
    # vector grow with n
    assert c >= 100032 * 50 * 4
    assert c - b >= (100032 - 1024) * (50 * 4 + 8)
    assert d - c >= (100032 * 50 * 4) - (b - a) - 1024 * 50 * 4
    assert d > c
    assert a % 256 == 0 and b % 256 == 0


@pytest.mark.parametrize("args", [(0, 10, 0), (10, 0, 0), (10, 513, 0), (10, 10, 7), (-5, 10, 1)])
def test_workspace_bytes_rejects(F, args):
    out = ctypes.c_size_t()
    assert F.lib.foa_workspace_bytes(*args, ctypes.byref(out)) == F.FOA_E_ARG
    assert F.lib.foa_workspace_bytes(10, 10, 0, None) == F.FOA_E_ARG


def test_init_rejects_before_device(F):
    ctx = ctypes.c_void_p()
    good = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    L = F.lib
    assert L.foa_init(None, 10, 10, 0, good, 1 << 30, None, -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 0, 10, 0, good, 1 << 30, None, -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 600, 0, good, 1 << 30, None, -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 10, 3, good, 1 << 30, None, -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 10, 0, None, 1 << 30, None, -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 10, 0, ctypes.c_void_p((1 << 20) + 8), 1 << 30, None,
                      -1.0) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 10, 0, good, 1 << 30, None, float("nan")) == F.FOA_E_ARG
    assert L.foa_init(ctypes.byref(ctx), 10, 10, 0, good, 16, None, -1.0) == F.FOA_E_NOMEM
    assert ctx.value is None


def test_null_context_calls(F):
    L = F.lib
    assert L.foa_push_snapshot(None, None, 0) == F.FOA_E_ARG
    assert L.foa_sync(None, None) == F.FOA_E_ARG
    assert L.foa_get_state(None, None, None, 1, None, None) == F.FOA_E_ARG
    assert L.foa_truncate(None, -1.0, 0, None, None) == F.FOA_E_ARG
    assert L.foa_modes(None, 1, None, None, None, None, None, 0, 0, 0, None) == F.FOA_E_ARG
    assert L.foa_indicators(None, 1, None, None, None) == F.FOA_E_ARG
    assert L.foa_destroy(None) == F.FOA_E_ARG
    assert L.foa_set_option(None, b"grid", 1) == F.FOA_E_ARG
    assert L.foa_batch_push(None, None, 0) == F.FOA_E_ARG
    assert L.foa_batch_destroy(None) == F.FOA_E_ARG


def test_status_strings(F):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8):
        assert F.status_str(code) not in ("", "unknown status")
    assert F.status_str(99) == "unknown status"
