"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/cbs.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2603_18527_amd import cbs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "cbs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:cbs|fgmres)_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("cbs_setup", "cbs_apply", "cbs_residual", "cbs_iterate", "fgmres_solve",
                     "cbs_adjoint_step", "cbs_loss_seed", "cbs_destroy", "cbs_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = cbs.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(cbs.SIGNATURES)


def test_version_string():
    assert b"gfx950" in cbs.load().cbs_version()


def _setup(batch, sizes, k2=1, dtype=cbs.CBS_C64, restart=0, flags=0, out=True):
    lib = cbs.load()
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * max(1, len(sizes)))(*sizes) if sizes is not None else None
    return lib.cbs_setup(ctypes.byref(h) if out else None, batch, n,
                         ctypes.c_void_p(k2) if k2 else None, None, None, dtype, restart, flags, None)


def test_setup_argument_errors_without_gpu():
    assert _setup(1, [64], out=False) == cbs.CBS_ERR_ARG
    assert _setup(0, [64]) == cbs.CBS_ERR_ARG
    assert _setup(1, [64], k2=0) == cbs.CBS_ERR_ARG
    assert _setup(1, [64], dtype=7) == cbs.CBS_ERR_ARG
    assert _setup(1, [64], restart=-1) == cbs.CBS_ERR_ARG
    assert _setup(1, [64], flags=8) == cbs.CBS_ERR_ARG
    assert "flag" in cbs.last_error()
    for bad in (8, 100, 2048, 0, -16):
        assert _setup(1, [bad]) == cbs.CBS_ERR_SIZE
        assert str(bad) in cbs.last_error()
    assert _setup(3, [64, 512, 96]) == cbs.CBS_ERR_SIZE


def test_calls_with_null_plan_fail_cleanly():
    lib = cbs.load()
    assert lib.cbs_apply(None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_residual(None, None, None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_iterate(None, None, None, 10, 1e-6, 10, None, None, None, 0, None) == cbs.CBS_ERR_ARG
    assert lib.fgmres_solve(None, None, None, 10, 4, 10, 1e-6, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_adjoint_step(None, None, None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_set_tile(None, 0, 16) == cbs.CBS_ERR_ARG
    lib.cbs_destroy(None)


def test_packing_offsets():
    assert cbs.offsets([16, 32, 64]) == [0, 256, 256 + 1024]
