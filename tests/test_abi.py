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
    assert _setup(1, [64], flags=16) == cbs.CBS_ERR_ARG
    assert "flag" in cbs.last_error()
    # undamped needs the Dirichlet reference, and takes no eps
    assert _setup(1, [64], flags=cbs.FLAG_UNDAMPED) == cbs.CBS_ERR_ARG
    assert "DIRICHLET" in cbs.last_error()
    assert _setup(1, [65], flags=cbs.FLAG_UNDAMPED | cbs.FLAG_DIRICHLET) == cbs.CBS_ERR_SIZE
    # Dirichlet sizes: 2(n+1) an FFT size, or n = 64 (direct DST-I); host-only size query
    out = ctypes.c_size_t()
    lib0 = cbs.load()
    for n_ok in (7, 63, 64, 511):
        n1 = (ctypes.c_int32 * 1)(n_ok)
        assert lib0.cbs_workspace_size(1, n1, cbs.CBS_C64, 0, cbs.FLAG_DIRICHLET, ctypes.byref(out)) == cbs.CBS_OK
    for n_bad in (8, 62, 65, 512):
        n1 = (ctypes.c_int32 * 1)(n_bad)
        assert lib0.cbs_workspace_size(1, n1, cbs.CBS_C64, 0, cbs.FLAG_DIRICHLET,
                                       ctypes.byref(out)) == cbs.CBS_ERR_SIZE
    lib = cbs.load()
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * 1)(63)
    eps = (ctypes.c_double * 1)(1.0)
    assert lib.cbs_setup(ctypes.byref(h), 1, n, ctypes.c_void_p(1), None, eps, cbs.CBS_C64, 0,
                         cbs.FLAG_UNDAMPED | cbs.FLAG_DIRICHLET, None) == cbs.CBS_ERR_ARG
    assert "eps" in cbs.last_error()
    for bad in (8, 100, 2048, 0, -16):
        assert _setup(1, [bad]) == cbs.CBS_ERR_SIZE
        assert str(bad) in cbs.last_error()
    assert _setup(3, [64, 512, 96]) == cbs.CBS_ERR_SIZE


def test_calls_with_null_plan_fail_cleanly():
    lib = cbs.load()
    assert lib.cbs_apply(None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_residual(None, None, None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_iterate(None, None, None, 10, 1e-6, 10, 0, None, None, None, 0, None) == cbs.CBS_ERR_ARG
    assert lib.fgmres_solve(None, None, None, 10, 4, 10, 1e-6, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_adjoint_step(None, None, None, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_set_tile(None, 0, 16) == cbs.CBS_ERR_ARG
    assert lib.cbs_iterate_async(None, None, None, 10, 1e-6, 10, 0, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.fgmres_solve_async(None, None, None, 10, 4, 10, 1e-6, None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_relres(None, None, None, 0, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_metric_matched_grad(None, None, None, None, None, None, None) == cbs.CBS_ERR_ARG
    lib.cbs_destroy(None)


def test_packing_offsets():
    assert cbs.offsets([16, 32, 64]) == [0, 256, 256 + 1024]


def test_workspace_size_without_gpu():
    small = cbs.workspace_size([64])
    assert small > 0 and small % 256 == 0
    assert cbs.workspace_size([64], cbs.CBS_C64, 0) == small
    assert cbs.workspace_size([64], cbs.CBS_C64, 10) > small        # FGMRES bases
    assert cbs.workspace_size([64], cbs.CBS_C128) > small           # complex128 fields
    assert cbs.workspace_size([64, 128]) > cbs.workspace_size([128])
    # at least the packed fields the plan keeps: 4 FP64 copies + 2 FP32 + 3 operator fields
    cells = 128 * 128 + 192 * 192
    assert cbs.workspace_size([128, 192]) >= cells * (4 * 16 + 2 * 8 + 3 * 8)
    lib = cbs.load()
    out = ctypes.c_size_t()
    n = (ctypes.c_int32 * 1)(100)
    assert lib.cbs_workspace_size(1, n, cbs.CBS_C64, 0, 0, ctypes.byref(out)) == cbs.CBS_ERR_SIZE
    n = (ctypes.c_int32 * 1)(64)
    assert lib.cbs_workspace_size(0, n, cbs.CBS_C64, 0, 0, ctypes.byref(out)) == cbs.CBS_ERR_ARG
    assert lib.cbs_workspace_size(1, n, 5, 0, 0, ctypes.byref(out)) == cbs.CBS_ERR_ARG
    assert lib.cbs_workspace_size(1, n, cbs.CBS_C64, -1, 0, ctypes.byref(out)) == cbs.CBS_ERR_ARG
    assert lib.cbs_workspace_size(1, n, cbs.CBS_C64, 0, 0, None) == cbs.CBS_ERR_ARG


def test_setup_ws_rejects_bad_workspace_without_gpu():
    # every check below fails before the library touches the device
    lib = cbs.load()
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * 1)(64)
    need = cbs.workspace_size([64])
    fake_k2 = ctypes.c_void_p(1 << 20)

    def setup(ws, nbytes):
        return lib.cbs_setup_ws(ctypes.byref(h), 1, n, fake_k2, None, None, cbs.CBS_C64, 0, 0,
                                ws, nbytes, None)
    assert setup(None, need) == cbs.CBS_ERR_ARG
    assert setup(ctypes.c_void_p((1 << 20) + 8), need) == cbs.CBS_ERR_WORKSPACE
    assert "aligned" in cbs.last_error()
    assert setup(ctypes.c_void_p(1 << 20), need - 256) == cbs.CBS_ERR_WORKSPACE
    assert "need" in cbs.last_error()
    assert h.value is None


def test_setup_cdr_argument_errors_without_gpu():
    # every check below fails before the library touches the device
    lib = cbs.load()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)

    def setup(sizes, bg, ks=fake, vel=fake, out=True, dtype=cbs.CBS_C64):
        n = (ctypes.c_int32 * max(1, len(sizes)))(*sizes)
        b = None if bg is None else (ctypes.c_double * len(bg))(*bg)
        return lib.cbs_setup_cdr(ctypes.byref(h) if out else None, len(sizes), n, ks, vel, b, dtype, None)

    good = [1.0, 0.3, -0.2, 0.5]
    assert setup([64], good, out=False) == cbs.CBS_ERR_ARG
    assert setup([64], good, ks=None) == cbs.CBS_ERR_ARG
    assert setup([64], good, vel=None) == cbs.CBS_ERR_ARG
    assert setup([64], None) == cbs.CBS_ERR_ARG
    assert setup([], good) == cbs.CBS_ERR_ARG
    assert setup([64], good, dtype=3) == cbs.CBS_ERR_ARG
    assert setup([100], good) == cbs.CBS_ERR_SIZE
    assert setup([64], [1.0, float("inf"), 0.0, 0.5]) == cbs.CBS_ERR_ARG
    # sigma0 = 0: L0 vanishes at xi = 0
    assert setup([64], [1.0, 0.3, -0.2, 0.0]) == cbs.CBS_ERR_ILLCOND
    # kappa0 |xi|^2 + sigma0 = 0 on the bin xi = (2 pi / 64, 0) with v0 . xi = 0 there
    a = 2 * 3.141592653589793 / 64
    assert setup([64], [1.0, 0.0, 0.7, -a * a]) == cbs.CBS_ERR_ILLCOND
    assert "vanishes" in cbs.last_error()
    assert setup([64, 32], good + [1.0, 0.0, 0.0, 0.0]) == cbs.CBS_ERR_ILLCOND
    assert "instance 1" in cbs.last_error()
    assert h.value is None
    assert lib.cbs_born_adjoint(None, fake, fake, None) == cbs.CBS_ERR_ARG


def test_workspace_covers_partial_dirichlet_column_tiles():
    # Dirichlet sizes are odd, so an instance of n columns has ceil(n / c)
    # column tiles.  At the narrowest compiled width (2) 32 instances of
    # n = 255 need 32 * 128 work items per list; cbs_workspace_size checks
    # every list it sizes against the tiles of every compiled width and
    # fails with CBS_ERR_WORKSPACE if one would not fit.
    for n in (143, 191, 255, 95, 7):
        sizes = [n] * 32
        ws = cbs.workspace_size(sizes, dirichlet=True)
        assert ws > 0 and ws % 256 == 0
        assert cbs.workspace_size(sizes + [n], dirichlet=True) > ws
    # the lists of a ragged Dirichlet batch fit too
    assert cbs.workspace_size([7, 255, 143, 191, 511, 63], dirichlet=True) > 0


def test_plan_layout_null_plan():
    lib = cbs.load()
    assert lib.cbs_plan_layout(None, None, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_set_col_threads(None, 512) == cbs.CBS_ERR_ARG


def test_apply_static_argument_errors_without_gpu():
    # every argument check of cbs_apply_static runs before the device is touched
    lib = cbs.load()
    fake = ctypes.c_void_p(0x1000)
    one = (ctypes.c_double * 17)(*([1.0] * 17))
    zero = (ctypes.c_double * 1)(0.0)

    def call(batch, sizes, k0=one, eps=one, dtype=cbs.CBS_C64, k2=fake, y=ctypes.c_void_p(0x2000), u=None):
        n = (ctypes.c_int32 * max(1, len(sizes)))(*sizes)
        return lib.cbs_apply_static(batch, n, k2, k0, eps, dtype, u, None, y, None)

    assert call(0, [64]) == cbs.CBS_ERR_ARG
    assert call(cbs.STATIC_MAX_BATCH + 1, [64] * 17) == cbs.CBS_ERR_ARG
    assert call(1, [64], k2=None) == cbs.CBS_ERR_ARG
    assert call(1, [64], y=None) == cbs.CBS_ERR_ARG
    assert call(1, [64], y=fake, u=fake) == cbs.CBS_ERR_ARG
    assert call(1, [64], dtype=5) == cbs.CBS_ERR_ARG
    assert call(1, [64], eps=zero) == cbs.CBS_ERR_ARG
    assert call(1, [100]) == cbs.CBS_ERR_SIZE
    # the spectral buffer holds 2^21 complex64 / 2^20 complex128 cells
    assert call(3, [1024] * 3) == cbs.CBS_ERR_WORKSPACE
    assert call(2, [1024, 16], dtype=cbs.CBS_C128) == cbs.CBS_ERR_WORKSPACE
    assert "scratch" in cbs.last_error()


def test_cdr_workspace_without_gpu():
    # the CDR plan's workspace holds one more operator-precision field (the
    # velocity) than a Helmholtz plan's, and no FGMRES bases
    ws = cbs.workspace_size_cdr([64, 128])
    assert ws > 0 and ws % 256 == 0
    assert ws > cbs.workspace_size([64, 128])
    assert cbs.workspace_size_cdr([64, 128], cbs.CBS_C128) > ws
    lib = cbs.load()
    out = ctypes.c_size_t()
    assert lib.cbs_workspace_size_cdr(1, (ctypes.c_int32 * 1)(100), cbs.CBS_C64, ctypes.byref(out)) == \
        cbs.CBS_ERR_SIZE
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * 1)(64)
    fake = ctypes.c_void_p(1 << 20)
    bg = (ctypes.c_double * 4)(1.0, 0.1, 0.1, 0.5)
    need = cbs.workspace_size_cdr([64])
    assert lib.cbs_setup_cdr_ws(ctypes.byref(h), 1, n, fake, fake, bg, cbs.CBS_C64, None, need, None) == \
        cbs.CBS_ERR_ARG
    assert lib.cbs_setup_cdr_ws(ctypes.byref(h), 1, n, fake, fake, bg, cbs.CBS_C64, fake, need - 256, None) == \
        cbs.CBS_ERR_WORKSPACE
    assert h.value is None
