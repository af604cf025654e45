"""Plans whose device memory is one caller-owned workspace (cbs_setup_ws, the
Python default: a torch tensor) against plans that allocate it themselves
(cbs_setup): the same kernels on the same inputs, bitwise equal results."""
import pytest
import torch

from gpu_helpers import random_problem, say
from paper_2603_18527_amd import cbs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_workspace_plans_match_self_allocated(dtype):
    sizes = [128, 64, 192]
    probs = [random_problem(n, seed=500 + i, source="point") for i, n in enumerate(sizes)]
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    k2 = cbs.pack([p.k2 for p in probs], tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    k0 = [p.k0sq for p in probs]
    a = cbs.Plan(k2, sizes, k0sq=k0, dtype=dtype, max_restart=6, torch_workspace=True)
    b = cbs.Plan(k2, sizes, k0sq=k0, dtype=dtype, max_restart=6, torch_workspace=False)
    say(f"[workspace] dtype={dtype} bytes={a._ws.numel()}")
    assert a._ws.numel() == cbs.workspace_size(sizes, dtype, 6)
    assert a.k0sq == b.k0sq and a.eps == b.eps
    assert torch.equal(a.apply(s, s), b.apply(s, s))
    ua, ub = a.zeros(), b.zeros()
    ra = a.iterate(ua, s, max_sweeps=400, rtol=1e-6, check_every=20)
    rb = b.iterate(ub, s, max_sweeps=400, rtol=1e-6, check_every=20)
    assert ra == rb and torch.equal(ua, ub)
    ua.zero_(), ub.zero_()
    fa = a.fgmres(ua, s, restart=6, sweeps=2, max_iters=60, rtol=1e-6)
    fb = b.fgmres(ub, s, restart=6, sweeps=2, max_iters=60, rtol=1e-6)
    assert fa == fb and torch.equal(ua, ub)
    a.close()
    b.close()
    assert a._ws is None


def test_workspace_too_small_is_rejected_on_gpu():
    p = random_problem(64, seed=510, source="point")
    k2 = cbs.pack([p.k2], torch.complex64)
    need = cbs.workspace_size([64])
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    lib = cbs.load()
    import ctypes
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * 1)(64)
    st = lib.cbs_setup_ws(ctypes.byref(h), 1, n, ctypes.c_void_p(k2.data_ptr()), None, None,
                          cbs.CBS_C64, 0, 0, ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == cbs.CBS_ERR_WORKSPACE and h.value is None
