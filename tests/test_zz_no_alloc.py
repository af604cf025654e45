"""cbs_apply_static (the entry point that allocates nothing: its scratch is a
fixed device array inside the library) against cbs_apply on a plan of the
same instances, k0^2 and eps: two calls in a row, the second on a smaller
batch, in FP32 and FP64.  Bar: the operator tolerance of the apply parity
tests (relative L2 and per-cell).  The two entry points run the same
transform arithmetic (a plan may tile its column launches differently, which
moves no result); FP32 results come out bitwise equal, FP64 ones to rounding
(the FP64 twiddles are evaluated on the device here, on the host for a plan).
Collected last: a failure here hides no other test."""
import numpy as np
import pytest
import torch

import synthetic as S
from paper_2603_18527_amd import cbs
from gpu_helpers import elem_err, random_problem, rel_err, say

pytestmark = pytest.mark.gpu

TOL = {cbs.CBS_C64: 1e-6, cbs.CBS_C128: 1e-13}
TDT = {cbs.CBS_C64: torch.complex64, cbs.CBS_C128: torch.complex128}
CALLS = {
    cbs.CBS_C64: ([1024, 512, 384, 288, 256, 192, 128, 64, 32, 16], [192, 64, 128]),
    cbs.CBS_C128: ([512, 384, 256, 128, 16, 32], [288, 64]),
}


def _case(sizes, dtype, seed):
    probs = [random_problem(n, seed=seed + i, cmax=1.5 + 0.25 * i, ppw=6.0 + (i % 5))
             for i, n in enumerate(sizes)]
    rng = np.random.default_rng(seed)
    tdt = TDT[dtype]
    k2 = cbs.pack([p.k2 for p in probs], tdt)
    u = cbs.pack([S.random_field_c(p.n, rng) for p in probs], tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    return probs, k2, u, s


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_static_apply_matches_plan_apply(dtype):
    for call, sizes in enumerate(CALLS[dtype]):
        cells = sum(n * n for n in sizes)
        assert cells * (8 if dtype == cbs.CBS_C64 else 16) <= cbs.STATIC_MAX_BYTES
        say(f"[apply_static] dtype={dtype} call {call}: sizes={sizes} ({cells} cells)")
        probs, k2, u, s = _case(sizes, dtype, 7100 + 100 * call + 10 * dtype)
        plan = cbs.Plan(k2, sizes, k0sq=[p.k0sq for p in probs], dtype=dtype)
        ref = plan.apply(u, s)
        ref_s = plan.apply(None, s)
        y = cbs.apply_static(k2, sizes, plan.k0sq, plan.eps, u, s)
        y_s = cbs.apply_static(k2, sizes, plan.k0sq, plan.eps, None, s)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(cbs.unpack(y, sizes), cbs.unpack(ref, sizes))):
            err, emax = rel_err(a, b), elem_err(a, b)
            say(f"   n={sizes[i]}: rel err {err:.2e}, max cell err / rms {emax:.2e}, "
                f"bitwise equal {bool(torch.equal(a, b))}")
            assert err <= TOL[dtype] and emax <= 10 * TOL[dtype]
        assert rel_err(y_s, ref_s) <= TOL[dtype]
        plan.close()


def test_static_apply_rejects_oversize_and_bad_arguments():
    # more cells than the fixed scratch holds: an error, nothing launched
    big = [1024] * 3
    k2 = torch.ones(sum(n * n for n in big), dtype=torch.complex64, device="cuda")
    with pytest.raises(cbs.CbsError) as e:
        cbs.apply_static(k2, big, [1.0] * 3, [1.0] * 3, None, k2)
    assert e.value.status == cbs.CBS_ERR_WORKSPACE
    small = [64]
    k2 = torch.ones(64 * 64, dtype=torch.complex64, device="cuda")
    with pytest.raises(cbs.CbsError) as e:
        cbs.apply_static(k2, small, [1.0], [0.0], None, k2)
    assert e.value.status == cbs.CBS_ERR_ARG
