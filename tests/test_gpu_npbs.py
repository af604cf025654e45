"""GPU NPBS step with a linear Fourier layer (cbs_npbs_step) against the FP64
oracle: u <- u + F^-1(wf F r) + wloc r with r = G(V u + s) - u (Sec. 4.1,
Eq. npbs_integral; App. E, Eq. lfl).  Bars: FP64 plans 1e-12 relative,
FP32 plans 1e-5 relative (a few FP32 roundings of O(1) terms per cell)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from paper_2603_18527_amd import cbs
from gpu_helpers import elem_err, plan_for, random_problem, rel_err, say, to_list

pytestmark = pytest.mark.gpu

TDT = {cbs.CBS_C64: torch.complex64, cbs.CBS_C128: torch.complex128}
TOL = {cbs.CBS_C64: 1e-5, cbs.CBS_C128: 1e-12}


def _weights(sizes, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    wf = [scale * S.random_field_c(n, rng) for n in sizes]
    wl = [scale * S.random_field_c(n, rng) for n in sizes]
    return wf, wl


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_npbs_steps_match_oracle(dtype):
    sizes = [128, 64, 192, 32]
    probs = [random_problem(n, seed=700 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs, dtype)
    tdt = TDT[dtype]
    rng = np.random.default_rng(71)
    u0 = [S.random_field_c(n, rng) for n in sizes]
    wf, wl = _weights(sizes, 72)
    u = cbs.pack(u0, tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    plan.npbs_step(u, s, cbs.pack(wf, tdt), cbs.pack(wl, tdt), count=3)
    torch.cuda.synchronize()
    for i, (ki, ug) in enumerate(zip(to_list(k2, sizes), to_list(u, sizes))):
        x = O.as_c(u0[i])
        for _ in range(3):
            x = O.npbs_step(ki, plan.k0sq[i], plan.eps[i], x, probs[i].source, wf[i], wl[i])
        e = rel_err(ug, x)
        emax = elem_err(ug, x)
        say(f"[npbs] dtype={dtype} instance {i} n={sizes[i]}: rel err {e:.2e}, max cell err / rms {emax:.2e}")
        assert e <= TOL[dtype]
        assert emax <= 10 * TOL[dtype]


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_npbs_steps_bench_sizes_two_lanes(dtype):
    # the fused NPBS chain at the benchmark's scale: a batch of 2^21+ cells
    # with every bridged size 128..1024 and 288, so the plan runs two lanes,
    # element by element against the oracle over two steps
    sizes = [1024, 1024, 512, 384, 288, 256, 192, 128]
    assert sum(n * n for n in sizes) >= 1 << 21
    probs = [random_problem(n, seed=760 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs, dtype)
    assert plan.layout()[0] == 2
    tdt = TDT[dtype]
    rng = np.random.default_rng(761)
    u0 = [S.random_field_c(n, rng) for n in sizes]
    wf, wl = _weights(sizes, 762)
    u = cbs.pack(u0, tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    plan.npbs_step(u, s, cbs.pack(wf, tdt), cbs.pack(wl, tdt), count=2)
    torch.cuda.synchronize()
    for i, (ki, ug) in enumerate(zip(to_list(k2, sizes), to_list(u, sizes))):
        x = O.as_c(u0[i])
        for _ in range(2):
            x = O.npbs_step(ki, plan.k0sq[i], plan.eps[i], x, probs[i].source, wf[i], wl[i])
        e, emax = rel_err(ug, x), elem_err(ug, x)
        say(f"[npbs bench sizes] dtype={dtype} n={sizes[i]}: rel err {e:.2e}, max cell err / rms {emax:.2e}")
        assert e <= TOL[dtype]
        assert emax <= 10 * TOL[dtype]


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_npbs_with_gamma_is_the_cbs_sweep(dtype):
    # Sec. 4.1: M = gamma gives the CBS step
    sizes = [64, 128]
    probs = [random_problem(n, seed=720 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs, dtype)
    tdt = TDT[dtype]
    gam = [O.gamma(ki, plan.k0sq[i], plan.eps[i]) for i, ki in enumerate(to_list(k2, sizes))]
    zero = cbs.pack([np.zeros((n, n)) for n in sizes], tdt)
    rng = np.random.default_rng(73)
    u0 = cbs.pack([S.random_field_c(n, rng) for n in sizes], tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    a, b = u0.clone(), u0.clone()
    plan.npbs_step(a, s, zero, cbs.pack(gam, tdt), count=2)
    plan.sweep(b, s, count=2)
    torch.cuda.synchronize()
    assert rel_err(a.cpu(), b.cpu()) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_npbs_exact_inverse_solves_in_one_step(dtype):
    # Sec. 4.1: M = (I - G V)^{-1} recovers the solution in one step; in a
    # homogeneous lossy medium that M is Fourier-diagonal, lambda / (lambda - v)
    n, k0sq, kappa = 64, 0.7, 0.25
    rng = np.random.default_rng(74)
    src = S.random_field_c(n, rng)
    h = S.homogeneous_lossy(n, k0sq, kappa, src)
    eps = 1.5 * kappa
    tdt = TDT[dtype]
    plan = cbs.Plan(cbs.pack([h.k2], tdt), [n], k0sq=[k0sq], eps=[eps], dtype=dtype)
    xi = 2 * math.pi * np.fft.fftfreq(n)
    lam = xi[:, None] ** 2 + xi[None, :] ** 2 - k0sq - 1j * eps
    v = 1j * (kappa - eps)
    u = cbs.pack([S.random_field_c(n, rng)], tdt)
    plan.npbs_step(u, cbs.pack([src], tdt), cbs.pack([lam / (lam - v)], tdt), None)
    torch.cuda.synchronize()
    exact = np.fft.ifft2(np.fft.fft2(src) / (xi[:, None] ** 2 + xi[None, :] ** 2 - k0sq - 1j * kappa))
    e = rel_err(to_list(u, [n])[0], torch.from_numpy(exact))
    say(f"[npbs exact inverse] dtype={dtype}: rel err {e:.2e}")
    assert e <= TOL[dtype]


def test_npbs_argument_errors():
    p = random_problem(32, seed=730)
    plan, k2 = plan_for([p])
    u = plan.zeros()
    w = plan.zeros()
    lib = cbs.load()
    ptr = cbs._ptr
    assert lib.cbs_npbs_step(plan._h, ptr(u), None, None, None, 1, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_npbs_step(plan._h, ptr(u), None, ptr(u), None, 1, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_npbs_step(plan._h, ptr(u), None, ptr(w), ptr(u), 1, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_npbs_step(plan._h, ptr(u), None, ptr(w), None, 0, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_npbs_step(None, ptr(u), None, ptr(w), None, 1, None) == cbs.CBS_ERR_ARG
