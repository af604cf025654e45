"""Shared helpers of the GPU tests: build plans from synthetic problems and
evaluate results with the FP64 oracle."""
import math
import sys

import numpy as np
import torch

import oracle as O
import synthetic as S
from paper_2603_18527_amd import cbs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def plan_for(problems, dtype=cbs.CBS_C64, restart=0, eps=None, guard=True):
    sizes = [p.n for p in problems]
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    k2 = cbs.pack([p.k2 for p in problems], tdt)
    plan = cbs.Plan(k2, sizes, k0sq=[p.k0sq for p in problems], eps=eps, dtype=dtype,
                    max_restart=restart, guard=guard)
    return plan, k2


def fields(problems, attr="source", dtype=torch.complex64):
    return cbs.pack([getattr(p, attr) for p in problems], dtype)


def to_list(t, sizes):
    return [x.cpu().to(torch.complex128) for x in cbs.unpack(t, sizes)]


def rel_err(a, b):
    a = torch.as_tensor(a).to(torch.complex128)
    b = torch.as_tensor(b).to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def elem_err(a, b):
    """Largest per-cell error relative to the field's RMS: max|a - b| / rms(b).
    Beside the relative L2 error this catches a few wrong cells in a large
    field (one cell off by 0.5 % of the RMS at 512^2 moves the L2 error by
    only 1e-5)."""
    a = torch.as_tensor(a).to(torch.complex128)
    b = torch.as_tensor(b).to(torch.complex128)
    rms = float(torch.linalg.vector_norm(b)) / math.sqrt(b.numel())
    return float(torch.max(torch.abs(a - b))) / rms


def peak_err(a, b):
    """Largest per-cell error relative to the field's peak: max|a - b| / max|b|
    (the bar for fields whose peak sits far above their RMS, where rounding
    errors follow the local magnitude)."""
    a = torch.as_tensor(a).to(torch.complex128)
    b = torch.as_tensor(b).to(torch.complex128)
    return float(torch.max(torch.abs(a - b))) / float(torch.max(torch.abs(b)))


def random_problem(n, seed, layer=None, cmax=2.5, ppw=8.0, source="random"):
    rng = np.random.default_rng(seed)
    layer = max(1, n // 8) if layer is None else layer
    c = S.minmax_map(S.gaussian_random_field(n, max(2.0, n / 16), rng), 1.0, cmax)
    if source == "random":
        src = S.random_field_c(n, rng)
    else:
        at = rng.integers(layer, n - layer, size=2)
        src = S.point_source(n, at)
    return S.velocity_problem(c, layer, ppw, src, cmin=1.0)
