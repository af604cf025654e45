"""Two-lane execution (sweep chains of a large batch split over two plan-owned
streams) against single-stream execution of the same plan: the kernels and the
per-instance reduction order are the same, so every result is bitwise equal."""
import numpy as np
import pytest
import torch

from gpu_helpers import random_problem, say
from paper_2603_18527_amd import cbs

pytestmark = pytest.mark.gpu

# 2,133,952 cells: above the 2^21-cell threshold at which a plan splits into lanes.
SIZES = [512, 128, 384, 256, 512, 192, 512, 256, 384, 512, 256, 512, 128, 512]
CMAX = [1.5, 2.0, 3.0, 2.5, 4.0, 1.8, 2.2, 3.5, 1.6, 2.8, 3.0, 1.7, 2.4, 3.2]


def _problems():
    assert sum(n * n for n in SIZES) >= 1 << 21
    return [random_problem(n, seed=400 + i, source="point", cmax=CMAX[i], ppw=6.0 + (i % 5))
            for i, n in enumerate(SIZES)]


@pytest.fixture(scope="module")
def plans():
    probs = _problems()
    k2 = cbs.pack([p.k2 for p in probs], torch.complex64)
    k0 = [p.k0sq for p in probs]
    lanes = cbs.Plan(k2, SIZES, k0sq=k0, max_restart=10)
    single = cbs.Plan(k2, SIZES, k0sq=k0, max_restart=10, lanes=False)
    for pl in (lanes, single):
        pl.set_tile(8, n=512)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    yield lanes, single, s
    lanes.close()
    single.close()


def test_sweep_chain_lanes_bitwise(plans):
    lanes, single, _ = plans
    g = torch.Generator(device="cpu").manual_seed(7)
    cells = sum(n * n for n in SIZES)
    u0 = torch.complex(torch.randn(cells, generator=g), torch.randn(cells, generator=g))
    s = torch.complex(torch.randn(cells, generator=g), torch.randn(cells, generator=g))
    u0, s = u0.to(torch.complex64).cuda(), s.to(torch.complex64).cuda()
    for count in (1, 2, 7):
        say(f"[lanes sweep] count={count}")
        ua, ub = u0.clone(), u0.clone()
        na = lanes.sweep(ua, s, count=count, norms=True)
        nb = single.sweep(ub, s, count=count, norms=True)
        torch.cuda.synchronize()
        assert torch.equal(ua, ub)
        assert torch.equal(na, nb)


@pytest.mark.parametrize("use_graph,stop", [(True, "born"), (False, "born"), (True, "physical")])
def test_iterate_lanes_bitwise(plans, use_graph, stop):
    # Instances converge at different sweep counts, so the work lists are
    # compacted (and the lanes rebuilt) along the way.
    lanes, single, s = plans
    say(f"[lanes iterate] graph={use_graph} stop={stop}")
    ua, ub = lanes.zeros(), single.zeros()
    a = lanes.iterate(ua, s, max_sweeps=900, rtol=1e-5, check_every=25, use_graph=use_graph, stop=stop)
    b = single.iterate(ub, s, max_sweeps=900, rtol=1e-5, check_every=25, use_graph=use_graph, stop=stop)
    its = np.array(a[0])
    say(f"   sweeps min {its.min()} max {its.max()}, status {a[2]}")
    assert a == b
    assert torch.equal(ua, ub)


def test_iterate_graph_vs_plain_with_lanes(plans):
    lanes, _, s = plans
    ua, ub = lanes.zeros(), lanes.zeros()
    a = lanes.iterate(ua, s, max_sweeps=300, rtol=1e-5, check_every=20, use_graph=True)
    b = lanes.iterate(ub, s, max_sweeps=300, rtol=1e-5, check_every=20, use_graph=False)
    assert a == b
    assert torch.equal(ua, ub)


def test_fgmres_lanes_bitwise(plans):
    lanes, single, s = plans
    say("[lanes fgmres]")
    ua, ub = lanes.zeros(), single.zeros()
    a = lanes.fgmres(ua, s, restart=10, sweeps=3, max_iters=40, rtol=1e-6)
    b = single.fgmres(ub, s, restart=10, sweeps=3, max_iters=40, rtol=1e-6)
    assert a == b
    assert torch.equal(ua, ub)


def test_lanes_follow_caller_stream(plans):
    # The caller's stream is a side stream: the forked lanes must be ordered
    # after the work queued before the call and before the work queued after.
    lanes, single, s = plans
    side = torch.cuda.Stream()
    ua, ub = lanes.zeros(), single.zeros()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        ua.copy_(s)           # queued on the side stream before the sweep
        lanes.sweep(ua, s, count=3, stream=side)
        out = ua * 2          # queued after it
    ub.copy_(s)
    single.sweep(ub, s, count=3)
    torch.cuda.synchronize()
    assert torch.equal(out, ub * 2)


def test_npbs_chain_lanes_bitwise(plans):
    lanes, single, s = plans
    g = torch.Generator(device="cpu").manual_seed(9)
    cells = sum(n * n for n in SIZES)

    def field(scale):
        return (scale * torch.complex(torch.randn(cells, generator=g),
                                      torch.randn(cells, generator=g))).to(torch.complex64).cuda()
    u0, wf, wl = field(1.0), field(0.3), field(0.3)
    for count in (1, 3):
        ua, ub = u0.clone(), u0.clone()
        lanes.npbs_step(ua, s, wf, wl, count=count)
        single.npbs_step(ub, s, wf, wl, count=count)
        torch.cuda.synchronize()
        assert torch.equal(ua, ub)
