"""GPU solvers against the FP64 oracle: stationary CBS (cbs_iterate) and
FGMRES (fgmres_solve), single instances and ragged batches.

Bar (per instance): the solvers keep their iterate in FP64 and stop when its
FP64 Born relative residual is <= rtol.  The solution handed back in an FP32
(complex64) plan is that iterate rounded to FP32; rounding alone moves the
residual by ~1e-7 * ||u|| / ||G s||, so the oracle's evaluation of the
returned FP32 solution must be <= 1e-5 (ten times rtol), and the reported
value -- the FP64 residual of that returned solution -- must agree with the
oracle's evaluation to 10 %.  FP64 plans return the iterate itself: the
oracle's evaluation must match the reported value to 1% and be <= rtol.  Sweep / Arnoldi-step counts match the oracle's (the
arithmetic is the same in exact arithmetic; FP32 noise and the check cadence
move the stop by at most a chunk)."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from paper_2603_18527_amd import cbs
from gpu_helpers import plan_for, random_problem, rel_err, say, to_list

pytestmark = pytest.mark.gpu


def _oracle_relres(k2, k0sq, eps, u, s):
    return O.born_relres(k2, k0sq, eps, u, s)


def _bar(dtype, reported, evaluated, rtol=1e-6):
    if dtype == cbs.CBS_C64:
        # the reported value is the FP64 residual of the returned (FP32-
        # rounded) solution: it agrees with the oracle's evaluation of that
        # solution to 10 %, and rounding keeps it within ten times rtol
        assert evaluated <= 10 * rtol
        assert abs(reported - evaluated) <= 0.1 * evaluated
    else:
        assert reported <= rtol
        assert evaluated <= rtol * 1.01
        assert abs(reported - evaluated) <= 0.01 * evaluated


@pytest.mark.parametrize("dtype,use_graph", [(cbs.CBS_C64, True), (cbs.CBS_C64, False),
                                             (cbs.CBS_C128, True)])
def test_iterate_blob64(dtype, use_graph):
    say(f"[iterate blob64] dtype={dtype} graph={use_graph}")
    p = S.blob_problem()
    plan, k2 = plan_for([p], dtype)
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    s = cbs.pack([p.source], tdt)
    u = plan.zeros()
    chunk = 25
    its, rel, stat = plan.iterate(u, s, max_sweeps=5000, rtol=1e-6, check_every=chunk,
                                  use_graph=use_graph)
    ki = to_list(k2, [64])[0]
    si = to_list(s, [64])[0]
    uo, mo, relo = O.cbs_iterate(ki, plan.k0sq[0], plan.eps[0], si, max_sweeps=5000, rtol=1e-6)
    ug = to_list(u, [64])[0]
    ev = _oracle_relres(ki, plan.k0sq[0], plan.eps[0], ug, si)
    say(f"   gpu sweeps {its[0]} relres {rel[0]:.3e} (oracle eval {ev:.3e}); oracle sweeps {mo}")
    assert stat[0] == cbs.INST_CONVERGED
    _bar(dtype, rel[0], ev)
    assert mo <= its[0] <= mo + chunk
    assert rel_err(ug, uo) <= 1e-4


def test_iterate_graph_matches_plain_bitwise():
    probs = [random_problem(n, seed=60 + n, source="point") for n in (64, 128)]
    plan, k2 = plan_for(probs)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    u1, u2 = plan.zeros(), plan.zeros()
    a = plan.iterate(u1, s, max_sweeps=3000, rtol=1e-6, check_every=20, use_graph=True)
    b = plan.iterate(u2, s, max_sweeps=3000, rtol=1e-6, check_every=20, use_graph=False)
    assert a == b
    assert torch.equal(u1, u2)


def test_batched_equals_per_instance_loop():
    # Ragged batch in one set of launches == one plan per instance (same
    # kernels, same per-instance reduction order => bitwise identical).
    sizes = [192, 64, 128, 64]
    say(f"[batched vs loop] sizes={sizes}")
    probs = [random_problem(n, seed=70 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    u = plan.zeros()
    its, rel, stat = plan.iterate(u, s, max_sweeps=4000, rtol=1e-6, check_every=20)
    us = cbs.unpack(u, sizes)
    for i, p in enumerate(probs):
        pi, ki = plan_for([p])
        si = cbs.pack([p.source], torch.complex64)
        ui = pi.zeros()
        it1, rel1, st1 = pi.iterate(ui, si, max_sweeps=4000, rtol=1e-6, check_every=20)
        say(f"   instance {i} n={p.n}: batched {its[i]} / loop {it1[0]} sweeps")
        assert it1[0] == its[i] and st1[0] == stat[i] == cbs.INST_CONVERGED
        assert rel1[0] == rel[i]
        assert torch.equal(ui.reshape(p.n, p.n), us[i])


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_iterate_physical_stop_rule(dtype):
    # rTol = ||s - A u|| / ||s|| (the paper's unified rule) tested in FP64 at
    # every chunk start: the GPU stops at the first multiple of check_every at
    # or after the oracle's first sweep with rTol <= rtol.
    k, rtol = 10, 1e-6
    p = S.blob_problem()
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    plan, k2 = plan_for([p], dtype)
    s = cbs.pack([p.source], tdt)
    u = plan.zeros()
    its, rel, stat = plan.iterate(u, s, max_sweeps=5000, rtol=rtol, check_every=k, stop="physical")
    ki, si = to_list(k2, [p.n])[0], to_list(s, [p.n])[0]
    _, m, relo, hist = O.cbs_iterate(ki, plan.k0sq[0], plan.eps[0], si, max_sweeps=5000, rtol=rtol,
                                     history=True, stop="physical")
    expect = k * -(-m // k)
    ug = to_list(u, [p.n])[0]
    ev = O.physical_relres(ki, ug, si)
    say(f"[physical stop] dtype={dtype}: gpu {its[0]} sweeps rTol {rel[0]:.3e} (oracle eval {ev:.3e}); "
        f"oracle first <= rtol at {m}")
    assert stat[0] == cbs.INST_CONVERGED
    assert its[0] % k == 0 and hist[m] <= rtol < hist[m - 1]
    if dtype == cbs.CBS_C128:
        assert its[0] == expect
        assert ev <= rtol and abs(ev - rel[0]) <= 0.01 * ev
    else:
        assert abs(its[0] - expect) <= k
        # rounding the FP64 iterate to FP32 moves A u by ~ unit * (|Lap u| + |k^2 u|)
        lap, ku = O.laplacian(ug), ki * ug
        bound = 16 * 2.0 ** -24 * float((torch.linalg.vector_norm(lap) + torch.linalg.vector_norm(ku))
                                        / torch.linalg.vector_norm(si))
        assert ev <= rtol + bound
        assert abs(ev - rel[0]) <= 0.1 * ev   # reported: FP64 residual of the returned field
    # the Born rule on the same problem is a different criterion
    u2 = plan.zeros()
    its_b, rel_b, _ = plan.iterate(u2, s, max_sweeps=5000, rtol=rtol, check_every=k)
    say(f"   Born rule: {its_b[0]} sweeps")
    assert its_b[0] != its[0]


def test_physical_stop_graph_plain_and_batched_bitwise():
    sizes = [128, 64, 192]
    probs = [random_problem(n, seed=610 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs)
    s = cbs.pack([q.source for q in probs], torch.complex64)
    ua, ub = plan.zeros(), plan.zeros()
    a = plan.iterate(ua, s, max_sweeps=3000, rtol=1e-6, check_every=20, stop="physical")
    b = plan.iterate(ub, s, max_sweeps=3000, rtol=1e-6, check_every=20, stop="physical",
                     use_graph=False)
    assert a == b and torch.equal(ua, ub)
    for i, q in enumerate(probs):
        pi, _ = plan_for([q])
        ui = pi.zeros()
        r = pi.iterate(ui, cbs.pack([q.source], torch.complex64), max_sweeps=3000, rtol=1e-6,
                       check_every=20, stop="physical")
        assert r[0][0] == a[0][i] and r[1][0] == a[1][i] and r[2][0] == a[2][i]
        assert torch.equal(ui, cbs.unpack(ua, sizes)[i].reshape(-1))
    with pytest.raises(ValueError):
        plan.iterate(ua, s, stop="l2")


def test_iterate_zero_source_and_max_sweeps():
    probs = [random_problem(64, seed=81, source="point"), random_problem(128, seed=82, source="point")]
    plan, k2 = plan_for(probs)
    s = cbs.pack([np.zeros((64, 64)), probs[1].source], torch.complex64)
    u = plan.zeros()
    its, rel, stat = plan.iterate(u, s, max_sweeps=30, rtol=1e-6, check_every=10)
    assert stat[0] == cbs.INST_CONVERGED and its[0] == 0 and rel[0] == 0.0
    assert stat[1] == cbs.INST_MAX_ITERS and 30 <= its[1] <= 40


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_fgmres_small_matches_oracle(dtype):
    say(f"[fgmres 64] dtype={dtype}")
    p = random_problem(64, seed=91, source="point", cmax=3.0, ppw=6.0)
    plan, k2 = plan_for([p], dtype, restart=10)
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    s = cbs.pack([p.source], tdt)
    u = plan.zeros()
    its, rel, stat = plan.fgmres(u, s, restart=10, sweeps=3, max_iters=500, rtol=1e-6)
    ki = to_list(k2, [64])[0]
    si = to_list(s, [64])[0]
    xo, ito, relo = O.fgmres(ki, plan.k0sq[0], plan.eps[0], si, restart=10, sweeps=3,
                             max_iters=500, rtol=1e-6)
    ug = to_list(u, [64])[0]
    ev = _oracle_relres(ki, plan.k0sq[0], plan.eps[0], ug, si)
    say(f"   gpu its {its[0]} relres {rel[0]:.3e} (oracle eval {ev:.3e}); oracle its {ito}")
    assert stat[0] == cbs.INST_CONVERGED
    _bar(dtype, rel[0], ev)
    if dtype == cbs.CBS_C128:
        assert its[0] == ito
        assert rel_err(ug, xo) <= 1e-8
    else:
        assert abs(its[0] - ito) <= 3


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_gmres_without_inner_sweeps_matches_oracle(dtype):
    # K = 0: no inner preconditioner, GMRES on B u = G s (periodic plan)
    p = random_problem(32, seed=93, source="point", cmax=2.0, ppw=8.0)
    plan, k2 = plan_for([p], dtype, restart=20)
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    s = cbs.pack([p.source], tdt)
    u = plan.zeros()
    its, rel, stat = plan.fgmres(u, s, restart=20, sweeps=0, max_iters=3000, rtol=1e-6)
    ki, si = to_list(k2, [32])[0], to_list(s, [32])[0]
    xo, ito, relo = O.fgmres(ki, plan.k0sq[0], plan.eps[0], si, restart=20, sweeps=0, max_iters=3000, rtol=1e-6)
    ug = to_list(u, [32])[0]
    ev = _oracle_relres(ki, plan.k0sq[0], plan.eps[0], ug, si)
    say(f"[gmres K=0] dtype={dtype}: gpu its {its[0]} relres {rel[0]:.3e} (oracle eval {ev:.3e}); oracle its {ito}")
    assert stat[0] == cbs.INST_CONVERGED
    _bar(dtype, rel[0], ev)
    if dtype == cbs.CBS_C128:
        assert its[0] == ito
        assert rel_err(ug, xo) <= 1e-8
    else:
        assert abs(its[0] - ito) <= 5


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
@pytest.mark.parametrize("sweeps", [0, 2])
def test_fgmres_one_step_on_an_eigenvector(dtype, sweeps):
    # Homogeneous lossy medium k^2 = k0^2 + i kappa: V is a constant, B = I - G V
    # is diagonal in Fourier space, so G s for one Fourier mode s is an
    # eigenvector of B and of P_K: the first Arnoldi step spans the solution
    # (the next Krylov vector vanishes up to rounding) and FGMRES stops there.
    n, k0sq, kappa = 32, 0.8, 0.3
    x = np.arange(n)
    mode = np.exp(2j * np.pi * (3 * x[:, None] + 5 * x[None, :]) / n)
    prob = S.homogeneous_lossy(n, k0sq, kappa, mode)
    plan, k2 = plan_for([prob], dtype, restart=10, eps=[1.5 * kappa])
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    s = cbs.pack([mode], tdt)
    u = plan.zeros()
    rtol = 1e-6 if dtype == cbs.CBS_C64 else 1e-12
    its, rel, stat = plan.fgmres(u, s, restart=10, sweeps=sweeps, max_iters=50, rtol=rtol)
    ki, si = to_list(k2, [n])[0], to_list(s, [n])[0]
    ev = _oracle_relres(ki, k0sq, 1.5 * kappa, to_list(u, [n])[0], si)
    say(f"[fgmres eigenvector] dtype={dtype} K={sweeps}: its {its[0]} rel {rel[0]:.2e} eval {ev:.2e}")
    assert stat[0] == cbs.INST_CONVERGED and its[0] == 1
    assert ev <= (1e-6 if dtype == cbs.CBS_C64 else 1e-12)


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
@pytest.mark.parametrize("solver", ["iterate", "fgmres"])
def test_zero_right_hand_side_in_a_batch(dtype, solver):
    # Degenerate instance: s = 0 from u = 0 is solved by u = 0 (G s = 0, so
    # the Born residual's reference norm is zero).  Beside an ordinary
    # instance in the same batch it must stop at once with u exactly zero and
    # no NaN, while the other instance converges as usual.
    probs = [random_problem(64, seed=90, source="point"), random_problem(128, seed=91, source="point")]
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    plan, k2 = plan_for(probs, dtype, restart=20)
    src = [np.zeros((64, 64), np.complex128), probs[1].source]
    s = cbs.pack(src, tdt)
    u = plan.zeros()
    if solver == "iterate":
        its, rel, stat = plan.iterate(u, s, max_sweeps=5000, rtol=1e-6, check_every=25)
    else:
        its, rel, stat = plan.fgmres(u, s, restart=20, sweeps=3, max_iters=2000, rtol=1e-6)
    torch.cuda.synchronize()
    say(f"[zero rhs] {solver} dtype={dtype}: iterations {its}, relres {rel}, status {stat}")
    u0, u1 = cbs.unpack(u, [64, 128])
    assert stat[0] == cbs.INST_CONVERGED and its[0] == 0 and rel[0] == 0.0
    assert bool(torch.all(u0 == 0))
    assert stat[1] == cbs.INST_CONVERGED and its[1] > 0
    assert bool(torch.all(torch.isfinite(torch.view_as_real(u1))))
    ev = _oracle_relres(to_list(k2, [64, 128])[1], plan.k0sq[1], plan.eps[1], to_list(u, [64, 128])[1],
                        to_list(s, [64, 128])[1])
    _bar(dtype, rel[1], ev)


def test_fgmres_grf256_full_size():
    # 256x256 random-field medium, FGMRES(30) with 4 CBS sweeps.
    say("[fgmres grf256]")
    p = S.grf_problem()
    plan, k2 = plan_for([p], restart=30)
    s = cbs.pack([p.source], torch.complex64)
    u = plan.zeros()
    its, rel, stat = plan.fgmres(u, s, restart=30, sweeps=4, max_iters=2500, rtol=1e-6)
    ki = to_list(k2, [256])[0]
    si = to_list(s, [256])[0]
    ev = _oracle_relres(ki, plan.k0sq[0], plan.eps[0], to_list(u, [256])[0], si)
    say(f"   gpu its {its[0]} relres {rel[0]:.3e} oracle eval {ev:.3e}")
    assert stat[0] == cbs.INST_CONVERGED
    _bar(cbs.CBS_C64, rel[0], ev)


def test_fgmres_ragged_batch():
    sizes = [128, 64, 192]
    probs = [random_problem(n, seed=95 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs, restart=15)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    u = plan.zeros()
    its, rel, stat = plan.fgmres(u, s, restart=15, sweeps=2, max_iters=1000, rtol=1e-6)
    for i, (ui, si, ki) in enumerate(zip(to_list(u, sizes), to_list(s, sizes), to_list(k2, sizes))):
        ev = _oracle_relres(ki, plan.k0sq[i], plan.eps[i], ui, si)
        say(f"   instance {i}: its {its[i]} relres {rel[i]:.3e} oracle {ev:.3e}")
        assert stat[i] == cbs.INST_CONVERGED
        _bar(cbs.CBS_C64, rel[i], ev)


@pytest.mark.parametrize("dtype", [cbs.CBS_C64, cbs.CBS_C128])
def test_iterate_and_fgmres_from_nonzero_initial_guess(dtype):
    # Sec. 3.1 Eq. CBS from u0 != 0: same sweep count as the oracle from the
    # same u0; FGMRES restarts from the true residual of u0.
    sizes = [64, 128]
    say(f"[nonzero u0] dtype={dtype}")
    probs = [random_problem(n, seed=140 + i, source="point") for i, n in enumerate(sizes)]
    plan, k2 = plan_for(probs, dtype, restart=12)
    tdt = torch.complex64 if dtype == cbs.CBS_C64 else torch.complex128
    rng = np.random.default_rng(5)
    u0 = cbs.pack([0.01 * S.random_field_c(n, rng) for n in sizes], tdt)
    s = cbs.pack([p.source for p in probs], tdt)
    u = u0.clone()
    its, rel, stat = plan.iterate(u, s, max_sweeps=5000, rtol=1e-6, check_every=20)
    v = u0.clone()
    fits, frel, fstat = plan.fgmres(v, s, restart=12, sweeps=2, max_iters=2000, rtol=1e-6)
    for i, (ki, si, u0i, ui, vi) in enumerate(zip(to_list(k2, sizes), to_list(s, sizes), to_list(u0, sizes),
                                                  to_list(u, sizes), to_list(v, sizes))):
        uo, mo, relo = O.cbs_iterate(ki, plan.k0sq[i], plan.eps[i], si, u0=u0i, max_sweeps=5000, rtol=1e-6)
        say(f"   instance {i}: gpu {its[i]} oracle {mo} sweeps; fgmres {fits[i]} its")
        assert stat[i] == cbs.INST_CONVERGED and mo <= its[i] <= mo + 20
        _bar(dtype, rel[i], _oracle_relres(ki, plan.k0sq[i], plan.eps[i], ui, si))
        assert fstat[i] == cbs.INST_CONVERGED
        _bar(dtype, frel[i], _oracle_relres(ki, plan.k0sq[i], plan.eps[i], vi, si))


def test_iterate_degenerate_cases():
    probs = [random_problem(64, seed=150, source="point"), random_problem(32, seed=151, source="point")]
    plan, k2 = plan_for(probs)
    s = cbs.pack([p.source for p in probs], torch.complex64)
    # no sweeps allowed: status MAX_ITERS, u unchanged
    u = plan.zeros()
    its, rel, stat = plan.iterate(u, s, max_sweeps=0, rtol=1e-6, check_every=5)
    assert its == [0, 0] and stat == [cbs.INST_MAX_ITERS] * 2 and float(torch.abs(u).max()) == 0.0
    assert abs(rel[0] - 1.0) < 1e-6 and abs(rel[1] - 1.0) < 1e-6   # r(0) = G s
    # a NaN in the source of instance 1: that instance diverges, instance 0 converges
    s2 = s.clone()
    s2[64 * 64 + 5] = float("nan")
    u = plan.zeros()
    its, rel, stat = plan.iterate(u, s2, max_sweeps=2000, rtol=1e-6, check_every=10)
    assert stat[0] == cbs.INST_CONVERGED and stat[1] == cbs.INST_DIVERGED
    # FGMRES with restart 1 (steepest-descent-like) still reaches the tolerance
    plan2, k2b = plan_for(probs[:1], restart=1)
    u = plan2.zeros()
    its, rel, stat = plan2.fgmres(u, cbs.pack([probs[0].source], torch.complex64), restart=1, sweeps=3,
                                  max_iters=5000, rtol=1e-6)
    ug = to_list(u, [probs[0].n])[0]
    ev = O.born_relres(to_list(k2b, [probs[0].n])[0], plan2.k0sq[0], plan2.eps[0], ug, probs[0].source)
    assert stat[0] == cbs.INST_CONVERGED
    _bar(cbs.CBS_C64, rel[0], ev)


def test_aliasing_and_argument_errors():
    probs = [random_problem(32, seed=160)]
    plan, k2 = plan_for(probs)
    u = plan.zeros()
    lib = cbs.load()
    ptr = lambda t: cbs._ptr(t)
    assert lib.cbs_apply(plan._h, ptr(u), None, ptr(u), None) == cbs.CBS_ERR_ARG
    assert lib.cbs_residual(plan._h, ptr(u), None, None, ptr(u), None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_sweep(plan._h, ptr(u), ptr(u), 1, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_sweep(plan._h, ptr(u), None, 0, None, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_iterate(plan._h, ptr(u), ptr(u), 10, 1e-6, 10, 0, None, None, None, 0, None) == cbs.CBS_ERR_ARG
    assert lib.cbs_iterate(plan._h, ptr(u), ptr(plan.zeros()), 10, 1e-6, 1, 0, None, None, None, 0, None) \
        == cbs.CBS_ERR_ARG
    for bad_stop in (-1, 2):
        assert lib.cbs_iterate(plan._h, ptr(u), ptr(plan.zeros()), 10, 1e-6, 10, bad_stop, None, None, None,
                               0, None) == cbs.CBS_ERR_ARG
        assert "stop" in cbs.last_error()
    assert lib.cbs_set_tile(plan._h, 32, 3) == cbs.CBS_ERR_ARG
    assert lib.cbs_set_tile(plan._h, 48, 16) == cbs.CBS_ERR_ARG
    with pytest.raises(ValueError):
        plan.apply(torch.zeros(10, dtype=torch.complex64, device="cuda"), None)
