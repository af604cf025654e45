"""Pins of the oracle's solvers: closed-form homogeneous solutions, dense
LAPACK solves on tiny grids, the outgoing 2D Green's function, and GMRES
invariants."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S


def _dense_helmholtz_numpy(k2):
    n = k2.shape[0]
    eye = np.eye(n * n).reshape(n * n, n, n)
    xi = 2 * math.pi * np.fft.fftfreq(n)
    xi2 = xi[:, None] ** 2 + xi[None, :] ** 2
    lap = np.fft.ifft2(np.fft.fft2(eye) * xi2).reshape(n * n, n * n).T
    return lap - np.diag(k2.reshape(-1))


def _problem16(seed=1):
    rng = np.random.default_rng(seed)
    c = S.minmax_map(S.gaussian_random_field(16, 3.0, rng), 1.0, 2.5)
    src = S.gaussian_pulse(16, (7, 9), 1.5)
    return S.velocity_problem(c, 4, 5.0, src, cmin=1.0)


def test_homogeneous_lossy_closed_form():
    # P5: k^2 = k0^2 + i kappa, eps = 1.5 kappa; the exact solution is
    # F^-1(s_hat / (|xi|^2 - k0^2 - i kappa)), evaluated here with numpy.fft.
    n, k0sq, kappa = 32, 0.8, 0.3
    rng = np.random.default_rng(0)
    s = S.random_field_c(n, rng)
    p = S.homogeneous_lossy(n, k0sq, kappa, s)
    xi = 2 * math.pi * np.fft.fftfreq(n)
    lam = xi[:, None] ** 2 + xi[None, :] ** 2 - k0sq - 1j * kappa
    exact = np.fft.ifft2(np.fft.fft2(s) / lam)
    u, m, rel = O.cbs_iterate(p.k2, k0sq, 1.5 * kappa, s, max_sweeps=500, rtol=1e-14)
    assert rel <= 1e-14
    assert np.max(np.abs(u.numpy() - exact)) <= 1e-12 * np.max(np.abs(exact))


def test_cbs_matches_dense_solve():
    # P6: CBS converges to the LAPACK solution of the pseudospectral A u = s.
    p = _problem16()
    eps = O.choose_eps(p.k2, p.k0sq)
    ref = np.linalg.solve(_dense_helmholtz_numpy(p.k2), p.source.reshape(-1)).reshape(16, 16)
    u, m, rel = O.cbs_iterate(p.k2, p.k0sq, eps, p.source, max_sweeps=20000, rtol=1e-13)
    assert rel <= 1e-13
    assert np.max(np.abs(u.numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    # The oracle's own dense solve agrees with the numpy-built one.
    assert np.max(np.abs(O.dense_solve(p.k2, p.source).numpy() - ref)) <= 1e-11 * np.max(np.abs(ref))
    # Physical residual of the converged iterate (the paper's rTol).
    assert O.physical_relres(p.k2, u, p.source) < 1e-10


def test_cbs_and_fgmres_match_dense_solve_32():
    # P6 at 32 x 32 (a 1024 x 1024 dense A): CBS and FGMRES(30) + P_4 both
    # reach the LAPACK solution.
    rng = np.random.default_rng(7)
    c = S.minmax_map(S.gaussian_random_field(32, 4.0, rng), 1.0, 2.0)
    src = S.gaussian_pulse(32, (13, 18), 1.5)
    p = S.velocity_problem(c, 6, 6.0, src, cmin=1.0)
    eps = O.choose_eps(p.k2, p.k0sq)
    ref = np.linalg.solve(_dense_helmholtz_numpy(p.k2), p.source.reshape(-1)).reshape(32, 32)
    u, m, rel = O.cbs_iterate(p.k2, p.k0sq, eps, p.source, max_sweeps=40000, rtol=1e-13)
    assert rel <= 1e-13
    assert np.max(np.abs(u.numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    x, its, rel = O.fgmres(p.k2, p.k0sq, eps, p.source, restart=30, sweeps=4, max_iters=5000, rtol=1e-13)
    assert rel <= 1e-13
    assert np.max(np.abs(x.numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_physical_stop_rule():
    # The paper's unified stopping rule rTol = ||s - A u|| / ||s|| (Sec. 5).
    # Pins: (i) the physical residual is L_eta applied to the Born residual,
    # s - A u = L_eta (G (V u + s) - u) (Prop. 3.1 key identity), here with
    # the Laplacian and k^2 on one side and the symbol lambda on the other;
    # (ii) the loop stops at the first sweep whose residual is <= rtol, with
    # the numpy-built dense A deciding on the returned iterate.
    p = _problem16(seed=3)
    eps = O.choose_eps(p.k2, p.k0sq)
    u, m, rel, hist = O.cbs_iterate(p.k2, p.k0sq, eps, p.source, max_sweeps=5000, rtol=1e-8,
                                    history=True, stop="physical")
    a = _dense_helmholtz_numpy(p.k2)
    e_dense = p.source.reshape(-1) - a @ u.numpy().reshape(-1)
    assert np.linalg.norm(e_dense) / np.linalg.norm(p.source) == pytest.approx(rel, rel=1e-9)
    assert rel <= 1e-8 < hist[-2] and len(hist) == m + 1
    r = O.cbs_residual(p.k2, p.k0sq, eps, u, p.source)
    l_eta_r = O.idft2(O.dft2(r) * O.symbol(16, p.k0sq, eps))
    e = O.as_c(p.source) - O.helmholtz(p.k2, u)
    assert torch.max(torch.abs(l_eta_r - e)) <= 1e-12 * torch.max(torch.abs(O.as_c(p.source)))
    # the Born rule on the same problem stops at a different sweep
    _, m_born, _ = O.cbs_iterate(p.k2, p.k0sq, eps, p.source, max_sweeps=5000, rtol=1e-8)
    assert m_born != m


@pytest.mark.parametrize("restart,sweeps", [(5, 1), (10, 4), (300, 2)])
def test_fgmres_matches_dense_solve(restart, sweeps):
    # P6 for FGMRES(m) with P_K: same solution as LAPACK.
    p = _problem16(seed=2)
    eps = O.choose_eps(p.k2, p.k0sq)
    ref = np.linalg.solve(_dense_helmholtz_numpy(p.k2), p.source.reshape(-1)).reshape(16, 16)
    x, its, rel = O.fgmres(p.k2, p.k0sq, eps, p.source, restart=restart, sweeps=sweeps,
                           max_iters=5000, rtol=1e-12)
    assert rel <= 1e-12
    assert np.max(np.abs(x.numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_fgmres_estimate_equals_true_residual_and_is_monotone():
    # GMRES invariant: the least-squares residual of step j equals the true
    # residual ||b - B x_j|| and never increases within a cycle.
    p = _problem16(seed=3)
    eps = O.choose_eps(p.k2, p.k0sq)
    ests = []
    for j in range(1, 7):
        x, its, rel, hist = O.fgmres(p.k2, p.k0sq, eps, p.source, restart=50, sweeps=2,
                                     max_iters=j, rtol=0.0, history=True)
        assert its == j
        # hist = [initial true residual, estimates..., final true residual]
        assert abs(hist[-2] - rel) <= 1e-10 * rel
        ests.append(rel)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(ests, ests[1:]))


def test_fgmres_k1_equals_diagonal_gamma_preconditioner():
    # P_1(v) = gamma v (Sec. 4.1: CBS uses the diagonal gamma in these coordinates).
    p = _problem16(seed=4)
    eps = O.choose_eps(p.k2, p.k0sq)
    v = O.as_c(S.random_field_c(16, np.random.default_rng(1)))
    assert torch.allclose(O.cbs_precondition(p.k2, p.k0sq, eps, v, 1), O.gamma(p.k2, p.k0sq, eps) * v,
                          rtol=0, atol=1e-15)


def test_gmres_without_inner_preconditioner():
    # K = 0 is P_0 = I: GMRES on B x = b.  One step from x = 0 is the best
    # multiple of b, with the closed-form residual
    # ||b|| sqrt(1 - |<B b, b>|^2 / (||B b||^2 ||b||^2)); the full space
    # (restart = number of unknowns) reaches LAPACK's solution.
    p = _problem16(seed=5)
    eps = O.choose_eps(p.k2, p.k0sq)
    b = O.green(O.as_c(p.source), p.k0sq, eps)
    bb = O.born_operator(p.k2, p.k0sq, eps, b)
    c = complex(torch.sum(bb.conj() * b))
    one = math.sqrt(1.0 - abs(c) ** 2 / (O.norm(bb) ** 2 * O.norm(b) ** 2))
    x, its, rel = O.fgmres(p.k2, p.k0sq, eps, p.source, restart=10, sweeps=0, max_iters=1, rtol=0.0)
    assert its == 1 and abs(rel - one) <= 1e-12 * one
    assert torch.allclose(x, b * (c / O.norm(bb) ** 2), rtol=0, atol=1e-14 * float(torch.abs(b).max()))
    ref = np.linalg.solve(_dense_helmholtz_numpy(p.k2), p.source.reshape(-1)).reshape(16, 16)
    x, its, rel = O.fgmres(p.k2, p.k0sq, eps, p.source, restart=256, sweeps=0, max_iters=256, rtol=1e-11)
    assert rel <= 1e-11 and its <= 256
    assert np.max(np.abs(x.numpy() - ref)) <= 1e-8 * np.max(np.abs(ref))


@pytest.mark.slow
def test_outgoing_greens_function_with_sponge():
    # P4: homogeneous lossless interior, absorbing sponge: the field of a unit
    # point source approximates the outgoing 2D Green's function
    # (i/4) H0^(1)(k0 r) (exp(-i omega t) convention, Im k^2 > 0 in the layer).
    # With the conjugate (incoming) sign the error is O(1).
    from scipy.special import hankel1

    n, layer = 128, 40
    k0 = 2 * math.pi / 12.0
    k0sq = k0 * k0
    i = np.arange(n)
    depth = np.maximum(np.maximum(layer - i, i - (n - layer - 1)), 0) / layer
    t = np.maximum(depth[:, None], depth[None, :])
    a = 1.0 * k0sq
    k2 = k0sq + 1j * a * t ** 2
    src = S.point_source(n, (n // 2, n // 2))
    u, m, rel = O.cbs_iterate(k2, k0sq, 2.0 * a, src, max_sweeps=20000, rtol=1e-9)
    assert rel <= 1e-9
    yy, xx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    r = np.hypot(yy, xx)
    sel = (r >= 6) & (r <= 18)
    g = 0.25j * hankel1(0, k0 * r[sel])
    got = u.numpy()[sel]
    err = np.linalg.norm(got - g) / np.linalg.norm(g)
    assert err < 0.1
    wrong = np.linalg.norm(got - np.conj(g)) / np.linalg.norm(g)
    assert wrong > 0.5
