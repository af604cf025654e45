"""Pins of the oracle's operators against the paper's propositions and the
CBS contraction property, on dense 16x16 (or smaller) systems."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S


def _dense_helmholtz_numpy(k2):
    """A = -Laplacian - diag(k2) built with numpy.fft (independent of the oracle)."""
    n = k2.shape[0]
    eye = np.eye(n * n).reshape(n * n, n, n)
    xi = 2 * math.pi * np.fft.fftfreq(n)
    xi2 = xi[:, None] ** 2 + xi[None, :] ** 2
    lap = np.fft.ifft2(np.fft.fft2(eye) * xi2).reshape(n * n, n * n).T
    return lap - np.diag(k2.reshape(-1))


def _small_problem(n=16, layer=4, seed=7):
    rng = np.random.default_rng(seed)
    c = S.minmax_map(S.gaussian_random_field(n, 3.0, rng), 1.0, 2.0)
    src = S.point_source(n, (n // 2, n // 2 + 1))
    return S.velocity_problem(c, layer, 6.0, src, cmin=1.0)


def test_key_identity_dense():
    # Prop. 3.1: I - G V = G A exactly.
    p = _small_problem()
    eps = O.choose_eps(p.k2, p.k0sq)
    n = p.n
    b = O.operator_matrix(lambda e: O.born_operator(p.k2, p.k0sq, eps, e), n).numpy()
    g = O.operator_matrix(lambda e: O.green(e, p.k0sq, eps), n).numpy()
    a = _dense_helmholtz_numpy(p.k2)
    assert np.max(np.abs(b - g @ a)) < 1e-12


def test_spectral_disk_and_condition_bounds():
    # Prop. 3.1 bounds when q = ||G V||_2 < 1: spectrum in |z - 1| <= q and
    # kappa_2(I - G V) <= (1 + q) / (1 - q).  k0^2 sits between grid
    # eigenvalues of -Laplacian, the medium is a small perturbation.
    n = 16
    h = (2 * math.pi / n) ** 2
    k0sq = 1.5 * h
    eta = 0.02
    rng = np.random.default_rng(3)
    k2 = k0sq + 0.03 * S.minmax_map(S.gaussian_random_field(n, 2.0, rng), -1.0, 1.0)
    gv = O.operator_matrix(lambda e: O.green(O.potential(k2, k0sq, eta) * e, k0sq, eta), n).numpy()
    q = np.linalg.norm(gv, 2)
    assert q < 1.0
    m = np.eye(n * n) - gv
    ev = np.linalg.eigvals(m)
    assert np.max(np.abs(ev - 1.0)) <= q + 1e-12
    sv = np.linalg.svd(m, compute_uv=False)
    assert sv[0] / sv[-1] <= (1 + q) / (1 - q) + 1e-9


def test_riesz_equivalence():
    # Prop. 4.1: ||(I - G V) x - G r|| = ||G (A x - r)||.
    p = _small_problem(seed=11)
    eps = O.choose_eps(p.k2, p.k0sq)
    rng = np.random.default_rng(5)
    x = O.as_c(S.random_field_c(p.n, rng))
    r = O.as_c(S.random_field_c(p.n, rng))
    lhs = O.norm(O.born_operator(p.k2, p.k0sq, eps, x) - O.green(r, p.k0sq, eps))
    ax = torch.from_numpy((_dense_helmholtz_numpy(p.k2) @ x.numpy().reshape(-1)).reshape(p.n, p.n))
    rhs = O.norm(O.green(ax - r, p.k0sq, eps))
    assert abs(lhs - rhs) <= 1e-12 * rhs


def test_cbs_contraction():
    # P8: with eps >= max|k^2 - k0^2| and min|V| > 0 the CBS iteration matrix
    # T = I - gamma (I - G V) has spectral radius and 2-norm below one.
    p = _small_problem(seed=2)
    eps = O.choose_eps(p.k2, p.k0sq)
    g = O.gamma(p.k2, p.k0sq, eps).reshape(-1).numpy()
    b = O.operator_matrix(lambda e: O.born_operator(p.k2, p.k0sq, eps, e), p.n).numpy()
    t = np.eye(p.n * p.n) - g[:, None] * b
    assert np.max(np.abs(np.linalg.eigvals(t))) < 1.0
    assert np.linalg.norm(t, 2) < 1.0 + 1e-12


def test_npbs_reductions():
    # Sec. 4.1: M = gamma gives the CBS step; M = (I - G V)^{-1} solves in one step.
    p = _small_problem(seed=4)
    eps = O.choose_eps(p.k2, p.k0sq)
    rng = np.random.default_rng(8)
    u0 = O.as_c(S.random_field_c(p.n, rng))
    r = O.cbs_residual(p.k2, p.k0sq, eps, u0, p.source)
    step_gamma = u0 + O.gamma(p.k2, p.k0sq, eps) * r
    assert torch.allclose(step_gamma, O.cbs_sweep(p.k2, p.k0sq, eps, u0, p.source), atol=0, rtol=0)
    b = O.operator_matrix(lambda e: O.born_operator(p.k2, p.k0sq, eps, e), p.n)
    m_exact = torch.linalg.inv(b)
    u1 = u0 + (m_exact @ r.reshape(-1)).reshape(p.n, p.n)
    ref = np.linalg.solve(_dense_helmholtz_numpy(p.k2), p.source.reshape(-1)).reshape(p.n, p.n)
    assert np.max(np.abs(u1.numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_npbs_linear_fourier_layer_reductions():
    # Sec. 4.1 with the linear Fourier layer of App. E as M:
    # (i) W^F = 0, W^loc = gamma is the CBS step;
    # (ii) in a homogeneous lossy medium V = v is constant, (I - G V)^{-1} is
    #     diagonal in Fourier space with entries lambda / (lambda - v), so that
    #     W^F (W^loc = 0) solves in one step from any u; the solution is the
    #     closed form F^-1(F s / (|xi|^2 - k^2)) evaluated with numpy.fft;
    # (iii) W^F = 1, W^loc = 0 gives M = identity: u + r = G (V u + s).
    p = _small_problem(seed=6)
    eps = O.choose_eps(p.k2, p.k0sq)
    rng = np.random.default_rng(9)
    u0 = O.as_c(S.random_field_c(p.n, rng))
    zero = torch.zeros(p.n, p.n, dtype=O.CDT)
    got = O.npbs_step(p.k2, p.k0sq, eps, u0, p.source, zero, O.gamma(p.k2, p.k0sq, eps))
    assert torch.equal(got, O.cbs_sweep(p.k2, p.k0sq, eps, u0, p.source))
    one = torch.ones(p.n, p.n, dtype=O.CDT)
    got = O.npbs_step(p.k2, p.k0sq, eps, u0, p.source, one, 0.0)
    assert torch.max(torch.abs(got - O.cbs_apply(p.k2, p.k0sq, eps, u0, p.source))) <= 1e-12
    n, k0sq, kappa = 24, 0.7, 0.25
    s = S.random_field_c(n, rng)
    h = S.homogeneous_lossy(n, k0sq, kappa, s)
    e = 1.5 * kappa
    lam = O.symbol(n, k0sq, e)
    v = complex(0.0, kappa - e)              # V = k^2 - k0^2 - i eps = i (kappa - eps)
    wf = lam / (lam - v)
    u1 = O.npbs_step(h.k2, k0sq, e, S.random_field_c(n, rng), s, wf, 0.0)
    xi = 2 * np.pi * np.fft.fftfreq(n)
    exact = np.fft.ifft2(np.fft.fft2(s) / (xi[:, None] ** 2 + xi[None, :] ** 2 - k0sq - 1j * kappa))
    assert np.max(np.abs(u1.numpy() - exact)) <= 1e-12 * np.max(np.abs(exact))
