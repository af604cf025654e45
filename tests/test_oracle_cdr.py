"""Pins of the oracle's convection-diffusion-reaction operators (App. B.1,
Eqs. cdr_pde to cdr_G_symbol): closed forms of spectral derivatives and of
A_cdr on band-limited fields, a single Fourier mode through G_cdr, the decay
rates of the textbook 1D convection-diffusion Green's function (which fix the
sign of the convection term), the split identity I - G V = G A with A taken
from the PDE, the reduction to the (separately pinned) Helmholtz Green
operator, and the adjoint against the dense conjugate transpose."""
import math

import numpy as np
import pytest
import torch

import oracle as O


def _grid(n):
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    return y, x


def _random_medium(n, seed, kappa0=1.5, vx0=0.4, vy0=-0.3, sigma0=0.8):
    rng = np.random.default_rng(seed)
    return O.CdrMedium(kappa=kappa0 + 0.3 * rng.standard_normal((n, n)),
                       vx=vx0 + 0.2 * rng.standard_normal((n, n)),
                       vy=vy0 + 0.2 * rng.standard_normal((n, n)),
                       sigma=sigma0 + 0.3 * rng.standard_normal((n, n)),
                       kappa0=kappa0, vx0=vx0, vy0=vy0, sigma0=sigma0)


def _c(a):
    return torch.from_numpy(np.asarray(a, dtype=np.complex128))


def test_spectral_derivatives_of_trig_polynomials():
    n = 16
    y, x = _grid(n)
    a = 2 * math.pi / n
    u = np.sin(3 * a * x) * np.cos(2 * a * y) + 1j * np.cos(a * x)
    ux = 3 * a * np.cos(3 * a * x) * np.cos(2 * a * y) - 1j * a * np.sin(a * x)
    uy = -2 * a * np.sin(3 * a * x) * np.sin(2 * a * y)
    assert torch.max(torch.abs(O.deriv_x(u) - _c(ux))) <= 1e-12
    assert torch.max(torch.abs(O.deriv_y(u) - _c(uy))) <= 1e-12


def test_single_mode_through_green_and_reference():
    # e^{i (xi_x x + xi_y y)} is an eigenfunction: L0 gives the factor
    # kappa0 |xi|^2 + i (vx0 xi_x + vy0 xi_y) + sigma0 (convection enters with +i)
    n = 16
    y, x = _grid(n)
    kx, ky = 2, -3
    xx, yy = 2 * math.pi * kx / n, 2 * math.pi * ky / n
    mode = np.exp(1j * (xx * x + yy * y))
    m = O.CdrMedium(np.full((n, n), 1.7), np.full((n, n), 0.6), np.full((n, n), -0.9),
                    np.full((n, n), 0.35), 1.7, 0.6, -0.9, 0.35)
    lam = 1.7 * (xx ** 2 + yy ** 2) + 1j * (0.6 * xx - 0.9 * yy) + 0.35
    assert torch.max(torch.abs(O.cdr_reference(mode, m) - _c(lam * mode))) <= 1e-12
    assert torch.max(torch.abs(O.green_cdr(mode, m) - _c(mode / lam))) <= 1e-12
    assert torch.max(torch.abs(O.green_cdr_adjoint(mode, m) - _c(mode / np.conj(lam)))) <= 1e-12
    # homogeneous medium: V = 0, so the apply is G s and A = L0
    assert torch.max(torch.abs(O.cdr_potential(mode, m))) <= 1e-12
    assert torch.max(torch.abs(O.cdr_operator(mode, m) - _c(lam * mode))) <= 1e-11


@pytest.mark.parametrize("axis", ["x", "y"])
def test_convection_diffusion_decay_rates(axis):
    # -kappa u'' + v u' + sigma u = s in 1D: away from the source u ~ e^{lam x}
    # with kappa lam^2 - v lam - sigma = 0; downstream (v > 0) decays with
    # lam- = (v - sqrt(v^2 + 4 kappa sigma)) / (2 kappa), upstream with lam+.
    # A smooth line source keeps the spectral solution equal to the periodised
    # continuous one; images are e^{-28} away.
    n, kappa, v, sigma, x0, w = 256, 1.0, 0.2, 0.05, 128, 3.0
    lam_p = (v + math.sqrt(v * v + 4 * kappa * sigma)) / (2 * kappa)
    lam_m = (v - math.sqrt(v * v + 4 * kappa * sigma)) / (2 * kappa)
    y, x = _grid(n)
    coord = x if axis == "x" else y
    src = np.exp(-((coord - x0) ** 2) / (2 * w * w))
    vx0, vy0 = (v, 0.0) if axis == "x" else (0.0, v)
    one = np.ones((n, n))
    m = O.CdrMedium(kappa * one, vx0 * one, vy0 * one, sigma * one, kappa, vx0, vy0, sigma)
    u = O.green_cdr(src, m).real.numpy()
    line = u[0, :] if axis == "x" else u[:, 0]
    for d in range(30, 35):
        down = line[x0 + d + 1] / line[x0 + d]
        up = line[x0 - d - 1] / line[x0 - d]
        assert abs(down / math.exp(lam_m) - 1) <= 1e-7
        assert abs(up / math.exp(-lam_p) - 1) <= 1e-7
    # and the upstream side really is the steeper one (sign of v . grad)
    assert line[x0 - 20] < line[x0 + 20]


def test_operator_closed_form_band_limited():
    # kappa, v, sigma and u band-limited well below N/2: spectral derivatives
    # are exact and A u has a closed form (product rule written out)
    n = 16
    y, x = _grid(n)
    a = 2 * math.pi / n
    kappa = 2.0 + 0.5 * np.cos(a * x)
    vx = 0.3 + 0.1 * np.sin(a * y)
    vy = -0.2 * np.ones((n, n))
    sigma = 1.0 + 0.25 * np.cos(a * (x + y))
    u = np.sin(2 * a * y) * np.exp(1j * a * x)
    au = (0.5j * a * a * np.sin(a * x) * u + 5 * a * a * kappa * u + 1j * a * vx * u
          + 2 * a * vy * np.cos(2 * a * y) * np.exp(1j * a * x) + sigma * u)
    m = O.CdrMedium(kappa, vx, vy, sigma, 2.0, 0.3, -0.2, 1.0)
    assert torch.max(torch.abs(O.cdr_operator(u, m) - _c(au))) <= 1e-12
    # the split: L0 u - V u is the same operator
    assert torch.max(torch.abs(O.cdr_reference(u, m) - O.cdr_potential(u, m) - _c(au))) <= 1e-12


def test_split_identity_dense():
    # Eq. cdr_identity: I - G V = G A, with A from the PDE (not L0 - V)
    n = 6
    m = _random_medium(n, 3)
    lhs = O.operator_matrix(lambda e: O.cdr_born_operator(m, e), n)
    rhs = O.operator_matrix(lambda e: O.green_cdr(O.cdr_operator(e, m), m), n)
    assert torch.max(torch.abs(lhs - rhs)) <= 1e-12 * torch.max(torch.abs(lhs))
    # the Born residual is G (s - A u) (Eq. cdr_integral)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    s = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    r1 = O.cdr_residual(m, u, s)
    r2 = O.green_cdr(O.cdr_physical_residual(m, u, s), m)
    assert torch.max(torch.abs(r1 - r2)) <= 1e-12 * torch.max(torch.abs(r1))


def test_dense_solve_is_fixed_point():
    # brute force: the LAPACK solution of A u = s has zero Born residual
    n = 8
    m = _random_medium(n, 5)
    rng = np.random.default_rng(6)
    s = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = O.operator_matrix(lambda e: O.cdr_operator(e, m), n)
    u = torch.linalg.solve(a, _c(s).reshape(-1)).reshape(n, n)
    assert O.norm(O.cdr_residual(m, u, s)) <= 1e-12 * O.norm(O.green_cdr(s, m))


def test_reduces_to_helmholtz_green():
    # v0 = 0: L0 = kappa0 (|xi|^2 + sigma0 / kappa0), the Helmholtz symbol with
    # k0^2 = -sigma0 / kappa0 and eta = 0, scaled by kappa0
    n = 16
    rng = np.random.default_rng(7)
    q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    one = np.ones((n, n))
    m = O.CdrMedium(2.5 * one, 0 * one, 0 * one, 0.7 * one, 2.5, 0.0, 0.0, 0.7)
    ref = O.green(_c(q), -0.7 / 2.5, 0.0) / 2.5
    assert torch.max(torch.abs(O.green_cdr(q, m) - ref)) <= 1e-13 * torch.max(torch.abs(ref))


def test_adjoint_against_dense_conjugate_transpose():
    n = 6
    m = _random_medium(n, 8)
    rmat = O.operator_matrix(lambda e: O.cdr_born_operator(m, e), n)
    rng = np.random.default_rng(9)
    e = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = (rmat.conj().T @ _c(e).reshape(-1)).reshape(n, n)
    got = O.cdr_born_adjoint(m, e)
    assert torch.max(torch.abs(got - ref)) <= 1e-12 * torch.max(torch.abs(ref))
    # G is not symmetric once v0 != 0 (odd part of the symbol)
    g = O.operator_matrix(lambda e: O.green_cdr(e, m), n)
    assert torch.max(torch.abs(g - g.T)) > 1e-3 * torch.max(torch.abs(g))


def test_loss_gradient_central_differences():
    n = 8
    m = _random_medium(n, 10)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    val, g = O.cdr_loss_and_grad(m, x, r)
    # closed form of the gradient: 2 R^H (R x - G r)
    e = O.cdr_born_operator(m, x) - O.green_cdr(r, m)
    assert torch.max(torch.abs(g - 2 * O.cdr_born_adjoint(m, e))) <= 1e-12 * torch.max(torch.abs(g))
    h = 1e-4
    for _ in range(6):
        iy, ix = rng.integers(0, n, size=2)
        for unit in (1.0, 1j):
            d = np.zeros((n, n), dtype=np.complex128)
            d[iy, ix] = unit * h
            fd = (float(O.cdr_loss(m, x + d, r)) - float(O.cdr_loss(m, x - d, r))) / (2 * h)
            an = float(g[iy, ix].real if unit == 1.0 else g[iy, ix].imag)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))   # quadratic: exact up to rounding
