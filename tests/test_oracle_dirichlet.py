"""Pins of the oracle's Dirichlet (DST-I) operators (App. C, "Newton linear
systems for nonlinear PDEs"): an independent library, closed-form
eigenfunctions of the five-point stencil, the stencil-built reference
operator and a dense solve."""
import math

import numpy as np
import pytest
import scipy.fft
import torch

import oracle as O
import synthetic as S


@pytest.mark.parametrize("n", [7, 15, 31])
def test_dst1_matches_scipy(n):
    # scipy's DST-I is y_k = 2 sum_j x_j sin(pi (j+1)(k+1)/(n+1))
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = scipy.fft.dst(x, type=1) / 2
    got = (O.dst1_matrix(n) @ torch.from_numpy(x)).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert torch.allclose(O.idst2(O.dst2(torch.from_numpy(np.outer(x, x)))),
                          torch.from_numpy(np.outer(x, x)), atol=1e-12)


@pytest.mark.parametrize("n,p,q", [(7, 1, 1), (15, 3, 11), (31, 31, 2)])
def test_sine_modes_are_stencil_eigenfunctions(n, p, q):
    # L_D phi = (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2)) phi for
    # phi_ij = sin(p pi i h) sin(q pi j h), i, j = 1..n, h = 1/(n+1)
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1)
    phi = np.outer(np.sin(p * math.pi * i * h), np.sin(q * math.pi * i * h))
    lam = 4 / h ** 2 * (math.sin(p * math.pi * h / 2) ** 2 + math.sin(q * math.pi * h / 2) ** 2)
    got = O.laplacian_dirichlet(phi).numpy()
    assert np.max(np.abs(got - lam * phi)) <= 1e-10 * lam
    assert O.dirichlet_eigs(n)[p - 1, q - 1] == pytest.approx(lam, rel=1e-14)


def test_green_dirichlet_inverts_the_stencil_reference():
    n, k0sq, eps = 15, 40.0, 25.0
    rng = np.random.default_rng(3)
    q = O.as_c(S.random_field_c(n, rng))
    lq = O.laplacian_dirichlet(q) - complex(k0sq, eps) * q
    assert torch.max(torch.abs(O.green_dirichlet(lq, k0sq, eps) - q)) <= 1e-12 * torch.max(torch.abs(q))


def test_dirichlet_cbs_matches_dense_solve():
    # a Newton-type operator J = L_D - k^2 with a smooth real k^2 (2 u_m)
    n = 15
    rng = np.random.default_rng(4)
    k2 = 100.0 + 60.0 * S.gaussian_random_field(n, 3.0, rng)
    s = S.random_field_c(n, rng)
    k0sq = 0.5 * (k2.min() + k2.max())
    eps = O.choose_eps(k2, k0sq)
    u, m, rel = O.cbs_iterate_dirichlet(k2, k0sq, eps, s, max_sweeps=20000, rtol=1e-12)
    assert rel <= 1e-12
    eye = np.eye(n * n).reshape(n * n, n, n)
    a = np.stack([O.laplacian_dirichlet(e).numpy().reshape(-1) for e in eye], axis=1) \
        - np.diag(k2.reshape(-1))
    ref = np.linalg.solve(a, s.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(u.numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert torch.max(torch.abs(O.helmholtz_dirichlet(k2, u) - O.as_c(s))) <= 1e-8 * np.max(np.abs(s))


def _dense_dirichlet_laplacian(n):
    # L_D = kron(L1, I) + kron(I, L1), L1 = tridiag(-1, 2, -1) / h^2
    h = 1.0 / (n + 1)
    l1 = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h ** 2
    return np.kron(l1, np.eye(n)) + np.kron(np.eye(n), l1)


@pytest.mark.parametrize("k0sq", [-50.0, 10.0, 300.0])
def test_undamped_green_is_the_inverse_reference(k0sq):
    # eps = 0: G = (L_D - k0^2)^-1 (App. B.2, Eq. newton_ref with no damping),
    # definite (k0^2 below the lowest eigenvalue 2 pi^2 ~ 19.6) or not
    n = 15
    rng = np.random.default_rng(7)
    q = S.random_field_c(n, rng)
    a = _dense_dirichlet_laplacian(n) - k0sq * np.eye(n * n)
    ref = np.linalg.solve(a, q.reshape(-1)).reshape(n, n)
    got = O.green_dirichlet(q, k0sq, 0.0).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_newton_born_identity_undamped():
    # I - G V = G J (Eq. newton_born_identity): with J = L_D - 2 diag(u_m),
    # J_0 = L_D - k0^2, k0^2 = 2 mean(u_m) - alpha and V = J_0 - J = 2 u_m - k0^2,
    # the Born residual G (V x + s) - x equals G (s - J x)
    n = 15
    rng = np.random.default_rng(8)
    x1 = np.arange(1, n + 1) / (n + 1)
    um = 5.0 + 3.0 * np.outer(np.sin(math.pi * x1), np.sin(2 * math.pi * x1))
    k2, k0sq = 2.0 * um, 2.0 * um.mean() - 4.0
    x = S.random_field_c(n, rng)
    s = S.random_field_c(n, rng)
    jac = _dense_dirichlet_laplacian(n) - np.diag(k2.reshape(-1))
    g = np.linalg.inv(_dense_dirichlet_laplacian(n) - k0sq * np.eye(n * n))
    ref = (g @ (s.reshape(-1) - jac @ x.reshape(-1))).reshape(n, n)
    got = O.cbs_residual_dirichlet(k2, k0sq, 0.0, x, s).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))
