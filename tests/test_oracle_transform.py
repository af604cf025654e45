"""Pins of the oracle's DFT, symbol and Green operator against things other
than itself: numpy.fft (an independent library), closed forms for single
Fourier modes (App. D), and operator invariants (App. C)."""
import math

import numpy as np
import pytest
import torch

import oracle as O


@pytest.mark.parametrize("n", [8, 16, 48, 64])
def test_dft_matches_numpy_fft(n):
    # P1: the naive DFT equals numpy's FFT (forward unnormalised, inverse 1/N^2).
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    f = O.dft2(O.as_c(x)).numpy()
    assert np.max(np.abs(f - np.fft.fft2(x))) <= 1e-12 * np.max(np.abs(f))
    b = O.idft2(O.as_c(x)).numpy()
    assert np.max(np.abs(b - np.fft.ifft2(x))) <= 1e-13 * np.max(np.abs(x))


def test_mode_index_keeps_nyquist_negative():
    # App. D: n in {-N/2, ..., N/2 - 1}.
    m = O.mode_index(8).tolist()
    assert m == [0, 1, 2, 3, -4, -3, -2, -1]


@pytest.mark.parametrize("n,modes", [(16, [(0, 0), (1, 0), (3, -5), (-8, 2), (-8, -8), (7, 7)]),
                                     (24, [(2, 11), (-12, 0), (-12, -12)])])
def test_green_single_mode_closed_form(n, modes):
    # P2: G e^{i xi.x} = e^{i xi.x} / (|xi|^2 - k0^2 - i eps), Nyquist included.
    k0sq, eps = 0.7, 0.35
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    for (p, q) in modes:
        xi_y, xi_x = 2 * math.pi * p / n, 2 * math.pi * q / n
        wave = np.exp(1j * (xi_y * y + xi_x * x))
        lam = xi_y ** 2 + xi_x ** 2 - k0sq - 1j * eps
        got = O.green(O.as_c(wave), k0sq, eps).numpy()
        # Nyquist waves are real-valued cosines on the grid (e^{i pi j} = (-1)^j), so
        # the closed form is exact for them as well.
        assert np.max(np.abs(got - wave / lam)) <= 1e-12 / abs(lam) * 10


def test_laplacian_single_mode():
    n = 16
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    p, q = 3, -2
    wave = np.exp(2j * math.pi * (p * y + q * x) / n)
    got = O.laplacian(O.as_c(wave)).numpy()
    xi2 = (2 * math.pi / n) ** 2 * (p * p + q * q)
    assert np.max(np.abs(got - xi2 * wave)) < 1e-12


def test_green_is_complex_symmetric_and_adjoint_symbol():
    # P3: the symbol is even in xi, so G^T = G; G^H = F^-1 diag(1/conj(lambda)) F.
    n, k0sq, eps = 8, 0.9, 0.4
    g = O.operator_matrix(lambda e: O.green(e, k0sq, eps), n)
    assert torch.max(torch.abs(g - g.T)) < 1e-14
    gh = O.operator_matrix(lambda e: O.green_adjoint(e, k0sq, eps), n)
    assert torch.max(torch.abs(gh - g.conj().T)) < 1e-14


def test_green_inverts_reference_operator():
    # G L_eta = I with L_eta = -Laplacian - (k0^2 + i eps), built from numpy.fft.
    n, k0sq, eps = 8, 1.1, 0.3
    eye = np.eye(n * n).reshape(n * n, n, n)
    xi = 2 * math.pi * np.fft.fftfreq(n)
    xi2 = xi[:, None] ** 2 + xi[None, :] ** 2
    lap = np.fft.ifft2(np.fft.fft2(eye) * xi2).reshape(n * n, n * n).T
    l_eta = lap - (k0sq + 1j * eps) * np.eye(n * n)
    g = O.operator_matrix(lambda e: O.green(e, k0sq, eps), n).numpy()
    assert np.max(np.abs(g @ l_eta - np.eye(n * n))) < 1e-12
