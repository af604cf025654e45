"""Pins of the oracle's loss gradient: central finite differences,
torch.autograd.gradcheck, and the closed-form adjoint recursion that the GPU
implements (derived from the CBS step, Sec. 3.1, and the metric-matched
residual, Sec. 4.2)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S


def _problem(n=8, layer=2, seed=0):
    rng = np.random.default_rng(seed)
    c = S.minmax_map(S.gaussian_random_field(n, 2.0, rng), 1.0, 2.0)
    p = S.velocity_problem(c, layer, 5.0, S.random_field_c(n, rng), cmin=1.0)
    u0 = S.random_field_c(n, rng)
    return p, u0


def _dirichlet_problem(n=7, seed=0):
    # Newton-type Jacobian J = L_D - 2 diag(u_m): k^2 = 2 u_m real and smooth
    rng = np.random.default_rng(seed)
    k2 = (100.0 + 60.0 * S.gaussian_random_field(n, 2.0, rng)).astype(np.complex128)
    p = S.Problem(n=n, layer=0, k2=k2, k0sq=float(0.5 * (k2.real.min() + k2.real.max())),
                  source=S.random_field_c(n, rng))
    return p, S.random_field_c(n, rng)


@pytest.mark.parametrize("weight,bc", [("gamma", "periodic"), ("one", "periodic"),
                                       ("physical", "periodic"), ("one", "dirichlet"),
                                       ("physical", "dirichlet")])
def test_loss_gradient_central_differences(weight, bc):
    # P11: central differences with h = 1e-3 on Re/Im u0 and Re/Im k^2.  The
    # loss is a high-degree polynomial in k^2, so the plain O(h^2) truncation
    # is ~1e-5 relative; Richardson extrapolation of D(h) and D(h/2) removes it
    # and the two then agree to ~1e-9.
    p, u0 = _problem() if bc == "periodic" else _dirichlet_problem()
    eps = O.choose_eps(p.k2, p.k0sq)
    steps = 3
    val, gu, gk = O.loss_and_grad(p.k2, p.k0sq, eps, u0, p.source, steps, weight, bc)
    h = 1e-3
    rng = np.random.default_rng(1)

    def central(fn, base, y, x, unit, hh):
        d = np.zeros_like(base)
        d[y, x] = unit * hh
        return (float(fn(base + d)) - float(fn(base - d))) / (2 * hh)

    f_u = lambda u: O.unrolled_loss(p.k2, p.k0sq, eps, u, p.source, steps, weight, bc=bc)
    f_k = lambda k: O.unrolled_loss(k, p.k0sq, eps, u0, p.source, steps, weight, bc=bc)
    for _ in range(6):
        y, x = rng.integers(0, p.n, size=2)
        for unit in (1.0, 1j):
            for fn, base, grad in ((f_u, u0, gu), (f_k, p.k2, gk)):
                d1 = central(fn, base, y, x, unit, h)
                d2 = central(fn, base, y, x, unit, h / 2)
                an = float(grad[y, x].real if unit == 1.0 else grad[y, x].imag)
                scale = max(1.0, abs(an))
                assert abs(d1 - an) <= 2e-4 * scale          # O(h^2) truncation
                assert abs((4 * d2 - d1) / 3 - an) <= 1e-8 * scale


def test_gradcheck_tiny():
    p, u0 = _problem(n=6, layer=1, seed=3)
    eps = O.choose_eps(p.k2, p.k0sq)
    k2 = O.as_c(p.k2).clone().requires_grad_(True)
    u = O.as_c(u0).clone().requires_grad_(True)
    s = O.as_c(p.source)
    assert torch.autograd.gradcheck(lambda a, b: O.unrolled_loss(a, p.k0sq, eps, b, s, 2, "gamma"),
                                    (k2, u), eps=1e-6, atol=1e-7, rtol=1e-5)


def adjoint_recursion(k2, k0sq, eps, u0, s, steps, weight="gamma"):
    """Closed-form reverse sweep (PyTorch convention grad = dRe + i dIm).

    Forward: u_{m+1} = u_m + g r_m, r_m = G(V u_m + s) - u_m, loss |W r_K|^2.
    Reverse: with seed mu = 2 W r_K, lam_K = (conj(V) G^H - I)(conj(W) mu);
    lam_m = lam_{m+1} + conj(V) G^H(conj(g) lam_{m+1}) - conj(g) lam_{m+1};
    dk2 += (-i/eps) lam_{m+1} conj(r_m) + G^H(conj(g) lam_{m+1}) conj(u_m),
    plus (-i/eps) mu conj(r_K) + G^H(conj(g) mu) conj(u_K) for W = gamma.
    For the physical loss |s - A u_K|^2 only the seed differs (see below).
    """
    v = O.potential(k2, k0sq, eps)
    g = O.gamma(k2, k0sq, eps)
    us = [O.as_c(u0)]
    for _ in range(steps):
        us.append(O.cbs_sweep(k2, k0sq, eps, us[-1], s))
    if weight == "physical":
        # loss |e|^2, e = s - A u_K: lam_K = -2 A^H e with A^H e = -Lap e -
        # conj(k^2) e, and dk2 = 2 conj(u_K) e (A depends on k^2 through -k^2 u)
        e = O.as_c(s) - O.helmholtz(k2, us[-1])
        lam = -2 * (O.laplacian(e) - O.as_c(k2).conj() * e)
        dk = 2 * us[-1].conj() * e
    else:
        rk = O.cbs_residual(k2, k0sq, eps, us[-1], s)
        w = g if weight == "gamma" else torch.ones_like(g)
        mu = 2 * w * rk
        gr = w.conj() * mu
        lam = v.conj() * O.green_adjoint(gr, k0sq, eps) - gr
        dk = (v.conj() * 0)
        dk = dk + O.green_adjoint(gr, k0sq, eps) * us[-1].conj()
        if weight == "gamma":
            dk = dk + (-1j / eps) * mu * rk.conj()
    for m in range(steps - 1, -1, -1):
        rm = O.cbs_residual(k2, k0sq, eps, us[m], s)
        t = O.green_adjoint(g.conj() * lam, k0sq, eps)
        dk = dk + (-1j / eps) * lam * rm.conj() + t * us[m].conj()
        lam = lam + v.conj() * t - g.conj() * lam
    return lam, dk


@pytest.mark.parametrize("weight", ["gamma", "one", "physical"])
def test_adjoint_recursion_matches_autograd(weight):
    # The hand-written reverse recursion (implemented by the GPU adjoint) equals
    # the oracle's autograd gradient at 32x32, K = 8.
    p, u0 = _problem(n=32, layer=4, seed=5)
    eps = O.choose_eps(p.k2, p.k0sq)
    val, gu, gk = O.loss_and_grad(p.k2, p.k0sq, eps, u0, p.source, 8, weight)
    lam, dk = adjoint_recursion(p.k2, p.k0sq, eps, u0, O.as_c(p.source), 8, weight)
    assert torch.max(torch.abs(lam - gu)) <= 1e-12 * torch.max(torch.abs(gu))
    assert torch.max(torch.abs(dk - gk)) <= 1e-12 * torch.max(torch.abs(gk))
