"""FP64 CPU oracle for the Convergent-Born-Series (CBS) operator.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it and shares no code with it.

Everything is plain PyTorch CPU arithmetic in complex128, written to be read
against the paper:

  * 2D DFT by explicit DFT matrices with the phase index j*n reduced modulo N
    in exact integer arithmetic (no FFT library);
  * Fourier pseudospectral reference operator L_eta = -Laplacian - (k0^2 + i eta),
    symbol lambda_n = |xi_n|^2 - k0^2 - i eta, xi = 2 pi n / N,
    n in {-N/2, ..., N/2 - 1} (App. D, "Periodic grid and Fourier modes" and
    "Discrete symbol"; App. C, Helmholtz case);
  * Green operator G q = F^-1 (F q / lambda) (App. D, the three-step recipe);
  * potential V = k^2 - k0^2 - i eta (Sec. 3.1 coefficient-only split; App. D);
  * CBS fixed-point step u <- u + gamma (G (V u + s) - u)  (Sec. 3.1, Eq. CBS)
    with gamma = i V / eta (the paper only says gamma is derived from V;
    this is the Osnabrugge et al. 2016 choice cited there);
  * Born residual r = G (V u + s) - u = G (s - A u)  (Sec. 4.1, Eqs.
    npbs_integral and npbs_iter);
  * FGMRES (Saad 1993, cited in Sec. 5.1.3) on B u = G s with B = I - G V
    (Prop. 3.1) and a flexible right preconditioner of K CBS sweeps;
  * the metric-matched residual loss (Sec. 4.2) and its gradient by torch
    autograd through this forward;
  * the convection-diffusion-reaction operators G_cdr, V_cdr, A_cdr and the
    CDR metric-matched objective (App. B.1, Eqs. cdr_pde to cdr_bs_loss_eq).

Notation: the paper's eta is the damping called eps here.  Fields are
(N, N) arrays indexed [y, x].
"""
from __future__ import annotations

import functools
import math
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

CDT = torch.complex128
RDT = torch.float64


def as_c(x) -> torch.Tensor:
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(x)
    return torch.as_tensor(x).to(CDT)


# ---------------------------------------------------------------------------
# Grid, DFT and symbol (App. D)
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=32)
def dft_matrix(n: int) -> torch.Tensor:
    """F[j, k] = exp(-2 pi i ((j k) mod n) / n); the phase index is reduced
    exactly in integers before scaling."""
    j = torch.arange(n, dtype=torch.int64)
    e = (j[:, None] * j[None, :]) % n
    ang = (-2.0 * math.pi / n) * e.to(RDT)
    return torch.polar(torch.ones_like(ang), ang)


def dft2(x: torch.Tensor) -> torch.Tensor:
    """Unnormalised forward 2D DFT along both axes: F x F^T (F is symmetric)."""
    f = dft_matrix(x.shape[-1])
    return f @ x @ f


def idft2(x: torch.Tensor) -> torch.Tensor:
    """Inverse 2D DFT: conj(F)/N on both axes."""
    n = x.shape[-1]
    fi = dft_matrix(n).conj() / n
    return fi @ x @ fi


def mode_index(n: int) -> torch.Tensor:
    """Signed Fourier index for DFT bin k: k for k < N/2, k - N otherwise, so
    the Nyquist bin maps to -N/2 (App. D)."""
    k = torch.arange(n, dtype=torch.int64)
    return torch.where(k >= n // 2, k - n, k)


def xi_squared(n: int) -> torch.Tensor:
    """|xi_n|^2 on the (N, N) grid of DFT bins, xi = 2 pi n / N (h = 1)."""
    m = mode_index(n).to(RDT)
    xi = 2.0 * math.pi * m / n
    return xi[:, None] ** 2 + xi[None, :] ** 2


def symbol(n: int, k0sq: float, eps: float) -> torch.Tensor:
    """lambda_n = |xi_n|^2 - (k0^2 + i eps)."""
    return xi_squared(n).to(CDT) - complex(k0sq, eps)


def green(q: torch.Tensor, k0sq: float, eps: float) -> torch.Tensor:
    """G q = F^-1 (F q / lambda)."""
    return idft2(dft2(q) / symbol(q.shape[-1], k0sq, eps))


def green_adjoint(q: torch.Tensor, k0sq: float, eps: float) -> torch.Tensor:
    """G^H q = F^-1 (F q / conj(lambda))  (App. C: G = F^-1 Lambda^-1 F)."""
    return idft2(dft2(q) / symbol(q.shape[-1], k0sq, eps).conj())


def laplacian(u: torch.Tensor) -> torch.Tensor:
    """-Laplacian u = F^-1 (|xi|^2 F u)  (App. D, relation to A)."""
    return idft2(dft2(u) * xi_squared(u.shape[-1]).to(CDT))


# ---------------------------------------------------------------------------
# Potential, preconditioner and operators (Sec. 3.1, Sec. 4.1)
# ---------------------------------------------------------------------------

def potential(k2, k0sq: float, eps: float) -> torch.Tensor:
    """V = k^2 - k0^2 - i eps."""
    return as_c(k2) - complex(k0sq, eps)


def gamma(k2, k0sq: float, eps: float) -> torch.Tensor:
    """gamma = i V / eps."""
    return 1j * potential(k2, k0sq, eps) / eps


def choose_eps(k2, k0sq: float) -> float:
    """Damping rule used throughout: eps = max over cells of |k^2 - k0^2|
    (the smallest eps for which the CBS contraction argument holds)."""
    return float(torch.max(torch.abs(as_c(k2) - k0sq)))


def cbs_apply(k2, k0sq, eps, u, s=None) -> torch.Tensor:
    """y = G (V u + s)."""
    q = potential(k2, k0sq, eps) * as_c(u)
    if s is not None:
        q = q + as_c(s)
    return green(q, k0sq, eps)


def cbs_residual(k2, k0sq, eps, u, s=None, rhs=None) -> torch.Tensor:
    """Born residual r = G (V u + s) - u (+ rhs)."""
    r = cbs_apply(k2, k0sq, eps, u, s) - as_c(u)
    if rhs is not None:
        r = r + as_c(rhs)
    return r


def cbs_sweep(k2, k0sq, eps, u, s=None, rhs=None) -> torch.Tensor:
    """One CBS step u + gamma * r(u)."""
    return as_c(u) + gamma(k2, k0sq, eps) * cbs_residual(k2, k0sq, eps, u, s, rhs)


def helmholtz(k2, u) -> torch.Tensor:
    """A u = -Laplacian u - k^2 u (pseudospectral)."""
    return laplacian(as_c(u)) - as_c(k2) * as_c(u)


def physical_relres(k2, u, s) -> float:
    """Paper's stopping quantity rTol = ||s - A u|| / ||s||  (Sec. 5)."""
    s = as_c(s)
    return float(torch.linalg.vector_norm(s - helmholtz(k2, u)) / torch.linalg.vector_norm(s))


def norm(x) -> float:
    return float(torch.linalg.vector_norm(as_c(x)))


def born_relres(k2, k0sq, eps, u, s) -> float:
    """||G (V u + s) - u|| / ||G s||, the preconditioned relative residual."""
    return norm(cbs_residual(k2, k0sq, eps, u, s)) / norm(green(as_c(s), k0sq, eps))


# ---------------------------------------------------------------------------
# Stationary CBS (Sec. 3.1, Eq. CBS)
# ---------------------------------------------------------------------------

def cbs_iterate(k2, k0sq, eps, s, u0=None, max_sweeps: int = 2500, rtol: float = 1e-6,
                history: bool = False, stop: str = "born"):
    """Run u <- u + gamma r(u) from u0 (zeros by default) until the relative
    residual is at most rtol: stop="born" measures ||r(u_m)|| / ||G s||, the
    Born (preconditioned) residual; stop="physical" the paper's unified rule
    rTol = ||s - A u_m|| / ||s|| (Sec. 5).  Returns (u, sweeps, relres[,
    history]).  `sweeps` is the number of updates applied; relres is that of
    the returned u."""
    s = as_c(s)
    u = torch.zeros_like(s) if u0 is None else as_c(u0).clone()
    g = gamma(k2, k0sq, eps)
    if stop not in ("born", "physical"):
        raise ValueError(stop)
    bnorm = norm(green(s, k0sq, eps)) if stop == "born" else norm(s)
    hist = []
    m = 0
    while True:
        r = cbs_residual(k2, k0sq, eps, u, s)
        if stop == "born":
            rel = norm(r) / bnorm
        else:
            rel = norm(s - helmholtz(k2, u)) / bnorm
        hist.append(rel)
        if rel <= rtol or m >= max_sweeps or not math.isfinite(rel):
            break
        u = u + g * r
        m += 1
    if history:
        return u, m, rel, hist
    return u, m, rel


# ---------------------------------------------------------------------------
# Dirichlet problems: five-point FD on the unit square, DST-I reference
# (App. C "Newton linear systems for nonlinear PDEs"; App. B, Newton-Born)
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=32)
def dst1_matrix(n: int) -> torch.Tensor:
    """S[j, k] = sin(pi (j+1)(k+1) / (n+1)), j, k = 0..n-1 (the DST-I; S is
    symmetric and S^-1 = 2/(n+1) S)."""
    j = torch.arange(1, n + 1, dtype=torch.int64)
    e = (j[:, None] * j[None, :]) % (2 * (n + 1))
    return torch.sin(math.pi * e.to(RDT) / (n + 1)).to(CDT)


def dst2(x: torch.Tensor) -> torch.Tensor:
    """2D DST-I along both axes: S x S."""
    s = dst1_matrix(x.shape[-1])
    return s @ x @ s


def idst2(x: torch.Tensor) -> torch.Tensor:
    """Inverse 2D DST-I: (2/(n+1))^2 S x S."""
    n = x.shape[-1]
    return (2.0 / (n + 1)) ** 2 * dst2(x)


def dirichlet_eigs(n: int) -> torch.Tensor:
    """Eigenvalues of the five-point negative Laplacian with h = 1/(n+1) on
    DST bins (p, q) = 1..n: 4/h^2 (sin^2(p pi h/2) + sin^2(q pi h/2))."""
    h = 1.0 / (n + 1)
    p = torch.arange(1, n + 1, dtype=RDT)
    m = 4.0 / h ** 2 * torch.sin(p * math.pi * h / 2) ** 2
    return m[:, None] + m[None, :]


def green_dirichlet(q, k0sq: float, eps: float) -> torch.Tensor:
    """G q = S^-1 (S q / lambda), lambda = eigs - k0^2 - i eps."""
    q = as_c(q)
    lam = dirichlet_eigs(q.shape[-1]).to(CDT) - complex(k0sq, eps)
    return idst2(dst2(q) / lam)


def green_adjoint_dirichlet(q, k0sq: float, eps: float) -> torch.Tensor:
    """G^H q = S^-1 (S q / conj(lambda)) (S^-1 S real symmetric up to scale)."""
    q = as_c(q)
    lam = dirichlet_eigs(q.shape[-1]).to(CDT) - complex(k0sq, eps)
    return idst2(dst2(q) / lam.conj())


def laplacian_dirichlet(u) -> torch.Tensor:
    """Five-point negative Laplacian with zero boundary values, h = 1/(n+1):
    (4 u_ij - u_i-1,j - u_i+1,j - u_i,j-1 - u_i,j+1) / h^2."""
    u = as_c(u)
    n = u.shape[-1]
    z = torch.zeros(n + 2, n + 2, dtype=CDT)
    z[1:-1, 1:-1] = u
    return (4 * u - z[:-2, 1:-1] - z[2:, 1:-1] - z[1:-1, :-2] - z[1:-1, 2:]) * (n + 1) ** 2


def cbs_residual_dirichlet(k2, k0sq, eps, u, s=None) -> torch.Tensor:
    """Born residual G (V u + s) - u with the Dirichlet G (V as in Sec. 3.1)."""
    q = potential(k2, k0sq, eps) * as_c(u)
    if s is not None:
        q = q + as_c(s)
    return green_dirichlet(q, k0sq, eps) - as_c(u)


def cbs_sweep_dirichlet(k2, k0sq, eps, u, s=None) -> torch.Tensor:
    return as_c(u) + gamma(k2, k0sq, eps) * cbs_residual_dirichlet(k2, k0sq, eps, u, s)


def helmholtz_dirichlet(k2, u) -> torch.Tensor:
    """A u = L_D u - k^2 u (a Newton Jacobian J = L_D - 2 diag(u_m) is k^2 = 2 u_m)."""
    return laplacian_dirichlet(u) - as_c(k2) * as_c(u)


def cbs_iterate_dirichlet(k2, k0sq, eps, s, max_sweeps: int = 2500, rtol: float = 1e-6):
    """Stationary CBS with the Dirichlet G until ||r|| / ||G s|| <= rtol."""
    s = as_c(s)
    u = torch.zeros_like(s)
    g = gamma(k2, k0sq, eps)
    bnorm = norm(green_dirichlet(s, k0sq, eps))
    m = 0
    while True:
        r = cbs_residual_dirichlet(k2, k0sq, eps, u, s)
        rel = norm(r) / bnorm
        if rel <= rtol or m >= max_sweeps or not math.isfinite(rel):
            return u, m, rel
        u = u + g * r
        m += 1


# ---------------------------------------------------------------------------
# Convection-diffusion-reaction (App. B.1, Eqs. cdr_pde to cdr_G_symbol;
# App. C, "CDR case", restates the symbol)
# ---------------------------------------------------------------------------
#
# L_cdr u = -div(kappa grad u) + v . grad u + sigma u with constant background
# kappa0, v0 = (vx0, vy0), sigma0; L0 = -kappa0 Lap + v0 . grad + sigma0 and
# V_cdr = L0 - L_cdr = div(dkappa grad) - dv . grad - dsigma.  On the
# periodic grid every derivative is spectral: d/dx = F^-1 diag(i xi_x) F with
# xi = 2 pi m / N on the signed index m of mode_index (Nyquist bin -N/2, as
# for |xi|^2).  x is the second (column) axis of an (N, N) field, y the first.

class CdrMedium:
    """Coefficient fields (real (N, N) arrays) and background constants."""

    def __init__(self, kappa, vx, vy, sigma, kappa0: float, vx0: float, vy0: float, sigma0: float):
        self.kappa = torch.as_tensor(np.asarray(kappa), dtype=RDT)
        self.vx = torch.as_tensor(np.asarray(vx), dtype=RDT)
        self.vy = torch.as_tensor(np.asarray(vy), dtype=RDT)
        self.sigma = torch.as_tensor(np.asarray(sigma), dtype=RDT)
        self.kappa0, self.vx0, self.vy0, self.sigma0 = float(kappa0), float(vx0), float(vy0), float(sigma0)

    @property
    def n(self) -> int:
        return self.kappa.shape[-1]


def wavenumbers(n: int) -> torch.Tensor:
    """xi = 2 pi m / N for DFT bin k, m = mode_index(k)."""
    return 2.0 * math.pi * mode_index(n).to(RDT) / n


def deriv_x(u) -> torch.Tensor:
    """Spectral d/dx (along the second axis): F^-1 (i xi_x F u)."""
    u = as_c(u)
    xi = wavenumbers(u.shape[-1]).to(CDT)
    return idft2(dft2(u) * (1j * xi)[None, :])


def deriv_y(u) -> torch.Tensor:
    """Spectral d/dy (along the first axis): F^-1 (i xi_y F u)."""
    u = as_c(u)
    xi = wavenumbers(u.shape[-1]).to(CDT)
    return idft2(dft2(u) * (1j * xi)[:, None])


def cdr_symbol(m: CdrMedium) -> torch.Tensor:
    """L0 on DFT bin (ky, kx): kappa0 |xi|^2 + i v0 . xi + sigma0 (Eq. cdr_G_symbol's denominator)."""
    xi = wavenumbers(m.n)
    xx, yy = xi[None, :], xi[:, None]
    return (m.kappa0 * (xx ** 2 + yy ** 2) + m.sigma0).to(CDT) + 1j * (m.vx0 * xx + m.vy0 * yy).to(CDT)


def green_cdr(q, m: CdrMedium) -> torch.Tensor:
    """G_cdr q = F^-1 (F q / L0(xi))  (Eq. cdr_G_symbol)."""
    return idft2(dft2(as_c(q)) / cdr_symbol(m))


def green_cdr_adjoint(q, m: CdrMedium) -> torch.Tensor:
    """G_cdr^H q = F^-1 (F q / conj(L0(xi)))."""
    return idft2(dft2(as_c(q)) / cdr_symbol(m).conj())


def cdr_reference(u, m: CdrMedium) -> torch.Tensor:
    """L0 u = -kappa0 Lap u + v0 . grad u + sigma0 u  (Eq. cdr_L0)."""
    u = as_c(u)
    return -m.kappa0 * (deriv_x(deriv_x(u)) + deriv_y(deriv_y(u))) \
        + m.vx0 * deriv_x(u) + m.vy0 * deriv_y(u) + m.sigma0 * u


def cdr_potential(u, m: CdrMedium) -> torch.Tensor:
    """V_cdr u = div(dkappa grad u) - dv . grad u - dsigma u  (Eq. cdr_V)."""
    u = as_c(u)
    dk = (m.kappa - m.kappa0).to(CDT)
    dvx, dvy = (m.vx - m.vx0).to(CDT), (m.vy - m.vy0).to(CDT)
    ds = (m.sigma - m.sigma0).to(CDT)
    ux, uy = deriv_x(u), deriv_y(u)
    return deriv_x(dk * ux) + deriv_y(dk * uy) - (dvx * ux + dvy * uy) - ds * u


def cdr_operator(u, m: CdrMedium) -> torch.Tensor:
    """A_cdr u = -div(kappa grad u) + v . grad u + sigma u  (Eq. cdr_pde),
    written from the PDE itself, not as L0 - V."""
    u = as_c(u)
    ux, uy = deriv_x(u), deriv_y(u)
    k = m.kappa.to(CDT)
    return -(deriv_x(k * ux) + deriv_y(k * uy)) + m.vx.to(CDT) * ux + m.vy.to(CDT) * uy \
        + m.sigma.to(CDT) * u


def cdr_apply(m: CdrMedium, u, s=None) -> torch.Tensor:
    """G_cdr (V_cdr u + s)."""
    q = cdr_potential(u, m)
    if s is not None:
        q = q + as_c(s)
    return green_cdr(q, m)


def cdr_residual(m: CdrMedium, u, s=None, rhs=None) -> torch.Tensor:
    """Born residual G_cdr (V_cdr u + s) - u (+ rhs) = G_cdr (s - A_cdr u) (+ rhs)
    (Eq. cdr_integral)."""
    r = cdr_apply(m, u, s) - as_c(u)
    if rhs is not None:
        r = r + as_c(rhs)
    return r


def cdr_physical_residual(m: CdrMedium, u, s) -> torch.Tensor:
    """s - A_cdr u."""
    return as_c(s) - cdr_operator(u, m)


def cdr_born_operator(m: CdrMedium, x) -> torch.Tensor:
    """R x = (I - G_cdr V_cdr) x  (Eq. cdr_identity)."""
    return as_c(x) - green_cdr(cdr_potential(x, m), m)


def cdr_born_adjoint(m: CdrMedium, e) -> torch.Tensor:
    """R^H e by reverse-mode autograd through R: the gradient (PyTorch's
    convention d/dRe + i d/dIm) of Re <e, R x> with respect to x."""
    e = as_c(e)
    x = torch.zeros_like(e).requires_grad_(True)
    val = torch.sum((e.conj() * cdr_born_operator(m, x)).real)
    (g,) = torch.autograd.grad(val, x)
    return g


def cdr_loss(m: CdrMedium, x, r) -> torch.Tensor:
    """|| G_cdr r - (I - G_cdr V_cdr) x ||^2, the residual of the metric-matched
    objective L_bs^{R_cdr} (Eq. cdr_bs_loss) for a network output x = M(G r)."""
    d = green_cdr(as_c(r), m) - cdr_born_operator(m, x)
    return torch.sum(d.real ** 2 + d.imag ** 2)


def cdr_loss_and_grad(m: CdrMedium, x, r):
    """(loss, dl/dx) by autograd, PyTorch's complex-gradient convention."""
    xt = as_c(x).clone().requires_grad_(True)
    val = cdr_loss(m, xt, r)
    (g,) = torch.autograd.grad(val, xt)
    return float(val.detach()), g


# ---------------------------------------------------------------------------
# NPBS step with a linear Fourier-layer preconditioner (Sec. 4.1; App. E)
# ---------------------------------------------------------------------------

def linear_fourier_layer(x, wf, wloc) -> torch.Tensor:
    """M(x) = F^-1 (W^F * F x) + W^loc * x: the linear Fourier layer LFL of
    App. E (Eq. lfl) on one complex channel, with spectral weights wf on the
    (N, N) grid of DFT bins and local weights wloc (a scalar or an (N, N)
    field; per cell it also stands for the fixed coefficient-branch factor
    that multiplies the residual branch in Eq. fno_impl)."""
    x = as_c(x)
    return idft2(as_c(wf) * dft2(x)) + as_c(wloc) * x


def npbs_step(k2, k0sq, eps, u, s, wf, wloc) -> torch.Tensor:
    """u + M(G (V u + s) - u) with M the linear Fourier layer (Sec. 4.1,
    Eq. npbs_integral)."""
    return as_c(u) + linear_fourier_layer(cbs_residual(k2, k0sq, eps, u, s), wf, wloc)


# ---------------------------------------------------------------------------
# Dense matrices for tiny grids (brute force pins)
# ---------------------------------------------------------------------------

def operator_matrix(fn: Callable[[torch.Tensor], torch.Tensor], n: int) -> torch.Tensor:
    """Dense (n^2, n^2) matrix of a linear map on (n, n) fields (row-major)."""
    eye = torch.eye(n * n, dtype=CDT).reshape(n * n, n, n)
    cols = fn(eye).reshape(n * n, n * n)     # row c = fn(e_c)
    return cols.T.contiguous()


def dense_solve(k2, s) -> torch.Tensor:
    """Exact solution of the pseudospectral system A u = s by LAPACK."""
    s = as_c(s)
    n = s.shape[-1]
    a = operator_matrix(lambda e: helmholtz(k2, e), n)
    return torch.linalg.solve(a, s.reshape(-1)).reshape(n, n)


# ---------------------------------------------------------------------------
# FGMRES on the Born-preconditioned system (Sec. 5.1.3; Saad 1993)
# ---------------------------------------------------------------------------

def born_operator(k2, k0sq, eps, x) -> torch.Tensor:
    """B x = x - G (V x) = G A x  (Prop. 3.1)."""
    return as_c(x) - cbs_apply(k2, k0sq, eps, x)


def cbs_precondition(k2, k0sq, eps, v, sweeps: int) -> torch.Tensor:
    """P_K(v): K CBS sweeps z <- z + gamma (G V z + v - z) from z = 0, an
    approximate inverse of B (K = 1 gives z = gamma v).  K = 0 stands for no
    inner preconditioner, P_0 = I (GMRES on B itself)."""
    if sweeps == 0:
        return as_c(v).clone()
    z = torch.zeros_like(as_c(v))
    for _ in range(sweeps):
        z = cbs_sweep(k2, k0sq, eps, z, None, v)
    return z


def _inner(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return torch.sum(a.conj() * b)


def fgmres(k2, k0sq, eps, s, x0=None, restart: int = 30, sweeps: int = 4,
           max_iters: int = 2500, rtol: float = 1e-6, history: bool = False):
    """Flexible GMRES(m) for B x = b, b = G s, right-preconditioned by P_K.

    Classical Gram-Schmidt applied twice (CGS2).  The small least-squares
    problem min ||beta e1 - H y|| is solved with LAPACK at every step (the
    definition; no Givens recurrence).  Returns (x, iterations, relres)
    where relres = ||b - B x|| / ||b|| of the returned x."""
    s = as_c(s)
    b = green(s, k0sq, eps)
    bnorm = norm(b)
    x = torch.zeros_like(s) if x0 is None else as_c(x0).clone()
    its = 0
    hist = []
    while True:
        r = b - born_operator(k2, k0sq, eps, x)
        beta = norm(r)
        rel = beta / bnorm
        hist.append(rel)
        if rel <= rtol or its >= max_iters:
            break
        vs = [r / beta]
        zs = []
        h = torch.zeros(restart + 1, restart, dtype=CDT)
        y = None
        for j in range(restart):
            z = cbs_precondition(k2, k0sq, eps, vs[j], sweeps)
            zs.append(z)
            w = born_operator(k2, k0sq, eps, z)
            for _ in range(2):
                coef = torch.stack([_inner(v, w) for v in vs])
                for i, v in enumerate(vs):
                    w = w - coef[i] * v
                h[: j + 1, j] += coef
            hn = norm(w)
            h[j + 1, j] = hn
            its += 1
            rhs = torch.zeros(j + 2, dtype=CDT)
            rhs[0] = beta
            y = torch.linalg.lstsq(h[: j + 2, : j + 1], rhs.unsqueeze(1)).solution.squeeze(1)
            est = norm(rhs - h[: j + 2, : j + 1] @ y) / bnorm
            hist.append(est)
            if est <= rtol or its >= max_iters or hn == 0.0:
                break
            vs.append(w / hn)
        for i in range(len(y)):
            x = x + y[i] * zs[i]
    if history:
        return x, its, rel, hist
    return x, its, rel


# ---------------------------------------------------------------------------
# Metric-matched loss and its gradient (Sec. 4.2)
# ---------------------------------------------------------------------------

def unrolled_loss(k2, k0sq, eps, u0, s, steps: int, weight: str = "gamma",
                  bc: str = "periodic") -> torch.Tensor:
    """ell = || W * (G s - (I - G V) u_K) ||^2 with u_{m+1} = u_m + gamma r(u_m).

    weight "gamma" uses W = gamma; "one" uses W = 1 (the residual of the
    metric-matched loss L_bs^{R_eta}, Sec. 4.2); "physical" measures the
    unpreconditioned residual instead, ell = || s - A u_K ||^2 (the residual
    of L_dir, Sec. 4, and of L_bs^{l2}, Sec. 4.2).  The ratio forms of these
    losses divide by ||G s||^2 or ||s||^2, constants the caller applies.
    eps and k0^2 are constants; k2 and u0 may require grad.
    bc="dirichlet" uses the five-point Dirichlet operators instead (the
    Newton-state instance of the metric-matched loss, App. B Eq. nl_bs_loss,
    with k^2 = 2 u_m).
    """
    if bc == "periodic":
        sweep, resid, hel = cbs_sweep, cbs_residual, helmholtz
    elif bc == "dirichlet":
        sweep, resid, hel = cbs_sweep_dirichlet, cbs_residual_dirichlet, helmholtz_dirichlet
    else:
        raise ValueError(bc)
    u = as_c(u0) if not torch.is_tensor(u0) else u0
    for _ in range(steps):
        u = sweep(k2, k0sq, eps, u, s)
    if weight == "physical":
        r = as_c(s) - hel(k2, u)
    else:
        r = resid(k2, k0sq, eps, u, s)
        if weight == "gamma":
            r = gamma(k2, k0sq, eps) * r
        elif weight != "one":
            raise ValueError(weight)
    return torch.sum(r.real ** 2 + r.imag ** 2)


def loss_and_grad(k2, k0sq, eps, u0, s, steps: int, weight: str = "gamma", bc: str = "periodic"):
    """Returns (loss, dl/du0, dl/dk2) with PyTorch's complex-gradient
    convention dl/dRe + i dl/dIm, computed by autograd through the oracle."""
    k2t = as_c(k2).clone().requires_grad_(True)
    u0t = as_c(u0).clone().requires_grad_(True)
    val = unrolled_loss(k2t, k0sq, eps, u0t, as_c(s), steps, weight, bc=bc)
    gu, gk = torch.autograd.grad(val, (u0t, k2t))
    return float(val.detach()), gu, gk
