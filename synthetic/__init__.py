"""Seeded synthetic Helmholtz problems (media and sources).

This module is the only code shared by the FP64 oracle and the GPU path, and
it holds none of the method's arithmetic: it draws random numbers and builds
input fields (squared wavenumber k(x)^2 with an absorbing sponge, and a source
field).  No Green operator, potential, preconditioner or iteration lives here.

The paper evaluates on OpenFWI velocity models (CurveVel-A, CurveFault-B:
256x256 interior, a 32-cell absorbing layer, velocities 1500-4500 m/s,
12 points per wavelength; Sec. 5.1 and App. G.1).  Those datasets are not
available, so the generators below produce stand-ins with the same shapes and
value ranges: Gaussian random-field velocities, layered media, Gaussian blobs.
Velocities are in km/s-like units (1.5-4.5) and the grid spacing is one cell.

Conventions (Sec. 3.1, App. D):
  * the grid is the full periodic FFT grid of N x N cells, rows = y, cols = x;
  * the outer L cells on every side form the absorbing layer, the interior is
    (N - 2L)^2 cells;
  * k(x) = omega / c(x); in the layer the real part of k^2 is copied from the
    nearest interior cell and the imaginary part grows as a * t^2 with t the
    normalised depth into the layer (a sponge; the paper names sponge layers
    or PML without a profile, Sec. 3.1);
  * a = 0.5 * max over the interior of |k^2 - k0^2|, which keeps every cell's
    |V| at least half of the damping eps used by the CBS preconditioner.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SIZES_RAGGED = (128, 192, 256, 384, 512)


@dataclasses.dataclass
class Problem:
    """One Helmholtz instance: A u = s with A = -Laplacian - k2 on an n x n grid."""

    n: int
    layer: int
    k2: np.ndarray          # complex128 (n, n): squared wavenumber incl. sponge
    k0sq: float             # reference squared wavenumber k0^2
    source: np.ndarray      # complex128 (n, n)
    omega: float = float("nan")
    meta: dict = dataclasses.field(default_factory=dict)


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    """Seed rule: seed = 1000 * config + instance, NumPy PCG64."""
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


def gaussian_random_field(n: int, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field with covariance ~ exp(-r^2 / (2 ell^2)).

    White noise filtered by exp(-|xi|^2 ell^2 / 4) in Fourier space.  Uses
    numpy.fft purely as a filter for input generation.
    """
    w = rng.standard_normal((n, n))
    xi = 2.0 * math.pi * np.fft.fftfreq(n)
    filt = np.exp(-(xi[:, None] ** 2 + xi[None, :] ** 2) * ell * ell / 4.0)
    return np.real(np.fft.ifft2(np.fft.fft2(w) * filt))


def minmax_map(g: np.ndarray, lo: float, hi: float) -> np.ndarray:
    gmin, gmax = float(g.min()), float(g.max())
    return lo + (g - gmin) / (gmax - gmin) * (hi - lo)


def interior_slice(n: int, layer: int):
    return slice(layer, n - layer)


def apply_sponge(k2_real: np.ndarray, layer: int, k0sq: float) -> np.ndarray:
    """Complex k^2 with a quadratic sponge in the outer `layer` cells.

    k2_real only needs valid values on the interior; the layer's real part is
    replaced by the nearest interior value.
    """
    n = k2_real.shape[0]
    if layer == 0:
        return k2_real.astype(np.complex128)
    idx = np.clip(np.arange(n), layer, n - layer - 1)
    re = k2_real[np.ix_(idx, idx)].astype(np.float64)
    i = np.arange(n)
    depth = np.maximum(np.maximum(layer - i, i - (n - layer - 1)), 0) / float(layer)
    t = np.maximum(depth[:, None], depth[None, :])
    interior = re[layer:n - layer, layer:n - layer]
    a = 0.5 * float(np.max(np.abs(interior - k0sq)))
    return re + 1j * a * t * t


def point_source(n: int, at) -> np.ndarray:
    s = np.zeros((n, n), np.complex128)
    s[at[0], at[1]] = 1.0
    return s


def gaussian_pulse(n: int, at, sigma: float) -> np.ndarray:
    y = np.arange(n)[:, None] - at[0]
    x = np.arange(n)[None, :] - at[1]
    return np.exp(-(x * x + y * y) / (2.0 * sigma * sigma)).astype(np.complex128)


def midpoint_k0sq(k2: np.ndarray, layer: int) -> float:
    """k0^2 = midpoint of the interior range of Re k^2 (a reading; the paper
    tunes its reference per dataset)."""
    n = k2.shape[0]
    sl = interior_slice(n, layer)
    re = np.real(k2[sl, sl])
    return 0.5 * (float(re.min()) + float(re.max()))


def velocity_problem(c: np.ndarray, layer: int, ppw: float, source: np.ndarray,
                     cmin: Optional[float] = None, meta: Optional[dict] = None) -> Problem:
    """k = omega / c with omega chosen so the shortest wavelength spans ppw cells."""
    n = c.shape[0]
    sl = interior_slice(n, layer)
    if cmin is None:
        cmin = float(c[sl, sl].min())
    omega = 2.0 * math.pi * cmin / ppw
    k2r = (omega / c) ** 2
    re = k2r[sl, sl]
    k0sq = 0.5 * (float(re.min()) + float(re.max()))
    k2 = apply_sponge(k2r, layer, k0sq)
    m = dict(meta or {})
    m.update(ppw=ppw)
    return Problem(n=n, layer=layer, k2=k2, k0sq=k0sq, source=source, omega=omega, meta=m)


# --------------------------------------------------------------------------
# The five workloads.  Each returns a list of Problem.
# --------------------------------------------------------------------------

def blob_problem(n: int = 64, layer: int = 16, seed_config: int = 1) -> Problem:
    """64x64 grid, 16-cell layer, k0 = 2 pi / 8, k^2 = k0^2 (1 + 0.5 g) with g a
    Gaussian blob (sigma 8 cells) at a seeded interior cell; point source at
    the grid centre."""
    rng = rng_for(seed_config, 0)
    k0 = 2.0 * math.pi / 8.0
    k0sq = k0 * k0
    cb = rng.integers(layer, n - layer, size=2)
    y = np.arange(n)[:, None] - cb[0]
    x = np.arange(n)[None, :] - cb[1]
    g = np.exp(-(x * x + y * y) / (2.0 * 8.0 ** 2))
    k2r = k0sq * (1.0 + 0.5 * g)
    k2 = apply_sponge(k2r, layer, k0sq)
    src = point_source(n, (n // 2, n // 2))
    return Problem(n=n, layer=layer, k2=k2, k0sq=k0sq, source=src, omega=k0,
                   meta=dict(config="blob64", blob_centre=tuple(int(v) for v in cb)))


def grf_problem(n: int = 256, layer: int = 32, seed_config: int = 2, instance: int = 0,
                cmax: float = 3.0, ppw: float = 10.0, ell: float = 16.0,
                pulse_sigma: Optional[float] = 2.0) -> Problem:
    """Random-field medium c in [1, cmax], omega for `ppw` cells per shortest
    wavelength; Gaussian pulse (or point source if pulse_sigma is None) at a
    seeded interior cell."""
    rng = rng_for(seed_config, instance)
    c = minmax_map(gaussian_random_field(n, ell, rng), 1.0, cmax)
    margin = layer + 4
    at = rng.integers(margin, n - margin, size=2)
    if pulse_sigma is None:
        src = point_source(n, at)
    else:
        src = gaussian_pulse(n, at, pulse_sigma)
    return velocity_problem(c, layer, ppw, src, cmin=1.0,
                            meta=dict(config=f"grf{n}", source_at=tuple(int(v) for v in at),
                                      cmax=cmax, seed=1000 * seed_config + instance))


def ragged_batch(count: int = 64, seed_config: int = 3, layer: int = 32,
                 sizes=SIZES_RAGGED) -> List[Problem]:
    """Ragged batch: N drawn uniformly from `sizes`, 6-12 points per wavelength,
    contrast 1.5-4, random-field media (correlation 16 cells), seeded interior
    point sources."""
    out = []
    for i in range(count):
        rng = rng_for(seed_config, i)
        n = int(rng.choice(np.asarray(sizes)))
        ppw = float(rng.uniform(6.0, 12.0))
        contrast = float(rng.uniform(1.5, 4.0))
        c = minmax_map(gaussian_random_field(n, 16.0, rng), 1.0, contrast)
        at = rng.integers(layer + 4, n - layer - 4, size=2)
        out.append(velocity_problem(c, layer, ppw, point_source(n, at), cmin=1.0,
                                    meta=dict(config="ragged", index=i, contrast=contrast,
                                              source_at=tuple(int(v) for v in at))))
    return out


def diff_batch(count: int = 16, n: int = 256, layer: int = 32, seed_config: int = 4):
    """Differentiation workload: random-field media with contrast 2 at 10
    points per wavelength; returns (problems, u0, s) with u0 and s drawn from a
    circular complex normal distribution (the paper's N(0, I) probes, Sec. 4)."""
    probs, u0s, ss = [], [], []
    for i in range(count):
        rng = rng_for(seed_config, i)
        c = minmax_map(gaussian_random_field(n, 16.0, rng), 1.0, 2.0)
        u0 = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
        s = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
        probs.append(velocity_problem(c, layer, 10.0, s, cmin=1.0,
                                      meta=dict(config="diff", index=i)))
        u0s.append(u0)
        ss.append(s)
    return probs, u0s, ss


def layered_batch(count: int = 8, n: int = 1024, layer: int = 64, seed_config: int = 5,
                  ppw: float = 8.0) -> List[Problem]:
    """High-wavenumber stress case: five horizontal layers with velocities in
    [1.5, 4.5] times (1 + 0.1 zeta), zeta a unit-variance random field
    (correlation 16 cells), the factor clipped at >= 0.75; 8 points per
    shortest wavelength; seeded interior point source."""
    out = []
    for i in range(count):
        rng = rng_for(seed_config, i)
        vel = rng.uniform(1.5, 4.5, size=5)
        rows = np.arange(n)
        band = np.clip(((rows - layer) * 5) // max(n - 2 * layer, 1), 0, 4)
        zeta = gaussian_random_field(n, 16.0, rng)
        zeta = (zeta - zeta.mean()) / zeta.std()
        c = vel[band][:, None] * np.maximum(1.0 + 0.1 * zeta, 0.75)
        at = rng.integers(layer + 4, n - layer - 4, size=2)
        out.append(velocity_problem(c, layer, ppw, point_source(n, at),
                                    meta=dict(config="layered", index=i,
                                              velocities=[float(v) for v in vel],
                                              source_at=tuple(int(v) for v in at))))
    return out


def homogeneous_lossy(n: int, k0sq: float, kappa: float, source: np.ndarray) -> Problem:
    """Periodic homogeneous lossy medium k^2 = k0^2 + i kappa (no layer)."""
    k2 = np.full((n, n), k0sq + 1j * kappa, np.complex128)
    return Problem(n=n, layer=0, k2=k2, k0sq=k0sq, source=source,
                   meta=dict(config="homogeneous_lossy", kappa=kappa))


def random_field_c(n: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Circular complex normal field (for probes and random operands)."""
    return scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)


def newton_batch(count: int = 100, n: int = 64, seed_config: int = 6, amplitude: float = 4.0,
                 level: float = 40.0):
    """Linearised Newton systems of -Lap u - u^2 - f = 0 on the unit square
    (App. B, App. F): Jacobians J = L_D - 2 diag(u_m) on n x n interior points
    with homogeneous Dirichlet boundaries, as Problems with k^2 = 2 u_m and the
    right-hand side r as source.  No Newton trajectories are available, so u_m
    is a smooth state built like the paper's perturbed initial guesses:
    level + amplitude * sum_{i,j<=4} c_ij sin(i pi x) sin(j pi y),
    c_ij ~ N(0, 0.1^2); r is a circular complex normal probe.  n = 64 is the
    paper's grid of interior points."""
    out = []
    x = np.arange(1, n + 1) / (n + 1)
    basis = [np.outer(np.sin((i + 1) * math.pi * x), np.sin((j + 1) * math.pi * x))
             for i in range(4) for j in range(4)]
    for b in range(count):
        rng = rng_for(seed_config, b)
        c = rng.normal(0.0, 0.1, size=16)
        um = level + amplitude * sum(ci * bi for ci, bi in zip(c, basis))
        out.append(Problem(n=n, layer=0, k2=(2.0 * um).astype(np.complex128), k0sq=None,
                           source=random_field_c(n, rng),
                           meta=dict(config="newton", instance=b, dirichlet=True)))
    return out


@dataclasses.dataclass
class CdrProblem:
    """One convection-diffusion-reaction instance: real coefficient fields,
    background constants (kappa0, vx0, vy0, sigma0) and a source."""
    n: int
    kappa: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    sigma: np.ndarray
    background: tuple
    source: np.ndarray


def cdr_problem(n: int, rng: np.random.Generator, ell: Optional[float] = None,
                kappa_range=(0.5, 1.5), v_mean=(0.4, -0.3), v_amp: float = 0.3,
                sigma_range=(0.25, 0.75)) -> CdrProblem:
    """Smooth random coefficients (periodic Gaussian random fields, correlation
    n / 16 cells unless given): diffusivity and reaction in the given ranges,
    velocity = v_mean + v_amp * (field in [-1, 1]) per component; background =
    the coefficient means; complex random source."""
    ell = max(2.0, n / 16.0) if ell is None else ell
    unit = lambda: minmax_map(gaussian_random_field(n, ell, rng), -1.0, 1.0)
    kappa = 0.5 * (kappa_range[0] + kappa_range[1]) + 0.5 * (kappa_range[1] - kappa_range[0]) * unit()
    vx = v_mean[0] + v_amp * unit()
    vy = v_mean[1] + v_amp * unit()
    sigma = 0.5 * (sigma_range[0] + sigma_range[1]) + 0.5 * (sigma_range[1] - sigma_range[0]) * unit()
    bg = (float(kappa.mean()), float(vx.mean()), float(vy.mean()), float(sigma.mean()))
    return CdrProblem(n=n, kappa=kappa, vx=vx, vy=vy, sigma=sigma, background=bg,
                      source=random_field_c(n, rng))


def cdr_batch(count: int = 64, seed_config: int = 7, sizes=SIZES_RAGGED) -> List[CdrProblem]:
    """Ragged convection-diffusion-reaction batch: N drawn uniformly from
    `sizes` (as the ragged Helmholtz batch), coefficients as in cdr_problem."""
    out = []
    for i in range(count):
        rng = rng_for(seed_config, i)
        n = int(rng.choice(np.asarray(sizes)))
        out.append(cdr_problem(n, rng))
    return out


def workload(name: str):
    """Problems for a named workload: blob64, grf256, ragged64, diff16, layered1024, newton64, cdr64."""
    if name == "blob64":
        return [blob_problem()]
    if name == "grf256":
        return [grf_problem()]
    if name == "ragged64":
        return ragged_batch()
    if name == "diff16":
        return diff_batch()[0]
    if name == "layered1024":
        return layered_batch()
    if name == "newton64":
        return newton_batch()
    if name == "cdr64":
        return cdr_batch()
    raise KeyError(name)
