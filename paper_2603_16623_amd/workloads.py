"""Seeded synthetic inputs for the gridless ring solve.

This module draws ring geometries, beam macroparticles and request streams.
It holds none of the model's arithmetic: weights, fields and pushes are
computed by the library (and, separately, by the test oracle) from the
arrays produced here.  Both sides receive identical arrays.

Units are the paper's normalised ones (lengths in k_p^-1, densities in n0,
Sec. "Theoretical framework").  A beam is a list of ultra-relativistic
macroparticles (x, y, xi, w) with w the number of physical particles in
units of n0 k_p^-3, or an analytic bi-Gaussian profile.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

WINDOW = 12.0  # xi extent of every configuration, in k_p^-1


# ----------------------------------------------------------------------------
# ring geometries (Sec. "Discretization of plasma species": rho_j0 = sum of
# the extents below j plus half its own extent)
# ----------------------------------------------------------------------------
def uniform_rings(n: int, r_max: float):
    dr = np.full(n, r_max / n)
    r0 = (np.arange(n) + 0.5) * (r_max / n)
    return r0, dr


def geometric_ratio(n: int, d_min: float, r_max: float) -> float:
    """Ratio g with d_min * (g**n - 1) / (g - 1) == r_max (bisection)."""
    if d_min * n >= r_max:
        raise ValueError("d_min * n already exceeds r_max")

    def extent(g):
        x = n * math.log(g)
        if x > 700.0:
            return math.inf
        return d_min * math.expm1(x) / (g - 1.0)

    lo, hi = 1.0 + 1e-15, 1.0 + 1.0 / n
    while extent(hi) < r_max:
        hi = 1.0 + 2.0 * (hi - 1.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if extent(mid) < r_max:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def geometric_rings(n: int, d_min: float, r_max: float):
    g = geometric_ratio(n, d_min, r_max)
    dr = d_min * g ** np.arange(n, dtype=np.float64)
    edges = np.concatenate([[0.0], np.cumsum(dr)])
    r0 = edges[:-1] + 0.5 * dr
    return r0, dr


# ----------------------------------------------------------------------------
# sources
# ----------------------------------------------------------------------------
@dataclass
class Particles:
    q: float
    x: np.ndarray
    y: np.ndarray
    xi: np.ndarray
    w: np.ndarray
    kind: str = "particles"


@dataclass
class GaussianBeam:
    q: float
    n_peak: float
    sigma_r: float
    sigma_xi: float
    xi_c: float
    kind: str = "gaussian"


@dataclass
class GaussianLaser:
    a0: float
    w0: float
    L: float
    xi_l: float
    kind: str = "laser"


def channel_density(r0: np.ndarray, w0: float) -> np.ndarray:
    """Parabolic channel n(r)/n0 = 1 + 4 r^2 / w0^4 (lengths in k_p^-1), the
    radial profile of the paper's laser-driven benchmark (Sec. "Validation
    benchmarks"), sampled at the rings' initial radii."""
    return 1.0 + 4.0 * np.asarray(r0, dtype=np.float64) ** 2 / w0 ** 4


def beam_number(n_peak: float, sigma_r: float, sigma_xi: float) -> float:
    """Physical particle count (units n0 k_p^-3) of a bi-Gaussian of peak n_peak."""
    return n_peak * (2.0 * math.pi) ** 1.5 * sigma_r ** 2 * sigma_xi


def gaussian_particles(rng: np.random.Generator, n_part: int, n_peak: float,
                       sigma_r: float, sigma_xi: float, xi_c: float,
                       q: float = -1.0) -> Particles:
    x = rng.normal(0.0, sigma_r, n_part)
    y = rng.normal(0.0, sigma_r, n_part)
    xi = rng.normal(xi_c, sigma_xi, n_part)
    w = np.full(n_part, beam_number(n_peak, sigma_r, sigma_xi) / n_part)
    return Particles(q, x, y, xi, w)


def witness_particles(rng, n_part, number, sigma_r, sigma_xi, xi_c, q=-1.0):
    x = rng.normal(0.0, sigma_r, n_part)
    y = rng.normal(0.0, sigma_r, n_part)
    xi = rng.normal(xi_c, sigma_xi, n_part)
    w = np.full(n_part, number / n_part)
    return Particles(q, x, y, xi, w)


# ----------------------------------------------------------------------------
# instances
# ----------------------------------------------------------------------------
@dataclass
class Instance:
    name: str
    r0: np.ndarray
    dr: np.ndarray
    dxi: float
    n_xi: int
    sources: List[object] = field(default_factory=list)
    dens: Optional[np.ndarray] = None

    @property
    def n_rings(self) -> int:
        return int(self.r0.shape[0])

    @property
    def ring_slices(self) -> int:
        return self.n_rings * self.n_xi


def config1(seed: int = 1, n_part: int = 10_000, analytic: bool = False,
            n_peak: float = 0.05, channel_w0: Optional[float] = None) -> Instance:
    """Linear regime: 1000 uniform rings to r=5, weak bi-Gaussian driver
    (in a parabolic channel with channel_w0)."""
    r0, dr = uniform_rings(1000, 5.0)
    sr, sx, xc = 0.1, 0.5, 2.0
    if analytic:
        src = [GaussianBeam(-1.0, n_peak, sr, sx, xc)]
    else:
        rng = np.random.default_rng(seed)
        src = [gaussian_particles(rng, n_part, n_peak, sr, sx, xc)]
    dens = None if channel_w0 is None else channel_density(r0, channel_w0)
    return Instance("linear-1000x1200", r0, dr, 0.01, 1200, src, dens)


def config2(seed: int = 2) -> Instance:
    """Nonlinear blowout: 20000 geometric rings to r=8, driver + witness."""
    r0, dr = geometric_rings(20_000, 1e-4, 8.0)
    rng = np.random.default_rng(seed)
    nd = beam_number(10.0, 0.05, 0.7)
    drv = gaussian_particles(rng, 50_000, 10.0, 0.05, 0.7, 2.8)
    wit = witness_particles(rng, 20_000, 0.2 * nd, 0.005, 0.1, 2.8 + 4.5)
    return Instance("blowout-20000x4000", r0, dr, 0.003, 4000, [drv, wit])


def batched_instance(rng: np.random.Generator, n_rings: int, n_xi: int,
                     n_drv: int = 10_000, n_wit: int = 4_000,
                     d_min: float = 1e-4, r_max: float = 8.0,
                     name: str = "batched") -> Instance:
    """One instance with batched-style spacing and randomly drawn beams."""
    r0, dr = geometric_rings(n_rings, d_min, r_max)
    n_peak = rng.uniform(0.5, 20.0)
    sr = rng.uniform(0.02, 0.2)
    sx = rng.uniform(0.3, 1.0)
    delay = rng.uniform(3.0, 6.0)
    xc = 4.0 * sx
    drv = gaussian_particles(rng, n_drv, n_peak, sr, sx, xc)
    wit = witness_particles(rng, n_wit, 0.2 * beam_number(n_peak, sr, sx),
                            sr / 10.0, 0.1, xc + delay)
    return Instance(name, r0, dr, WINDOW / n_xi, n_xi, [drv, wit])


def log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def config3(seed: int = 3, n_inst: int = 512, n_xi: int = 2000,
            n_min: int = 1000, n_max: int = 8000) -> List[Instance]:
    """Batched: independent instances with log-uniform ring counts."""
    children = np.random.SeedSequence(seed).spawn(n_inst)
    out = []
    for k, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = log_uniform_int(rng, n_min, n_max)
        out.append(batched_instance(rng, n, n_xi, name=f"batched-{k}"))
    return out


@dataclass
class Request:
    arrival: float
    instance: Instance


def config4_stream(seed: int = 4, rate: float = 2000.0, duration: float = 60.0,
                   n_min: int = 500, n_max: int = 50_000, xi_min: int = 500,
                   xi_max: int = 8000, max_requests: Optional[int] = None):
    """Poisson request stream; instances are built lazily by the caller."""
    ss = np.random.SeedSequence(seed)
    gap_rng = np.random.default_rng(ss.spawn(1)[0])
    t, k = 0.0, 0
    specs = []
    while True:
        t += gap_rng.exponential(1.0 / rate)
        if t > duration or (max_requests is not None and k >= max_requests):
            break
        specs.append((t, k))
        k += 1
    children = np.random.SeedSequence(seed + 1000).spawn(max(1, len(specs)))

    def build(k: int) -> Instance:
        rng = np.random.default_rng(children[k])
        n = log_uniform_int(rng, n_min, n_max)
        n_xi = int(rng.integers(xi_min, xi_max + 1))
        return batched_instance(rng, n, n_xi, name=f"request-{k}")

    return specs, build


def config5(seed: int = 5) -> Instance:
    """Large laser-driven instance: 2e5 geometric rings to r=15."""
    r0, dr = geometric_rings(200_000, 1e-5, 15.0)
    rng = np.random.default_rng(seed)
    wit = witness_particles(rng, 100_000, 0.05, 0.002, 0.1, 6.5)
    las = GaussianLaser(2.0, 2.0, 1.0, 2.0)
    return Instance("laser-200000x8000", r0, dr, 0.0015, 8000, [las, wit])


def small_instance(seed: int, n_rings: int = 96, n_xi: int = 60,
                   n_peak: float = 2.0, sigma_r: float = 0.15,
                   geometric: bool = True, laser: bool = False,
                   n_part: int = 3000, dxi: float = 0.02,
                   channel_w0: Optional[float] = None) -> Instance:
    """Small nonlinear instance for parity tests (several tiles, ragged tail);
    with channel_w0, a parabolic channel instead of uniform density."""
    rng = np.random.default_rng(seed)
    if geometric:
        r0, dr = geometric_rings(n_rings, 2e-3, 3.0)
    else:
        r0, dr = uniform_rings(n_rings, 3.0)
    sx = 0.3
    xc = 4.0 * sx
    src: List[object] = [gaussian_particles(rng, n_part, n_peak, sigma_r, sx, xc)]
    if laser:
        src.append(GaussianLaser(1.0, 1.0, 0.6, 0.8))
    dens = None if channel_w0 is None else channel_density(r0, channel_w0)
    return Instance(f"small-{n_rings}x{n_xi}", r0, dr, dxi, n_xi, src, dens)
