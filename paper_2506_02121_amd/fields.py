"""Seeded synthetic microlens fields and the named workloads.

This module only draws inputs.  It holds none of the method's arithmetic, so
both the HIP path and the CPU oracle can be fed from it without sharing code.

Field recipe (paper Sec. 2.1, the definition of the microlens convergence):
  kappa_star = pi * theta_star^2 * N * <m> / A_star with theta_star = 1, a
  circular field of area pi R^2, so R^2 = sum(m_i) / kappa_star.  <m> is the
  sample mean of the drawn masses, which makes sum(m_i) = kappa_star * pi R^2
  exact for every realisation.
Positions are area-uniform in the disk (r = R sqrt(u), theta = 2 pi v).
Masses are either all 1 or drawn from a Salpeter power law dN/dm ~ m^-2.35 on
[0.08, 1] by inverse-CDF sampling.

Every draw uses numpy.random.default_rng([seed, config_id, realisation]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SALPETER_SLOPE = 2.35
SALPETER_LO = 0.08
SALPETER_HI = 1.0


@dataclass
class StarField:
    """N point masses plus the macro-model: smooth convergence and shear."""

    x: np.ndarray
    y: np.ndarray
    m: np.ndarray
    kappa_s: float
    gamma: float
    kappa_star: float
    radius: float
    # rectangular field: (kappa_star, c1, c2, t), corner c1 + i c2 and the
    # Taylor degree t of the sheet; None for a circular field
    sheet: Optional[tuple] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Grid:
    """Pixelised source-plane window: pixel (r, c) has its centre at
    (center_re - half_width + (c + 0.5) * h, center_im - half_height + (r + 0.5) * h)."""

    center_re: float
    center_im: float
    half_width: float
    half_height: float
    nx: int
    ny: int


@dataclass
class Workload:
    name: str
    field: Optional[StarField]
    m_steps: int
    grid: Optional[Grid] = None
    precision: str = "fp64"
    fields: list = field(default_factory=list)   # batched workloads only


def rng_for(seed: int, config_id: int, realisation: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(config_id), int(realisation)])


def salpeter_masses(rng: np.random.Generator, n: int, lo: float = SALPETER_LO,
                    hi: float = SALPETER_HI, slope: float = SALPETER_SLOPE) -> np.ndarray:
    """Inverse-CDF draw from p(m) ~ m^-slope on [lo, hi]."""
    u = rng.random(n)
    a = 1.0 - slope
    return (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)


def uniform_disk(rng: np.random.Generator, n: int, radius: float):
    u = rng.random(n)
    v = rng.random(n)
    r = radius * np.sqrt(u)
    t = 2.0 * np.pi * v
    return r * np.cos(t), r * np.sin(t)


def make_field(rng: np.random.Generator, n: int, kappa_star: float, kappa_s: float,
               gamma: float, masses: str = "equal") -> StarField:
    if masses == "equal":
        m = np.ones(n)
    elif masses == "salpeter":
        m = salpeter_masses(rng, n)
    else:
        raise ValueError(f"unknown mass function {masses!r}")
    radius = float(np.sqrt(m.sum() / kappa_star))
    x, y = uniform_disk(rng, n, radius)
    return StarField(x=np.ascontiguousarray(x), y=np.ascontiguousarray(y),
                     m=np.ascontiguousarray(m), kappa_s=float(kappa_s),
                     gamma=float(gamma), kappa_star=float(kappa_star), radius=radius)


def make_rect_field(rng: np.random.Generator, n: int, kappa_star: float, kappa_s: float,
                    gamma: float, aspect: float, t: int, masses: str = "equal") -> StarField:
    """A rectangular field (Sec. 4.2): positions uniform in [-c1, c1] x
    [-c2, c2] with c2 = aspect * c1 and area 4 c1 c2 = pi sum(m_i) / kappa_star
    (the same definition of kappa_star as for the disk)."""
    if masses == "equal":
        m = np.ones(n)
    elif masses == "salpeter":
        m = salpeter_masses(rng, n)
    else:
        raise ValueError(f"unknown mass function {masses!r}")
    area = np.pi * m.sum() / kappa_star
    c1 = float(np.sqrt(area / (4.0 * aspect)))
    c2 = float(aspect * c1)
    x = (2.0 * rng.random(n) - 1.0) * c1
    y = (2.0 * rng.random(n) - 1.0) * c2
    return StarField(x=np.ascontiguousarray(x), y=np.ascontiguousarray(y),
                     m=np.ascontiguousarray(m), kappa_s=float(kappa_s), gamma=float(gamma),
                     kappa_star=float(kappa_star), radius=float(np.hypot(c1, c2)),
                     sheet=(float(kappa_star), c1, c2, int(t)))


def rect_field(seed: int, n: int, kappa_star: float = 0.4, kappa_s: float = 0.0,
               gamma: float = 0.3, aspect: float = 1.5, t: int = 9, masses: str = "equal",
               tag: int = 98) -> StarField:
    """A free-form seeded rectangular field for tests (config id `tag`)."""
    return make_rect_field(rng_for(seed, tag, n), n, kappa_star, kappa_s, gamma, aspect, t,
                           masses)


def random_field(seed: int, n: int, kappa_star: float = 0.4, kappa_s: float = 0.0,
                 gamma: float = 0.3, masses: str = "equal", tag: int = 99) -> StarField:
    """A free-form seeded field for tests (config id `tag`)."""
    return make_field(rng_for(seed, tag, n), n, kappa_star, kappa_s, gamma, masses)


def tiny_field(seed: int = 0) -> StarField:
    """N=10, m_i=1, kappa_star=0.3, kappa_s=0, gamma=0.3."""
    return make_field(rng_for(seed, 0), 10, 0.3, 0.0, 0.3, "equal")


def workload(name: str, seed: int = 0) -> Workload:
    """The six named workloads.

    tiny     N=10 equal masses, 1,000 phase steps (oracle finishes in seconds)
    n1k      N=1,000 Salpeter, kappa_star=0.4, kappa_s=0.2, gamma=0.45,
             10,000 steps, crossing map 1024^2 over 20x20
    n10k     N=10,000 equal masses, kappa_star=0.5, kappa_s=0, gamma=0.3,
             20,000 steps, crossing map 2048^2 and distance map over 40x40
    n10k_mixed  the n10k field in mixed precision
    batched  256 realisations, N log-uniform in [50, 5000], kappa_star in
             U[0.1, 0.8], gamma in U[0, 0.6], kappa_s=0, Salpeter masses,
             4,000 steps each
    rect     a rectangular field (Sec. 4.2) over the region that the n10k
             source map (40x40 at kappa_s=0, gamma=0.3) sees without stars,
             |x| <= 20/(1+gamma), |y| <= 20/(1-gamma), enlarged by s = 1.25:
             N=437 equal masses, kappa_star=0.5, c2/c1 = (1+gamma)/(1-gamma),
             sheet Taylor degree t = 87 (App. B's rule for error 1e-8 where
             |z| < |c|/1.25), 20,000 steps, the n10k grid
    """
    if name == "rect":
        g = 0.3
        f = make_rect_field(rng_for(seed, 5), 437, 0.5, 0.0, g, (1 + g) / (1 - g), 87, "equal")
        return Workload(name, f, 20000, Grid(0.0, 0.0, 20.0, 20.0, 2048, 2048))
    if name == "tiny":
        return Workload(name, tiny_field(seed), 1000)
    if name == "n1k":
        f = make_field(rng_for(seed, 1), 1000, 0.4, 0.2, 0.45, "salpeter")
        return Workload(name, f, 10000, Grid(0.0, 0.0, 10.0, 10.0, 1024, 1024))
    if name in ("n10k", "n10k_mixed"):
        f = make_field(rng_for(seed, 2), 10000, 0.5, 0.0, 0.3, "equal")
        return Workload(name, f, 20000, Grid(0.0, 0.0, 20.0, 20.0, 2048, 2048),
                        precision="mixed" if name == "n10k_mixed" else "fp64")
    if name == "batched":
        fields = []
        for r in range(256):
            rng = rng_for(seed, 4, r)
            n = int(round(np.exp(rng.uniform(np.log(50.0), np.log(5000.0)))))
            ks = float(rng.uniform(0.1, 0.8))
            g = float(rng.uniform(0.0, 0.6))
            fields.append(make_field(rng, n, ks, 0.0, g, "salpeter"))
        return Workload(name, None, 4000, precision="mixed", fields=fields)
    raise ValueError(f"unknown workload {name!r}")
