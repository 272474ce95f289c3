"""Seeded synthetic inputs for the Fresnel-diffraction workloads.

This module only describes and draws inputs: shape parameters, wavelengths,
distances, target sets and random coefficients.  It holds none of the method's
arithmetic (no quadrature, chirp, NUFFT or sum), so both the GPU library's
tests and the CPU oracle can take their inputs from it.

Random draws use ``numpy.random.Generator(PCG64(201005978 + workload_id))``.

Workloads (sizes follow the paper's own test geometries, secs. 3.1-3.2):
  1 disk        R = 1, Fresnel number R^2/(lambda z) = 10, 6x20 GL panels x m=40
                (4,800 nodes), 100x100 target grid on [-1.5, 1.5)^2.
  2 starfish    r(t) = 1 + 0.3 cos 5t, Fresnel number 20 at the maximum radius
                1.3 (lambda z = 0.0845), 20x20 GL panels x m=100 (40,000
                nodes); 1000x1000 grid on [-1.5, 1.5)^2 and 1e5 random points
                uniform in the disk |x| < 1.5.
  3 starshade   24 petals, disc radius a = 6 m, tip radius R = 12 m,
                A(r) = exp(-((r-6)/6)^6), z = 3.7e7 m, lambda in {0.5, 0.75,
                1.0} um; m = 320, n_p = 100, n_d = 720, m_d = 320 (998,400
                nodes); 1e6 random points in a 2.4 m pupil and a 2048^2 grid
                on [-2.4, 2.4)^2.
  4 batch       256 random star-shaped shapes (smooth radial Fourier curves and
                polygons), node counts uniform in [1e4, 4e5], 64 wavelengths
                log-spaced in [0.5, 1.0] um, z = 1e5 m, 512^2 grids on
                [-1.5, 1.5)^2.
  5 gradient    workload 3's occulter with each petal edge perturbed by 8 sine
                modes (384 real coefficients ~ N(0, (1e-3 m)^2)); 512^2 grid
                on [-2.4, 2.4)^2, pupil mask k1^2 + k2^2 < 256^2, 3 wavelengths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 201005978


def rng(workload_id: int, stream: int = 0) -> np.random.Generator:
    """Seeded generator for a workload (stream separates independent draws)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + workload_id, stream]))


# ------------------------------------------------------------------ shapes
@dataclass
class RadialCurve:
    """r(t) = r0 + sum_{k=1}^K a[k-1] cos kt + b[k-1] sin kt; GL panels x q; m radial."""
    r0: float
    a: np.ndarray
    b: np.ndarray
    panels: int
    q: int
    m: int

    @property
    def n_nodes(self) -> int:
        return self.panels * self.q * self.m


@dataclass
class Polygon:
    """CCW polygon vertices; q GL nodes per edge; m radial."""
    vx: np.ndarray
    vy: np.ndarray
    q: int
    m: int

    @property
    def n_nodes(self) -> int:
        return len(self.vx) * self.q * self.m


@dataclass
class Starshade:
    """Np petals, disc radius a, tip radius R, apodisation exp(-((r-a)/b)^p);
    m radial x np angular nodes per petal, nd x md disc nodes; optional edge
    perturbation coef (2*Np*K)."""
    Np: int
    a: float
    R: float
    b: float
    p: float
    m: int
    np_: int
    nd: int
    md: int
    coef: np.ndarray | None = None
    K: int = 0

    @property
    def n_nodes(self) -> int:
        return self.nd * self.md + self.Np * self.np_ * self.m


@dataclass
class Grid:
    n1: int
    n2: int
    h1: float
    h2: float
    xc: float = 0.0
    yc: float = 0.0

    @property
    def M(self) -> int:
        return self.n1 * self.n2


@dataclass
class Workload:
    name: str
    shape: object
    lam: float
    z: float
    grid: Grid | None = None
    points: tuple | None = None            # (xi, eta) float64 arrays
    pupil: float | None = None             # the points lie in the disk |x| < pupil
    occulter: bool = False
    lams: list = field(default_factory=list)


def disk_points_uniform(n: int, radius: float, g: np.random.Generator):
    """n points uniform in the disk |x| < radius: r = radius sqrt(U), t = 2 pi U'."""
    r = radius * np.sqrt(g.random(n))
    t = 2.0 * math.pi * g.random(n)
    return r * np.cos(t), r * np.sin(t)


def workload(wid: int, reduced: bool = False) -> Workload:
    """The seeded inputs of workload ``wid`` (1..5).  ``reduced`` picks the
    smaller geometry that the oracle can also run in seconds (5 only)."""
    if wid == 1:
        shape = RadialCurve(1.0, np.zeros(0), np.zeros(0), panels=6, q=20, m=40)
        # Fresnel number R^2/(lambda z) = 10 -> lambda z = 0.1
        return Workload("disk_R1_F10", shape, lam=5.0e-7, z=2.0e5,
                        grid=Grid(100, 100, 0.03, 0.03))
    if wid == 2:
        a = np.zeros(5)
        a[4] = 0.3
        shape = RadialCurve(1.0, a, np.zeros(5), panels=20, q=20, m=100)
        g = rng(2)
        pts = disk_points_uniform(100_000, 1.5, g)
        # Fresnel number 20 at the maximum radius 1.3 -> lambda z = 1.69/20
        return Workload("starfish_F20", shape, lam=5.0e-7, z=0.0845 / 5.0e-7,
                        grid=Grid(1000, 1000, 0.003, 0.003), points=pts, pupil=1.5)
    if wid == 3:
        shape = Starshade(24, 6.0, 12.0, 6.0, 6.0, m=320, np_=100, nd=720, md=320)
        g = rng(3)
        pts = disk_points_uniform(1_000_000, 2.4, g)
        return Workload("starshade24", shape, lam=0.5e-6, z=3.7e7,
                        grid=Grid(2048, 2048, 4.8 / 2048, 4.8 / 2048), points=pts, pupil=2.4,
                        occulter=True, lams=[0.5e-6, 0.75e-6, 1.0e-6])
    if wid == 5:
        K = 8
        g = rng(5)
        coef = g.normal(0.0, 1.0e-3, size=2 * 24 * K)
        if reduced:
            shape = Starshade(24, 6.0, 12.0, 6.0, 6.0, m=64, np_=32, nd=230, md=64,
                              coef=coef, K=K)
            grid = Grid(128, 128, 4.8 / 128, 4.8 / 128)
        else:
            shape = Starshade(24, 6.0, 12.0, 6.0, 6.0, m=320, np_=100, nd=720, md=320,
                              coef=coef, K=K)
            grid = Grid(512, 512, 4.8 / 512, 4.8 / 512)
        return Workload("starshade24_grad" + ("_reduced" if reduced else ""), shape,
                        lam=0.5e-6, z=3.7e7, grid=grid, occulter=True,
                        lams=[0.5e-6, 0.75e-6, 1.0e-6])
    raise ValueError(f"unknown workload {wid}")


def pupil_mask(n: int) -> np.ndarray:
    """Integer pupil mask k1^2 + k2^2 < (n/2)^2 on an n x n grid (k1 fastest)."""
    k = np.arange(-(n // 2), n - n // 2)
    K1, K2 = np.meshgrid(k, k, indexing="xy")
    return (K1 * K1 + K2 * K2 < (n // 2) ** 2).ravel()


def batch_shapes(count: int = 256, nmin: int = 10_000, nmax: int = 400_000,
                 workload_id: int = 4):
    """Random star-shaped instances: radius r(t) = 1 + p(t), p a Fourier series
    with K ~ U{8..32} modes, a_k, b_k ~ N(0, 0.05^2), scaled down if needed so
    |p| <= 0.7.  Even instances are smooth radial curves (GL panels of q = 16);
    odd instances are polygons with 2K vertices at jittered angles on r(t).
    Node counts N_i ~ U{nmin..nmax} with boundary:radial ~ 4:1."""
    g = rng(workload_id)
    shapes = []
    tt = np.linspace(0.0, 2.0 * math.pi, 4096, endpoint=False)
    for i in range(count):
        K = int(g.integers(8, 33))
        a = g.normal(0.0, 0.05, K)
        b = g.normal(0.0, 0.05, K)
        k = np.arange(1, K + 1)[:, None]
        p = (a[:, None] * np.cos(k * tt) + b[:, None] * np.sin(k * tt)).sum(0)
        s = min(1.0, 0.7 / max(1e-300, np.abs(p).max()))
        a, b = a * s, b * s
        Ni = int(g.integers(nmin, nmax + 1))
        n_b = max(16, int(round(2.0 * math.sqrt(Ni))))
        m = max(2, int(round(Ni / n_b)))
        if i % 2 == 0:
            q = 16
            panels = max(1, int(round(n_b / q)))
            shapes.append(RadialCurve(1.0, a, b, panels=panels, q=q, m=m))
        else:
            V = 2 * K
            jit = g.uniform(-0.3, 0.3, V) * (2.0 * math.pi / V)
            th = 2.0 * math.pi * np.arange(V) / V + jit
            kk = np.arange(1, K + 1)[:, None]
            r = 1.0 + (a[:, None] * np.cos(kk * th) + b[:, None] * np.sin(kk * th)).sum(0)
            q = max(2, int(round(n_b / V)))
            shapes.append(Polygon(r * np.cos(th), r * np.sin(th), q=q, m=m))
    return shapes


def batch_lambdas(count: int = 64) -> np.ndarray:
    """Wavelengths log-spaced in [0.5, 1.0] um: 0.5e-6 * 2^(l/(count-1))."""
    return 0.5e-6 * 2.0 ** (np.arange(count) / (count - 1))


BATCH_Z = 1.0e5
BATCH_GRID = Grid(512, 512, 3.0 / 512, 3.0 / 512)
