"""Seeded particle-set generators for the five benchmark workloads and the test cases.

Every generator draws with ``numpy.random.default_rng(seed)`` in a fixed order
(positions, then jitter, then velocities, then per-set scalars) and returns a
``ParticleSet`` of float64 arrays in *caller order*.  Nothing here evaluates the SPH
kernel, the equation of state, the tree or the integrator; the only physics is the
analytic density profile of each initial condition, used to place particles and to
pick their starting smoothing length and thermal energy.

Workloads (sizes as used by the benchmark; every generator also takes a smaller size
so that the CPU reference finishes in seconds):

* ``lattice_box``  -- jittered cubic lattice in the unit cube (16^3 = 4096 by default).
* ``sod_tube``     -- 3D Sod-type tube, two lattices with spacing ratio 2:1 that give
                      rho = 1, P = 1 on the left and rho = 0.125, P = 0.1 on the right
                      (the initial state of the paper's Sod test, Sec. 3.1, eq. (11)).
* ``polytrope_n1`` -- n = 1 polytrope, rho ~ sin(pi r)/(pi r) in the unit sphere.
* ``ensemble``     -- many independent jittered boxes of uneven size (segments).
* ``evrard``       -- cold gas sphere with rho ~ 1/r.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = 5.0 / 3.0


@dataclasses.dataclass
class ParticleSet:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    h: np.ndarray
    u: np.ndarray
    seg_offsets: np.ndarray | None = None  # int64[n_seg+1] or None for one set
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_seg(self) -> int:
        return 1 if self.seg_offsets is None else int(self.seg_offsets.shape[0] - 1)

    def fields(self):
        return dict(x=self.x, y=self.y, z=self.z, vx=self.vx, vy=self.vy, vz=self.vz,
                    m=self.m, h=self.h, u=self.u)

    def copy(self) -> "ParticleSet":
        return ParticleSet(**{k: v.copy() for k, v in self.fields().items()},
                           seg_offsets=None if self.seg_offsets is None else self.seg_offsets.copy(),
                           meta=dict(self.meta))

    def subset(self, idx: np.ndarray) -> "ParticleSet":
        return ParticleSet(**{k: np.ascontiguousarray(v[idx]) for k, v in self.fields().items()},
                           meta=dict(self.meta))


def _make(x, y, z, vx, vy, vz, m, h, u, seg_offsets=None, **meta) -> ParticleSet:
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    so = None if seg_offsets is None else np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.int64))
    return ParticleSet(f(x), f(y), f(z), f(vx), f(vy), f(vz), f(m), f(h), f(u), so, dict(meta))


def _cell_centres(nx, ny, nz, dx, origin=(0.0, 0.0, 0.0)):
    """Lattice points at cell centres (i + 1/2) dx, x fastest."""
    i = (np.arange(nx) + 0.5) * dx + origin[0]
    j = (np.arange(ny) + 0.5) * dx + origin[1]
    k = (np.arange(nz) + 0.5) * dx + origin[2]
    zz, yy, xx = np.meshgrid(k, j, i, indexing="ij")
    return xx.ravel(), yy.ravel(), zz.ravel()


def lattice_box(n_side: int = 16, seed: int = 1001, jitter: float = 0.1, v_sigma: float = 0.01,
                h_factor: float = 1.2, u0: float = 1.0, total_mass: float = 1.0) -> ParticleSet:
    """Jittered n_side^3 lattice in the unit cube, equal masses summing to total_mass,
    fixed h = h_factor * dx, uniform u, Gaussian velocities (sigma = v_sigma)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_side
    x, y, z = _cell_centres(n_side, n_side, n_side, dx)
    n = x.size
    if jitter:
        j = rng.uniform(-jitter * dx, jitter * dx, size=(3, n))
        x, y, z = x + j[0], y + j[1], z + j[2]
    v = rng.normal(0.0, v_sigma, size=(3, n)) if v_sigma else np.zeros((3, n))
    return _make(x, y, z, v[0], v[1], v[2], np.full(n, total_mass / n), np.full(n, h_factor * dx),
                 np.full(n, u0), name="lattice_box", n_side=n_side, dx=dx, seed=seed)


def sod_tube(ny: int = 56, seed: int = 1002, h_factor: float = 1.2) -> ParticleSet:
    """3D Sod-type tube in [0,1] x [0,0.1] x [0,0.1].

    Left half [0, 0.5]: (5 ny) x ny x ny lattice, spacing dx = 0.1/ny, rho = 1, P = 1.
    Right half [0.5, 1]: (5 ny/2) x (ny/2) x (ny/2) lattice, spacing 2 dx, rho = 0.125,
    P = 0.1.  Equal masses m = dx^3 (so rho_L = 1 exactly), v = 0, gamma = 5/3 gives
    u_L = 1.5 and u_R = 1.2.  h = h_factor (m / rho)^(1/3) from the lattice density.
    ny = 56 gives 878,080 + 109,760 = 987,840 particles.  The lattice is not jittered
    (the seed is recorded but unused)."""
    if ny % 2:
        raise ValueError("ny must be even")
    dx = 0.1 / ny
    xl, yl, zl = _cell_centres(5 * ny, ny, ny, dx)
    xr, yr, zr = _cell_centres(5 * ny // 2, ny // 2, ny // 2, 2 * dx, origin=(0.5, 0.0, 0.0))
    x, y, z = np.concatenate([xl, xr]), np.concatenate([yl, yr]), np.concatenate([zl, zr])
    n, nl = x.size, xl.size
    m = np.full(n, dx ** 3)
    rho = np.where(np.arange(n) < nl, 1.0, 0.125)
    P = np.where(np.arange(n) < nl, 1.0, 0.1)
    u = P / ((GAMMA - 1.0) * rho)
    h = h_factor * np.cbrt(m / rho)
    zero = np.zeros(n)
    return _make(x, y, z, zero, zero, zero, m, h, u, name="sod_tube", ny=ny, dx=dx, n_left=nl, seed=seed)


def _isotropic(rng, n):
    mu = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    s = np.sqrt(1.0 - mu * mu)
    return s * np.cos(phi), s * np.sin(phi), mu


def _polytrope_mass(r):
    """Enclosed mass of rho = (pi/4) sin(pi r)/(pi r) in the unit sphere; M(1) = 1."""
    return (np.sin(np.pi * r) - np.pi * r * np.cos(np.pi * r)) / np.pi


def polytrope_n1(n: int = 4194304, seed: int = 1003, h_factor: float = 1.2) -> ParticleSet:
    """n = 1 polytrope: equal-mass particles with radii drawn by inverting M(r) (FP64
    bisection) and isotropic directions; G = M = R = 1, rho_c = pi/4, K = 2/pi so that
    P = K rho^2 is hydrostatic; u = K rho / (gamma - 1); v = 0;
    h0 = h_factor (m / max(rho, 1e-4 rho_c))^(1/3)."""
    rng = np.random.default_rng(seed)
    target = rng.uniform(0.0, 1.0, size=n)
    lo, hi = np.zeros(n), np.ones(n)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = _polytrope_mass(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    r = 0.5 * (lo + hi)
    ex, ey, ez = _isotropic(rng, n)
    rho_c = math.pi / 4.0
    pr = np.pi * r
    rho = rho_c * np.where(pr > 0, np.sin(pr) / np.where(pr > 0, pr, 1.0), 1.0)
    K = 2.0 / math.pi
    m = np.full(n, 1.0 / n)
    h = h_factor * np.cbrt(m / np.maximum(rho, 1e-4 * rho_c))
    u = K * rho / (GAMMA - 1.0)
    zero = np.zeros(n)
    return _make(r * ex, r * ey, r * ez, zero, zero, zero, m, h, u, name="polytrope_n1", seed=seed,
                 G=1.0, soft_eps=0.01, theta=0.5)


def ensemble(n_boxes: int = 256, seed: int = 1004, n_min: int = 2048, n_max: int = 65536,
             side_lo: int = 13, side_hi: int = 40, jitter: float = 0.1, v_sigma: float = 0.01,
             h_factor: float = 1.2) -> ParticleSet:
    """Batched ensemble of independent jittered unit-cube lattices.

    Box i has n_i^3 particles, n_i = clip(round(cbrt(exp(U(ln n_min, ln n_max)))),
    side_lo, side_hi); rho0_i ~ U(0.5, 2) (m_i = rho0_i / n_i^3), u_i ~ U(0.5, 2),
    h = h_factor dx_i fixed, v ~ N(0, v_sigma^2).  Boxes are concatenated; seg_offsets
    marks them."""
    rng = np.random.default_rng(seed)
    sides = np.clip(np.rint(np.cbrt(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_boxes)))),
                    side_lo, side_hi).astype(np.int64)
    rho0 = rng.uniform(0.5, 2.0, size=n_boxes)
    u0 = rng.uniform(0.5, 2.0, size=n_boxes)
    parts, offs = [], [0]
    for b in range(n_boxes):
        s = int(sides[b])
        dx = 1.0 / s
        x, y, z = _cell_centres(s, s, s, dx)
        k = x.size
        j = rng.uniform(-jitter * dx, jitter * dx, size=(3, k))
        v = rng.normal(0.0, v_sigma, size=(3, k))
        parts.append((x + j[0], y + j[1], z + j[2], v[0], v[1], v[2], np.full(k, rho0[b] / k),
                      np.full(k, h_factor * dx), np.full(k, u0[b])))
        offs.append(offs[-1] + k)
    cols = [np.concatenate([p[c] for p in parts]) for c in range(9)]
    return _make(*cols, seg_offsets=np.array(offs, dtype=np.int64), name="ensemble", seed=seed,
                 sides=sides, rho0=rho0, u0=u0)


def evrard(n: int = 16777216, seed: int = 1005, u0: float = 0.05, h_factor: float = 1.2) -> ParticleSet:
    """Evrard-style cold sphere: rho = 1/(2 pi r) in the unit sphere (M(r) = r^2, so
    r = sqrt(U)), isotropic directions, m = 1/N, u = u0 (G = M = R = 1), v = 0,
    h0 = h_factor (m / rho)^(1/3) from the analytic density."""
    rng = np.random.default_rng(seed)
    r = np.sqrt(rng.uniform(0.0, 1.0, size=n))
    ex, ey, ez = _isotropic(rng, n)
    rho = 1.0 / (2.0 * math.pi * np.maximum(r, 1e-6))
    m = np.full(n, 1.0 / n)
    zero = np.zeros(n)
    return _make(r * ex, r * ey, r * ez, zero, zero, zero, m, h_factor * np.cbrt(m / rho), np.full(n, u0),
                 name="evrard", seed=seed, G=1.0, soft_eps=0.005, theta=0.5)


def uniform_random(n: int, seed: int, h: float | tuple = 0.05, box: float = 1.0, v_sigma: float = 0.1,
                   u_range=(0.5, 2.0)) -> ParticleSet:
    """Uniform random points in [0, box]^3 with per-particle h drawn from [h/2, h] (or a
    given (lo, hi) range), masses in [0.5, 1.5]/n, u in u_range, Gaussian velocities."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, box, size=(3, n))
    v = rng.normal(0.0, v_sigma, size=(3, n))
    hl, hh = (h / 2.0, h) if np.isscalar(h) else h
    hh_ = rng.uniform(hl, hh, size=n)
    m = rng.uniform(0.5, 1.5, size=n) / n
    u = rng.uniform(u_range[0], u_range[1], size=n)
    return _make(p[0], p[1], p[2], v[0], v[1], v[2], m, hh_, u, name="uniform_random", seed=seed)


def fig1_points():
    """The ten particles of the paper's Fig. 1 (tree topology), read off the TikZ
    drawing: the outer square is [-2.5, 2.5]^2 and each bullet sits at the anchor point
    given in the drawing.  Returned in key space: X = x, Y = -y (the figure numbers the
    quadrants NW, NE, SW, SE, i.e. y grows downward), Z = 0.  Box: lo = (-2.5, -2.5, 0),
    hi = (2.5, 2.5, 0); root cell side 5."""
    pts = [
        (1.5, 1.5),        # cell 11
        (-0.69, 2.02),     # cell 101
        (-2.2, 0.05),      # cell 102
        (-0.25, -0.5),     # cell 121
        (0.8, -0.7),       # cell 130
        (-1.74, -0.8),     # cell 120
        (-2.4, -1.35),     # cell 1220
        (-1.755, -2.225),  # cell 1223
        (2.025, -0.25),    # cell 1311
        (1.4, -0.875),     # cell 1312
    ]
    x = np.array([p[0] for p in pts])
    y = -np.array([p[1] for p in pts])
    z = np.zeros(len(pts))
    box = np.array([-2.5, -2.5, 0.0, 2.5, 2.5, 0.0])
    return x, y, z, box
