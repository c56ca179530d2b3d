"""Seeded synthetic inputs for the Lagrangian particle model.

This module only *describes* workloads: release point, schedule, physical
constants, wind fields, rain region and grid geometry.  It holds none of the
model's arithmetic (no interpolation, random numbers, stepping or binning), so
both the FP64 oracle and the HIP library can be fed from it without sharing any
of the method.

Workloads (the paper's own numbers are given where it states them):

* ``c0``  -- uniform-weather analogue of the paper's "artificial" case
  (Sec. 4, caption of Fig. 3: constant wind along x, no vertical wind),
  1e4 particles, 1 h at dt = 10 s, mass gridded on 100 x 100 x 20 cells.
* ``c1``  -- 1e6 particles, 6 h at dt = 5 s, one gridded 200 x 200 x 30 wind
  field (stands in for the paper's ALADIN "real weather", which is not
  available), parabolic K_z, dry and wet deposition, two nuclides.
* ``c2``  -- 1.6e7 particles, 24 h, 25 hourly 400 x 400 x 40 fields,
  continuous release over the first 6 h.

Field layout (device and host alike): float32 ``[nt][nz][ny][nx][ncomp]`` with
cell-centred nodes at ``x0 + (i + 1/2) dx`` (same in y, z) and node times
``t0 + k dt_field``; ``ncomp`` is 2 (u, v; w = 0) or 3 (u, v, w).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field as dc_field, replace
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "Source", "Schedule", "Physics", "Rain", "Field", "Grid", "Case",
    "c0", "c1", "c2", "c3", "c4", "wind_field", "rain_region", "uniform_field",
    "uniform_state", "replace", "Receptors", "load_receptors", "with_theta",
    "THETA0", "THETA_HIDDEN",
]


@dataclass(frozen=True)
class Source:
    """Point source (Sec. 2: particles are released from a point source in
    each time step).  ``q`` is the release rate in relative units per second
    (Sec. 4: the emission is scaled to the particle count), ``wind_scale``
    multiplies the sampled wind, ``v_d`` is the dry-deposition velocity and
    ``scenario`` is the second Philox key word."""
    xs: float = 0.0
    ys: float = 0.0
    h: float = 50.0
    q: float = 1.0
    wind_scale: float = 1.0
    v_d: float = 0.0
    scenario: int = 0


@dataclass(frozen=True)
class Schedule:
    """Release schedule (Sec. 3.2: the emission profile and the maximum
    particle count are known a priori).  Global particle id ``g`` is born at
    step ``floor(g * s_release / n_total)``.  A run may hold only a subset of
    the ids: local index ``i`` is global id ``id_base + i * id_stride``."""
    n_total: int
    s_release: int
    n_local: Optional[int] = None
    id_base: int = 0
    id_stride: int = 1

    @property
    def local_count(self) -> int:
        if self.n_local is not None:
            return int(self.n_local)
        return int((self.n_total - self.id_base + self.id_stride - 1) // self.id_stride)

    def subset(self, stride: int, base: int = 0) -> "Schedule":
        n = (self.n_total - base + stride - 1) // stride
        return replace(self, n_local=n, id_base=base, id_stride=stride)


@dataclass(frozen=True)
class Rain:
    """Elliptical rain region: centre, semi-axes, rotation and the width of
    the linear edge (in units of the elliptical radius)."""
    cx: float = 0.0
    cy: float = 0.0
    a: float = 1.0
    b: float = 1.0
    angle: float = 0.0
    edge: float = 0.1


@dataclass(frozen=True)
class Physics:
    """Physical constants of one run.

    kz_kind: 0 = constant ``Kz_const``; 1 = parabolic
    ``kappa_ustar (z + z0) (1 - z/H_mix)``; 2 = Eq. (3) with Phi = 1,
    ``kappa_ustar (z + z0) (1 - z/H_mix)^2``; 3 = Eq. (3) with the heat
    similarity function of (z + z0) inv_L.
    """
    dt: float
    Kh: float
    kz_kind: int = 0
    Kz_const: float = 0.0
    kappa_ustar: float = 0.2
    z0: float = 0.25
    H_mix: float = 1000.0
    H_lid: float = 1000.0
    h_s: float = 40.0
    lambdas: Tuple[float, ...] = (1e-6,)
    Lambda0: float = 0.0
    rain: Rain = Rain()
    seed: int = 0
    inv_L: float = 0.0    # kz_kind 3: inverse Monin-Obukhov length (1/m)
    chain: int = 0        # 1: decay chain 0 -> 1 -> ..., parent released
    dep_mode: int = 0     # 1: stochastic deposition (removal), 0: mass depletion

    @property
    def n_nuc(self) -> int:
        return len(self.lambdas)


@dataclass
class Field:
    """Gridded wind, float32 ``[nt][nz][ny][nx][ncomp]``.  ``bounded``: a
    particle whose (x, y) leaves ``[x0, x0 + nx dx) x [y0, y0 + ny dy)`` is
    inactivated (Sec. 3.2: particles become inactive at the predefined
    boundaries of the simulated area).  ``z_levels`` (optional, increasing,
    length nz) replaces the uniform node heights ``(k + 1/2) dz``."""
    data: np.ndarray
    x0: float
    y0: float
    dx: float
    dy: float
    dz: float
    t0: float = 0.0
    dt_field: float = 3600.0
    z_levels: Optional[np.ndarray] = None
    bounded: bool = True

    def __post_init__(self):
        assert self.data.dtype == np.float32 and self.data.ndim == 5
        assert self.data.shape[-1] in (2, 3)
        self.data = np.ascontiguousarray(self.data)
        if self.z_levels is not None:
            self.z_levels = np.ascontiguousarray(self.z_levels, dtype=np.float32)
            assert self.z_levels.shape == (self.nz,)

    nt = property(lambda self: self.data.shape[0])
    nz = property(lambda self: self.data.shape[1])
    ny = property(lambda self: self.data.shape[2])
    nx = property(lambda self: self.data.shape[3])
    ncomp = property(lambda self: self.data.shape[4])


@dataclass(frozen=True)
class Grid:
    """Rectangular output grid; mode 0 = nearest cell, 1 = cloud-in-cell
    (bilinear/trilinear about cell centres).  ``density``: divide by the cell
    volume (3-D) or area (2-D)."""
    nx: int
    ny: int
    nz: int
    x0: float
    y0: float
    z0: float
    dx: float
    dy: float
    dz: float
    mode: int = 1
    density: bool = False


@dataclass
class Case:
    name: str
    source: Source
    schedule: Schedule
    physics: Physics
    field: Field
    conc_grid: Grid
    dep_grid: Grid
    n_steps: int
    out_every: int = 60

    def output_steps(self):
        """Steps after which the concentration is gridded (Sec. 3.2: every
        n-th step), plus the final step."""
        s = [k for k in range(self.n_steps) if (k + 1) % self.out_every == 0]
        if not s or s[-1] != self.n_steps - 1:
            s.append(self.n_steps - 1)
        return s

    def with_(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# field builders
# ---------------------------------------------------------------------------

def uniform_field(u: float, v: float = 0.0, w: Optional[float] = None,
                  bounded: bool = False) -> Field:
    """A 1 x 1 x 1 field: with clamp-to-edge sampling it is uniform
    everywhere (the paper's homogeneous "artificial" weather)."""
    comps = [u, v] if w is None else [u, v, w]
    data = np.array(comps, dtype=np.float32).reshape(1, 1, 1, 1, len(comps))
    return Field(data, x0=-0.5, y0=-0.5, dx=1.0, dy=1.0, dz=1.0,
                 bounded=bounded)


def _wind_params(rng: np.random.Generator):
    u_ref = rng.uniform(3.0, 8.0)
    theta0 = rng.uniform(0.0, 2.0 * math.pi)
    pairs = [(m, n) for m in range(3) for n in range(3) if (m, n) != (0, 0)]
    modes = []
    for _ in range(4):
        a = rng.uniform(0.0, math.pi / 8.0)
        m, n = pairs[int(rng.integers(0, len(pairs)))]
        phi = rng.uniform(0.0, 2.0 * math.pi)
        modes.append((a, m, n, phi))
    return u_ref, theta0, modes


def wind_field_hour(seed: int, nx: int, ny: int, nz: int, dx: float, dy: float,
                    dz: float, x0: float, y0: float):
    """One hourly wind field [nz][ny][nx][2] in float64.

    Direction: theta0 plus four seeded Fourier modes over the domain;
    speed: power law u_ref (max(z, 1 m)/10)^0.2; no vertical wind."""
    rng = np.random.default_rng(seed)
    u_ref, theta0, modes = _wind_params(rng)
    Lx, Ly = nx * dx, ny * dy
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    zc = (np.arange(nz) + 0.5) * dz
    X, Y = np.meshgrid(xc, yc)          # [ny][nx]
    theta = np.full_like(X, theta0)
    for a, m, n, phi in modes:
        theta += a * np.sin(2.0 * math.pi * (m * X / Lx + n * Y / Ly) + phi)
    speed = u_ref * (np.maximum(zc, 1.0) / 10.0) ** 0.2     # [nz]
    out = np.empty((nz, ny, nx, 2))
    out[..., 0] = speed[:, None, None] * np.cos(theta)[None]
    out[..., 1] = speed[:, None, None] * np.sin(theta)[None]
    return out


def _rng_after_wind(seed: int) -> np.random.Generator:
    """The generator of ``seed`` after the wind parameters were drawn: the
    rain region of a gridded workload continues the same seeded stream."""
    rng = np.random.default_rng(seed)
    _wind_params(rng)
    return rng


def rain_region(rng: np.random.Generator, dx: float) -> Rain:
    cx = rng.uniform(-10e3, 10e3)
    cy = rng.uniform(-10e3, 10e3)
    a = rng.uniform(3e3, 10e3)
    b = rng.uniform(3e3, 10e3)
    ang = rng.uniform(0.0, math.pi)
    return Rain(cx=cx, cy=cy, a=a, b=b, angle=ang, edge=dx / min(a, b))


def wind_field(seeds, nx, ny, nz, dx=250.0, dy=250.0, dz=40.0,
               bounded=True) -> Field:
    """Stack hourly fields (one seed per hour) into a Field centred on the
    origin."""
    x0, y0 = -nx * dx / 2.0, -ny * dy / 2.0
    hours = [wind_field_hour(s, nx, ny, nz, dx, dy, dz, x0, y0) for s in seeds]
    data = np.stack(hours).astype(np.float32)
    return Field(data, x0=x0, y0=y0, dx=dx, dy=dy, dz=dz, t0=0.0,
                 dt_field=3600.0, bounded=bounded)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def c0(n_total: int = 10_000, n_steps: int = 360) -> Case:
    """Uniform wind 5 m/s along x, K_h = 50, K_z = 10 m^2/s, one nuclide with
    lambda = 1e-6 1/s, no deposition, reflecting ground and a lid at 1000 m,
    dt = 10 s (the paper's time step, Sec. 2), Philox seed 0.  Source at
    (0, 0, 50 m); continuous release over the whole run.  Mass per cell on a
    100 x 100 x 20 grid of 100 x 100 x 50 m with origin (-1000, -5000, 0)."""
    src = Source(xs=0.0, ys=0.0, h=50.0, q=1.0)
    sch = Schedule(n_total=n_total, s_release=n_steps)
    phys = Physics(dt=10.0, Kh=50.0, kz_kind=0, Kz_const=10.0,
                   H_mix=1000.0, H_lid=1000.0, lambdas=(1e-6,), seed=0)
    fld = uniform_field(5.0, 0.0, bounded=False)
    g3 = Grid(100, 100, 20, -1000.0, -5000.0, 0.0, 100.0, 100.0, 50.0,
              mode=1, density=False)
    g2 = Grid(100, 100, 1, -1000.0, -5000.0, 0.0, 100.0, 100.0, 1.0,
              mode=1, density=False)
    return Case("c0", src, sch, phys, fld, g3, g2, n_steps, out_every=60)


def _gridded_physics(rain: Rain) -> Physics:
    return Physics(dt=5.0, Kh=50.0, kz_kind=1, kappa_ustar=0.4 * 0.5, z0=0.25,
                   H_mix=1000.0, H_lid=1000.0, h_s=40.0,
                   lambdas=(1e-6, 1e-5), Lambda0=1e-5, rain=rain, seed=0)


def c1(n_total: int = 1_000_000, n_steps: int = 4320, s_release: Optional[int] = None,
       field_seed: int = 1) -> Case:
    """1e6 particles, 6 h at dt = 5 s, steady 200 x 200 x 30 wind field on
    250/250/40 m nodes over [-25, 25] km^2 x [0, 1200] m."""
    nx = ny = 200
    nz = 30
    fld = wind_field([field_seed], nx, ny, nz, 250.0, 250.0, 40.0)
    rain = rain_region(_rng_after_wind(field_seed), 250.0)
    src = Source(xs=0.0, ys=0.0, h=50.0, q=1.0, wind_scale=1.0, v_d=0.002)
    sch = Schedule(n_total=n_total, s_release=s_release or n_steps)
    g3 = Grid(nx, ny, nz, fld.x0, fld.y0, 0.0, 250.0, 250.0, 40.0, mode=1,
              density=True)
    g2 = Grid(nx, ny, 1, fld.x0, fld.y0, 0.0, 250.0, 250.0, 1.0, mode=1,
              density=True)
    return Case("c1", src, sch, _gridded_physics(rain), fld, g3, g2, n_steps,
                out_every=60)


def c2(n_total: int = 16_000_000, n_steps: int = 17280, s_release: int = 4320,
       n_hours: int = 25) -> Case:
    """1.6e7 particles, 24 h at dt = 5 s, 25 hourly 400 x 400 x 40 fields
    (seeds 1000 + k), continuous release over the first 6 h."""
    nx = ny = 400
    nz = 40
    fld = wind_field([1000 + k for k in range(n_hours)], nx, ny, nz,
                     250.0, 250.0, 40.0)
    rain = rain_region(_rng_after_wind(1), 250.0)
    src = Source(xs=0.0, ys=0.0, h=50.0, q=1.0, wind_scale=1.0, v_d=0.002)
    sch = Schedule(n_total=n_total, s_release=s_release)
    g3 = Grid(nx, ny, nz, fld.x0, fld.y0, 0.0, 250.0, 250.0, 40.0, mode=1,
              density=True)
    g2 = Grid(nx, ny, 1, fld.x0, fld.y0, 0.0, 250.0, 250.0, 1.0, mode=1,
              density=True)
    return Case("c2", src, sch, _gridded_physics(rain), fld, g3, g2, n_steps,
                out_every=60)


def c3(seed: int = 3, n_scen: int = 64, n_steps: int = 4320, scale: float = 1.0):
    """Ensemble of release scenarios on the gridded 6 h workload: per
    scenario a particle count log-uniform in [1e4, 1e6] (times ``scale``),
    source height U(10, 200) m, release rate U(0.5, 2) and wind scale
    U(0.8, 1.2), drawn as whole vectors in that order from ``seed``; the
    scenario index is the Philox scenario key.  Returns (base case, sources,
    counts)."""
    rng = np.random.default_rng(seed)
    counts = np.round(10.0 ** rng.uniform(4.0, 6.0, n_scen) * scale).astype(np.int64)
    counts = np.maximum(counts, 1)
    h = rng.uniform(10.0, 200.0, n_scen)
    q = rng.uniform(0.5, 2.0, n_scen)
    sw = rng.uniform(0.8, 1.2, n_scen)
    base = c1(n_total=int(counts.max()), n_steps=n_steps)
    sources = [replace(base.source, h=float(h[c]), q=float(q[c]), wind_scale=float(sw[c]),
                       scenario=c) for c in range(n_scen)]
    return base, sources, [int(n) for n in counts]


def uniform_state(n: int, box, seed: int):
    """Seeded particle state spread uniformly over ``box`` =
    ((x_lo, x_hi), (y_lo, y_hi), (z_lo, z_hi)), mass 1; float32 SoA."""
    rng = np.random.default_rng(seed)
    (xl, xh), (yl, yh), (zl, zh) = box
    x = rng.uniform(xl, xh, n).astype(np.float32)
    y = rng.uniform(yl, yh, n).astype(np.float32)
    z = rng.uniform(zl, zh, n).astype(np.float32)
    m = np.ones(n, dtype=np.float32)
    return x, y, z, m


# ---------------------------------------------------------------------------
# receptor workload (source inversion): gradients of a receptor misfit with
# respect to theta = (h, q, s_w, v_d)
# ---------------------------------------------------------------------------

THETA0 = (50.0, 1.0, 1.0, 0.002)        # where the gradient is taken
THETA_HIDDEN = (80.0, 1.3, 1.1, 0.003)  # source that made the observations


@dataclass(frozen=True)
class Receptors:
    """Receptor points and the Gaussian kernel that turns particle
    activities into their concentrations: horizontal width ``sigma_h`` (m),
    vertical width ``sigma_z`` (m, mirrored at the ground) and the time
    weight of one output step ``weight`` (s)."""
    x: Tuple[float, ...]
    y: Tuple[float, ...]
    z: Tuple[float, ...]
    sigma_h: float = 250.0
    sigma_z: float = 40.0
    weight: float = 300.0

    @property
    def n(self) -> int:
        return len(self.x)


def with_theta(case: Case, theta) -> Case:
    """The case with source height, release rate, wind scale and deposition
    velocity set to ``theta``."""
    h, q, sw, vd = (float(t) for t in theta)
    return case.with_(source=replace(case.source, h=h, q=q, wind_scale=sw, v_d=vd))


def c4(n_total: int = 1_000_000, n_steps: int = 4320, seed: int = 0) -> Case:
    """The 1e6-particle 6 h gridded workload at theta0 (h = 50 m, q = 1,
    s_w = 1, v_d = 0.002 m/s) with Philox seed ``seed``; output every 60
    steps (the checkpoint interval of the gradient)."""
    c = c1(n_total=n_total, n_steps=n_steps)
    c = c.with_(physics=replace(c.physics, seed=seed))
    return with_theta(c, THETA0)


def load_receptors(path: str):
    """Receptors and observations stored as JSON (written by the script
    next to the file).  Returns (Receptors, observations, meta)."""
    import json
    with open(path) as f:
        d = json.load(f)
    r = Receptors(tuple(d["x"]), tuple(d["y"]), tuple(d["z"]), d["sigma_h"], d["sigma_z"],
                  d["weight"])
    return r, np.asarray(d["observations"], dtype=np.float64), d
