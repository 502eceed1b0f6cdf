"""Seeded synthetic scene generators (inputs only; none of the solver's arithmetic).

This module produces initial particle states for the rigid-body workloads the
solver is measured and tested on.  It draws positions, velocities and masses,
and nothing else: rest poses, centres of mass, contacts and every other quantity
of the PBD-R method are computed independently by the solver and by the FP64
reference, never here.

Shapes follow the paper's packing of primitives (Sec. IV-B "Shape
Representations"): equal-radius spheres on a uniform lattice with spacing 2r,
i.e. touching but not overlapping.  Workload sizes and distributions:

* ``drop_cubes``    8 lattice cubes 4x4x4, r = 0.05 m, 1 kg per particle, drop
                    heights U(0.5, 2) m, velocity N(0, 0.5) m/s per body.
* ``cuboid_rain``   1000 cuboids with per-axis sizes U{3..8}, r = 0.01 m,
                    density U(500, 2000) kg/m^3, uniform random orientation,
                    centres in a 2 x 2 x 4 m box.
* ``dense_pile``    20k mixed cuboid / sphere-lattice bodies, log-normal counts
                    (mean 100, clipped [8, 1024]), r = 0.01 m, walled 4 x 4 m bin.
* ``batch_scenes``  many independent small scenes (log-normal 100-5000
                    particles, 1-50 bodies) with per-scene gravity and friction.
* ``serving_trace`` Poisson arrivals of rollout requests.

Arrays are structure-of-arrays: ``x`` and ``v`` are float32 ``[3, N]``,
``mass`` float32 ``[N]``, ``body_start`` int32 ``[B + 1]`` (particles of body b
are ``body_start[b]:body_start[b+1]``; bodies are contiguous and non-empty).
All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GROUND = (0.0, 0.0, 1.0, 0.0)  # half-space n.x >= d + r with n = +z, d = 0


@dataclasses.dataclass
class Scene:
    """One scene: state, body partition and solver parameters (SI units)."""

    x: np.ndarray            # float32 [3, N]
    v: np.ndarray            # float32 [3, N]
    mass: np.ndarray         # float32 [N]
    body_start: np.ndarray   # int32 [B + 1]
    radius: float
    dt_frame: float = 1.0 / 240.0
    substeps: int = 4
    iterations: int = 10
    gravity: tuple = (0.0, 0.0, -9.81)
    mu: float = 0.4
    planes: tuple = (GROUND,)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_bodies(self) -> int:
        return int(self.body_start.shape[0] - 1)

    def body_of_particle(self) -> np.ndarray:
        counts = np.diff(self.body_start)
        return np.repeat(np.arange(self.n_bodies, dtype=np.int32), counts)

    def copy(self) -> "Scene":
        return dataclasses.replace(self, x=self.x.copy(), v=self.v.copy(),
                                   mass=self.mass.copy(),
                                   body_start=self.body_start.copy())


# ----------------------------------------------------------------------------
# shape primitives (lattice offsets about the lattice centre, spacing 2r)
# ----------------------------------------------------------------------------

def lattice_box(nx: int, ny: int, nz: int, spacing: float) -> np.ndarray:
    """Offsets [3, nx*ny*nz] of a box lattice, centred on the lattice centre."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()]).astype(np.float64)
    pts -= np.array([[nx - 1], [ny - 1], [nz - 1]], dtype=np.float64) / 2.0
    return pts * spacing


def lattice_ball(target: int, spacing: float) -> np.ndarray:
    """Lattice points inside a ball whose volume holds about ``target`` cells."""
    rad = (3.0 * target / (4.0 * math.pi)) ** (1.0 / 3.0)  # in lattice units
    k = int(math.ceil(rad)) + 1
    g = np.arange(-k, k + 1, dtype=np.float64)
    ix, iy, iz = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()])
    keep = (pts ** 2).sum(axis=0) <= rad * rad
    pts = pts[:, keep]
    if pts.shape[1] == 0:
        pts = np.zeros((3, 1))
    return pts * spacing


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix (Shoemake's unit-quaternion method)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    qw, qx = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qy, qz = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def _bounding_radius(offsets: np.ndarray, r: float) -> float:
    return float(np.sqrt((offsets ** 2).sum(axis=0)).max()) + r


def _assemble(parts: List[np.ndarray], vels: List[np.ndarray], masses: List[float]):
    counts = [p.shape[1] for p in parts]
    x = np.concatenate(parts, axis=1).astype(np.float32)
    v = np.concatenate([np.repeat(vv.reshape(3, 1), c, axis=1) for vv, c in zip(vels, counts)],
                       axis=1).astype(np.float32)
    m = np.concatenate([np.full(c, mm, dtype=np.float32) for mm, c in zip(masses, counts)])
    bs = np.zeros(len(parts) + 1, dtype=np.int32)
    bs[1:] = np.cumsum(counts)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m, bs


def _place(rng, radii, lo, hi, gap, max_tries=20000):
    """Rejection-sample non-overlapping bounding spheres inside [lo, hi]."""
    centres = np.zeros((len(radii), 3))
    placed_r = np.zeros(len(radii))
    for i, rb in enumerate(radii):
        for _ in range(max_tries):
            c = lo + rb + rng.random(3) * (hi - lo - 2 * rb)
            if i == 0:
                break
            d = np.sqrt(((centres[:i] - c) ** 2).sum(axis=1))
            if np.all(d >= placed_r[:i] + rb + gap):
                break
        else:
            raise RuntimeError("could not place body %d without overlap" % i)
        centres[i] = c
        placed_r[i] = rb
    return centres


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def drop_cubes(seed: int = 0, n_cubes: int = 8, side: int = 4, radius: float = 0.05,
               frames: int = 200) -> Scene:
    """8 lattice cubes (4x4x4, 512 particles) dropped on the ground.

    Unit mass per particle; centre heights U(0.5, 2) m, horizontal centres
    U(-1, 1) m, axis-aligned, one N(0, 0.5^2) velocity per body and component.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    off = lattice_box(side, side, side, 2 * radius)
    rb = _bounding_radius(off, radius)
    parts, vels = [], []
    centres = np.zeros((n_cubes, 3))
    for i in range(n_cubes):
        for _ in range(100000):
            c = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2.0)])
            if i == 0 or np.all(np.sqrt(((centres[:i] - c) ** 2).sum(axis=1)) >= 2 * rb + 1e-3):
                break
        centres[i] = c
        parts.append(off + c.reshape(3, 1))
        vels.append(rng.normal(0.0, 0.5, size=3))
    x, v, m, bs = _assemble(parts, vels, [1.0] * n_cubes)
    return Scene(x, v, m, bs, radius=radius, name="drop_cubes_8x64")


def _cuboid_bodies(rng, n_bodies, radius, size_lo=3, size_hi=8):
    offs, masses = [], []
    for _ in range(n_bodies):
        nx, ny, nz = rng.integers(size_lo, size_hi + 1, size=3)
        rho = rng.uniform(500.0, 2000.0)
        rot = random_rotation(rng)
        offs.append(rot @ lattice_box(int(nx), int(ny), int(nz), 2 * radius))
        masses.append(rho * (2 * radius) ** 3)
    return offs, masses


def cuboid_rain(seed: int = 0, n_bodies: int = 1000, radius: float = 0.01,
                box=(2.0, 2.0, 4.0)) -> Scene:
    """1000 randomly oriented cuboid lattices (sizes U{3..8} per axis) in a 2x2x4 m box.

    Density U(500, 2000) kg/m^3, so each particle has mass rho (2r)^3.  Bodies
    are rejection-sampled so no two particles of different bodies start closer
    than 2r and every particle starts above the ground (z >= r).  Zero initial
    velocity.  E[N] = 5.5^3 * 1000, about 166k particles.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    offs, masses = _cuboid_bodies(rng, n_bodies, radius)
    radii = [_bounding_radius(o, radius) for o in offs]
    lo = np.array([-box[0] / 2, -box[1] / 2, 0.0])
    hi = np.array([box[0] / 2, box[1] / 2, box[2]])
    centres = _place(rng, radii, lo, hi, gap=1e-4)
    parts = [o + c.reshape(3, 1) for o, c in zip(offs, centres)]
    vels = [np.zeros(3)] * n_bodies
    x, v, m, bs = _assemble(parts, vels, masses)
    return Scene(x, v, m, bs, radius=radius, name="cuboid_rain_1000")


def dense_pile(seed: int = 0, n_bodies: int = 20000, radius: float = 0.01,
               half_width: float = 2.0, sigma: float = 0.5, mean_count: float = 100.0,
               gap_frac: float = 0.05, speed: float = 0.5, packed: bool = False) -> Scene:
    """20k mixed bodies packed tightly into a walled 4 x 4 m bin.

    Particle counts are log-normal (sigma 0.5, mean 100), clipped to [8, 1024];
    half the bodies are near-cubic cuboids, half are lattice balls.  Bodies are
    shelf-packed in layers with a gap of ``gap_frac * r`` between bounding
    spheres, with random orientations and N(0, speed^2) velocities, so contacts
    start within the first substeps.  Solver settings: 8 substeps x 20
    iterations, walls at x, y = +-2 m.

    ``packed``: the same bodies without rotation, shelf-packed by their
    bounding boxes (gap ``gap_frac * r`` between the boxes of the particle
    spheres) from the ground up: a pile that is dense from the start, with
    faces of neighbouring bodies in contact when gap_frac < 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mu_ln = math.log(mean_count) - 0.5 * sigma * sigma
    counts = np.clip(np.round(rng.lognormal(mu_ln, sigma, size=n_bodies)), 8, 1024).astype(int)
    offs, masses = [], []
    for c in counts:
        if rng.random() < 0.5:
            a = max(2, int(round(c ** (1.0 / 3.0))))
            b = max(2, int(round(math.sqrt(c / a))))
            cz = max(1, int(round(c / (a * b))))
            o = lattice_box(a, b, cz, 2 * radius)
        else:
            o = lattice_ball(int(c), 2 * radius)
        rot = random_rotation(rng)
        offs.append(o if packed else rot @ o)
        masses.append(rng.uniform(500.0, 2000.0) * (2 * radius) ** 3)
    if packed:
        return _box_packed_pile(rng, offs, masses, radius, half_width, gap_frac, speed)
    radii = np.array([_bounding_radius(o, radius) for o in offs])
    gap = gap_frac * radius
    # shelf packing: rows along x, rows stacked along y, layers along z
    centres = np.zeros((n_bodies, 3))
    lo = -half_width + radius * 0.5
    hi = half_width - radius * 0.5
    x0, y0, z0 = lo, lo, 0.0
    row_h, layer_h = 0.0, 0.0
    for i, rb in enumerate(radii):
        d = 2 * rb + gap
        if x0 + d > hi:
            x0 = lo
            y0 += row_h
            row_h = 0.0
        if y0 + d > hi:
            y0 = lo
            z0 += layer_h
            layer_h = 0.0
        centres[i] = (x0 + d / 2, y0 + d / 2, z0 + d / 2)
        x0 += d
        row_h = max(row_h, d)
        layer_h = max(layer_h, d)
    parts = [o + c.reshape(3, 1) for o, c in zip(offs, centres)]
    vels = [rng.normal(0.0, speed, size=3) for _ in range(n_bodies)]
    x, v, m, bs = _assemble(parts, vels, masses)
    walls = ((1.0, 0.0, 0.0, -half_width), (-1.0, 0.0, 0.0, -half_width),
             (0.0, 1.0, 0.0, -half_width), (0.0, -1.0, 0.0, -half_width))
    return Scene(x, v, m, bs, radius=radius, substeps=8, iterations=20,
                 planes=(GROUND,) + walls, name="dense_pile_20k")


def _box_packed_pile(rng, offs, masses, radius, half_width, gap_frac, speed) -> Scene:
    """Bodies shelf-packed by bounding boxes (rows along x, rows along y,
    layers along z, from z = 0 up) in the walled bin of ``dense_pile``."""
    gap = gap_frac * radius
    lo_b = -half_width + radius * 0.5
    hi_b = half_width - radius * 0.5
    x0, y0, z0 = lo_b, lo_b, 0.0
    row_h, layer_h = 0.0, 0.0
    parts = []
    for o in offs:
        omin, omax = o.min(axis=1) - radius, o.max(axis=1) + radius
        ext = omax - omin + gap
        if x0 + ext[0] > hi_b:
            x0 = lo_b
            y0 += row_h
            row_h = 0.0
        if y0 + ext[1] > hi_b:
            y0 = lo_b
            z0 += layer_h
            layer_h = 0.0
        parts.append(o + (np.array([x0, y0, z0]) - omin).reshape(3, 1))
        x0 += ext[0]
        row_h = max(row_h, ext[1])
        layer_h = max(layer_h, ext[2])
    vels = [rng.normal(0.0, speed, size=3) for _ in offs]
    x, v, m, bs = _assemble(parts, vels, masses)
    walls = ((1.0, 0.0, 0.0, -half_width), (-1.0, 0.0, 0.0, -half_width),
             (0.0, 1.0, 0.0, -half_width), (0.0, -1.0, 0.0, -half_width))
    return Scene(x, v, m, bs, radius=radius, substeps=8, iterations=20,
                 planes=(GROUND,) + walls, name="dense_pile_20k")


def small_scene(rng: np.random.Generator, n_target: int, radius: float = 0.01,
                gravity_z: Optional[float] = None, mu: Optional[float] = None, max_bodies: int = 50) -> Scene:
    """A scene of cuboid bodies (as in ``cuboid_rain``) totalling about n_target particles.

    Bodies are drawn until the target is reached (at least 1, at most
    ``max_bodies``); the spawn box grows with the body count.  Gravity magnitude
    U(5, 15) along -z and friction U(0, 1) unless given.
    """
    offs, masses = [], []
    total = 0
    while total < n_target and len(offs) < max_bodies:
        o, mm = _cuboid_bodies(rng, 1, radius)
        offs += o
        masses += mm
        total += o[0].shape[1]
    radii = [_bounding_radius(o, radius) for o in offs]
    side = 0.3 + 0.25 * len(offs) ** (1.0 / 3.0)
    lo = np.array([-side / 2, -side / 2, 0.0])
    hi = np.array([side / 2, side / 2, 2 * side])
    centres = _place(rng, radii, lo, hi, gap=1e-4)
    parts = [o + c.reshape(3, 1) for o, c in zip(offs, centres)]
    vels = [np.zeros(3)] * len(offs)
    x, v, m, bs = _assemble(parts, vels, masses)
    gz = -rng.uniform(5.0, 15.0) if gravity_z is None else gravity_z
    mu_s = rng.uniform(0.0, 1.0) if mu is None else mu
    return Scene(x, v, m, bs, radius=radius, gravity=(0.0, 0.0, gz), mu=mu_s,
                 name="small_%d" % total)


def batch_scenes(seed: int = 0, n_scenes: int = 4096, lo: int = 100, hi: int = 5000) -> List[Scene]:
    """Independent scenes with log-normal sizes (1st/99th percentile 100/5000 particles).

    ln N ~ N(ln 707, 0.841^2) clipped to [lo, hi]; bodies as in ``cuboid_rain``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.clip(np.exp(rng.normal(math.log(707.0), 0.841, size=n_scenes)), lo, hi).astype(int)
    return [small_scene(rng, int(s)) for s in sizes]


@dataclasses.dataclass
class Request:
    arrival_s: float
    scene: Scene
    frames: int
    request_id: int


def serving_trace(seed: int = 0, rate_hz: float = 200.0, duration_s: float = 2.0,
                  lo: int = 200, hi: int = 50000, h_lo: int = 50, h_hi: int = 500,
                  max_bodies: int = 256) -> List[Request]:
    """Poisson arrivals of rollout requests.

    Target sizes log-uniform in [lo, hi] particles (built like ``small_scene``
    with at most ``max_bodies`` bodies, so the largest scenes hold about 42k
    particles), horizons uniform in {h_lo..h_hi} frames.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out: List[Request] = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        sc = small_scene(rng, n, max_bodies=max_bodies)
        out.append(Request(t, sc, int(rng.integers(h_lo, h_hi + 1)), len(out)))
    return out


def single_body(offsets: np.ndarray, centre=(0.0, 0.0, 0.0), velocity=(0.0, 0.0, 0.0),
                mass: float = 1.0, radius: float = 0.05, **kw) -> Scene:
    """A scene with one body made of the given lattice offsets (for tests)."""
    c = np.asarray(centre, dtype=np.float64).reshape(3, 1)
    x, v, m, bs = _assemble([offsets + c], [np.asarray(velocity, dtype=np.float64)], [mass])
    return Scene(x, v, m, bs, radius=radius, **kw)


def from_bodies(parts, vels, masses, radius: float, **kw) -> Scene:
    """A scene from explicit per-body particle positions [3, n_b], velocities and masses."""
    x, v, m, bs = _assemble([np.asarray(p, dtype=np.float64) for p in parts],
                            [np.asarray(vv, dtype=np.float64) for vv in vels],
                            list(masses))
    return Scene(x, v, m, bs, radius=radius, **kw)


WORKLOADS = {
    "drop_cubes_8x64": drop_cubes,
    "cuboid_rain_1000": cuboid_rain,
    "dense_pile_20k": dense_pile,
}
