"""Test scenes built from explicit bodies (inputs only)."""
import math

import numpy as np

from paper_2603_14634_amd import scenes


def touching_bodies(sizes, r=0.01, seed=0, speed=0.3, pen=0.6, **kw):
    """Bodies of the given particle counts (partial lattice cubes, random
    orientation) in a row along x, each moved so that its closest particle pair
    with the previous body is 2r - pen*r apart."""
    rng = np.random.default_rng(seed)
    parts, vels, masses = [], [], []
    prev = None
    for n in sizes:
        if n == 1:
            off = np.zeros((3, 1))
        else:
            a = int(math.ceil(n ** (1.0 / 3.0)))
            off = scenes.lattice_box(a, a, a, 2 * r)[:, :n]
            off = off - off.mean(axis=1, keepdims=True)
        off = scenes.random_rotation(rng) @ off
        pts = off + np.array([[0.0], [0.0], [0.1 + np.abs(off[2]).max()]])
        if prev is not None:
            pts[0] += prev[0].max() + 2 * r - pts[0].min() + 4 * r
            for _ in range(200):
                d = np.sqrt(((pts[:, :, None] - prev[:, None, :]) ** 2).sum(axis=0)).min()
                if abs(d - (2 - pen) * r) < 1e-4 * r:
                    break
                pts[0] -= d - (2 - pen) * r
        parts.append(pts)
        prev = pts
        vels.append(rng.normal(0, speed, size=3))
        masses.append(rng.uniform(0.01, 0.03))
    return scenes.from_bodies(parts, vels, masses, radius=r, **kw)


def interleaved_lattices(n_pairs, r=0.01, depth=0.2, seed=0, **kw):
    """Pairs of 4 x 4 x 4 lattices, the second shifted by half the x spacing
    into the first: the x spacing is (4 - 2 depth) r, so a particle between two
    of the other body's on its x row is 2r - depth r from each (two contacts),
    one at a row's end from one.  112 contact pairs per body; the pairs sit in
    a grid 24r / 12r / 12r apart, above the ground."""
    rng = np.random.default_rng(seed)
    pitch = (4.0 - 2.0 * depth) * r
    g = np.arange(4)
    X, Y, Z = np.meshgrid(g * pitch, g * 2.5 * r, g * 2.5 * r, indexing="ij")
    lattice = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    side = int(math.ceil(n_pairs ** (1.0 / 3.0)))
    parts, vels, masses = [], [], []
    for k in range(n_pairs):
        o = np.array([[(k % side) * 24 * r], [((k // side) % side) * 12 * r], [0.2 + (k // (side * side)) * 12 * r]])
        a = lattice + o
        b = a.copy()
        b[0] += pitch / 2.0
        for pts in (a, b):
            parts.append(pts)
            vels.append(rng.normal(0.0, 0.02, size=3))
            masses.append(float(rng.uniform(0.01, 0.03)))
    return scenes.from_bodies(parts, vels, masses, radius=r, **kw)
