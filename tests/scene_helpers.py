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
