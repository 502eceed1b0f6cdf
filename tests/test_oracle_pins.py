"""Pins of the FP64 reference against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form,
an exact identity, a library routine, a different algorithm, or brute force.
They are CPU-only.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2603_14634_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _body_scene(off, centre=(0.0, 0.0, 0.0), velocity=(0.0, 0.0, 0.0), mass=1.0, radius=0.05, **kw):
    return scenes.single_body(off, centre=centre, velocity=velocity, mass=mass, radius=radius, **kw)


def _run(orc, sc, n_substeps=1, accel=None, **pkw):
    p = orc.params_for(sc, **pkw)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v, mx = orc.substep(p, rest, sc.x, sc.v, accel=accel, n_substeps=n_substeps)
    return x, v, mx, p, rest


# --------------------------------------------------------------------------
# integration step (Alg. 1, first loop): discrete free fall closed form
# --------------------------------------------------------------------------

def test_free_fall_matches_symplectic_euler_closed_form(orc):
    g = np.array([0.3, -0.2, -9.81])
    v0 = np.array([0.5, 0.1, 2.0])
    sc = _body_scene(scenes.lattice_box(4, 3, 5, 0.1), centre=(0.1, -0.2, 3.0), velocity=v0,
                     gravity=tuple(g), planes=())
    n = 37
    v0 = sc.v[:, 0].astype(np.float64)        # the state is stored in FP32
    x, v, mx, p, _ = _run(orc, sc, n_substeps=n)
    h = p.h
    # v_n = v0 + n h g ; x_n = x0 + n h v0 + h^2 g n(n+1)/2
    v_ref = v0 + n * h * g
    x_ref = sc.x.astype(np.float64) + (n * h * v0 + h * h * g * n * (n + 1) / 2.0)[:, None]
    assert mx == 0
    np.testing.assert_allclose(v, np.repeat(v_ref[:, None], sc.n, axis=1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x, x_ref, rtol=1e-12, atol=1e-12)


def test_constant_velocity_without_gravity(orc):
    v0 = np.array([-1.5, 0.25, 0.75])
    sc = _body_scene(scenes.lattice_box(3, 3, 3, 0.1), centre=(0.0, 0.0, 1.0), velocity=v0,
                     gravity=(0.0, 0.0, 0.0), planes=())
    v0 = sc.v[:, 0].astype(np.float64)
    x, v, _, p, _ = _run(orc, sc, n_substeps=25)
    np.testing.assert_allclose(x, sc.x + (25 * p.h * v0)[:, None], rtol=0, atol=1e-13)
    np.testing.assert_allclose(v, np.repeat(v0[:, None], sc.n, axis=1), rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# ground contact and friction (constraint (1)) on a single particle
# --------------------------------------------------------------------------

def _particle(z, vt=(0.0, 0.0), r=0.05, mu=0.0, iterations=1):
    return _body_scene(np.zeros((3, 1)), centre=(0.0, 0.0, z), velocity=(vt[0], vt[1], 0.0),
                       radius=r, gravity=(0.0, 0.0, 0.0), mu=mu, iterations=iterations)


def test_ground_pushes_out_exactly_the_penetration(orc):
    r = 0.05
    sc = _particle(r - 1e-3)
    pen = r - float(sc.x[2, 0])           # penetration of the FP32-stored start
    x, v, _, p, _ = _run(orc, sc)
    assert x[2, 0] == pytest.approx(r, abs=1e-15)
    assert v[2, 0] == pytest.approx(pen / p.h, rel=1e-12)
    assert x[0, 0] == 0.0 and x[1, 0] == 0.0


@pytest.mark.parametrize("speed_scale", [0.5, 3.0])
def test_ground_friction_static_and_kinetic(orc, speed_scale):
    r, mu = 0.05, 0.4
    sc0 = _particle(r - 1e-3, mu=mu)
    pen = r - float(sc0.x[2, 0])
    h = sc0.dt_frame / sc0.substeps
    ut = speed_scale * mu * pen          # tangential displacement over the substep
    sc = _particle(r - 1e-3, vt=(ut / h * 0.6, ut / h * 0.8), mu=mu)
    x, v, _, p, _ = _run(orc, sc)
    u = h * sc.v[:2, 0].astype(np.float64)
    ut = float(np.linalg.norm(u))
    moved = x[:2, 0] - sc.x[:2, 0].astype(np.float64)
    if ut <= mu * pen:       # static: the whole tangential displacement is removed
        np.testing.assert_allclose(moved, 0.0, atol=1e-15)
    else:                    # kinetic: it shrinks by mu * pen
        np.testing.assert_allclose(moved, u * (1.0 - mu * pen / ut), rtol=1e-12, atol=1e-16)
    assert x[2, 0] == pytest.approx(r, abs=1e-15)


# --------------------------------------------------------------------------
# particle-particle contact (constraint (2)): mass split and momentum
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m1,m2", [(1.0, 1.0), (1.0, 3.0)])
def test_pair_contact_splits_penetration_by_inverse_mass(orc, m1, m2):
    r, pen = 0.05, 2e-3
    d = 2 * r - pen
    sc = scenes.from_bodies([np.array([[-d / 2], [0.0], [0.0]]), np.array([[d / 2], [0.0], [0.0]])],
                            [np.zeros(3), np.zeros(3)], [m1, m2], radius=r,
                            gravity=(0.0, 0.0, 0.0), planes=(), iterations=1)
    x, v, mx, _, _ = _run(orc, sc)
    assert mx == 1
    pen = 2 * r - (float(sc.x[0, 1]) - float(sc.x[0, 0]))
    w1, w2 = 1.0 / m1, 1.0 / m2
    assert x[0, 0] - sc.x[0, 0] == pytest.approx(-pen * w1 / (w1 + w2), rel=1e-9)
    assert x[0, 1] - sc.x[0, 1] == pytest.approx(pen * w2 / (w1 + w2), rel=1e-9)
    assert m1 * v[0, 0] + m2 * v[0, 1] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_particle_bodies_move_only_by_contact(orc, seed):
    # three one-particle bodies on the x axis, overlapping by pen: a one-particle
    # body has no shape-matching goal offset and no rotational inertia, so only
    # the pair corrections act, along x; the middle one has two neighbours.
    rng = np.random.default_rng(seed)
    r, pen = 0.01, 0.006
    m = rng.uniform(0.005, 0.05, size=3)
    xs = np.array([0.0, 2 * r - pen, 2 * (2 * r - pen)]) + rng.uniform(-1, 1)
    sc = scenes.from_bodies([np.array([[x], [0.25], [0.5]]) for x in xs], [np.zeros(3)] * 3, list(m),
                            radius=r, gravity=(0.0, 0.0, 0.0), planes=(), mu=0.0, iterations=1)
    x, v, mx, _, _ = _run(orc, sc)
    assert mx == 2
    m = sc.mass.astype(np.float64)                        # stored in FP32
    x0 = sc.x.astype(np.float64)
    np.testing.assert_array_equal(x[1:], x0[1:])          # nothing moves in y or z
    gaps = np.diff(x0[0])
    corr = [m[1] / (m[0] + m[1]) * (2 * r - gaps[0]) / 2, m[2] / (m[1] + m[2]) * (2 * r - gaps[1]) / 2]
    expect = x0[0] + np.array([-corr[0],
                               m[0] / (m[0] + m[1]) * (2 * r - gaps[0]) / 2 - corr[1],
                               m[1] / (m[1] + m[2]) * (2 * r - gaps[1]) / 2])
    np.testing.assert_allclose(x[0], expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("avg", ["own", "none"])
@pytest.mark.parametrize("seed", [0, 1])
def test_pair_weight_modes_on_a_chain(orc, avg, seed):
    # the chain of the test above under the two other pair weights: 1/n_p
    # (each particle averages over its own list) and 1 (plain sum).  The middle
    # particle has two neighbours, the ends one, so the modes differ there and
    # at the ends by a factor of two.
    rng = np.random.default_rng(20 + seed)
    r, pen = 0.01, 0.006
    m = rng.uniform(0.005, 0.05, size=3)
    xs = np.array([0.0, 2 * r - pen, 2 * (2 * r - pen)]) + rng.uniform(-1, 1)
    flags = orc.PP_AVG_OWN if avg == "own" else orc.PP_AVG_NONE
    sc = scenes.from_bodies([np.array([[x], [0.25], [0.5]]) for x in xs], [np.zeros(3)] * 3, list(m),
                            radius=r, gravity=(0.0, 0.0, 0.0), planes=(), mu=0.0, iterations=1)
    x, v, mx, p, _ = _run(orc, sc, flags=flags)
    assert mx == 2
    m = sc.mass.astype(np.float64)
    x0 = sc.x.astype(np.float64)
    gaps = np.diff(x0[0])
    p01, p12 = 2 * r - gaps[0], 2 * r - gaps[1]
    # inverse-mass shares of each pair: w_a / (w_a + w_b) = m_b / (m_a + m_b)
    a0, a1 = m[1] / (m[0] + m[1]), m[0] / (m[0] + m[1])
    b1, b2 = m[2] / (m[1] + m[2]), m[1] / (m[1] + m[2])
    wmid = 0.5 if avg == "own" else 1.0                 # the middle particle's own weight
    expect = x0[0] + np.array([-a0 * p01, wmid * (a1 * p01 - b1 * p12), b2 * p12])
    np.testing.assert_allclose(x[0], expect, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(x[1:], x0[1:])
    np.testing.assert_allclose(v[0] * p.h, x[0] - x0[0], rtol=0, atol=1e-15)
    P = (m * v[0]).sum()
    if avg == "none":          # equal and opposite corrections: momentum kept
        assert P == pytest.approx(0.0, abs=1e-12 * np.abs(m * v[0]).max())
    else:                      # 1/n_p is not symmetric: the ends push twice as hard
        assert abs(P) > 1e-3 * np.abs(m * v[0]).max()


def _sliding_pair(m1, m2, s, mu, r=0.05, pen=4e-3):
    # Two one-particle bodies with h = 1/1024 s (dt_frame 1/256 s, 4 substeps;
    # every product below is exact in FP32).  Particle 0 starts at (-a, -h s, 0)
    # moving +s along y, particle 1 at (a, h s, 0) moving -s: after the
    # integration step both lie on the x axis, so the contact normal is x and
    # their relative displacement since X_init, (0, 2 h s, 0), is tangential.
    h = 1.0 / 1024.0
    a = (2 * r - pen) / 2
    sc = scenes.from_bodies([np.array([[-a], [-h * s], [0.0]]), np.array([[a], [h * s], [0.0]])],
                            [np.array([0.0, s, 0.0]), np.array([0.0, -s, 0.0])], [m1, m2], radius=r,
                            gravity=(0.0, 0.0, 0.0), planes=(), mu=mu, iterations=1,
                            dt_frame=1.0 / 256.0, substeps=4)
    return sc, h


@pytest.mark.parametrize("kind", ["static", "kinetic"])
@pytest.mark.parametrize("m1,m2", [(1.0, 1.0), (0.5, 2.5)])
def test_pair_friction_static_and_kinetic(orc, kind, m1, m2):
    mu, pen = 0.5, 4e-3
    # |u_t| = 2 h s against mu * pen = 2e-3: 1e-3 (static) or 6e-3 (kinetic)
    s = 0.512 if kind == "static" else 3.072
    sc, h = _sliding_pair(m1, m2, s, mu, pen=pen)
    x, v, mx, p, _ = _run(orc, sc)
    assert mx == 1 and p.h == h
    x0 = sc.x.astype(np.float64)
    sv = float(sc.v[1, 0])
    assert h * sv + x0[1, 0] == 0.0                    # exactly on the x axis after prediction
    m = sc.mass.astype(np.float64)
    w = 1.0 / m
    al = w / w.sum()                                   # each particle's share of the pair
    pe = 2 * sc.radius - (x0[0, 1] - x0[0, 0])         # penetration of the stored positions
    ut = 2 * h * sv
    removed = ut if kind == "static" else mu * pe      # tangential displacement taken away
    moved = x - x0
    # normal: the penetration, split by inverse mass
    np.testing.assert_allclose(moved[0], [-al[0] * pe, al[1] * pe], rtol=1e-13, atol=1e-17)
    # tangential: the relative slip shrinks by `removed`, split the same way
    np.testing.assert_allclose(moved[1], [h * sv - al[0] * removed, -h * sv + al[1] * removed],
                               rtol=1e-13, atol=1e-17)
    slip = moved[1, 0] - moved[1, 1]
    if kind == "static":
        assert abs(slip) <= 1e-15                       # the slip is removed entirely
    else:
        assert slip == pytest.approx(ut - mu * pe, rel=1e-12)
    np.testing.assert_array_equal(moved[2], 0.0)
    np.testing.assert_allclose(v * h, moved, rtol=0, atol=1e-16)
    np.testing.assert_allclose((m * v).sum(axis=1), (m * sc.v.astype(np.float64)).sum(axis=1), rtol=0,
                               atol=1e-13)


@pytest.mark.parametrize("flags", [0, 1])
def test_sliding_block_velocity_in_both_update_modes(orc, flags):
    # A 3x2 lattice plate (one body) starts a depth pen inside the ground,
    # sliding along a diagonal of the plane with no gravity.  Iteration 1 pushes
    # every particle out by pen and kinetic friction removes mu * pen of the
    # tangential displacement; iterations 2 and 3 find nothing to correct, and
    # shape matching and the momentum constraint leave the uniform motion alone.
    # With either velocity update (incremental, or standard PBD's
    # (X_K - X_init) / h) the velocity after K = 3 iterations is the whole
    # substep's displacement over h.
    r, pen, mu = 0.05, 1e-3, 0.4
    vt = np.array([0.6, 0.8]) * 2.0
    sc = _body_scene(scenes.lattice_box(3, 2, 1, 2 * r), centre=(0.1, -0.2, r - pen),
                     velocity=(vt[0], vt[1], 0.0), radius=r, gravity=(0.0, 0.0, 0.0), mu=mu, iterations=3)
    x, v, _, p, _ = _run(orc, sc, flags=flags)
    h = p.h
    x0 = sc.x.astype(np.float64)
    pe = r - x0[2, 0]
    u = h * sc.v[:2, 0].astype(np.float64)
    un = float(np.linalg.norm(u))
    assert un > mu * pe                                     # kinetic
    moved = x - x0
    np.testing.assert_allclose(moved[:2], np.repeat((u * (1.0 - mu * pe / un))[:, None], sc.n, axis=1),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(x[2], r, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v, moved / h, rtol=0, atol=1e-12)


def test_standard_and_incremental_velocity_agree_in_contact(orc):
    # In exact arithmetic V_{i+1} = V_i + dX_i / h and (X_{i+1} - X_init) / h
    # are the same after every iteration, momentum correction included; in FP64
    # the two branches agree to rounding, also with contacts, shape matching
    # and the momentum correction all acting.
    sc = scenes.drop_cubes(seed=1)
    p = orc.params_for(sc)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v, _ = orc.substep(p, rest, sc.x, sc.v, n_substeps=4 * 150)   # first cubes have landed
    assert (x[2] < sc.radius).any()
    xi, vi, _ = orc.substep(p, rest, x, v)
    xs, vs, _ = orc.substep(orc.params_for(sc, flags=orc.STD_VELOCITY), rest, x, v)
    np.testing.assert_allclose(vs * p.h, xs - x, rtol=0, atol=1e-12 * p.h * np.abs(vs).max())
    np.testing.assert_allclose(xs, xi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(vs, vi, rtol=0, atol=1e-9 * np.abs(vi).max())
    assert np.abs(vi - v).max() > 1e-2                       # the contacts did act


def test_symmetric_averaging_conserves_total_momentum(orc):
    rng = np.random.default_rng(7)
    r = 0.05
    off = scenes.lattice_box(3, 3, 3, 2 * r)
    parts, vels, masses = [], [], []
    for k in range(6):
        parts.append(scenes.random_rotation(rng) @ off + rng.uniform(-0.25, 0.25, size=(3, 1)))
        vels.append(rng.normal(0, 1.0, size=3))
        masses.append(rng.uniform(0.5, 2.0))
    for mu in (0.0, 0.4):
        sc = scenes.from_bodies(parts, vels, masses, radius=r, gravity=(0.0, 0.0, 0.0), planes=(), mu=mu)
        x, v, mx, _, rest = _run(orc, sc, n_substeps=20)
        assert mx >= 2
        P0 = (sc.v.astype(np.float64) * rest.mass).sum(axis=1)
        P1 = (v * rest.mass).sum(axis=1)
        np.testing.assert_allclose(P1, P0, rtol=0, atol=1e-12 * np.abs(P0).max())


def _amplification(orc, sc, flags, seeds=3, eps=1e-9, rest=None, threads=1):
    """Largest change of the reference's substep per unit of a random velocity
    perturbation of eps (a position perturbation of h eps), applied only where
    it leaves the FP32 velocity unchanged, so the FP32 predicted positions and
    the neighbour lists stay the same.  rest: the rest pose (default: the
    scene's positions)."""
    p = orc.params_for(sc, flags=flags, threads=threads)
    if rest is None:
        rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v = sc.x.astype(np.float64), sc.v.astype(np.float64)
    x1, _, _ = orc.substep(p, rest, x, v)
    h = sc.dt_frame / sc.substeps
    xt = orc.predict32(p, sc.x, sc.v)
    out = 0.0
    for seed in range(seeds):
        vp = v + np.random.default_rng(seed).normal(0.0, eps, size=v.shape)
        keep = vp.astype(np.float32) != v.astype(np.float32)
        vp[keep] = v[keep]
        assert np.array_equal(orc.predict32(p, sc.x, vp.astype(np.float32)), xt)
        x2, _, _ = orc.substep(p, rest, x, vp)
        out = max(out, float(np.abs(x2 - x1).max()) / (h * eps))
    return out


def test_plain_pair_sum_is_ill_conditioned_on_face_contacts(orc):
    """Pair weights (averaging reading): with 1/max(n_p, n_q) the Jacobi
    iteration contracts perturbations, while the plain sum over-corrects
    where particles of large bodies touch several others and amplifies a
    perturbation of 1e-12 m hundreds of times.  On smaller bodies the plain
    sum contracts too.  (This is why the GPU gate of the plain-sum mode uses
    the smaller bodies.)"""
    from scene_helpers import touching_bodies

    big = touching_bodies([27, 1024, 8, 700, 125, 900, 513], seed=3)
    small = touching_bodies([27, 64, 8, 125], seed=3)
    assert _amplification(orc, big, 0) < 3.0
    assert _amplification(orc, big, 2 << 8) > 100.0
    assert _amplification(orc, small, 2 << 8) < 3.0


def test_packed_pile_is_ill_conditioned_until_its_overlaps_resolve(orc):
    """A pile packed with overlapping faces (300 bodies of the dense-pile
    recipe, 30k particles): in its first substep the Jacobi iteration
    amplifies a perturbation of 1e-12 m about a hundred times, while the
    overlaps are pushed apart; three frames later, resting in contact at the
    same density, it contracts again (amplification of a few).  (This is why
    the GPU's settled-density gate settles a pile of randomly oriented bodies
    instead of packing one face to face.)"""
    import os

    from paper_2603_14634_amd import scenes

    threads = max(1, min(8, os.cpu_count() or 1))
    sc = scenes.dense_pile(0, n_bodies=300, gap_frac=-0.1, packed=True)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    assert _amplification(orc, sc, 0, seeds=2, threads=threads) > 30.0
    p = orc.params_for(sc, threads=threads)
    x, v, _ = orc.substep(p, rest, sc.x.astype(np.float64), sc.v.astype(np.float64), n_substeps=3 * sc.substeps)
    later = sc.copy()
    later.x, later.v = x.astype(np.float32), v.astype(np.float32)
    assert _amplification(orc, later, 0, seeds=2, rest=rest, threads=threads) < 10.0


# --------------------------------------------------------------------------
# shape matching: polar decomposition (Mueller et al. 2005)
# --------------------------------------------------------------------------

def _higham_polar(A):
    """Newton iteration X <- (X + X^-T)/2 (Higham 1986); orthogonal polar factor."""
    X = A.copy()
    for _ in range(100):
        Xn = 0.5 * (X + np.linalg.inv(X).T)
        if np.abs(Xn - X).max() < 1e-15:
            return Xn
        X = Xn
    return X


def _kabsch(A):
    U, s, Vt = np.linalg.svd(A)
    d = np.sign(np.linalg.det(U @ Vt))
    return U @ np.diag([1.0, 1.0, d]) @ Vt


def test_polar_recovers_the_rotation_of_a_rigid_motion(orc):
    rng = np.random.default_rng(3)
    q = scenes.lattice_box(4, 3, 2, 0.1)
    m = rng.uniform(0.5, 2.0, size=q.shape[1])
    q = q - (q * m).sum(axis=1, keepdims=True) / m.sum()
    for _ in range(20):
        R0 = scenes.random_rotation(rng)
        x = R0 @ q + rng.normal(size=(3, 1))
        c = (x * m).sum(axis=1) / m.sum()
        A = ((x - c[:, None]) * m) @ q.T
        np.testing.assert_allclose(orc.polar(A), R0, atol=1e-13)


def test_body_state_of_rigid_motions(orc):
    # x = t + R0 q, v = V + w x (R0 q) for every body: the centre is t, the
    # rotation R0, P = M V and L = I w with I = sum m (|r|^2 1 - r r^T)
    rng = np.random.default_rng(11)
    parts = [scenes.lattice_box(3, 4, 5, 0.1), scenes.lattice_box(2, 2, 6, 0.1), scenes.lattice_box(4, 4, 4, 0.1)]
    x0 = np.concatenate(parts, axis=1)
    bs = np.concatenate([[0], np.cumsum([q.shape[1] for q in parts])]).astype(np.int32)
    m = rng.uniform(0.5, 2.0, size=x0.shape[1])
    rest = orc.Body(x0, m, bs)
    x, v = np.zeros_like(x0), np.zeros_like(x0)
    want = []
    for b in range(3):
        sl = slice(bs[b], bs[b + 1])
        R0, t, V, w = scenes.random_rotation(rng), rng.normal(size=3), rng.normal(size=3), rng.normal(size=3)
        r = R0 @ rest.q[:, sl]
        x[:, sl] = t[:, None] + r
        v[:, sl] = V[:, None] + np.cross(w, r.T).T
        mb = m[sl]
        inertia = sum(mi * (ri @ ri * np.eye(3) - np.outer(ri, ri)) for mi, ri in zip(mb, r.T))
        want.append((t, R0, mb.sum() * V, inertia @ w))
    com, rot, P, L = orc.body_state(rest, x, v)
    for b, (t, R0, Pw, Lw) in enumerate(want):
        np.testing.assert_allclose(com[b], t, atol=1e-13)
        np.testing.assert_allclose(rot[b], R0, atol=1e-12)
        np.testing.assert_allclose(P[b], Pw, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(L[b], Lw, rtol=1e-11, atol=1e-12)


def test_polar_matches_newton_polar_and_library_svd(orc):
    rng = np.random.default_rng(4)
    for _ in range(200):
        A = rng.normal(size=(3, 3))
        R = orc.polar(A)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-13)
        np.testing.assert_allclose(R, _kabsch(A), atol=1e-10)
        if np.linalg.det(A) > 0:
            np.testing.assert_allclose(R, _higham_polar(A), atol=1e-10)
        S = R.T @ A                          # symmetric at the optimum
        np.testing.assert_allclose(S, S.T, atol=1e-12)


def test_polar_maximises_trace_over_rotations(orc):
    rng = np.random.default_rng(5)
    for _ in range(20):
        A = rng.normal(size=(3, 3))
        if np.linalg.det(A) > 0:
            A[:, 0] *= -1.0                  # reflections: optimum is not the polar factor
        R = orc.polar(A)
        best = np.trace(R.T @ A)
        for _ in range(200):
            Q = scenes.random_rotation(rng)
            assert np.trace(Q.T @ A) <= best + 1e-12


def test_polar_degenerate_ranks(orc):
    assert np.allclose(orc.polar(np.zeros((3, 3))), np.eye(3))
    rng = np.random.default_rng(6)
    a, b = rng.normal(size=3), rng.normal(size=3)
    A2 = np.outer(a, rng.normal(size=3)) + np.outer(b, rng.normal(size=3))   # rank 2: unique
    np.testing.assert_allclose(orc.polar(A2), _kabsch(A2), atol=1e-10)
    A1 = np.outer(a, b)                                                      # rank 1: R b ∥ a
    R1 = orc.polar(A1)
    np.testing.assert_allclose(R1.T @ R1, np.eye(3), atol=1e-13)
    np.testing.assert_allclose(R1 @ b / np.linalg.norm(b), a / np.linalg.norm(a), atol=1e-12)


def test_pinv_sym3_matches_library(orc):
    rng = np.random.default_rng(8)
    for rank in (3, 2, 1, 0):
        for _ in range(10):
            B = rng.normal(size=(3, rank))
            S = B @ B.T
            np.testing.assert_allclose(orc.pinv_sym3(S), np.linalg.pinv(S, rcond=1e-10, hermitian=True),
                                       atol=1e-9 * max(1.0, np.abs(np.linalg.pinv(S)).max()))


def test_rigid_body_at_its_goal_does_not_move(orc):
    rng = np.random.default_rng(9)
    off = scenes.lattice_box(4, 2, 3, 0.1)
    sc = _body_scene(off, centre=(0.0, 0.0, 1.0), gravity=(0.0, 0.0, 0.0), planes=())
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    R0 = scenes.random_rotation(rng)
    x0 = R0 @ rest.q + np.array([[0.3], [-0.1], [0.7]])
    p = orc.params_for(sc)
    x, v, _ = orc.substep(p, rest, x0, np.zeros_like(x0))
    np.testing.assert_allclose(x, x0, atol=1e-14)
    np.testing.assert_allclose(v, 0.0, atol=1e-11)


# --------------------------------------------------------------------------
# momentum conservation constraint (Eqs. (4)-(5)) on arbitrary states
# --------------------------------------------------------------------------

def _mom(m, x, v):
    c = (m[:, None] * x).sum(axis=0) / m.sum()
    P = (m[:, None] * v).sum(axis=0)
    L = (m[:, None] * np.cross(x - c, v)).sum(axis=0)
    return c, P, L


@pytest.mark.parametrize("flags", [0, 2, 4])
def test_momentum_constraint_restores_pre_shape_matching_momentum(orc, flags):
    rng = np.random.default_rng(10 + flags)
    n, h = 17, 1e-3
    m = rng.uniform(0.2, 2.0, size=n)
    xb, vb = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    xa, va = xb + 0.1 * rng.normal(size=(n, 3)), vb + rng.normal(size=(n, 3))
    x, v = orc.enforce_momentum(m, xb, vb, xa, va, h, flags, radius=0.01)
    _, Pb, Lb = _mom(m, xb, vb)
    ca, Pa, La = _mom(m, xa, va)
    P = (m[:, None] * v).sum(axis=0)
    L = (m[:, None] * np.cross(xa - ca, v)).sum(axis=0)   # about the corrected state's r
    np.testing.assert_allclose(P, Pa if flags & 2 else Pb, atol=1e-12)
    np.testing.assert_allclose(L, La if flags & 4 else Lb, atol=1e-12)
    # the correction is one rigid velocity field dv - w x r, applied to x times dt
    dv = v - va
    np.testing.assert_allclose(x - xa, h * dv, atol=1e-15)
    r = xa - ca
    Amat = np.zeros((3 * n, 6))
    for i in range(n):
        Amat[3 * i:3 * i + 3, :3] = np.eye(3)
        rx, ry, rz = r[i]
        Amat[3 * i:3 * i + 3, 3:] = np.array([[0, rz, -ry], [-rz, 0, rx], [ry, -rx, 0]])  # -w x r
    sol, res, *_ = np.linalg.lstsq(Amat, dv.ravel(), rcond=None)
    np.testing.assert_allclose(Amat @ sol, dv.ravel(), atol=1e-12)


def test_free_spin_keeps_angular_momentum_only_with_the_constraint(orc):
    r = 0.05
    off = scenes.lattice_box(4, 4, 4, 2 * r)
    w0 = np.array([1.0, 2.0, -3.0])
    v = np.cross(w0, off.T).T + np.array([[0.3], [0.0], [0.1]])
    res = {}
    for flags in (0, orc.NO_ANG_MOM):
        sc = _body_scene(off, centre=(0.1, 0.2, 0.3), mass=0.5, radius=r, gravity=(0.0, 0.0, 0.0), planes=())
        sc.v[:] = v
        x0, v0 = sc.x.astype(np.float64), sc.v.astype(np.float64)
        x1, v1, _, p, rest = _run(orc, sc, flags=flags)
        _, P0, L0 = _mom(rest.mass, x0.T, v0.T)
        _, P1, L1 = _mom(rest.mass, x1.T, v1.T)
        res[flags] = np.abs(L1 - L0).max() / np.abs(L0).max()
        np.testing.assert_allclose(P1, P0, atol=1e-13)
        d0 = np.linalg.norm(x0[:, :, None] - x0[:, None, :], axis=0)
        d1 = np.linalg.norm(x1[:, :, None] - x1[:, None, :], axis=0)
        np.testing.assert_allclose(d1, d0, atol=1e-9)      # rigid: pairwise distances kept
    # with the constraint the residual is far below the drift it removes
    assert res[0] < 1e-9
    assert res[orc.NO_ANG_MOM] > 1e-6


# --------------------------------------------------------------------------
# velocity update (Sec. III-B): V_i = (X_i - X_init)/dt holds as an invariant
# --------------------------------------------------------------------------

def test_incremental_velocity_equals_position_difference(orc):
    sc = scenes.drop_cubes(seed=1)
    p = orc.params_for(sc)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v, _ = orc.substep(p, rest, sc.x, sc.v, n_substeps=4 * 150)   # first cubes have landed
    assert (x[2] < sc.radius).any()
    x1, v1, _ = orc.substep(p, rest, x, v)
    np.testing.assert_allclose(v1 * p.h, x1 - x, rtol=0, atol=1e-9 * p.h * np.abs(v1).max())


def test_resting_cube_stays_at_rest(orc):
    r = 0.05
    sc = _body_scene(scenes.lattice_box(4, 4, 4, 2 * r), centre=(0.0, 0.0, 0.15 + r), radius=r)
    p = orc.params_for(sc)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v = sc.x.astype(np.float64), sc.v.astype(np.float64)
    zs = []
    for _ in range(20):
        x, v, _ = orc.substep(p, rest, x, v, n_substeps=200)
        zs.append(x[2].mean())
    assert max(zs) - min(zs) < 1e-9                 # no secular drift
    assert abs(zs[-1] - (0.15 + r)) < 0.01 * r      # penetration well below r
    assert np.abs(v).max() <= p.h * 9.81


# --------------------------------------------------------------------------
# neighbour search: brute force over all pairs, and the index structure
# --------------------------------------------------------------------------

def _brute_force_lists(xt32, body, rs):
    n = xt32.shape[1]
    r2 = np.float32(rs * rs)
    out = []
    for i in range(n):
        d = xt32 - xt32[:, i:i + 1]                       # float32 subtraction
        s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]     # float32, no fused ops
        ok = (s < r2) & (body != body[i])
        ok[i] = False
        out.append(np.nonzero(ok)[0].astype(np.uint32))
    return out


def _random_cloud(rng, n, n_bodies, extent):
    x = rng.uniform(-extent, extent, size=(3, n)).astype(np.float32)
    body = np.sort(rng.integers(0, n_bodies, size=n)).astype(np.int32)
    return x, body


@pytest.mark.parametrize("case", ["cloud", "lattice", "pile"])
def test_neighbour_lists_equal_brute_force(orc, case):
    rng = np.random.default_rng(11)
    r = 0.01
    if case == "cloud":
        xt, body = _random_cloud(rng, 1500, 40, 0.12)
    elif case == "lattice":   # exact lattice spacing 2r: touching pairs sit on the predicate edge
        off = scenes.lattice_box(6, 6, 6, 2 * r)
        x = np.concatenate([off, off + np.array([[12 * r], [0.0], [0.0]]),
                            off + np.array([[6 * r], [11 * r], [1e-3]])], axis=1)
        xt = x.astype(np.float32)
        body = np.repeat(np.arange(3, dtype=np.int32), off.shape[1])
    else:
        sc = scenes.dense_pile(seed=2, n_bodies=40, half_width=0.3, gap_frac=-4.0)
        xt, body = sc.x, sc.body_of_particle()
    for bits in (10, 14):
        p = orc.make_params(1e-3, 1, r, hash_bits=bits, nbr_cap=64)
        idx = orc.index(p, body, xt)
        ref = _brute_force_lists(xt, body, 2 * r)
        assert idx["max_count"] == max(len(a) for a in ref)
        assert idx["max_count"] <= 64
        for i in range(xt.shape[1]):
            c = int(idx["nbr_count"][i])
            np.testing.assert_array_equal(idx["nbr"][i, :c], ref[i])
    assert sum(len(a) for a in ref) > 0


def test_sorted_order_and_cell_tables(orc):
    rng = np.random.default_rng(12)
    xt, body = _random_cloud(rng, 3000, 50, 0.3)
    p = orc.make_params(1e-3, 1, 0.01, hash_bits=11)
    idx = orc.index(p, body, xt)
    key = idx["key"]
    assert key.max() < (1 << 11)
    order = np.lexsort((np.arange(xt.shape[1]), key))      # by key, ties by id
    np.testing.assert_array_equal(idx["sorted_id"], order)
    cnt = np.bincount(key, minlength=1 << 11).astype(np.uint32)
    np.testing.assert_array_equal(idx["cell_count"], cnt)
    np.testing.assert_array_equal(idx["cell_start"], (np.cumsum(cnt) - cnt).astype(np.uint32))


def test_cell_keys_hand_computed(orc):
    # cell edge 1 (inverse exact), origin 0: the cell of (a+0.5, b+0.5, c+0.5) is (a, b, c)
    p = orc.make_params(1e-3, 1, 0.25, cell_size=1.0, hash_bits=10)
    pts = np.array([
        [0.5, 0.5, 0.5],      # (0,0,0) -> 0
        [1.5, 0.5, 0.5],      # (1,0,0) -> bit 0
        [0.5, 1.5, 0.5],      # (0,1,0) -> bit 1
        [0.5, 0.5, 1.5],      # (0,0,1) -> bit 2
        [2.5, 0.5, 0.5],      # (2,0,0) -> bit 3
        [3.5, 2.5, 1.5],      # (3,2,1) -> bits 0,3 | 4 | 2 = 29
        [-0.5, 0.5, 0.5],     # (-1,0,0) wraps to 1023: x bits at 0,3,6,9 -> 585 (low 10 bits)
        [1024.5, 0.5, 0.5],   # 1024 wraps to 0 -> 0
        [1e30, 0.5, 0.5],     # clamped to 2^24, a multiple of 1024 -> 0
    ], dtype=np.float32).T
    np.testing.assert_array_equal(orc.cell_keys(p, pts), [0, 1, 2, 4, 8, 29, 585, 0, 0])


def test_predict32_is_the_fp32_recipe(orc):
    rng = np.random.default_rng(13)
    x = rng.uniform(-3, 3, size=(3, 1000)).astype(np.float32)
    v = rng.normal(size=(3, 1000)).astype(np.float32)
    a = rng.normal(size=(3, 1000)).astype(np.float32)
    p = orc.make_params(1.0 / 960.0, 1, 0.01, gravity=(0.1, -0.2, -9.81))
    xt = orc.predict32(p, x, v, a)
    h = np.float32(1.0 / 960.0)
    g = np.array([0.1, -0.2, -9.81], dtype=np.float32)[:, None]
    vt = v + h * (g + a)                       # float32 ops, each rounded
    np.testing.assert_array_equal(xt, x + h * vt)
    # the FP32 prediction is within FP32 rounding of the FP64 one
    x64 = x.astype(np.float64) + (1.0 / 960.0) * (v + (1.0 / 960.0) * (g.astype(np.float64) + a))
    assert np.abs(xt - x64).max() < 4 * np.finfo(np.float32).eps * 4


# --------------------------------------------------------------------------
# paper Tests 1-3 (Table I closed forms, Table II parameters)
# --------------------------------------------------------------------------

def _paper_box(golden, mu, gravity):
    r = golden["not_in_paper"]["sphere_radius_m"]
    n = golden["spheres_per_axis"]
    off = scenes.lattice_box(n, n, n, 2 * r)
    half = (n - 1) * r
    return _body_scene(off, centre=(0.0, 0.0, half + r), mass=golden["box_mass_kg"] / n ** 3, radius=r,
                       dt_frame=1.0 / golden["frame_rate_hz"], substeps=golden["substeps"],
                       iterations=golden["iterations"], mu=mu, gravity=gravity)


def _load_golden():
    with open(os.path.join(GOLDEN, "paper_tests_1_3.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("test_id", [1, 2, 3])
def test_paper_closed_forms_tests_1_to_3(orc, test_id):
    gd = _load_golden()
    g = gd["not_in_paper"]["g_m_per_s2"]
    M = gd["box_mass_kg"]
    t_end = 2.0
    frames = int(round(t_end * gd["frame_rate_hz"]))
    if test_id == 3:
        th = gd["slope_angle_test_3_rad"]
        sc = _paper_box(gd, gd["mu_tests_1_3"], (g * math.sin(th), 0.0, -g * math.cos(th)))
    else:
        mu = gd["mu_tests_1_3"] if test_id == 1 else gd["mu_test_2"]
        sc = _paper_box(gd, mu, (0.0, 0.0, -g))
    p = orc.params_for(sc)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    x, v = sc.x.astype(np.float64), sc.v.astype(np.float64)
    lam = (rest.mass * (rest.q[0] ** 2 + rest.q[1] ** 2)).sum()     # discrete I_zz
    for _ in range(frames):
        acc = np.zeros_like(x)
        if test_id == 1:
            acc[0] = gd["force_test_1_N"] / M                          # force at the centre of mass
        elif test_id == 2:
            c = (x * rest.mass).sum(axis=1) / M
            alpha = gd["torque_test_2_Nm"] / lam                       # a_p = alpha z x r_p
            acc[0] = -alpha * (x[1] - c[1])
            acc[1] = alpha * (x[0] - c[0])
        x, v, _ = orc.substep(p, rest, x, v, accel=acc, n_substeps=sc.substeps)
    c = (x * rest.mass).sum(axis=1) / M
    if test_id == 1:
        ref = 0.5 * (gd["force_test_1_N"] - gd["mu_tests_1_3"] * M * g) / M * t_end ** 2
        assert c[0] == pytest.approx(ref, rel=0.03)
    elif test_id == 3:
        th = gd["slope_angle_test_3_rad"]
        ref = 0.5 * (g * math.sin(th) - gd["mu_tests_1_3"] * g * math.cos(th)) * t_end ** 2
        assert c[0] == pytest.approx(ref, rel=0.05)
    else:
        A = ((x - c[:, None]) * rest.mass) @ rest.q.T
        R = orc.polar(A)
        theta = math.atan2(R[1, 0], R[0, 0])
        ref = 0.5 * gd["torque_test_2_Nm"] / lam * t_end ** 2
        assert theta == pytest.approx(ref, rel=0.03)
        assert abs(c[0]) < 1e-6 and abs(c[1]) < 1e-6
