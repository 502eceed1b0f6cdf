"""GPU parity of scene pools (many small scenes, one workgroup each).

Per scene and substep, against the FP64 reference on the same FP32 start:
FP32 predicted positions, neighbour counts and lists bit-exact; displacement
X_K - X_init within 1e-5 r; positions within 1e-5 r + ulp32 and velocities
within 1e-5 r / h + 2 ulp32.  A scene's result must not depend on the other
scenes of the pool or on the launch shape.
"""
import math
import os

import numpy as np
import pytest

from paper_2603_14634_amd import binding as B
from paper_2603_14634_amd import scenes

from scene_helpers import touching_bodies

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load_library()


def _tol_v(r, h, xo, vo, flags):
    """Velocity tolerance: 1e-5 r / h plus two FP32 ulps of V.  Standard PBD's
    update (PBDR_FLAG_STD_VELOCITY) forms V from positions held in FP32 world
    coordinates, (fl(X_init + dX) - X_init) / h, as the paper's solver does; that
    rounding of the position, up to one ulp of x per h, is part of the mode."""
    tol = 1e-5 * r / h + 2 * _ulp32(vo)
    if flags & B.FLAG_STD_VELOCITY:
        tol = tol + _ulp32(xo) / h
    return tol


def _ulp32(a):
    return np.spacing(np.abs(np.asarray(a, dtype=np.float32))).astype(np.float64)


def _pool_params(sc, cap=32, flags=0):
    return B.params_for(sc, nbr_cap=cap, flags=flags)


def _check_scene(orc, pool, slot, sc, x, v, cap=32, flags=0, label=""):
    """The scene in `slot` has just run one substep from (x, v)."""
    xg, vg = pool.read_state(slot)
    dg = pool.read_debug(slot, B.DEBUG_DELTA).astype(np.float64)
    p = orc.params_for(sc, nbr_cap=cap, flags=flags, threads=THREADS)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    xt_o = orc.predict32(p, x, v)
    np.testing.assert_array_equal(pool.read_debug(slot, B.DEBUG_XT), xt_o)
    idx = orc.index(p, rest.body_of_particle(), xt_o)
    cnt = pool.read_debug(slot, B.DEBUG_NBR_COUNT)
    np.testing.assert_array_equal(cnt, idx["nbr_count"])
    nbr = pool.read_debug(slot, B.DEBUG_NBR)
    stored = np.minimum(cnt, cap)
    for j in range(int(stored.max())):
        rows = np.nonzero(stored > j)[0]
        np.testing.assert_array_equal(nbr[j, rows], idx["nbr"][rows, j])
    xo, vo, _ = orc.substep(p, rest, x, v)
    r, h = sc.radius, sc.dt_frame / sc.substeps
    d_err = np.abs(dg - (xo - x.astype(np.float64)))
    v_err = np.abs(vg.astype(np.float64) - vo)
    print("[pool] %s n=%d bodies=%d: max |d err| %.3g  max |v err| %.3g  contacts max %d"
          % (label, sc.n, sc.n_bodies, d_err.max(), v_err.max(), int(cnt.max())), flush=True)
    assert np.all(d_err <= 1e-5 * r), "displacement error %.3g" % d_err.max()
    assert np.all(np.abs(xg.astype(np.float64) - xo) <= 1e-5 * r + _ulp32(xo))
    assert np.all(v_err <= _tol_v(r, h, xo, vo, flags)), "velocity error %.3g" % v_err.max()
    return int(cnt.max())


def _mixed_scenes():
    """Scenes of every size class, with contacts in the first substep, and
    per-scene gravity and friction."""
    out = []
    for k, sizes in enumerate([[1], [1, 1, 1], [27, 64, 8], [100, 27], [255, 256, 257],
                               [511, 513, 64, 1, 7], [700, 800, 900, 512], [1000] * 5,
                               [27] * 80, [1000] * 12]):        # the last two run the large-scene kernel
        sc = touching_bodies(sizes, seed=10 + k)
        sc.gravity = (0.5 * k, -0.3, -5.0 - k)
        sc.mu = 0.1 * k
        sc.name = "touching %s" % sizes
        out.append(sc)
    return out


def _new_pool(scs, cap=32, flags=0, max_scenes=None):
    n = sum(s.n for s in scs)
    nb = sum(s.n_bodies for s in scs)
    return B.Pool(_pool_params(scs[0], cap=cap, flags=flags), max_scenes or len(scs), max(n, 1), max(nb, 1))


def test_pool_substep_matches_reference(orc):
    scs = _mixed_scenes()
    pool = _new_pool(scs)
    print("[pool] device allows scenes of up to %d particles" % pool.info().max_scene_particles, flush=True)
    slots = [pool.add(sc) for sc in scs]
    pool.substep(1)
    contacts = [_check_scene(orc, pool, sl, sc, sc.x, sc.v, label=sc.name) for sl, sc in zip(slots, scs)]
    assert max(contacts) >= 1
    # a later substep, from the reference's own state after 3 frames
    for sl, sc in zip(slots, scs):
        p = orc.params_for(sc, threads=THREADS)
        rest = orc.Body(sc.x, sc.mass, sc.body_start)
        x, v, _ = orc.substep(p, rest, sc.x, sc.v, n_substeps=3 * sc.substeps)
        sc2 = sc.copy()
        sc2.x, sc2.v = x.astype(np.float32), v.astype(np.float32)
        pool.remove(sl)
        sl2 = pool.add(sc2)
        pool.step_slots([sl2], [0])            # nothing runs
        pool.substep(1)
        # rest pose comes from the new start state: compare with a reference built the same way
        _check_scene(orc, pool, sl2, sc2, sc2.x, sc2.v, label=sc.name + " (3 frames on)")
        pool.remove(sl2)
    pool.close()


def test_pool_flags_match_reference(orc):
    scs = [touching_bodies([27, 64, 8, 125], seed=3)]
    for flags in (B.FLAG_STD_VELOCITY, B.FLAG_NO_LIN_MOM, B.FLAG_NO_ANG_MOM, B.PP_AVG_OWN, B.PP_AVG_NONE):
        pool = _new_pool(scs, flags=flags)
        sl = pool.add(scs[0])
        pool.substep(1)
        _check_scene(orc, pool, sl, scs[0], scs[0].x, scs[0].v, flags=flags, label="flags %#x" % flags)
        pool.close()


def test_pool_sampled_scenes_of_the_full_batch(orc):
    """The 4096-scene batch as benchmarked: every size class present; sampled
    scenes (the largest, the smallest and a spread) checked after one substep."""
    batch = scenes.batch_scenes(0)
    pool = _new_pool(batch)
    slots = [pool.add(sc) for sc in batch]
    pool.substep(1)
    order = np.argsort([sc.n for sc in batch])
    pick = sorted(set([int(order[0]), int(order[-1])] + [int(order[j]) for j in np.linspace(1, len(batch) - 2, 6).astype(int)]))
    for j in pick:
        _check_scene(orc, pool, slots[j], batch[j], batch[j].x, batch[j].v, label="batch scene %d" % j)
    pool.close()


def test_pool_sampled_batch_scenes_in_contact(orc):
    """16 scenes of the 4096-scene batch (spread over its sizes) after 250
    reference frames, when every body has landed: one substep of each, from
    the reference state rounded to FP32 (rest pose: that state, on both
    sides).  Nearly every scene rests on the ground, and some bodies on each other."""
    batch = scenes.batch_scenes(0)
    order = np.argsort([sc.n for sc in batch])
    pick = [int(order[j]) for j in np.linspace(0, len(batch) - 1, 16).astype(int)]
    moved = []
    for j in pick:
        sc = batch[j]
        p = orc.params_for(sc, threads=THREADS)
        rest = orc.Body(sc.x, sc.mass, sc.body_start)
        x, v, _ = orc.substep(p, rest, sc.x, sc.v, n_substeps=250 * sc.substeps)
        sc2 = sc.copy()
        sc2.x, sc2.v = x.astype(np.float32), v.astype(np.float32)
        moved.append(sc2)
    pool = _new_pool(moved)
    slots = [pool.add(sc) for sc in moved]
    pool.substep(1)
    contacts = [_check_scene(orc, pool, sl, sc, sc.x, sc.v, label="batch scene %d after 250 frames" % j)
                for sl, sc, j in zip(slots, moved, pick)]
    print("[pool] pair contacts per sampled scene: %s" % contacts, flush=True)
    grounded = sum(float(sc.x[2].min()) < 1.001 * sc.radius for sc in moved)
    print("[pool] scenes resting on the ground: %d of %d" % (grounded, len(moved)), flush=True)
    assert grounded >= 12                                             # on the ground
    assert max(contacts) >= 1                                         # and bodies on bodies
    pool.close()


def test_pool_step_graph_replays_equal_direct_launches():
    """pbdr_pool_step replays a captured graph of the class launches (fork and
    join included); pbdr_pool_step_slots launches them directly.  Replayed
    several times, with other work and synchronisations between the replays,
    and captured again after the resident set changes, the states stay
    bitwise equal to the direct launches'."""
    import torch

    scs = scenes.batch_scenes(3, n_scenes=48)
    graphed, direct = _new_pool(scs), _new_pool(scs)
    sg = [graphed.add(sc) for sc in scs]
    sd = [direct.add(sc) for sc in scs]
    scratch = torch.zeros(1 << 20, device="cuda")
    for rep in range(6):
        if rep == 3:                       # a new resident set: the graph is captured again
            graphed.remove(sg[5])
            direct.remove(sd[5])
            sg[5] = sd[5] = None
        graphed.step(2)
        direct.step_slots([s for s in sd if s is not None], [2] * sum(s is not None for s in sd))
        scratch.add_(1.0)                  # eager work between the replays
        torch.cuda.synchronize()
        for a, b in zip(sg, sd):
            if a is None:
                continue
            xa, va = graphed.read_state(a)
            xb, vb = direct.read_state(b)
            np.testing.assert_array_equal(xa, xb)
            np.testing.assert_array_equal(va, vb)
    graphed.close()
    direct.close()


def test_scene_result_is_the_same_alone_in_a_mix_and_for_every_launch_shape():
    scs = _mixed_scenes()
    target = scs[-2]                            # 2912 particles: several register sets per lane
    frames = 20
    alone = _new_pool([target])
    s0 = alone.add(target)
    alone.step(frames)
    xa, va = alone.read_state(s0)
    alone.close()

    rng = np.random.default_rng(1)
    others = scenes.batch_scenes(2, n_scenes=40)
    mix_list = others[:20] + [target] + others[20:]
    mix = _new_pool(mix_list)
    slots = [mix.add(sc) for sc in mix_list]
    t = slots[20]
    mix.tuning = [1, 2, 2, 4, 8, 16, 16]
    for _ in range(frames):                     # one frame at a time, others with varied horizons
        busy = [s for s in slots if s == t or rng.random() < 0.7]
        mix.step_slots(busy, [1 if s == t else int(rng.integers(0, 3)) for s in busy])
    xm, vm = mix.read_state(t)
    np.testing.assert_array_equal(xm, xa)
    np.testing.assert_array_equal(vm, va)
    mix.close()

    for waves in (8, 16):                       # 6 and 3 register sets per lane
        pool = _new_pool([target])
        s = pool.add(target)
        w = pool.tuning
        w[5] = waves                            # class of 2049..4096 particles
        pool.tuning = w
        pool.step(frames)
        x, v = pool.read_state(s)
        np.testing.assert_array_equal(x, xa)
        np.testing.assert_array_equal(v, va)
        pool.close()


def test_autotune_restores_state_and_keeps_results():
    batch = scenes.batch_scenes(3, n_scenes=64)
    ref = _new_pool(batch)
    rs = [ref.add(sc) for sc in batch]
    ref.step(5)
    want = [ref.read_state(s) for s in rs]
    ref.close()
    pool = _new_pool(batch)
    ss = [pool.add(sc) for sc in batch]
    ms = pool.autotune(n_frames=2, repeats=1)
    print("[pool] tuned waves %s, ms per class %s" % (pool.tuning, ["%.3f" % m for m in ms]), flush=True)
    pool.step(5)
    for s, (x, v) in zip(ss, want):
        gx, gv = pool.read_state(s)
        np.testing.assert_array_equal(gx, x)
        np.testing.assert_array_equal(gv, v)
    pool.close()


def test_admission_capacity_and_slot_reuse():
    batch = scenes.batch_scenes(4, n_scenes=12)
    n_cap = sum(sc.n for sc in batch[:6])
    pool = B.Pool(_pool_params(batch[0]), 8, n_cap, 64 * 8)
    slots = [pool.try_add(sc) for sc in batch[:6]]
    assert all(s is not None for s in slots)
    info = pool.info()
    assert info.scenes_used == 6 and info.particles_used == n_cap and info.largest_free_particles == 0
    assert pool.try_add(batch[6]) is None       # no particle range left: refused, nothing changes
    assert pool.info().scenes_used == 6
    pool.remove(slots[2])
    assert pool.info().largest_free_particles == batch[2].n
    with pytest.raises(B.PbdrError):
        pool.remove(slots[2])                   # already free
    small = min(batch[6:], key=lambda sc: sc.n)
    if small.n <= batch[2].n:
        s = pool.add(small)                     # reuses the freed slot and range
        pool.step(2)
        pool.check(s)
        assert pool.info().scenes_used == 6
    pool.close()


def test_capacity_overflow_and_non_finite_are_latched_per_scene():
    r = 0.01
    lat = scenes.lattice_box(4, 4, 4, 2 * r)
    # interpenetrating lattices offset by half a spacing on every axis: 8 neighbours each
    dense = scenes.from_bodies([lat + 0.5, lat + 0.5 + r], [np.zeros(3), np.zeros(3)], [0.01, 0.01], radius=r)
    quiet = scenes.batch_scenes(5, n_scenes=1)[0]
    pool = _new_pool([dense, quiet], cap=4)
    a = pool.add(dense)
    b = pool.add(quiet)
    pool.substep(1)
    assert pool.status(a) == B.ERR_CAPACITY
    assert pool.status(b) == B.OK
    with pytest.raises(B.PbdrError):
        pool.check(a)
    mx = __import__("ctypes").c_int32()
    pool._lib.pbdr_pool_check(pool._h, a, __import__("ctypes").byref(mx))
    assert mx.value == 8
    pool.close()
    bad = quiet.copy()
    bad.v, bad.x = bad.v.copy(), bad.x.copy()
    bad.v[2, 0] = 3e38
    bad.x[0, 0] = 3e38                          # finite input whose inertia overflows FP32
    pool = _new_pool([bad])
    s = pool.add(bad)
    pool.step(2)
    assert pool.status(s) == B.ERR_NONFINITE
    pool.close()


def test_pool_rejects_bad_scenes():
    sc = scenes.batch_scenes(6, n_scenes=1)[0]
    big = scenes.single_body(scenes.lattice_box(41, 40, 40, 0.02), radius=0.01)
    many = touching_bodies([1] * 257)
    pool = B.Pool(_pool_params(sc), 4, big.n + sc.n, 400)
    with pytest.raises(B.PbdrError):
        pool.add(big)                           # above the largest pooled scene (65535 particles)
    with pytest.raises(B.PbdrError):
        pool.add(many)                          # more bodies than a pooled scene holds (256)
    pool.add(sc)
    pool.close()


def test_large_scenes_alone_and_among_small_ones():
    """Scenes above the register-resident limits (more than 8192 particles or
    64 bodies) share a pool with small ones; each result is the same alone."""
    big = touching_bodies([900] * 11, seed=7)           # 9900 particles
    wide = touching_bodies([27] * 90, seed=8)           # 90 bodies
    small = scenes.batch_scenes(9, n_scenes=10)
    frames = 6
    want = {}
    for sc in (big, wide):
        pool = _new_pool([sc])
        s = pool.add(sc)
        pool.step(frames)
        want[id(sc)] = pool.read_state(s)
        pool.close()
    mix_list = small[:5] + [big] + small[5:] + [wide]
    pool = _new_pool(mix_list)
    slots = [pool.add(sc) for sc in mix_list]
    for _ in range(frames):
        pool.step(1)
    for sc, sl in zip(mix_list, slots):
        if id(sc) in want:
            x, v = pool.read_state(sl)
            np.testing.assert_array_equal(x, want[id(sc)][0])
            np.testing.assert_array_equal(v, want[id(sc)][1])
        else:
            pool.check(sl)
    pool.close()
