"""GPU parity of scene batches (many scenes stepped by the multi-workgroup kernels).

Per scene and substep, against the FP64 reference on the same FP32 start: FP32
predicted positions, neighbour counts and lists bit-exact; displacement
X_K - X_init within 1e-5 r; positions within 1e-5 r + ulp32 and velocities
within 1e-5 r / h + 2 ulp32.  A scene's result must not depend on the other
scenes of the batch or on how many frames the others are stepped, and equals
the single-scene solver's.
"""
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


def _check_scene(orc, batch, slot, sc, x, v, cap=32, flags=0, label=""):
    """The scene in `slot` has just run one substep from (x, v)."""
    xg, vg = batch.read_state(slot)
    dg = batch.read_debug(slot, B.DEBUG_DELTA).astype(np.float64)
    p = orc.params_for(sc, nbr_cap=cap, flags=flags, threads=THREADS)
    rest = orc.Body(sc.x, sc.mass, sc.body_start)
    xt_o = orc.predict32(p, x, v)
    np.testing.assert_array_equal(batch.read_debug(slot, B.DEBUG_XT), xt_o)
    idx = orc.index(p, rest.body_of_particle(), xt_o)
    cnt = batch.read_debug(slot, B.DEBUG_NBR_COUNT)
    np.testing.assert_array_equal(cnt, idx["nbr_count"])
    nbr = batch.read_debug(slot, B.DEBUG_NBR)
    stored = np.minimum(cnt, cap)
    for j in range(int(stored.max()) if sc.n else 0):
        rows = np.nonzero(stored > j)[0]
        np.testing.assert_array_equal(nbr[j, rows], idx["nbr"][rows, j])
    xo, vo, _ = orc.substep(p, rest, x, v)
    r, h = sc.radius, sc.dt_frame / sc.substeps
    d_err = np.abs(dg - (xo - x.astype(np.float64)))
    v_err = np.abs(vg.astype(np.float64) - vo)
    print("[batch] %s n=%d bodies=%d: max |d err| %.3g  max |v err| %.3g  contacts max %d"
          % (label, sc.n, sc.n_bodies, d_err.max(), v_err.max(), int(cnt.max())), flush=True)
    assert np.all(d_err <= 1e-5 * r), "displacement error %.3g" % d_err.max()
    assert np.all(np.abs(xg.astype(np.float64) - xo) <= 1e-5 * r + _ulp32(xo))
    assert np.all(v_err <= _tol_v(r, h, xo, vo, flags)), "velocity error %.3g" % v_err.max()
    return int(cnt.max())


def _scenes():
    """Scenes with contacts in the first substep, per-scene gravity and friction,
    bodies from 1 to 1000 particles."""
    out = []
    for k, sizes in enumerate([[1000] * 12, [27] * 80, [511, 513, 64, 1, 7], [700, 800, 900, 512]]):
        sc = touching_bodies(sizes, seed=40 + k)
        sc.gravity = (0.5 * k, -0.3, -5.0 - k)
        sc.mu = 0.15 * (k + 1)
        sc.name = "touching %s" % sizes[:3]
        out.append(sc)
    return out


def _new_batch(scs, max_scenes=None, spare=1.0):
    n = sum(s.n for s in scs)
    nb = sum(s.n_bodies for s in scs)
    return B.Batch(B.params_for(scs[0]), max_scenes or len(scs), max(int(n * spare), 1), max(int(nb * spare), 1))


def test_batch_substep_matches_reference(orc):
    scs = _scenes()
    batch = _new_batch(scs)
    slots = [batch.add(sc) for sc in scs]
    batch.substep(1)
    contacts = 0
    for sl, sc in zip(slots, scs):
        contacts = max(contacts, _check_scene(orc, batch, sl, sc, sc.x, sc.v, label=sc.name))
    assert contacts >= 1
    batch.close()


@pytest.mark.parametrize("flags", [B.FLAG_STD_VELOCITY, B.FLAG_NO_LIN_MOM, B.FLAG_NO_ANG_MOM, B.PP_AVG_OWN,
                                   B.PP_AVG_NONE])
def test_batch_flags_match_reference(orc, flags):
    # bodies of 1 to 1000 particles (the larger ones take FP64 shape-matching sums)
    scs = _scenes()[2:4] + _scenes()[:1]
    batch = B.Batch(B.params_for(scs[0], flags=flags), len(scs), sum(s.n for s in scs),
                    sum(s.n_bodies for s in scs))
    slots = [batch.add(sc) for sc in scs]
    batch.substep(1)
    for sl, sc in zip(slots, scs):
        _check_scene(orc, batch, sl, sc, sc.x, sc.v, flags=flags, label="%s flags %#x" % (sc.name, flags))
    batch.close()


def test_batch_equals_single_scene_solver_and_is_independent_of_the_mix():
    scs = _scenes()
    frames = [7, 3, 5, 4]
    batch = _new_batch(scs, max_scenes=6, spare=1.5)
    slots = [batch.add(sc) for sc in scs]
    # uneven horizons: steps of 2 frames until each scene is done
    left = dict(zip(slots, frames))
    while any(left.values()):
        live = [s for s in slots if left[s] > 0]
        step = [min(2, left[s]) for s in live]
        batch.step_slots(live, step)
        for s, f in zip(live, step):
            left[s] -= f
    mixed = {s: batch.read_state(s) for s in slots}
    batch.close()
    for sc, s, f in zip(scs, slots, frames):
        alone = _new_batch([sc])
        a = alone.add(sc)
        alone.step(f)
        xa, va = alone.read_state(a)
        alone.close()
        np.testing.assert_array_equal(mixed[s][0], xa)
        np.testing.assert_array_equal(mixed[s][1], va)
        solver = B.Solver(B.params_for(sc), sc.x, sc.v, sc.mass, sc.body_start)
        solver.step(f)
        xs, vs = solver.read_state()
        solver.close()
        print("[batch] %s: %d frames, same alone, in the mix and as a single scene" % (sc.name, f), flush=True)
        np.testing.assert_array_equal(xa, xs)
        np.testing.assert_array_equal(va, vs)


def test_batch_admission_removal_and_reuse():
    scs = _scenes()
    batch = _new_batch(scs[:2], max_scenes=3)
    info = batch.info()
    assert info.max_scenes == 3 and info.scenes_used == 0
    s0 = batch.add(scs[0])
    s1 = batch.add(scs[1])
    assert batch.try_add(scs[2]) is None                   # no particles left
    info = batch.info()
    assert info.scenes_used == 2 and info.particles_used == scs[0].n + scs[1].n
    batch.step(2)
    batch.check()
    x0, _ = batch.read_state(s0)
    x1, v1 = batch.read_state(s1)
    batch.remove(s1)
    assert batch.info().particles_used == scs[0].n
    s2 = batch.add(scs[1])                                 # into the freed ranges
    batch.step_slots([s2], [2])                            # s0 stays
    x2, v2 = batch.read_state(s2)
    np.testing.assert_array_equal(x2, x1)
    np.testing.assert_array_equal(v2, v1)
    np.testing.assert_array_equal(batch.read_state(s0)[0], x0)
    with pytest.raises(B.PbdrError):
        batch.step_slots([s0, s0], [1, 1])
    with pytest.raises(B.PbdrError):
        batch.remove(s1 if s1 != s2 else 2)
    batch.close()


def test_batch_rejects_bad_scenes():
    sc = touching_bodies([1025], seed=3)                    # a body above 1024 particles
    batch = B.Batch(B.params_for(sc), 2, 4096, 16)
    with pytest.raises(B.PbdrError):
        batch.add(sc)
    bad = touching_bodies([8, 8], seed=4)
    bad.x[0, 3] = np.nan
    with pytest.raises(B.PbdrError):
        batch.add(bad)
    assert batch.info().scenes_used == 0
    batch.close()
