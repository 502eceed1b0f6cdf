"""Scheduling logic of the serving engine on a simulated pool (no GPU).

The fake pool has the real pool's admission rule (a scene needs a free slot
and a free range of particles) and a simulated clock: a tick costs a fixed
time per resident particle-frame.
"""
import dataclasses

import numpy as np
import pytest

from paper_2603_14634_amd.serving import ServingEngine


@dataclasses.dataclass
class _Scene:
    n: int
    tag: int


@dataclasses.dataclass
class _Req:
    arrival_s: float
    scene: _Scene
    frames: int
    request_id: int


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class _FakePool:
    """Admission as in the real pool; two lanes (scenes above `big` particles on
    lane 1) whose launches take simulated time and run side by side."""

    def __init__(self, clock, capacity, slots, cost_per_particle_frame=1e-6, big=10 ** 9):
        self.clock, self.capacity, self.max_slots = clock, capacity, slots
        self.resident = {}
        self.frames = {}
        self.cost = cost_per_particle_frame
        self.big = big
        self.peak = 0
        self.admitted = []
        self.busy_until = [0.0, 0.0]
        self.lane_launches = [0, 0]

    def try_add(self, scene):
        used = sum(s.n for s in self.resident.values())
        if len(self.resident) >= self.max_slots or used + scene.n > self.capacity:
            return None
        slot = min(set(range(self.max_slots)) - set(self.resident))
        self.resident[slot] = scene
        self.frames[slot] = 0
        self.admitted.append(scene.tag)
        self.peak = max(self.peak, used + scene.n)
        return slot

    def lane_of(self, slot):
        return 1 if self.resident[slot].n > self.big else 0

    def remove(self, slot):
        del self.resident[slot]
        del self.frames[slot]

    def launch(self, lane, slots, frames):
        assert self.done(lane)
        work = 0
        for s, f in zip(slots, frames):
            assert self.lane_of(s) == lane
            self.frames[s] += f
            work = max(work, self.resident[s].n * f)      # one workgroup per scene: the largest sets the pace
        self.busy_until[lane] = self.clock.t + 1e-4 + self.cost * work
        self.lane_launches[lane] += 1

    def done(self, lane):
        return self.clock.t >= self.busy_until[lane]

    def read_state(self, slot):
        assert self.done(self.lane_of(slot))
        sc = self.resident[slot]
        return np.full((3, sc.n), sc.tag, np.float32), np.full((3, sc.n), self.frames[slot], np.float32)

    def check(self, slot):
        return 0


def _engine(capacity=1000, slots=8, fpt=1, big=10 ** 9):
    clk = _Clock()
    pool = _FakePool(clk, capacity, slots, big=big)
    return ServingEngine(pool, frames_per_tick=fpt, clock=clk, sleep=clk.sleep), pool


def test_every_request_completes_with_its_own_horizon():
    eng, pool = _engine(fpt=3)
    rng = np.random.default_rng(0)
    reqs = [_Req(float(t), _Scene(int(n), j), int(h), j)
            for j, (t, n, h) in enumerate(zip(np.sort(rng.uniform(0, 0.05, 40)), rng.integers(10, 300, 40),
                                              rng.integers(1, 20, 40)))]
    out = eng.run(reqs)
    assert out["completed"] == 40 and not out["rejected"]
    for o in out["outcomes"]:
        req = reqs[o.request_id]
        assert o.frames == req.frames
        assert np.all(o.v == req.frames)             # exactly its horizon, never more
        assert np.all(o.x == req.scene.tag)          # its own scene
        assert o.arrival_s <= o.admitted_s <= o.done_s
    assert pool.peak <= 1000
    assert out["p99_ms"] >= out["p50_ms"] > 0


def test_a_request_that_does_not_fit_yet_does_not_block_smaller_ones():
    eng, pool = _engine(capacity=1000)
    reqs = [_Req(0.0, _Scene(900, 0), 50, 0), _Req(0.001, _Scene(500, 1), 5, 1), _Req(0.002, _Scene(50, 2), 5, 2)]
    out = eng.run(reqs)
    assert out["completed"] == 3
    assert pool.admitted.index(2) < pool.admitted.index(1)     # the small one went ahead
    done = {o.request_id: o for o in out["outcomes"]}
    assert done[1].admitted_s >= done[0].done_s - 1e-12        # 500 waited for the 900 to leave


def test_requests_are_admitted_in_arrival_order_when_they_fit():
    eng, pool = _engine(capacity=10_000, slots=64)
    reqs = [_Req(0.0001 * j, _Scene(10 + j, j), 3, j) for j in range(30)]
    eng.run(reqs)
    assert pool.admitted == list(range(30))


def test_a_request_that_can_never_fit_is_rejected():
    eng, pool = _engine(capacity=100)
    reqs = [_Req(0.0, _Scene(50, 0), 2, 0), _Req(0.0, _Scene(500, 1), 2, 1)]
    out = eng.run(reqs, capacity_check=lambda sc: sc.n <= 100)
    assert out["rejected"] == [1] and out["completed"] == 1


def test_large_scenes_tick_on_their_own_lane():
    eng, pool = _engine(capacity=100_000, slots=16, big=5000)
    reqs = [_Req(0.0, _Scene(20_000, 0), 40, 0)] + [_Req(0.001 * j, _Scene(300, j), 20, j) for j in range(1, 9)]
    out = eng.run(reqs)
    assert out["completed"] == 9
    done = {o.request_id: o for o in out["outcomes"]}
    # the small scenes finish long before the large one: they never waited for its frames
    assert max(done[j].done_s for j in range(1, 9)) < 0.5 * done[0].done_s
    assert pool.lane_launches[1] == 40 and pool.lane_launches[0] >= 20


def test_engine_rejects_bad_settings():
    with pytest.raises(ValueError):
        ServingEngine(object(), frames_per_tick=0)


class _Stream:
    """Stands in for a torch stream (no GPU)."""


class _FakeRoutedPool:
    """The pool side of HybridBackend: launch classes by size, POOL_CLASSES above `big`."""

    def __init__(self, big):
        self.big = big
        self.resident = {}
        self.device = "cpu"
        self.launched = []

    def class_for(self, scene):
        from paper_2603_14634_amd import binding as B

        return B.POOL_CLASSES if scene.n > self.big else 0

    def slot_class(self, slot):
        return 0

    def try_add(self, scene):
        slot = len(self.resident)
        self.resident[slot] = scene
        return slot

    def step_slots_on(self, lane, stream, slots, frames):
        self.launched.append((lane, list(slots), list(frames)))

    def read_state(self, slot):
        return ("pool", slot)

    def check(self, slot):
        return 0

    def remove(self, slot):
        del self.resident[slot]


class _FakeBatch(_FakeRoutedPool):
    def __init__(self, capacity):
        super().__init__(big=0)
        self.capacity = capacity
        self.stream = _Stream()
        self.steps = []

    def info(self):
        return type("Info", (), {"max_particles": self.capacity, "max_bodies": self.capacity // 16})()

    def try_add(self, scene):
        if sum(s.n for s in self.resident.values()) + scene.n > self.capacity:
            return None
        return super().try_add(scene)

    def step_slots(self, slots, frames):
        self.steps.append((list(slots), list(frames)))

    def read_state(self, slot):
        return ("batch", slot)


def test_hybrid_backend_routes_by_shape_and_keeps_slot_spaces_apart(monkeypatch):
    import torch

    from paper_2603_14634_amd import serving

    class _Event:
        def record(self, stream):
            pass

        def query(self):
            return True

    monkeypatch.setattr(torch.cuda, "Stream", lambda device=None: _Stream())
    monkeypatch.setattr(torch.cuda, "Event", _Event)
    pool, batch = _FakeRoutedPool(big=1000), _FakeBatch(capacity=5000)
    hb = serving.HybridBackend(pool, batch)
    assert hb.lanes == 4 and hb.batch_lane == 3
    def scene(n, tag):
        sc = _Scene(n, tag)
        sc.n_bodies = max(1, n // 100)
        return sc

    small, large, huge = scene(500, 0), scene(3000, 1), scene(4000, 2)
    s_small, s_large = hb.try_add(small), hb.try_add(large)
    assert s_small < hb.FIRST_BATCH <= s_large
    assert hb.try_add(huge) is None                          # the batch arena is full for now
    assert hb.lane_of(s_small) < hb.pool_lanes and hb.lane_of(s_large) == hb.batch_lane
    hb.launch(hb.batch_lane, [s_large], [2])
    assert batch.steps == [([s_large - hb.FIRST_BATCH], [2])] and hb.done(hb.batch_lane)
    assert hb.read_state(s_large) == ("batch", s_large - hb.FIRST_BATCH)
    assert hb.read_state(s_small) == ("pool", s_small)
    assert hb.fits_ever(huge) is True and hb.fits_ever(scene(6000, 3)) is False
    hb.remove(s_large)
    assert not batch.resident and hb.try_add(huge) is not None
