"""Rollout serving with continuous batching on a scene pool.

Requests (a scene and a horizon in frames) arrive over time.  Every resident
request lives in a slot of one ``binding.Pool``; admission is by the pool's
HBM arena: a request is admitted as soon as a slot, a particle range and a body
range are free, in arrival order, without blocking smaller requests behind a
larger one that does not fit yet.  Each tick of a lane advances every resident
request of that lane by up to ``frames_per_tick`` frames in the same few
launches (one workgroup per scene), so requests that arrive while others run
join the next tick and their work overlaps on the device.  Scenes of the
large-scene kernel have a lane of their own, ticking at their own pace beside
the small scenes.  A request's result is its scene's state after
its horizon; it does not depend on the other requests (the pool computes every
scene alone).

This module is host-side scheduling only; all stepping runs in libpbdr.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Outcome:
    request_id: int
    arrival_s: float
    admitted_s: float
    done_s: float
    particles: int
    frames: int
    x: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclasses.dataclass
class _Active:
    request: object
    left: int
    admitted_s: float
    lane: int


class ServingEngine:
    """Continuous batching over a pool-like backend with independent lanes.

    The backend provides ``try_add(scene) -> slot or None``, ``lane_of(slot)``,
    ``launch(lane, slots, frames)`` (asynchronous), ``done(lane) -> bool`` (the
    lane's last launch has finished), ``read_state(slot) -> (x, v)``,
    ``check(slot)`` and ``remove(slot)``; ``PoolBackend`` wraps a
    ``binding.Pool``.  Scenes of the large-scene kernel run on their own lane,
    so their long frames do not hold back the small scenes' ticks.
    """

    def __init__(self, backend, frames_per_tick: int = 1, keep_results: bool = True, substeps: int = 4,
                 clock=time.perf_counter, sleep=time.sleep, lanes: Optional[int] = None, poll_s: float = 5e-5):
        if frames_per_tick < 1:
            raise ValueError("frames_per_tick must be >= 1")
        self.backend = backend
        self.frames_per_tick = frames_per_tick
        self.keep_results = keep_results
        self.substeps = substeps
        self.clock = clock
        self.sleep = sleep
        self.lanes = lanes if lanes is not None else getattr(backend, "lanes", 2)
        self.poll_s = poll_s

    def run(self, requests: List, capacity_check=None) -> Dict:
        """Serves the requests (each with ``arrival_s``, ``scene``, ``frames``,
        ``request_id``) in real time; returns the outcomes and statistics.
        ``capacity_check(scene) -> bool`` tells whether a scene could ever fit
        (an empty pool); requests that never fit are rejected."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.request_id)))
        queue: List = []
        active: Dict[int, _Active] = {}
        in_flight: Dict[int, List] = {}          # lane -> [(slot, frames)]
        outcomes: List[Outcome] = []
        rejected: List[int] = []
        ticks, peak_active, busy = 0, 0, [0.0] * self.lanes
        started = [0.0] * self.lanes
        t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            # admission in arrival order; a request that does not fit yet does
            # not hold back later ones
            still = []
            for req in queue:
                slot = self.backend.try_add(req.scene)
                if slot is None:
                    if capacity_check is not None and not capacity_check(req.scene):
                        rejected.append(req.request_id)
                    else:
                        still.append(req)
                    continue
                active[slot] = _Active(req, req.frames, self.clock() - t0, self.backend.lane_of(slot))
            queue = still
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival_s - (self.clock() - t0)))
                elif queue:        # nothing runs and nothing fits: cannot happen with capacity_check
                    rejected.extend(r.request_id for r in queue)
                    queue = []
                continue
            peak_active = max(peak_active, len(active))
            progressed = False
            for lane in range(self.lanes):
                if lane in in_flight:
                    if not self.backend.done(lane):
                        continue
                    busy[lane] += self.clock() - t0 - started[lane]
                    for s, f in in_flight.pop(lane):
                        a = active[s]
                        a.left -= f
                        if a.left > 0:
                            continue
                        if self.keep_results:
                            x, v = self.backend.read_state(s)
                        else:
                            self.backend.check(s)
                            x = v = None
                        req = a.request
                        outcomes.append(Outcome(req.request_id, req.arrival_s, a.admitted_s, self.clock() - t0,
                                                req.scene.n, req.frames, x, v))
                        self.backend.remove(s)
                        del active[s]
                    progressed = True
                mine = sorted(s for s, a in active.items() if a.lane == lane)
                if not mine:
                    continue
                frames = [min(self.frames_per_tick, active[s].left) for s in mine]
                started[lane] = self.clock() - t0
                self.backend.launch(lane, mine, frames)
                in_flight[lane] = list(zip(mine, frames))
                ticks += 1
                progressed = True
            if not progressed:
                self.sleep(self.poll_s)
        makespan = self.clock() - t0
        lat = np.array([o.latency_s for o in outcomes]) if outcomes else np.zeros(0)
        wait = np.array([o.admitted_s - o.arrival_s for o in outcomes]) if outcomes else np.zeros(0)
        psub = float(sum(o.particles * o.frames for o in outcomes)) * self.substeps
        return {
            "outcomes": outcomes,
            "rejected": rejected,
            "completed": len(outcomes),
            "ticks": ticks,
            "peak_active": peak_active,
            "makespan_s": makespan,
            "busy_s": max(busy) if busy else 0.0,
            "particle_substeps": psub,
            "throughput": psub / makespan if makespan > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_wait_ms": float(wait.mean() * 1e3) if wait.size else None,
        }


class PoolBackend:
    """``binding.Pool`` as the engine's backend.  Launch classes are grouped by
    the length of their frames, one lane (and stream) each: the register-
    resident classes up to 4096 particles (side by side within the lane), the
    largest register-resident class, and the large-scene kernel."""

    LANE_OF_CLASS = (0, 0, 0, 0, 0, 0, 1, 2)

    def __init__(self, pool):
        import torch

        self.pool = pool
        self.lanes = 3
        self.streams = [torch.cuda.Stream(device=pool.device) for _ in range(self.lanes)]
        self.events = [None] * self.lanes

    def try_add(self, scene):
        return self.pool.try_add(scene)

    def lane_of(self, slot):
        return self.LANE_OF_CLASS[self.pool.slot_class(slot)]

    def launch(self, lane, slots, frames):
        import torch

        st = self.streams[lane]
        self.pool.step_slots_on(lane, st, slots, frames)
        ev = torch.cuda.Event()
        ev.record(st)
        self.events[lane] = ev

    def done(self, lane):
        ev = self.events[lane]
        return ev is None or ev.query()

    def read_state(self, slot):
        return self.pool.read_state(slot)

    def check(self, slot):
        return self.pool.check(slot)

    def remove(self, slot):
        self.pool.remove(slot)


class HybridBackend(PoolBackend):
    """The pool for the scenes its register-resident classes hold; every scene
    the pool would give to its large-scene kernel (one workgroup walking tens of
    thousands of particles, tens of milliseconds per frame) goes instead to a
    scene batch (``binding.Batch``): all of them are stepped together by the
    multi-workgroup kernels, one set of launches per frame for the whole batch,
    on a lane of its own beside the pool's.  The batch's HBM arena admits them
    as the pool's admits the small ones.  A scene's result depends only on the
    scene: it is routed by its shape alone, and neither the pool nor the batch
    lets scenes interact."""

    FIRST_BATCH = 1 << 20          # slot numbers of batch scenes start here

    def __init__(self, pool, batch):
        super().__init__(pool)
        self.batch = batch
        self.pool_lanes = self.lanes
        self.batch_lane = self.lanes
        self.lanes += 1
        self.streams.append(batch.stream)
        self.events.append(None)

    def routes_to_batch(self, scene) -> bool:
        from . import binding as B

        return self.pool.class_for(scene) == B.POOL_CLASSES

    def try_add(self, scene):
        if not self.routes_to_batch(scene):
            return self.pool.try_add(scene)
        slot = self.batch.try_add(scene)
        return None if slot is None else self.FIRST_BATCH + slot

    def fits_ever(self, scene) -> bool:
        """Whether the scene could be admitted into an empty backend."""
        if self.routes_to_batch(scene):
            info = self.batch.info()
            return scene.n <= info.max_particles and scene.n_bodies <= info.max_bodies
        return scene.n <= self.pool.info().max_particles

    def lane_of(self, slot):
        return self.batch_lane if slot >= self.FIRST_BATCH else super().lane_of(slot)

    def launch(self, lane, slots, frames):
        if lane != self.batch_lane:
            return super().launch(lane, slots, frames)
        import torch

        self.batch.step_slots([s - self.FIRST_BATCH for s in slots], frames)
        ev = torch.cuda.Event()
        ev.record(self.batch.stream)
        self.events[lane] = ev

    def read_state(self, slot):
        if slot >= self.FIRST_BATCH:
            return self.batch.read_state(slot - self.FIRST_BATCH)
        return super().read_state(slot)

    def check(self, slot):
        if slot >= self.FIRST_BATCH:
            return self.batch.check()
        return super().check(slot)

    def remove(self, slot):
        if slot >= self.FIRST_BATCH:
            return self.batch.remove(slot - self.FIRST_BATCH)
        return super().remove(slot)


def batch_for_budget(params, budget_bytes: int, max_scenes: int = 1024, particles_per_body: int = 16,
                     device="cuda:0"):
    """The largest scene batch (in particles) whose workspace fits the HBM budget,
    on a stream of its own."""
    import torch

    from . import binding as B

    def size(n):
        return B.batch_bytes(params, max_scenes, n, max(1, n // particles_per_body))

    lo, hi = 1, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        b = size(mid)
        if 0 < b <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    if not 0 < size(lo) <= budget_bytes:
        raise ValueError("budget too small for a scene batch")
    return B.Batch(params, max_scenes, lo, max(1, lo // particles_per_body), device=device,
                   stream=torch.cuda.Stream(device=device))


def pool_for_budget(params, budget_bytes: int, max_scenes: int = 4096, particles_per_body: int = 16, device="cuda:0"):
    """The largest pool (in particles) whose workspace fits the HBM budget."""
    from . import binding as B

    lo, hi = 1, 1 << 28
    while lo < hi:
        mid = (lo + hi + 1) // 2
        nb = max(1, mid // particles_per_body)
        if B.pool_bytes(params, max_scenes, mid, nb) <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    if B.pool_bytes(params, max_scenes, lo, max(1, lo // particles_per_body)) > budget_bytes:
        raise ValueError("budget too small for a pool")
    return B.Pool(params, max_scenes, lo, max(1, lo // particles_per_body), device=device)
