#!/usr/bin/env python3
"""Throughput of the PBD-R solver substep on one MI355X.

Workloads: ``dense_pile_20k`` (default), ``cuboid_rain_1000`` and
``drop_cubes_8x64`` run one scene through the single-scene solver;
``batch_4096`` steps 4096 independent scenes (log-normal 100-5000 particles)
in a scene pool; ``serving`` serves Poisson-arriving rollout requests with
continuous batching and reports p50/p99 latency beside throughput.

Default workload: ``dense_pile_20k`` -- 20k mixed cuboid and lattice-ball
bodies (log-normal counts, mean 100; about 2.0M particles, r = 0.01 m) in a
walled 4 x 4 m bin, dt = 1/240 s, 8 substeps x 20 iterations per frame,
seeded synthetic input, timed after 240 untimed frames in which the pile
settles into contact.  A "step" is one frame: 8 full substeps (prediction,
hash-grid neighbour search, 20 Jacobi iterations of contacts + shape matching
+ momentum constraint, velocity update), replayed from a HIP graph.

Prints one JSON line:
  value          particle-substeps per second over the timed frames (inputs
                 resident in HBM, HIP events on the solver's stream)
  roofline       the dominant kernel (one solver iteration over all bodies):
                 algorithmic bytes per launch / its average duration, timed
                 live with HIP events on the same stream, against 8 TB/s;
                 beside it the whole substep against the same peak
  cpu_baseline   the FP64 reference on this host's cores for a bounded sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_2603_14634_amd", "csrc", f)
               for f in ("pbdr_kernels.hip", "pbdr_math.h", "pbdr_device.h")]
PROFILES = os.path.join(ROOT, "profiles")


def iterate_bytes_per_particle(kbar: float) -> float:
    """Algorithmic HBM bytes of one iteration per particle.

    Reads X_init (12), delta_i (12), V_i (12), q (12), mass (4), list length
    (4) and 4 bytes per neighbour id; writes delta_{i+1} (12) and V_{i+1} (12).
    Neighbour positions are other particles' already-counted data.
    """
    return 84.0 + 4.0 * kbar


def iterate_bytes_per_body() -> float:
    """body_start (8), body mass (4), rotation written (36)."""
    return 48.0


def substep_bytes_per_particle(iterations: int, kbar: float, hash_bits: int) -> float:
    """Algorithmic bytes of one particle-substep, B = 112 + 16 P + 4 k + K (84 + 4 k).

    Per substep: prediction (read x, v: 24; write X_init, delta_0, V_0: 36),
    key (4), P sort passes of 8-bit digits over (key, id) pairs (16 each), cell
    table (about 20), neighbour build (24 + 4 k); then K iterations of 84 + 4 k
    (``iterate_bytes_per_particle``).  k = mean neighbour count, P = ceil(bits / 8).
    """
    passes = (hash_bits + 7) // 8
    return 112.0 + 16.0 * passes + 4.0 * kbar + iterations * iterate_bytes_per_particle(kbar)


# untimed frames before the warm-up: the pile settles into contact, the rain
# lands, so that the timed frames carry contacts and partner waits
SETTLE_FRAMES = {"dense_pile_20k": 240, "cuboid_rain_1000": 120}


def source_digest() -> str:
    """Digest of the single-scene kernel sources (the iteration kernel and what it includes)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of the iteration kernel `kernel` on this workload
    from the committed rocprofv3 counter summary, or None when there is none,
    it covers another kernel, or it was taken on a different kernel source."""
    try:
        vals = {}
        with open(os.path.join(PROFILES, "k_iterate_%s_traffic.txt" % workload)) as f:
            for line in f:
                if ":" in line:
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256_16") != source_digest() or vals.get("kernel") != kernel:
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def measured_copy_gbs(mib: int = 1024, reps: int = 5) -> float:
    """HBM bandwidth a plain device-to-device copy reaches on this GPU (bytes
    read + written per second, GB/s), beside the datasheet peak."""
    import torch

    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


def host_cpu() -> str:
    """CPU model and logical CPU count of this host."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s, %d logical CPUs" % (model, os.cpu_count() or 1)


class Roctx:
    """roctx ranges of the profiler SDK, when its library is present: the timed
    frames (and the calibration copy) are named ranges in a trace."""

    def __init__(self):
        import ctypes

        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.lib is not None:
            self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]

    def begin(self, name: str):
        if self.lib is not None:
            self.lib.roctxRangePushA(name.encode())

    def end(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


def oracle_threads(requested: int) -> int:
    return max(1, min(requested, os.cpu_count() or 1))


def cpu_baseline(sc, budget_s: float, threads: int):
    from oracle import oracle as ref
    import numpy as np

    p = ref.params_for(sc, threads=threads)
    rest = ref.Body(sc.x, sc.mass, sc.body_start)
    x, v = sc.x.astype(np.float64), sc.v.astype(np.float64)
    t0 = time.perf_counter()
    x, v, _ = ref.substep(p, rest, x, v, n_substeps=1)
    one = time.perf_counter() - t0
    extra = int(max(0, min(15, budget_s / max(one, 1e-6) - 1)))
    t1 = time.perf_counter()
    if extra:
        ref.substep(p, rest, x, v, n_substeps=extra)
    total = one + (time.perf_counter() - t1)
    subs = 1 + extra
    return {"value": sc.n * subs / total, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": "%d substeps of %s from its initial state (%d particles, K=%d), FP64, %d OpenMP threads"
                      % (subs, sc.name, sc.n, sc.iterations, threads), "host": host_cpu()}


def pool_bytes_per_particle_substep(iterations: int, kbar: float) -> float:
    """Algorithmic bytes of one particle-substep: the iteration's 84 + 4 k per
    iteration (as for the single-scene iteration kernel) plus predict (x, v
    read, X_init, delta, V written: 60) and the neighbour build (24 + 4 k)."""
    return iterations * iterate_bytes_per_particle(kbar) + 60.0 + 24.0 + 4.0 * kbar


def cpu_baseline_scenes(scs, budget_s: float, label: str, threads: int):
    """The FP64 reference over whole scenes, one substep each, until the budget is spent."""
    from oracle import oracle as ref

    done_n, used, count = 0, 0.0, 0
    for sc in scs:
        p = ref.params_for(sc, threads=threads)
        rest = ref.Body(sc.x, sc.mass, sc.body_start)
        t0 = time.perf_counter()
        ref.substep(p, rest, sc.x, sc.v, n_substeps=1)
        used += time.perf_counter() - t0
        done_n += sc.n
        count += 1
        if used > budget_s:
            break
    return {"value": done_n / used, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": "one substep of each of the first %d scenes of %s (%d particles), FP64, %d OpenMP threads"
                      % (count, label, done_n, threads), "host": host_cpu()}


def bench_pool(args):
    import torch
    from paper_2603_14634_amd import binding as B
    from paper_2603_14634_amd import scenes

    batch = scenes.batch_scenes(args.seed)
    N = sum(sc.n for sc in batch)
    NB = sum(sc.n_bodies for sc in batch)
    S = batch[0].substeps
    print("[bench] batch_4096: %d scenes, %d particles, %d bodies" % (len(batch), N, NB), file=sys.stderr, flush=True)
    pool = B.Pool(B.params_for(batch[0]), len(batch), N, NB)
    slots = [pool.add(sc) for sc in batch]
    stream = pool.stream
    tuned = pool.autotune(n_frames=2, repeats=1)
    print("[bench] tuned waves per class %s (ms %s)" % (pool.tuning, ["%.2f" % t for t in tuned]), file=sys.stderr,
          flush=True)
    # a step is one frame of every scene: pbdr_pool_step replays the captured
    # graph of the class launches (captured on the first call)
    for _ in range(max(1, args.warmup)):
        pool.step(1)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        pool.step(1)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    mx = 0
    for sl in slots:
        mx = max(mx, pool.check(sl))
    value = N * S * args.steps / (ms / 1e3)
    # the same frames as direct launches (pbdr_pool_step_slots over every scene)
    ones = [1] * len(slots)
    pool.step_slots(slots, ones)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        pool.step_slots(slots, ones)
    t1.record(stream)
    torch.cuda.synchronize()
    direct = N * S * args.steps / (t0.elapsed_time(t1) / 1e3)
    # per-scene launches of the single-scene solver on a sample, for comparison
    rng = np.random.default_rng(args.seed)
    pick = rng.choice(len(batch), 16, replace=False)
    tot_n, tot_ms = 0, 0.0
    for j in pick:
        sv = B.Solver.from_scene(batch[j])
        sv.step(1)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sv.stream)
        sv.step(8)
        e1.record(sv.stream)
        torch.cuda.synchronize()
        tot_ms += e0.elapsed_time(e1)
        tot_n += batch[j].n
        sv.close()
    per_scene = tot_n * S * 8 / (tot_ms / 1e3)
    print("[bench] %d frames in %.3f ms: %.4g particle-substeps/s from the graph (direct launches: %.4g; "
          "per-scene launches: %.4g)" % (args.steps, ms, value, direct, per_scene), file=sys.stderr, flush=True)
    bpps = pool_bytes_per_particle_substep(batch[0].iterations, 0.0)
    achieved = value * bpps / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_pool (one workgroup per scene, all substeps of the call), replayed from a HIP graph",
            "us_per_call": round(ms * 1e3 / args.steps, 1), "bytes_per_particle_substep": bpps,
            "note": "state stays on chip across iterations, so HBM carries far less than the algorithmic bytes"}
    cpu = None if args.no_cpu_baseline else cpu_baseline_scenes(batch, args.cpu_budget_s, "batch_4096",
                                                                     oracle_threads(args.cpu_threads))
    line = {
        "metric": "particle-substeps/s at stated error vs FP64 oracle",
        "value": round(value, 1), "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch_4096", "scenes": len(batch), "particles": N, "bodies": NB, "substeps": S,
                   "iterations": batch[0].iterations, "seed": args.seed, "max_neighbours": mx,
                   "per_scene_launch_rate": round(per_scene, 1), "direct_launch_rate": round(direct, 1),
                   "tuned_waves": pool.tuning},
        "roofline": roof, "cpu_baseline": cpu,
    }
    pool.close()
    print(json.dumps(line), flush=True)


def bench_serving(args):
    from paper_2603_14634_amd import binding as B
    from paper_2603_14634_amd import scenes
    from paper_2603_14634_amd.serving import (HybridBackend, PoolBackend, ServingEngine, batch_for_budget,
                                              pool_for_budget)

    reqs = scenes.serving_trace(args.seed, rate_hz=args.rate, duration_s=args.window)
    params = B.params_for(reqs[0].scene)
    large = args.large_gib << 30 if args.serving_backend == "hybrid" else 0
    pool = pool_for_budget(params, (args.budget_gib << 30) - large, max_scenes=4096)
    batch = batch_for_budget(params, large) if large else None
    backend = HybridBackend(pool, batch) if batch is not None else PoolBackend(pool)
    eng = ServingEngine(backend, frames_per_tick=args.frames_per_tick, keep_results=False)
    # warm-up: one tiny request compiles nothing new but touches every path once
    eng.run([scenes.Request(0.0, reqs[0].scene, 1, -1)])
    print("[bench] serving: %d requests at %.0f/s over %.2f s, pool of %d particles (%.1f GiB), %s backend"
          % (len(reqs), args.rate, args.window, pool.info().max_particles, pool.info().workspace_bytes / 2 ** 30,
             args.serving_backend), file=sys.stderr, flush=True)
    out = eng.run(reqs)
    print("[bench] served %d in %.2f s: p50 %.1f ms, p99 %.1f ms, %.4g particle-substeps/s, peak %d resident"
          % (out["completed"], out["makespan_s"], out["p50_ms"], out["p99_ms"], out["throughput"],
             out["peak_active"]), file=sys.stderr, flush=True)
    # latency by where the requests ran: the pool's register-resident classes,
    # or the large-scene route (the scene batch, or the pool's large-scene kernel)
    by_id = {r.request_id: r for r in reqs}
    split = {}
    for o in out["outcomes"]:
        big = pool.class_for(by_id[o.request_id].scene) == B.POOL_CLASSES
        split.setdefault("large" if big else "small", []).append(o.latency_s * 1e3)
    split = {k: {"requests": len(v), "p50": round(float(np.percentile(v, 50)), 2),
                 "p99": round(float(np.percentile(v, 99)), 2)} for k, v in sorted(split.items())}
    print("[bench] latency by route: %s" % split, file=sys.stderr, flush=True)
    bpps = pool_bytes_per_particle_substep(reqs[0].scene.iterations, 0.0)
    busy_rate = out["particle_substeps"] / out["busy_s"] if out["busy_s"] > 0 else 0.0
    achieved = busy_rate * bpps / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_pool and the batch's multi-workgroup kernels over the ticks (time the GPU was stepping)",
            "bytes_per_particle_substep": bpps}
    cpu = None if args.no_cpu_baseline else cpu_baseline_scenes([r.scene for r in reqs], args.cpu_budget_s,
                                                                "the serving trace", oracle_threads(args.cpu_threads))
    line = {
        "metric": "particle-substeps/s at stated error vs FP64 oracle; p50/p99 rollout latency",
        "value": round(out["throughput"], 1), "unit": "particle-substeps/s", "n_gpus": 1,
        "steps": out["ticks"], "warmup": 1, "ms_per_step": round(out["busy_s"] * 1e3 / max(out["ticks"], 1), 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "latency_ms": {"p50": round(out["p50_ms"], 2), "p99": round(out["p99_ms"], 2),
                       "mean_queue_wait": round(out["mean_wait_ms"], 2), "by_route": split},
        "config": {"workload": "serving", "rate_hz": args.rate, "window_s": args.window, "requests": len(reqs),
                   "completed": out["completed"], "rejected": len(out["rejected"]),
                   "peak_resident": out["peak_active"], "frames_per_tick": args.frames_per_tick,
                   "hbm_budget_gib": args.budget_gib, "backend": args.serving_backend,
                   "large_scene_gib": args.large_gib if args.serving_backend == "hybrid" else 0,
                   "makespan_s": round(out["makespan_s"], 3), "seed": args.seed},
        "roofline": roof, "cpu_baseline": cpu,
    }
    pool.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed frames")
    ap.add_argument("--warmup", type=int, default=20, help="untimed frames")
    ap.add_argument("--workload", default="dense_pile_20k")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--hash-bits", type=int, default=0, help="override the hash-grid key bits (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iteration-launches", action="store_true",
                    help="one launch per solver iteration even where the substep could run them as one")
    ap.add_argument("--no-graph", action="store_true",
                    help="direct kernel launches instead of replaying a captured graph (counter runs)")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=16, help="OpenMP threads of the FP64 reference baseline")
    ap.add_argument("--iter-launches", type=int, default=200, help="launches timed for the roofline")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (3 times), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: Poisson arrival rate (requests/s)")
    ap.add_argument("--window", type=float, default=1.0, help="serving: seconds of arrivals")
    ap.add_argument("--budget-gib", type=int, default=16, help="serving: HBM budget of the scene pool")
    ap.add_argument("--frames-per-tick", type=int, default=2, help="serving: frames per scheduling tick")
    ap.add_argument("--serving-backend", choices=("hybrid", "pool"), default="hybrid",
                    help="serving: large scenes in a scene batch (hybrid) or in the pool's large-scene kernel")
    ap.add_argument("--large-gib", type=int, default=4, help="serving: HBM budget of the scene batch")
    ap.add_argument("--settle", type=int, default=None,
                    help="untimed frames before the warm-up (default: 240 for dense_pile_20k, so the pile has "
                         "settled into contact, 120 for cuboid_rain_1000, so the rain has landed, else 0)")
    args = ap.parse_args()
    if args.workload == "serving":
        # the serving lanes (pool and batch) and the pool's side-by-side classes
        # use about a dozen streams; give each its own hardware queue (read when
        # HIP starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
    if args.gpus != 1:
        print("bench.py measures one GPU only; runs on several GPUs are not supported "
              "(independent scenes would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_14634_amd import binding as B
    from paper_2603_14634_amd import scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batch_4096":
        return bench_pool(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        cal = Roctx()
        cal.begin("calibration copy")
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        cal.end()
        print("[bench] calibration copy: %d bytes read and %d bytes written per launch" % (nbytes, nbytes),
              file=sys.stderr, flush=True)
        del src, dst
    copy_gbs = measured_copy_gbs()
    sc = scenes.WORKLOADS[args.workload](args.seed)
    print("[bench] workload %s: %d particles, %d bodies" % (sc.name, sc.n, sc.n_bodies), file=sys.stderr,
          flush=True)
    flags = (B.FLAG_ITERATION_LAUNCHES if args.iteration_launches else 0) | (B.FLAG_NO_GRAPH if args.no_graph else 0)
    solver = B.Solver.from_scene(sc, hash_bits=args.hash_bits, flags=flags)
    stream = solver.stream
    settle = args.settle if args.settle is not None else SETTLE_FRAMES.get(args.workload, 0)
    if settle:
        print("[bench] settling %d frames (untimed)" % settle, file=sys.stderr, flush=True)
        done = 0
        while done < settle:
            chunk = min(40, settle - done)
            solver.step(chunk)
            solver.check()
            done += chunk
            print("[bench]   settled %d frames" % done, file=sys.stderr, flush=True)
        # the neighbour statistics restart here (setting the same state clears
        # them), so the mean list length is that of the warm-up and timed frames
        xd = torch.empty((3, sc.n), dtype=torch.float32, device="cuda")
        vd = torch.empty_like(xd)
        solver.read_state_device(xd, vd)
        solver.set_state(xd, vd)
        del xd, vd
    solver.step(args.warmup)
    torch.cuda.synchronize()
    solver.check()

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    marks = Roctx()
    marks.begin("timed frames: %s" % sc.name)
    wall0 = time.perf_counter()
    t_start.record(stream)
    solver.step(args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    marks.end()
    ms = t_start.elapsed_time(t_end)
    solver.check()
    max_nbr, kbar = solver.neighbour_stats()
    psubs = sc.n * sc.substeps * args.steps
    value = psubs / (ms / 1e3)
    print("[bench] %d frames in %.3f ms (wall %.3f s): %.4g particle-substeps/s" % (args.steps, ms, wall, value),
          file=sys.stderr, flush=True)

    # dominant kernel: the iteration kernel of the substep, one Jacobi
    # iteration over all bodies per launch, or all K of them where the
    # substep runs them as one launch (iteration_kernel 2).  Each launch
    # carries a pair of HIP events bound to its own dispatch on the solver's
    # stream (begin and end of the kernel, no marker packets between), so the
    # average is the kernel's duration; the back-to-back rate (which adds the
    # gap between dependent launches) is reported beside it.
    info = solver.info()
    per_launch = sc.iterations if info.iteration_kernel == 2 else 1
    solver.launch_iterations(10)
    torch.cuda.synchronize()
    n_it = args.iter_launches
    it_ms = float(np.mean(solver.time_iterations(n_it))) / 1e3
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    solver.launch_iterations(n_it)
    k1.record(stream)
    torch.cuda.synchronize()
    interval_ms = k0.elapsed_time(k1) / n_it
    bytes_launch = per_launch * (sc.n * iterate_bytes_per_particle(kbar) + sc.n_bodies * iterate_bytes_per_body())
    achieved = bytes_launch / (it_ms / 1e3) / 1e9
    timed_kernel = {0: "k_iterate", 1: "k_iterate_dense", 2: "k_iterate_resident"}[info.iteration_kernel]
    traffic = measured_traffic(sc.name, timed_kernel)
    kernel = {0: "k_iterate (one Jacobi iteration, all bodies, one launch)",
              1: "k_iterate_dense (one Jacobi iteration, all bodies, one launch of 4-wave workgroups)",
              2: "k_iterate_resident (the %d Jacobi iterations of a substep, all bodies, one launch)" % per_launch}
    sub_b = substep_bytes_per_particle(sc.iterations, kbar, info.hash_bits)
    sub_gbs = value * sub_b / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel[info.iteration_kernel],
            "iterations_per_launch": per_launch, "measured_copy_gbs": round(copy_gbs, 1),
            "avg_launch_us": round(it_ms * 1e3, 3), "launch_interval_us": round(interval_ms * 1e3, 3),
            "bytes_per_launch": int(bytes_launch), "particles_per_launch": sc.n,
            "mean_neighbours": round(kbar, 4),
            # HBM bytes the counters saw per launch, over the same duration
            "counter_frac": (round(traffic / (it_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None),
            # the whole substep (index build + K iterations) on the survey's byte model
            "substep": {"bytes_per_particle_substep": round(sub_b, 1), "achieved": round(sub_gbs, 2),
                        "frac": round(sub_gbs / HBM_PEAK_GBS, 4)}}
    print("[bench] iteration kernel %.2f us/launch (%.2f us apart back to back), %.1f GB/s algorithmic"
          % (it_ms * 1e3, interval_ms * 1e3, achieved), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 reference on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(sc, args.cpu_budget_s, oracle_threads(args.cpu_threads))

    line = {
        "metric": "particle-substeps/s at stated error vs FP64 oracle",
        "value": round(value, 1),
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "particles": sc.n, "bodies": sc.n_bodies, "substeps": sc.substeps,
                   "iterations": sc.iterations, "dt_frame": sc.dt_frame, "radius": sc.radius, "seed": args.seed,
                   "max_neighbours": max_nbr, "settled_frames": settle,
                   "accuracy": "per substep |dX - dX_ref| <= 1e-5 r (tests)"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
