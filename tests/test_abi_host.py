"""C-ABI checks that need no GPU: exports, header, struct layout, validation."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2603_14634_amd import binding as B
from paper_2603_14634_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbdr.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pbdr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = B.load_library()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTED) == declared
    assert lib.pbdr_abi_version() == 1


def test_header_compiles_as_c_and_struct_layout_matches_binding(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "pbdr.h"
int main(void) {
  printf("%zu %zu %d %d %zu %zu\n", offsetof(pbdr_scene_info, iteration_kernel),
         offsetof(pbdr_scene_info, max_body_particles), PBDR_MAX_TIMED_LAUNCHES, PBDR_MAX_PLANES,
         sizeof(pbdr_batch_info), offsetof(pbdr_batch_info, workspace_bytes));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pbdr_params), offsetof(pbdr_params, planes),
         offsetof(pbdr_params, flags), sizeof(pbdr_scene_desc), sizeof(pbdr_scene_info),
         offsetof(pbdr_scene_info, workspace_bytes), sizeof(pbdr_pool_scene_desc),
         offsetof(pbdr_pool_scene_desc, gravity), sizeof(pbdr_pool_info), offsetof(pbdr_pool_info, workspace_bytes));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(prog),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = [int(t) for t in out]
    want = [B.SceneInfo.iteration_kernel.offset, B.SceneInfo.max_body_particles.offset, B.MAX_TIMED_LAUNCHES,
            B.MAX_PLANES, ctypes.sizeof(B.BatchInfo), B.BatchInfo.workspace_bytes.offset, ctypes.sizeof(B.Params), B.Params.planes.offset, B.Params.flags.offset, ctypes.sizeof(B.SceneDesc),
            ctypes.sizeof(B.SceneInfo), B.SceneInfo.workspace_bytes.offset, ctypes.sizeof(B.PoolSceneDesc),
            B.PoolSceneDesc.gravity.offset, ctypes.sizeof(B.PoolInfo), B.PoolInfo.workspace_bytes.offset]
    assert got == want


def test_latched_conditions_map_to_statuses():
    # each condition alone, then mixes: a list over capacity is reported first
    # (it can make partner waits give up too), then a non-finite state
    assert B.condition_status(0) == B.OK
    assert B.condition_status(B.COND_CAPACITY) == B.ERR_CAPACITY
    assert B.condition_status(B.COND_NONFINITE) == B.ERR_NONFINITE
    assert B.condition_status(B.COND_INTERNAL) == B.ERR_DEVICE
    assert "internal" in B.last_error()
    assert B.condition_status(B.COND_PARTNER_WAIT) == B.ERR_DEVICE
    assert "partner" in B.last_error()
    assert B.condition_status(B.COND_CAPACITY | B.COND_PARTNER_WAIT) == B.ERR_CAPACITY
    assert B.condition_status(B.COND_NONFINITE | B.COND_PARTNER_WAIT | B.COND_INTERNAL) == B.ERR_NONFINITE
    assert B.condition_status(0xF) == B.ERR_CAPACITY
    assert "last frame" in B.last_error()


def _params(**kw):
    sc = scenes.drop_cubes(0)
    return sc, B.params_for(sc, **kw)


def test_scene_bytes_and_parameter_validation():
    sc, p = _params()
    nbytes = B.scene_bytes(p, sc.n, sc.n_bodies)
    assert nbytes > 0 and nbytes % 256 == 0
    bad = [
        dict(substeps=0), dict(iterations=-1), dict(radius=0.0), dict(dt_frame=float("nan")),
        dict(mu=-0.1), dict(nbr_cap=65), dict(hash_bits=5), dict(hash_bits=29), dict(flags=0x8),
        dict(flags=3 << 8), dict(cell_size=0.05), dict(planes=[(0.0, 0.0, 2.0, 0.0)]),
    ]
    for kw in bad:
        sc2 = scenes.drop_cubes(0)
        args = dict(gravity=sc2.gravity, mu=sc2.mu, planes=sc2.planes)
        base = dict(dt_frame=sc2.dt_frame, substeps=sc2.substeps, iterations=sc2.iterations, radius=sc2.radius)
        base.update({k: v for k, v in kw.items() if k in base})
        args.update({k: v for k, v in kw.items() if k not in base})
        pp = B.make_params(**base, **args)
        assert B.scene_bytes(pp, sc.n, sc.n_bodies) == 0, kw
        assert B.last_error() != ""
    assert B.scene_bytes(p, sc.n, 0) == 0          # particles without bodies
    for ok_flags in (B.FLAG_ITERATION_LAUNCHES, B.FLAG_NO_GRAPH | B.FLAG_ITERATION_LAUNCHES):
        assert B.scene_bytes(B.params_for(sc, flags=ok_flags), sc.n, sc.n_bodies) == nbytes
    assert B.scene_bytes(B.params_for(sc, flags=0x40), sc.n, sc.n_bodies) == 0
    assert B.scene_bytes(p, 0, 0) > 0              # an empty scene is valid


def _create(p, x, v, m, bs, ws=None, ws_bytes=1 << 20):
    lib = B.load_library()
    desc = B.SceneDesc(x.shape[1], bs.shape[0] - 1, x.ctypes.data, v.ctypes.data, m.ctypes.data,
                       bs.ctypes.data, None)
    h = ctypes.c_void_p()
    st = lib.pbdr_scene_create(ctypes.byref(p), ctypes.byref(desc), ws, ws_bytes, None, ctypes.byref(h))
    return st, h


def test_create_rejects_bad_scenes_before_any_device_call():
    sc, p = _params()
    x, v, m, bs = sc.x, sc.v, sc.mass, sc.body_start.copy()
    # every failure below is detected on the host; no workspace or GPU is needed
    st, h = _create(p, x, v, m, bs, ws=None)
    assert st == B.ERR_WORKSPACE and not h.value
    st, _ = _create(p, x, v, m, bs, ws=ctypes.c_void_p(0x1001))
    assert st == B.ERR_WORKSPACE and "aligned" in B.last_error()
    st, _ = _create(p, x, v, m, bs, ws=ctypes.c_void_p(0x1000), ws_bytes=16)
    assert st == B.ERR_WORKSPACE
    bad_bs = bs.copy()
    bad_bs[3] = bad_bs[2]
    st, _ = _create(p, x, v, m, bad_bs, ws=ctypes.c_void_p(0x1000))
    assert st == B.ERR_INVALID_ARG and "empty" in B.last_error()
    bad_bs = bs.copy()
    bad_bs[-1] += 1
    st, _ = _create(p, x, v, m, bad_bs, ws=ctypes.c_void_p(0x1000))
    assert st == B.ERR_INVALID_ARG
    bad_m = m.copy()
    bad_m[5] = -1.0
    st, _ = _create(p, x, v, bad_m, bs, ws=ctypes.c_void_p(0x1000))
    assert st == B.ERR_INVALID_ARG and "mass" in B.last_error()
    bad_x = x.copy()
    bad_x[1, 7] = np.inf
    st, _ = _create(p, bad_x, v, m, bs, ws=ctypes.c_void_p(0x1000))
    assert st == B.ERR_INVALID_ARG and "not finite" in B.last_error()
    big = scenes.single_body(scenes.lattice_box(11, 10, 10, 0.02), radius=0.01)
    pb = B.params_for(big)
    st, _ = _create(pb, big.x, big.v, big.mass, big.body_start, ws=ctypes.c_void_p(0x1000))
    assert st == B.ERR_INVALID_ARG and "max 1024" in B.last_error()


def test_pool_bytes_and_create_validation_before_device_work():
    sc, p = _params()
    lib = B.load_library()
    nbytes = B.pool_bytes(p, 16, 10000, 200)
    assert nbytes > 0 and nbytes % 256 == 0
    assert B.pool_bytes(p, 32, 10000, 200) > nbytes
    for bad in [(0, 100, 10), (4, 0, 10), (4, 100, 0)]:
        assert B.pool_bytes(p, *bad) == 0
    h = ctypes.c_void_p()
    assert lib.pbdr_pool_create(ctypes.byref(p), 4, 100, 10, None, 1 << 20, None, ctypes.byref(h)) == B.ERR_WORKSPACE
    assert lib.pbdr_pool_create(ctypes.byref(p), 4, 100, 10, ctypes.c_void_p(0x1001), 1 << 20, None,
                                ctypes.byref(h)) == B.ERR_WORKSPACE
    assert lib.pbdr_pool_create(ctypes.byref(p), 4, 100, 10, ctypes.c_void_p(0x1000), 16, None,
                                ctypes.byref(h)) == B.ERR_WORKSPACE
    bad = B.make_params(sc.dt_frame, 0, sc.iterations, sc.radius)
    assert lib.pbdr_pool_create(ctypes.byref(bad), 4, 100, 10, ctypes.c_void_p(0x1000), 1 << 30, None,
                                ctypes.byref(h)) == B.ERR_INVALID_ARG
    assert not h.value


def test_null_handles_are_rejected():
    lib = B.load_library()
    assert lib.pbdr_pool_step(None, 1) == B.ERR_INVALID_ARG
    assert lib.pbdr_pool_substep(None, 1) == B.ERR_INVALID_ARG
    assert lib.pbdr_pool_remove(None, 0) == B.ERR_INVALID_ARG
    assert lib.pbdr_pool_read_state(None, 0, None, None, 0) == B.ERR_INVALID_ARG
    assert lib.pbdr_pool_autotune(None, 1, 1, None) == B.ERR_INVALID_ARG
    lib.pbdr_pool_destroy(None)
    assert lib.pbdr_scene_step(None, 1) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_substep(None, 1) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_read_state(None, None, None, 0) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_launch_iterations(None, 1) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_time_iterations(None, 1, None) == B.ERR_INVALID_ARG
    assert lib.pbdr_pool_class_for(None, 1, 1, None, None) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_set_stream(None, None) == B.ERR_INVALID_ARG
    assert lib.pbdr_scene_read_bodies(None, None, None, None, None) == B.ERR_INVALID_ARG
    for name, args in (("pbdr_batch_add", (None, None, None)), ("pbdr_batch_remove", (None, 0)),
                       ("pbdr_batch_step", (None, 1)), ("pbdr_batch_step_slots", (None, 0, None, None)),
                       ("pbdr_batch_substep", (None, 1)), ("pbdr_batch_read_state", (None, 0, None, None, 0)),
                       ("pbdr_batch_read_debug", (None, 0, 0, None)), ("pbdr_batch_check", (None, None)),
                       ("pbdr_batch_info_get", (None, None))):
        assert getattr(lib, name)(*args) == B.ERR_INVALID_ARG, name
    lib.pbdr_batch_destroy(None)
    lib.pbdr_scene_destroy(None)


def test_solver_refuses_to_run_without_gpu_or_library(monkeypatch):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    sc = scenes.drop_cubes(0)
    with pytest.raises(RuntimeError):
        B.Solver.from_scene(sc)
    with pytest.raises(RuntimeError):
        B.Pool(B.params_for(sc), 4, 1000, 10)
