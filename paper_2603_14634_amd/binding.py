"""ctypes binding of libpbdr (include/pbdr.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts numpy /
torch arguments to the C ABI and back.  Device memory comes from torch (one
uint8 workspace tensor per scene) and work is enqueued on torch's current HIP
stream.  Importing works without a GPU; creating a ``Solver`` needs the built
library and a GPU, and raises if either is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbdr.so")

OK, ERR_INVALID_ARG, ERR_WORKSPACE, ERR_DEVICE, ERR_CAPACITY, ERR_NONFINITE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
FLAG_STD_VELOCITY, FLAG_NO_LIN_MOM, FLAG_NO_ANG_MOM, FLAG_NO_GRAPH = 0x1, 0x2, 0x4, 0x10
FLAG_ITERATION_LAUNCHES = 0x20
PP_AVG_MAX, PP_AVG_OWN, PP_AVG_NONE = 0, 1 << 8, 2 << 8
DEBUG_XT, DEBUG_KEYS, DEBUG_SORTED, DEBUG_CELL_START, DEBUG_CELL_COUNT = 1, 2, 3, 4, 5
DEBUG_NBR_COUNT, DEBUG_NBR, DEBUG_DELTA = 6, 7, 8
MAX_PLANES = 8
MAX_TIMED_LAUNCHES = 4096
COND_CAPACITY, COND_NONFINITE, COND_INTERNAL, COND_PARTNER_WAIT = 0x1, 0x2, 0x4, 0x8

EXPORTED = [
    "pbdr_abi_version", "pbdr_last_error", "pbdr_condition_status", "pbdr_scene_bytes", "pbdr_scene_create",
    "pbdr_scene_set_accel", "pbdr_scene_set_stream", "pbdr_scene_step", "pbdr_scene_substep", "pbdr_scene_set_state",
    "pbdr_scene_read_state", "pbdr_scene_read_bodies", "pbdr_scene_read_rest", "pbdr_scene_check", "pbdr_scene_neighbour_stats",
    "pbdr_scene_read_debug", "pbdr_scene_info_get", "pbdr_scene_launch_iterations",
    "pbdr_scene_time_iterations", "pbdr_scene_destroy", "pbdr_scene_create_static",
    "pbdr_pool_bytes", "pbdr_pool_create", "pbdr_pool_add", "pbdr_pool_remove", "pbdr_pool_step",
    "pbdr_pool_step_slots", "pbdr_pool_substep", "pbdr_pool_read_state", "pbdr_pool_read_debug",
    "pbdr_pool_check", "pbdr_pool_get_tuning", "pbdr_pool_set_tuning", "pbdr_pool_autotune",
    "pbdr_pool_info_get", "pbdr_pool_destroy", "pbdr_pool_step_slots_on", "pbdr_pool_slot_class",
    "pbdr_pool_class_for",
    "pbdr_batch_bytes", "pbdr_batch_create", "pbdr_batch_add", "pbdr_batch_remove", "pbdr_batch_step",
    "pbdr_batch_step_slots", "pbdr_batch_substep", "pbdr_batch_read_state", "pbdr_batch_read_debug",
    "pbdr_batch_check", "pbdr_batch_info_get", "pbdr_batch_destroy",
]
POOL_MAX_PARTICLES, POOL_MAX_BODIES, POOL_CLASSES, POOL_LANES = 65535, 256, 7, 4


class Params(ctypes.Structure):
    _fields_ = [
        ("dt_frame", ctypes.c_double),
        ("substeps", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("gravity", ctypes.c_double * 3),
        ("friction_mu", ctypes.c_double),
        ("radius", ctypes.c_double),
        ("search_radius", ctypes.c_double),
        ("cell_size", ctypes.c_double),
        ("grid_origin", ctypes.c_double * 3),
        ("hash_bits", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("planes", (ctypes.c_double * 4) * MAX_PLANES),
        ("flags", ctypes.c_uint32),
        ("nbr_cap", ctypes.c_int32),
    ]


class SceneDesc(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int32),
        ("n_bodies", ctypes.c_int32),
        ("x", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("body_start", ctypes.c_void_p),
        ("rest_q", ctypes.c_void_p),
    ]


class SceneInfo(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int32),
        ("n_bodies", ctypes.c_int32),
        ("hash_bits", ctypes.c_int32),
        ("nbr_cap", ctypes.c_int32),
        ("substep_h", ctypes.c_double),
        ("search_radius", ctypes.c_double),
        ("cell_size", ctypes.c_double),
        ("waves_per_block", ctypes.c_int32),
        ("iteration_blocks", ctypes.c_int32),
        ("max_body_particles", ctypes.c_int32),
        ("iteration_kernel", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class PoolSceneDesc(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int32),
        ("n_bodies", ctypes.c_int32),
        ("x", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("body_start", ctypes.c_void_p),
        ("gravity", ctypes.c_double * 3),
        ("friction_mu", ctypes.c_double),
    ]


class PoolInfo(ctypes.Structure):
    _fields_ = [
        ("max_scenes", ctypes.c_int32), ("scenes_used", ctypes.c_int32),
        ("max_particles", ctypes.c_int32), ("particles_used", ctypes.c_int32),
        ("largest_free_particles", ctypes.c_int32),
        ("max_bodies", ctypes.c_int32), ("bodies_used", ctypes.c_int32), ("largest_free_bodies", ctypes.c_int32),
        ("max_scene_particles", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("max_scenes", ctypes.c_int32), ("scenes_used", ctypes.c_int32),
        ("max_particles", ctypes.c_int32), ("particles_used", ctypes.c_int32),
        ("largest_free_particles", ctypes.c_int32),
        ("max_bodies", ctypes.c_int32), ("bodies_used", ctypes.c_int32),
        ("max_keys", ctypes.c_int32), ("largest_free_keys", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class PbdrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("pbdr status %d: %s" % (status, message))
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libpbdr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpbdr.so is not built (expected at %s); run "
                           "`python -m paper_2603_14634_amd.build`" % path)
    # torch first: its HIP runtime has the same soname as the one libpbdr links,
    # so the library then binds to it and the process holds a single runtime
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.pbdr_abi_version.restype = i32
    lib.pbdr_last_error.restype = ctypes.c_char_p
    lib.pbdr_condition_status.restype = i32
    lib.pbdr_condition_status.argtypes = [ctypes.c_uint32]
    lib.pbdr_scene_bytes.restype = sz
    lib.pbdr_scene_bytes.argtypes = [ctypes.POINTER(Params), i32, i32]
    lib.pbdr_scene_create.restype = i32
    lib.pbdr_scene_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(SceneDesc), vp, sz, vp,
                                      ctypes.POINTER(vp)]
    for name, args in [("pbdr_scene_set_accel", [vp, vp]), ("pbdr_scene_set_stream", [vp, vp]),
                       ("pbdr_scene_step", [vp, i32]),
                       ("pbdr_scene_substep", [vp, i32]), ("pbdr_scene_set_state", [vp, vp, vp, i32]),
                       ("pbdr_scene_read_state", [vp, vp, vp, i32]), ("pbdr_scene_read_rest", [vp, vp]),
                       ("pbdr_scene_read_bodies", [vp, vp, vp, vp, vp]),
                       ("pbdr_scene_check", [vp, ctypes.POINTER(i32)]),
                       ("pbdr_scene_neighbour_stats", [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
                       ("pbdr_scene_read_debug", [vp, i32, vp]),
                       ("pbdr_scene_launch_iterations", [vp, i32]),
                       ("pbdr_scene_time_iterations", [vp, i32, vp]),
                       ("pbdr_scene_info_get", [vp, ctypes.POINTER(SceneInfo)])]:
        fn = getattr(lib, name)
        fn.restype = i32
        fn.argtypes = args
    lib.pbdr_scene_destroy.restype = None
    lib.pbdr_scene_destroy.argtypes = [vp]
    pi32 = ctypes.POINTER(i32)
    lib.pbdr_pool_bytes.restype = sz
    lib.pbdr_pool_bytes.argtypes = [ctypes.POINTER(Params), i32, i32, i32]
    lib.pbdr_pool_create.restype = i32
    lib.pbdr_pool_create.argtypes = [ctypes.POINTER(Params), i32, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    for name, args in [("pbdr_pool_add", [vp, ctypes.POINTER(PoolSceneDesc), pi32]), ("pbdr_pool_remove", [vp, i32]),
                       ("pbdr_pool_step", [vp, i32]), ("pbdr_pool_step_slots", [vp, i32, vp, vp]),
                       ("pbdr_pool_substep", [vp, i32]), ("pbdr_pool_read_state", [vp, i32, vp, vp, i32]),
                       ("pbdr_pool_read_debug", [vp, i32, i32, vp]), ("pbdr_pool_check", [vp, i32, pi32]),
                       ("pbdr_pool_get_tuning", [vp, vp]), ("pbdr_pool_set_tuning", [vp, vp]),
                       ("pbdr_pool_autotune", [vp, i32, i32, vp]),
                       ("pbdr_pool_info_get", [vp, ctypes.POINTER(PoolInfo)]),
                       ("pbdr_pool_step_slots_on", [vp, i32, vp, i32, vp, vp]),
                       ("pbdr_pool_slot_class", [vp, i32, pi32]),
                       ("pbdr_pool_class_for", [vp, i32, i32, vp, pi32])]:
        fn = getattr(lib, name)
        fn.restype = i32
        fn.argtypes = args
    lib.pbdr_pool_destroy.restype = None
    lib.pbdr_pool_destroy.argtypes = [vp]
    lib.pbdr_batch_bytes.restype = sz
    lib.pbdr_batch_bytes.argtypes = [ctypes.POINTER(Params), i32, i32, i32]
    lib.pbdr_batch_create.restype = i32
    lib.pbdr_batch_create.argtypes = [ctypes.POINTER(Params), i32, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    for name, args in [("pbdr_batch_add", [vp, ctypes.POINTER(PoolSceneDesc), pi32]),
                       ("pbdr_batch_remove", [vp, i32]), ("pbdr_batch_step", [vp, i32]),
                       ("pbdr_batch_step_slots", [vp, i32, vp, vp]), ("pbdr_batch_substep", [vp, i32]),
                       ("pbdr_batch_read_state", [vp, i32, vp, vp, i32]),
                       ("pbdr_batch_read_debug", [vp, i32, i32, vp]), ("pbdr_batch_check", [vp, pi32]),
                       ("pbdr_batch_info_get", [vp, ctypes.POINTER(BatchInfo)])]:
        fn = getattr(lib, name)
        fn.restype = i32
        fn.argtypes = args
    lib.pbdr_batch_destroy.restype = None
    lib.pbdr_batch_destroy.argtypes = [vp]
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().pbdr_last_error().decode()


def condition_status(conditions: int) -> int:
    """Status the library reports for a set of latched device-condition bits."""
    return int(load_library().pbdr_condition_status(conditions))


def _check(status: int):
    if status != OK:
        raise PbdrError(status, last_error())


def make_params(dt_frame: float, substeps: int, iterations: int, radius: float,
                gravity: Sequence[float] = (0.0, 0.0, -9.81), mu: float = 0.4,
                planes: Sequence[Sequence[float]] = ((0.0, 0.0, 1.0, 0.0),),
                search_radius: float = 0.0, cell_size: float = 0.0, grid_origin=(0.0, 0.0, 0.0),
                hash_bits: int = 0, nbr_cap: int = 0, flags: int = 0) -> Params:
    p = Params()
    p.dt_frame = dt_frame
    p.substeps = substeps
    p.iterations = iterations
    p.gravity[:] = [float(g) for g in gravity]
    p.friction_mu = mu
    p.radius = radius
    p.search_radius = search_radius
    p.cell_size = cell_size
    p.grid_origin[:] = [float(o) for o in grid_origin]
    p.hash_bits = hash_bits
    if len(planes) > MAX_PLANES:
        raise ValueError("at most %d planes" % MAX_PLANES)
    p.n_planes = len(planes)
    for j, pl in enumerate(planes):
        p.planes[j][:] = [float(c) for c in pl]
    p.flags = flags
    p.nbr_cap = nbr_cap
    return p


def params_for(scene, **kw) -> Params:
    """Parameters of a ``scenes.Scene``; keyword arguments override."""
    args = dict(gravity=scene.gravity, mu=scene.mu, planes=scene.planes)
    args.update(kw)
    return make_params(scene.dt_frame, scene.substeps, scene.iterations, scene.radius, **args)


def scene_bytes(params: Params, n_particles: int, n_bodies: int) -> int:
    return int(load_library().pbdr_scene_bytes(ctypes.byref(params), n_particles, n_bodies))


def _host_f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


class Solver:
    """One scene resident in GPU memory (a torch uint8 workspace)."""

    def __init__(self, params: Params, x, v, mass, body_start, rest_q=None, device: str = "cuda:0",
                 stream=None, static_workspace: bool = False):
        """static_workspace: place the scene in the library's static device
        workspace (pbdr_scene_create_static) instead of a torch allocation."""
        import torch

        self._lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP GPU is required")
        self.device = torch.device(device)
        self.params = params
        self._x = _host_f32(x, (3, np.asarray(x).shape[1]))
        n = self._x.shape[1]
        self._v = _host_f32(v, (3, n))
        self._m = _host_f32(mass, (n,))
        self._bs = np.ascontiguousarray(body_start, dtype=np.int32)
        self._q = None if rest_q is None else _host_f32(rest_q, (3, n))
        self.n, self.n_bodies = n, int(self._bs.shape[0] - 1)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        desc = SceneDesc(n, self.n_bodies, self._x.ctypes.data, self._v.ctypes.data, self._m.ctypes.data,
                         self._bs.ctypes.data, None if self._q is None else self._q.ctypes.data)
        handle = ctypes.c_void_p()
        self._accel = None
        if static_workspace:
            fn = self._lib.pbdr_scene_create_static
            fn.restype = ctypes.c_int32
            fn.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(SceneDesc), ctypes.c_void_p,
                           ctypes.POINTER(ctypes.c_void_p)]
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(fn(ctypes.byref(params), ctypes.byref(desc), ctypes.c_void_p(self.stream.cuda_stream),
                          ctypes.byref(handle)))
            self._h = handle
            return
        nbytes = self._lib.pbdr_scene_bytes(ctypes.byref(params), n, self.n_bodies)
        if nbytes == 0:
            raise PbdrError(ERR_INVALID_ARG, last_error())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        _check(self._lib.pbdr_scene_create(ctypes.byref(params), ctypes.byref(desc),
                                           self.workspace.data_ptr(), int(nbytes),
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self._h = handle
        self.workspace.record_stream(self.stream)   # the allocator waits for this stream's work on free

    @classmethod
    def from_scene(cls, scene, device: str = "cuda:0", **param_overrides) -> "Solver":
        return cls(params_for(scene, **param_overrides), scene.x, scene.v, scene.mass, scene.body_start,
                   device=device)

    # -- stepping ---------------------------------------------------------
    def step(self, n_frames: int = 1):
        _check(self._lib.pbdr_scene_step(self._h, n_frames))

    def substep(self, n_substeps: int = 1):
        _check(self._lib.pbdr_scene_substep(self._h, n_substeps))

    def set_stream(self, stream):
        """Moves later work to ``stream`` (a torch stream) after the current one drains."""
        _check(self._lib.pbdr_scene_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream
        if self.workspace is not None:
            self.workspace.record_stream(stream)

    def set_accel(self, accel):
        """accel: torch float32 device tensor [3, N] (kept alive here) or None."""
        if accel is None:
            self._accel = None
            _check(self._lib.pbdr_scene_set_accel(self._h, None))
            return
        if tuple(accel.shape) != (3, self.n) or accel.dtype.__str__() != "torch.float32" or not accel.is_cuda:
            raise ValueError("accel must be a float32 CUDA tensor of shape (3, N)")
        self._accel = accel.contiguous()
        _check(self._lib.pbdr_scene_set_accel(self._h, ctypes.c_void_p(self._accel.data_ptr())))

    # -- state ------------------------------------------------------------
    def set_state(self, x, v):
        if hasattr(x, "is_cuda") and x.is_cuda:
            _check(self._lib.pbdr_scene_set_state(self._h, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(v.data_ptr()), 1))
        else:
            xx, vv = _host_f32(x, (3, self.n)), _host_f32(v, (3, self.n))
            _check(self._lib.pbdr_scene_set_state(self._h, xx.ctypes.data, vv.ctypes.data, 0))

    def read_state(self):
        x = np.empty((3, self.n), dtype=np.float32)
        v = np.empty((3, self.n), dtype=np.float32)
        _check(self._lib.pbdr_scene_read_state(self._h, x.ctypes.data, v.ctypes.data, 0))
        return x, v

    def read_state_device(self, x, v):
        _check(self._lib.pbdr_scene_read_state(self._h, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(v.data_ptr()), 1))

    def read_bodies(self):
        """Per-body (com [B,3], R [B,3,3], P [B,3], L [B,3]) of the current state, FP64."""
        B = self.n_bodies
        com, rot, P, L = np.zeros((B, 3)), np.zeros((B, 3, 3)), np.zeros((B, 3)), np.zeros((B, 3))
        _check(self._lib.pbdr_scene_read_bodies(self._h, com.ctypes.data, rot.ctypes.data, P.ctypes.data,
                                                L.ctypes.data))
        return com, rot, P, L

    def read_rest(self):
        q = np.empty((3, self.n), dtype=np.float32)
        _check(self._lib.pbdr_scene_read_rest(self._h, q.ctypes.data))
        return q

    def check(self) -> int:
        mx = ctypes.c_int32()
        _check(self._lib.pbdr_scene_check(self._h, ctypes.byref(mx)))
        return int(mx.value)

    def status(self) -> int:
        mx = ctypes.c_int32()
        return int(self._lib.pbdr_scene_check(self._h, ctypes.byref(mx)))

    def neighbour_stats(self):
        mx, mean = ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.pbdr_scene_neighbour_stats(self._h, ctypes.byref(mx), ctypes.byref(mean)))
        return int(mx.value), float(mean.value)

    def launch_iterations(self, n_launches: int):
        """Measurement aid: n back-to-back launches of the iteration kernel alone."""
        _check(self._lib.pbdr_scene_launch_iterations(self._h, n_launches))

    def time_iterations(self, n_launches: int) -> np.ndarray:
        """Measurement aid: n launches of the iteration kernel, each timed by HIP
        events bound to its own dispatch; returns the durations in microseconds."""
        out = np.zeros(n_launches, dtype=np.float32)
        _check(self._lib.pbdr_scene_time_iterations(self._h, n_launches, out.ctypes.data))
        return out

    def info(self) -> SceneInfo:
        out = SceneInfo()
        _check(self._lib.pbdr_scene_info_get(self._h, ctypes.byref(out)))
        return out

    def read_debug(self, what: int) -> np.ndarray:
        info = self.info()
        n, T, cap = self.n, 1 << info.hash_bits, info.nbr_cap
        shapes = {DEBUG_XT: ((3, n), np.float32), DEBUG_KEYS: ((n,), np.uint32),
                  DEBUG_SORTED: ((n,), np.uint32), DEBUG_CELL_START: ((T,), np.uint32),
                  DEBUG_CELL_COUNT: ((T,), np.uint32), DEBUG_NBR_COUNT: ((n,), np.uint32),
                  DEBUG_NBR: ((cap, n), np.uint32), DEBUG_DELTA: ((3, n), np.float32)}
        shape, dt = shapes[what]
        out = np.empty(shape, dtype=dt)
        _check(self._lib.pbdr_scene_read_debug(self._h, what, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pbdr_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pool_bytes(params: Params, max_scenes: int, max_particles: int, max_bodies: int) -> int:
    return int(load_library().pbdr_pool_bytes(ctypes.byref(params), max_scenes, max_particles, max_bodies))


class Pool:
    """Many small scenes resident together (include/pbdr.h, scene pools)."""

    def __init__(self, params: Params, max_scenes: int, max_particles: int, max_bodies: int,
                 device: str = "cuda:0", stream=None):
        import torch

        self._lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP GPU is required")
        self.device = torch.device(device)
        self.params = params
        nbytes = self._lib.pbdr_pool_bytes(ctypes.byref(params), max_scenes, max_particles, max_bodies)
        if nbytes == 0:
            raise PbdrError(ERR_INVALID_ARG, last_error())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        _check(self._lib.pbdr_pool_create(ctypes.byref(params), max_scenes, max_particles, max_bodies,
                                          self.workspace.data_ptr(), int(nbytes),
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self._h = handle
        self.workspace.record_stream(self.stream)
        self.sizes = {}

    def try_add(self, scene):
        """Adds a ``scenes.Scene``; returns its slot, or None if it does not fit now."""
        x = _host_f32(scene.x, (3, scene.n))
        v = _host_f32(scene.v, (3, scene.n))
        m = _host_f32(scene.mass, (scene.n,))
        bs = np.ascontiguousarray(scene.body_start, dtype=np.int32)
        desc = PoolSceneDesc(scene.n, scene.n_bodies, x.ctypes.data, v.ctypes.data, m.ctypes.data, bs.ctypes.data)
        desc.gravity[:] = [float(g) for g in scene.gravity]
        desc.friction_mu = float(scene.mu)
        slot = ctypes.c_int32(-1)
        st = self._lib.pbdr_pool_add(self._h, ctypes.byref(desc), ctypes.byref(slot))
        if st == ERR_CAPACITY:
            return None
        _check(st)
        self.sizes[int(slot.value)] = scene.n
        return int(slot.value)

    def add(self, scene) -> int:
        slot = self.try_add(scene)
        if slot is None:
            raise PbdrError(ERR_CAPACITY, last_error())
        return slot

    def remove(self, slot: int):
        _check(self._lib.pbdr_pool_remove(self._h, slot))
        self.sizes.pop(slot, None)

    def step(self, n_frames: int = 1):
        _check(self._lib.pbdr_pool_step(self._h, n_frames))

    def step_slots(self, slots, frames):
        s = np.ascontiguousarray(slots, dtype=np.int32)
        f = np.ascontiguousarray(frames, dtype=np.int32)
        if s.shape != f.shape:
            raise ValueError("slots and frames differ in length")
        _check(self._lib.pbdr_pool_step_slots(self._h, int(s.shape[0]), s.ctypes.data, f.ctypes.data))

    def step_slots_on(self, lane: int, stream, slots, frames):
        """Asynchronous launch of the listed slots on a torch stream through a launch lane."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        f = np.ascontiguousarray(frames, dtype=np.int32)
        if s.shape != f.shape:
            raise ValueError("slots and frames differ in length")
        _check(self._lib.pbdr_pool_step_slots_on(self._h, lane, ctypes.c_void_p(stream.cuda_stream), int(s.shape[0]),
                                                 s.ctypes.data, f.ctypes.data))
        self.workspace.record_stream(stream)   # the allocator waits for this lane's work as well

    def slot_class(self, slot: int) -> int:
        c = ctypes.c_int32()
        _check(self._lib.pbdr_pool_slot_class(self._h, slot, ctypes.byref(c)))
        return int(c.value)

    def class_for(self, scene) -> int:
        """Launch class the scene would get here (POOL_CLASSES = the large-scene kernel)."""
        bs = np.ascontiguousarray(scene.body_start, dtype=np.int32)
        c = ctypes.c_int32()
        _check(self._lib.pbdr_pool_class_for(self._h, int(scene.n), int(bs.shape[0] - 1), bs.ctypes.data,
                                             ctypes.byref(c)))
        return int(c.value)

    def substep(self, n_substeps: int = 1):
        _check(self._lib.pbdr_pool_substep(self._h, n_substeps))

    def read_state(self, slot: int):
        n = self.sizes[slot]
        x = np.empty((3, n), dtype=np.float32)
        v = np.empty((3, n), dtype=np.float32)
        _check(self._lib.pbdr_pool_read_state(self._h, slot, x.ctypes.data, v.ctypes.data, 0))
        return x, v

    def status(self, slot: int) -> int:
        mx = ctypes.c_int32()
        return int(self._lib.pbdr_pool_check(self._h, slot, ctypes.byref(mx)))

    def check(self, slot: int) -> int:
        mx = ctypes.c_int32()
        _check(self._lib.pbdr_pool_check(self._h, slot, ctypes.byref(mx)))
        return int(mx.value)

    def read_debug(self, slot: int, what: int) -> np.ndarray:
        n = self.sizes[slot]
        cap = self.params.nbr_cap or 32
        shapes = {DEBUG_XT: ((3, n), np.float32), DEBUG_NBR_COUNT: ((n,), np.uint32),
                  DEBUG_NBR: ((cap, n), np.uint32), DEBUG_DELTA: ((3, n), np.float32)}
        shape, dt = shapes[what]
        out = np.empty(shape, dtype=dt)
        _check(self._lib.pbdr_pool_read_debug(self._h, slot, what, out.ctypes.data))
        return out

    @property
    def tuning(self):
        w = np.zeros(POOL_CLASSES, dtype=np.int32)
        _check(self._lib.pbdr_pool_get_tuning(self._h, w.ctypes.data))
        return [int(a) for a in w]

    @tuning.setter
    def tuning(self, waves):
        w = np.ascontiguousarray(waves, dtype=np.int32)
        if w.shape != (POOL_CLASSES,):
            raise ValueError("one entry per size class")
        _check(self._lib.pbdr_pool_set_tuning(self._h, w.ctypes.data))

    def autotune(self, n_frames: int = 2, repeats: int = 2):
        ms = np.zeros(POOL_CLASSES, dtype=np.float64)
        _check(self._lib.pbdr_pool_autotune(self._h, n_frames, repeats, ms.ctypes.data))
        return [float(a) for a in ms]

    def info(self) -> PoolInfo:
        out = PoolInfo()
        _check(self._lib.pbdr_pool_info_get(self._h, ctypes.byref(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pbdr_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_bytes(params: Params, max_scenes: int, max_particles: int, max_bodies: int) -> int:
    return int(load_library().pbdr_batch_bytes(ctypes.byref(params), max_scenes, max_particles, max_bodies))


def _pool_desc(scene):
    """A pool/batch scene descriptor and the host arrays it points to."""
    x = _host_f32(scene.x, (3, scene.n))
    v = _host_f32(scene.v, (3, scene.n))
    m = _host_f32(scene.mass, (scene.n,))
    bs = np.ascontiguousarray(scene.body_start, dtype=np.int32)
    desc = PoolSceneDesc(scene.n, scene.n_bodies, x.ctypes.data, v.ctypes.data, m.ctypes.data, bs.ctypes.data)
    desc.gravity[:] = [float(g) for g in scene.gravity]
    desc.friction_mu = float(scene.mu)
    return desc, (x, v, m, bs)


class Batch:
    """Many large scenes stepped together by the multi-workgroup kernels
    (include/pbdr.h, scene batches)."""

    def __init__(self, params: Params, max_scenes: int, max_particles: int, max_bodies: int,
                 device: str = "cuda:0", stream=None):
        import torch

        self._lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP GPU is required")
        self.device = torch.device(device)
        self.params = params
        nbytes = self._lib.pbdr_batch_bytes(ctypes.byref(params), max_scenes, max_particles, max_bodies)
        if nbytes == 0:
            raise PbdrError(ERR_INVALID_ARG, "invalid batch capacities or parameters")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        _check(self._lib.pbdr_batch_create(ctypes.byref(params), max_scenes, max_particles, max_bodies,
                                           self.workspace.data_ptr(), int(nbytes),
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self._h = handle
        self.workspace.record_stream(self.stream)
        self.sizes = {}

    def try_add(self, scene):
        """Adds a ``scenes.Scene``; returns its slot, or None if it does not fit now."""
        desc, keep = _pool_desc(scene)
        slot = ctypes.c_int32(-1)
        st = self._lib.pbdr_batch_add(self._h, ctypes.byref(desc), ctypes.byref(slot))
        del keep
        if st == ERR_CAPACITY:
            return None
        _check(st)
        self.sizes[int(slot.value)] = scene.n
        return int(slot.value)

    def add(self, scene) -> int:
        slot = self.try_add(scene)
        if slot is None:
            raise PbdrError(ERR_CAPACITY, last_error())
        return slot

    def remove(self, slot: int):
        _check(self._lib.pbdr_batch_remove(self._h, slot))
        self.sizes.pop(slot, None)

    def step(self, n_frames: int = 1):
        _check(self._lib.pbdr_batch_step(self._h, n_frames))

    def step_slots(self, slots, frames):
        s = np.ascontiguousarray(slots, dtype=np.int32)
        f = np.ascontiguousarray(frames, dtype=np.int32)
        if s.shape != f.shape:
            raise ValueError("slots and frames differ in length")
        _check(self._lib.pbdr_batch_step_slots(self._h, int(s.shape[0]), s.ctypes.data, f.ctypes.data))

    def substep(self, n_substeps: int = 1):
        _check(self._lib.pbdr_batch_substep(self._h, n_substeps))

    def read_state(self, slot: int):
        n = self.sizes[slot]
        x = np.empty((3, n), dtype=np.float32)
        v = np.empty((3, n), dtype=np.float32)
        _check(self._lib.pbdr_batch_read_state(self._h, slot, x.ctypes.data, v.ctypes.data, 0))
        return x, v

    def check(self) -> int:
        mx = ctypes.c_int32()
        _check(self._lib.pbdr_batch_check(self._h, ctypes.byref(mx)))
        return int(mx.value)

    def read_debug(self, slot: int, what: int) -> np.ndarray:
        n = self.sizes[slot]
        cap = self.params.nbr_cap or 32
        shapes = {DEBUG_XT: ((3, n), np.float32), DEBUG_NBR_COUNT: ((n,), np.uint32),
                  DEBUG_NBR: ((cap, n), np.uint32), DEBUG_DELTA: ((3, n), np.float32)}
        shape, dt = shapes[what]
        out = np.empty(shape, dtype=dt)
        _check(self._lib.pbdr_batch_read_debug(self._h, slot, what, out.ctypes.data))
        return out

    def info(self) -> BatchInfo:
        out = BatchInfo()
        _check(self._lib.pbdr_batch_info_get(self._h, ctypes.byref(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pbdr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
