"""Python binding of the FP64 PBD-R reference (``pbdr_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this module.

``build()`` compiles ``liborc.so`` next to this file with gcc (``-O2
-ffp-contract=off -fno-fast-math -fopenmp``); ``load()`` builds it when it is
missing.  The functions below take and return numpy arrays in the same
structure-of-arrays layout the C code uses.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pbdr_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

STD_VELOCITY = 1
NO_LIN_MOM = 2
NO_ANG_MOM = 4
PP_AVG_MAX, PP_AVG_OWN, PP_AVG_NONE = 0, 1 << 8, 2 << 8


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("mu", ctypes.c_double),
        ("radius", ctypes.c_double),
        ("search_radius", ctypes.c_double),
        ("cell_size", ctypes.c_double),
        ("grid_origin", ctypes.c_double * 3),
        ("planes", (ctypes.c_double * 4) * 8),
        ("iterations", ctypes.c_int32),
        ("hash_bits", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("nbr_cap", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("n_threads", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = ctypes.CDLL(LIB)
        _lib.orc_index.restype = ctypes.c_int32
        _lib.orc_substep.restype = ctypes.c_int32
        _lib.orc_run.restype = ctypes.c_int32
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def default_hash_bits(n: int) -> int:
    """k = max(10, ceil(log2(8n))), at most 28."""
    return int(min(28, max(10, math.ceil(math.log2(max(8 * n, 2))))))


def make_params(h: float, iterations: int, radius: float, gravity=(0.0, 0.0, -9.81), mu: float = 0.4,
                planes=((0.0, 0.0, 1.0, 0.0),), search_radius: Optional[float] = None,
                cell_size: Optional[float] = None, grid_origin=(0.0, 0.0, 0.0),
                hash_bits: int = 10, nbr_cap: int = 32, flags: int = 0, threads: int = 1) -> OrcParams:
    p = OrcParams()
    p.h = h
    p.gravity[:] = list(gravity)
    p.mu = mu
    p.radius = radius
    p.search_radius = 2 * radius if search_radius is None else search_radius
    p.cell_size = p.search_radius * (1.0 + 2.0 ** -10) if cell_size is None else cell_size
    p.grid_origin[:] = list(grid_origin)
    if len(planes) > 8:
        raise ValueError("at most 8 planes")
    for j, pl in enumerate(planes):
        p.planes[j][:] = list(pl)
    p.n_planes = len(planes)
    p.iterations = iterations
    p.hash_bits = hash_bits
    p.nbr_cap = nbr_cap
    p.flags = flags
    p.n_threads = threads
    return p


def params_for(scene, **kw) -> OrcParams:
    """Parameters of a ``scenes.Scene`` (substep h = dt_frame / substeps)."""
    kw.setdefault("hash_bits", default_hash_bits(scene.n))
    return make_params(scene.dt_frame / scene.substeps, scene.iterations, scene.radius,
                       gravity=scene.gravity, mu=scene.mu, planes=scene.planes, **kw)


class Body:
    """Rest pose of a scene: per-particle q and per-body mass (FP64)."""

    def __init__(self, x0: np.ndarray, mass: np.ndarray, body_start: np.ndarray):
        lib = load()
        self.n = int(x0.shape[1])
        self.nb = int(body_start.shape[0] - 1)
        self.mass = _f64(mass)
        self.body_start = np.ascontiguousarray(body_start, dtype=np.int32)
        self.q = np.zeros((3, self.n))
        self.body_mass = np.zeros(self.nb)
        lib.orc_rest_pose(ctypes.c_int32(self.n), ctypes.c_int32(self.nb), _p(self.body_start),
                          _p(self.mass), _p(_f64(x0)), _p(self.q), _p(self.body_mass))

    def body_of_particle(self) -> np.ndarray:
        return np.repeat(np.arange(self.nb, dtype=np.int32), np.diff(self.body_start))


def substep(p: OrcParams, rest: Body, x: np.ndarray, v: np.ndarray, accel=None, n_substeps: int = 1):
    """Runs ``n_substeps`` substeps from (x, v); returns (x, v, max_neighbours)."""
    lib = load()
    xx, vv = _f64(x).copy(), _f64(v).copy()
    acc = None if accel is None else _f64(accel)
    mx = lib.orc_run(ctypes.byref(p), ctypes.c_int32(rest.n), ctypes.c_int32(rest.nb),
                     _p(rest.body_start), _p(rest.mass), _p(rest.body_mass), _p(rest.q),
                     _p(acc), _p(xx), _p(vv), ctypes.c_int32(n_substeps))
    return xx, vv, int(mx)


def body_state(rest: Body, x: np.ndarray, v: np.ndarray):
    """Per-body (com [B,3], R [B,3,3], P [B,3], L [B,3]) of the state (x, v), FP64."""
    lib = load()
    B = rest.nb
    com, rot, P, L = np.zeros((B, 3)), np.zeros((B, 3, 3)), np.zeros((B, 3)), np.zeros((B, 3))
    lib.orc_body_state(ctypes.c_int32(rest.n), ctypes.c_int32(B), _p(rest.body_start), _p(rest.mass),
                       _p(rest.q), _p(_f64(x)), _p(_f64(v)), _p(com), _p(rot), _p(P), _p(L))
    return com, rot, P, L


def predict32(p: OrcParams, x, v, accel=None) -> np.ndarray:
    lib = load()
    x32, v32 = _f32(x), _f32(v)
    a32 = None if accel is None else _f32(accel)
    out = np.zeros_like(x32)
    lib.orc_predict32(ctypes.c_int32(x32.shape[1]), ctypes.byref(p), _p(x32), _p(v32), _p(a32), _p(out))
    return out


def cell_keys(p: OrcParams, xt32) -> np.ndarray:
    lib = load()
    xt = _f32(xt32)
    out = np.zeros(xt.shape[1], dtype=np.uint32)
    lib.orc_cell_keys(ctypes.c_int32(xt.shape[1]), ctypes.byref(p), _p(xt), _p(out))
    return out


def index(p: OrcParams, body: np.ndarray, xt32) -> dict:
    """Keys, stable (key, id) order, cell tables and neighbour lists of FP32 positions."""
    lib = load()
    xt = _f32(xt32)
    n = xt.shape[1]
    T = 1 << p.hash_bits
    out = dict(key=np.zeros(n, np.uint32), sorted_id=np.zeros(n, np.uint32),
               cell_start=np.zeros(T, np.uint32), cell_count=np.zeros(T, np.uint32),
               nbr_count=np.zeros(n, np.uint32),
               nbr=np.zeros((n, p.nbr_cap), np.uint32))
    mx = lib.orc_index(ctypes.c_int32(n), ctypes.byref(p), _p(np.ascontiguousarray(body, np.int32)),
                       _p(xt), _p(out["key"]), _p(out["sorted_id"]), _p(out["cell_start"]),
                       _p(out["cell_count"]), _p(out["nbr_count"]), _p(out["nbr"]))
    out["max_count"] = int(mx)
    return out


def polar(A: np.ndarray) -> np.ndarray:
    lib = load()
    a = _f64(A).reshape(3, 3).copy()
    r = np.zeros((3, 3))
    lib.orc_polar(_p(a), _p(r))
    return r


def pinv_sym3(S: np.ndarray, cutoff: Optional[float] = None) -> np.ndarray:
    """Pseudo-inverse dropping eigenvalues <= cutoff (default 1e-12 * trace)."""
    lib = load()
    s = _f64(S).reshape(3, 3).copy()
    if cutoff is None:
        cutoff = 1e-12 * float(np.trace(s))
    out = np.zeros((3, 3))
    lib.orc_pinv_sym3(_p(s), ctypes.c_double(cutoff), _p(out))
    return out


def enforce_momentum(mass, xb, vb, xa, va, h: float, flags: int = 0, radius: float = 0.0):
    """Eqs. (4)-(5) on one body; positions/velocities are AoS [n, 3]."""
    lib = load()
    n = len(mass)
    xo = np.zeros((n, 3))
    vo = np.zeros((n, 3))
    lib.orc_enforce_momentum(ctypes.c_int32(n), _p(_f64(mass)), _p(_f64(xb)), _p(_f64(vb)),
                             _p(_f64(xa)), _p(_f64(va)), ctypes.c_double(h), ctypes.c_double(radius),
                             ctypes.c_uint32(flags), _p(xo), _p(vo))
    return xo, vo
