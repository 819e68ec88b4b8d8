"""ctypes front end of the FP64 oracle (test infrastructure only).

Every function here only converts arguments; the computation is in
``merf_oracle.c``.  See that file's header for the readings of the paper the
oracle takes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "merf_oracle.c")
_LIB = os.path.join(_HERE, "libmerf_oracle.so")
_lib = None

MAX_LEVELS = 4
MAX_SEG = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("L", C.c_int32), ("B", C.c_int32), ("R", C.c_int32), ("C", C.c_int32),
                ("num_blocks", C.c_int32), ("occ_levels", C.c_int32),
                ("block_index", C.c_void_p), ("blocks", C.c_void_p), ("planes", C.c_void_p),
                ("occ_res", C.c_int32 * MAX_LEVELS), ("occ", C.c_void_p * MAX_LEVELS),
                ("m_density", C.c_double), ("m_feature", C.c_double),
                ("mlp_in", C.c_int32), ("mlp_hidden", C.c_int32), ("mlp", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("c2w", C.c_double * 12), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("step", C.c_double), ("t_min", C.c_double), ("delta_mode", C.c_int32),
                ("want_fragile", C.c_int32), ("eps_occ", C.c_double), ("eps_int", C.c_double)]


RAY_STATS_FIELDS = ["visited", "evaluated", "contributing", "sum_w", "T", "segments", "fragile",
                    "cd0", "cd1", "cd2", "f0", "f1", "f2", "f3"]
_STATS_DTYPE = np.dtype([(n, np.float64) for n in RAY_STATS_FIELDS])

_SAMPLE_DTYPE = np.dtype([("p", np.float64, 3), ("delta", np.float64), ("alpha", np.float64),
                          ("T", np.float64), ("evaluated", np.int32), ("segment", np.int32)])


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    d3 = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.or_region.argtypes = [d3]
    lib.or_region.restype = C.c_int
    lib.or_map_region.argtypes = [C.c_int, d3, d3]
    lib.or_unmap_region.argtypes = [C.c_int, d3, d3]
    lib.or_contract.argtypes = [d3, d3]
    lib.or_candidates.argtypes = [d3, d3, d3]
    lib.or_candidates.restype = C.c_int
    lib.or_segments.argtypes = [d3, d3, d3, d3, np.ctypeslib.ndpointer(np.int32), d3, d3]
    lib.or_segments.restype = C.c_int
    lib.or_dequant.argtypes = [C.c_int, C.c_double]
    lib.or_dequant.restype = C.c_double
    lib.or_features.argtypes = [C.POINTER(_Scene), d3, d3]
    lib.or_occupied.argtypes = [C.POINTER(_Scene), d3]
    lib.or_occupied.restype = C.c_int
    lib.or_encode.argtypes = [d3, d3, d3, d3]
    lib.or_mlp.argtypes = [C.POINTER(_Scene), d3, d3]
    lib.or_render_ray.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), d3, d3, d3, C.c_void_p,
                                  C.c_void_p, C.c_int]
    lib.or_render_ray.restype = C.c_int
    lib.or_camera_ray.argtypes = [C.POINTER(_Camera), C.c_int, C.c_int, d3, d3]
    lib.or_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_int, C.POINTER(_Params),
                              d3, C.c_void_p, C.c_int, C.c_int, C.c_int]
    lib.or_render.restype = C.c_long
    lib.or_max_threads.restype = C.c_int
    _lib = lib
    return lib


class OracleScene:
    """Holds a synth.Scene's arrays alive behind the oracle's own struct."""

    def __init__(self, scene):
        self.scene = scene
        s = _Scene()
        s.L, s.B, s.R, s.C = scene.L, scene.B, scene.R, scene.C
        self._bi = np.ascontiguousarray(scene.block_index, np.int32)
        self._blocks = np.ascontiguousarray(scene.blocks, np.uint8)
        self._planes = np.ascontiguousarray(scene.planes, np.uint8)
        self._occ = [np.ascontiguousarray(o, np.uint8) for _, o in scene.occ]
        self._mlp = np.ascontiguousarray(scene.mlp, np.float32)
        s.num_blocks = self._blocks.shape[0]
        s.occ_levels = len(self._occ)
        s.block_index = self._bi.ctypes.data
        s.blocks = self._blocks.ctypes.data if self._blocks.size else None
        s.planes = self._planes.ctypes.data
        for i, (r, _) in enumerate(scene.occ):
            s.occ_res[i] = r
            s.occ[i] = self._occ[i].ctypes.data
        s.m_density, s.m_feature = float(scene.m_density), float(scene.m_feature)
        s.mlp_in, s.mlp_hidden = scene.mlp_in, scene.mlp_hidden
        s.mlp = self._mlp.ctypes.data
        self.s = s

    def ptr(self):
        return C.byref(self.s)


def _as_oscene(scene) -> OracleScene:
    return scene if isinstance(scene, OracleScene) else OracleScene(scene)


def _params(step, t_min, delta_mode, fragile, eps_occ, eps_int) -> _Params:
    p = _Params()
    p.step, p.t_min, p.delta_mode, p.want_fragile = float(step), float(t_min), int(delta_mode), int(bool(fragile))
    p.eps_occ, p.eps_int = float(eps_occ), float(eps_int)
    return p


def _cams(cams):
    n = len(cams)
    arr = (_Camera * n)()
    for i in range(n):
        c = arr[i]
        for k, v in enumerate(np.asarray(cams.c2w[i], np.float64).reshape(12)):
            c.c2w[k] = float(v)
        c.fx, c.fy, c.cx, c.cy = [float(v) for v in np.asarray(cams.intr[i], np.float64)]
        c.width, c.height = int(cams.size[i, 0]), int(cams.size[i, 1])
    return arr


def max_threads() -> int:
    return int(load().or_max_threads())


def render(scene, cams, step: Optional[float] = None, t_min: float = 2e-4, delta_mode: int = 0,
           fragile: bool = True, stats: bool = True, nthreads: int = 0, rows_stride: int = 1,
           row_offset: int = 0, eps_occ: float = 3e-6, eps_int: float = 1e-3):
    """Render cameras; returns (rgba[N,4] float64, stats structured array or None)."""
    lib = load()
    os_ = _as_oscene(scene)
    if step is None:
        step = os_.scene.step
    n = 0
    for i in range(len(cams)):
        h = int(cams.size[i, 1])
        rows = len(range(row_offset, h, max(rows_stride, 1)))
        n += rows * int(cams.size[i, 0])
    out = np.zeros((n, 4), np.float64)
    st = np.zeros(n, _STATS_DTYPE) if (stats or fragile) else None
    carr = _cams(cams)
    p = _params(step, t_min, delta_mode, fragile, eps_occ, eps_int)
    got = lib.or_render(os_.ptr(), carr, len(cams), C.byref(p), out,
                        st.ctypes.data if st is not None else None, int(nthreads), int(rows_stride),
                        int(row_offset))
    assert got == n
    return out, st


def render_ray(scene, o, d, step: Optional[float] = None, t_min: float = 2e-4, delta_mode: int = 0,
               fragile: bool = True, log_cap: int = 200000, eps_occ: float = 3e-6, eps_int: float = 1e-3):
    """One ray; returns (rgba[4], stats record, samples structured array)."""
    lib = load()
    os_ = _as_oscene(scene)
    if step is None:
        step = os_.scene.step
    out = np.zeros(4, np.float64)
    st = np.zeros(1, _STATS_DTYPE)
    log = np.zeros(log_cap, _SAMPLE_DTYPE)
    p = _params(step, t_min, delta_mode, fragile, eps_occ, eps_int)
    n = lib.or_render_ray(os_.ptr(), C.byref(p), np.asarray(o, np.float64).copy(),
                          np.asarray(d, np.float64).copy(), out, st.ctypes.data, log.ctypes.data, log_cap)
    return out, st[0], log[:min(n, log_cap)]


def contract(x):
    lib = load()
    x = np.asarray(x, np.float64)
    flat = x.reshape(-1, 3)
    y = np.zeros_like(flat)
    for i in range(flat.shape[0]):
        yi = np.zeros(3)
        lib.or_contract(np.ascontiguousarray(flat[i]), yi)
        y[i] = yi
    return y.reshape(x.shape)


def region(x) -> int:
    return int(load().or_region(np.ascontiguousarray(x, np.float64)))


def map_region(reg: int, x):
    y = np.zeros(3)
    load().or_map_region(int(reg), np.ascontiguousarray(x, np.float64), y)
    return y


def unmap_region(reg: int, y):
    x = np.zeros(3)
    load().or_unmap_region(int(reg), np.ascontiguousarray(y, np.float64), x)
    return x


def candidates(o, d):
    c = np.zeros(12)
    n = load().or_candidates(np.ascontiguousarray(o, np.float64), np.ascontiguousarray(d, np.float64), c)
    return c[:n]


def segments(o, d):
    """Returns (ta[n], tb[n], region[n], ya[n,3], yb[n,3])."""
    ta, tb = np.zeros(MAX_SEG), np.zeros(MAX_SEG)
    reg = np.zeros(MAX_SEG, np.int32)
    ya, yb = np.zeros((MAX_SEG, 3)), np.zeros((MAX_SEG, 3))
    n = load().or_segments(np.ascontiguousarray(o, np.float64), np.ascontiguousarray(d, np.float64),
                           ta, tb, reg, ya, yb)
    return ta[:n], tb[:n], reg[:n], ya[:n], yb[:n]


def features(scene, p):
    os_ = _as_oscene(scene)
    t = np.zeros(8)
    load().or_features(os_.ptr(), np.ascontiguousarray(p, np.float64), t)
    return t


def occupied(scene, p) -> bool:
    os_ = _as_oscene(scene)
    return bool(load().or_occupied(os_.ptr(), np.ascontiguousarray(p, np.float64)))


def dequant(b: int, m: float) -> float:
    return float(load().or_dequant(int(b), float(m)))


def encode(cd, f, d):
    x = np.zeros(34)
    load().or_encode(np.ascontiguousarray(cd, np.float64), np.ascontiguousarray(f, np.float64),
                     np.ascontiguousarray(d, np.float64), x)
    return x


def mlp(scene, x):
    os_ = _as_oscene(scene)
    y = np.zeros(3)
    load().or_mlp(os_.ptr(), np.ascontiguousarray(x, np.float64), y)
    return y


def camera_rays(cams, cam_index: int, rows, cols):
    """Origins and unit directions of the given pixels, as the oracle computes them."""
    lib = load()
    carr = _cams(cams.subset(cam_index))
    rows, cols = np.atleast_1d(rows), np.atleast_1d(cols)
    o = np.zeros((rows.size, 3))
    d = np.zeros((rows.size, 3))
    for k, (i, j) in enumerate(zip(rows, cols)):
        oi, di = np.zeros(3), np.zeros(3)
        lib.or_camera_ray(C.byref(carr[0]), int(i), int(j), oi, di)
        o[k], d[k] = oi, di
    return o, d
