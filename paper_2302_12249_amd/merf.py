"""ctypes binding of the C ABI in include/merf.h (argument marshalling only).

Every step of rendering runs in the HIP library ``libmerf_hip.so`` built for
gfx950; this module only converts numpy / torch arguments.  Importing it on a
machine without the built library raises immediately: there is no fallback.
PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmerf_hip.so")

MERF_OK = 0
MERF_E_INVALID = -1
MERF_E_OOM = -2
MERF_E_DEVICE = -3
MAX_OCC_LEVELS = 4
STATS_FIELDS = ["rays", "occ_lookups", "visited", "evaluated", "contributing", "terminated"]

PREC = {"f32": 0, "fp32": 0, "f16": 1, "fp16": 1, "bf16": 2}
# feature precision: fp32 interpolation of the codes, every code dequantised
# to float16 first, or appearance interpolated from float16 operands
FEAT = {"f32": 0, "fp32": 0, "f16": 1, "fp16": 1, "f16_interp": 2}


class MerfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"merf error {code}: {msg}")
        self.code = code


class merf_scene_desc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("grid_res", C.c_int32), ("block_size", C.c_int32),
                ("plane_res", C.c_int32), ("channels", C.c_int32), ("num_blocks", C.c_int32),
                ("block_index", C.c_void_p), ("blocks", C.c_void_p), ("planes", C.c_void_p),
                ("occ_levels", C.c_int32), ("occ_res", C.c_int32 * MAX_OCC_LEVELS),
                ("occ", C.c_void_p * MAX_OCC_LEVELS), ("m_density", C.c_float), ("m_feature", C.c_float),
                ("mlp_in", C.c_int32), ("mlp_hidden", C.c_int32), ("mlp_params", C.c_void_p)]


class merf_camera(C.Structure):
    _fields_ = [("c2w", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class merf_render_params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("step", C.c_float), ("t_min", C.c_float),
                ("delta_mode", C.c_int32), ("mlp_prec", C.c_int32), ("feat_prec", C.c_int32),
                ("skip_mode", C.c_int32), ("tile_order", C.c_int32), ("stats_dev", C.c_void_p)]


EXPORTS = ["merf_scene_upload", "merf_render", "merf_render_noalloc", "merf_free", "merf_last_error",
           "merf_set_hbm_budget", "merf_hbm_in_use", "merf_scene_bytes", "merf_dequantize",
           "merf_occupancy_pyramid", "merf_distance_grid", "merf_octant_extent_grid"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(path)
    lib.merf_scene_upload.argtypes = [C.POINTER(merf_scene_desc), C.POINTER(C.c_void_p)]
    lib.merf_scene_upload.restype = C.c_int
    lib.merf_render.argtypes = [C.c_void_p, C.POINTER(merf_camera), C.c_int32, C.POINTER(merf_render_params),
                                C.c_void_p, C.c_void_p]
    lib.merf_render.restype = C.c_int
    lib.merf_render_noalloc.argtypes = lib.merf_render.argtypes
    lib.merf_render_noalloc.restype = C.c_int
    lib.merf_free.argtypes = [C.c_void_p]
    lib.merf_free.restype = C.c_int
    lib.merf_last_error.argtypes = []
    lib.merf_last_error.restype = C.c_char_p
    lib.merf_set_hbm_budget.argtypes = [C.c_size_t]
    lib.merf_set_hbm_budget.restype = C.c_int
    lib.merf_hbm_in_use.argtypes = []
    lib.merf_hbm_in_use.restype = C.c_size_t
    lib.merf_scene_bytes.argtypes = [C.c_void_p]
    lib.merf_scene_bytes.restype = C.c_size_t
    lib.merf_dequantize.argtypes = [C.c_void_p, C.c_int64, C.c_float, C.c_int32, C.c_void_p, C.c_void_p]
    lib.merf_dequantize.restype = C.c_int
    lib.merf_occupancy_pyramid.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                           C.POINTER(C.c_void_p), C.c_void_p]
    lib.merf_occupancy_pyramid.restype = C.c_int
    lib.merf_distance_grid.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_int32), C.c_int32, C.c_void_p,
                                       C.c_void_p]
    lib.merf_distance_grid.restype = C.c_int
    lib.merf_octant_extent_grid.argtypes = lib.merf_distance_grid.argtypes
    lib.merf_octant_extent_grid.restype = C.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().merf_last_error().decode()


def _check(rc: int):
    if rc != MERF_OK:
        raise MerfError(rc, last_error())


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def scene_desc(scene):
    """Build a merf_scene_desc for a synth.Scene-like object.  Returns
    (desc, keepalive) -- keepalive must outlive any call using desc."""
    d = merf_scene_desc()
    d.struct_size = C.sizeof(merf_scene_desc)
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a

    def ptr(a, dt):
        """Address of a numpy array, or of a contiguous cuda tensor of the
        same element size (blocks, planes, occupancy levels and MLP may be
        device memory)."""
        if hasattr(a, "data_ptr") and getattr(a, "is_cuda", False):
            assert a.is_contiguous() and a.element_size() == np.dtype(dt).itemsize
            keep.append(a)
            return a.data_ptr()
        return _ptr(arr(a, dt))

    bi = arr(scene.block_index, np.int32)               # read on the host by the upload
    d.grid_res, d.block_size, d.plane_res, d.channels = scene.L, scene.B, scene.R, scene.C
    d.num_blocks = int(scene.blocks.shape[0])
    d.block_index = _ptr(bi)
    d.blocks = ptr(scene.blocks, np.uint8) if d.num_blocks else None
    d.planes = ptr(scene.planes, np.uint8)
    d.occ_levels = len(scene.occ)
    for i, (r, o) in enumerate(scene.occ):
        d.occ_res[i] = int(r)
        d.occ[i] = ptr(o, np.uint8)
    d.m_density, d.m_feature = float(scene.m_density), float(scene.m_feature)
    d.mlp_in, d.mlp_hidden = scene.mlp_in, scene.mlp_hidden
    d.mlp_params = ptr(scene.mlp, np.float32)
    return d, keep


def scene_upload(scene) -> int:
    """merf_scene_upload: returns the opaque scene handle (an int)."""
    lib = load()
    d, keep = scene_desc(scene)
    h = C.c_void_p()
    _check(lib.merf_scene_upload(C.byref(d), C.byref(h)))
    del keep
    return h.value


def merf_free(handle: int):
    _check(load().merf_free(C.c_void_p(handle)))


def set_hbm_budget(nbytes: int):
    _check(load().merf_set_hbm_budget(int(nbytes)))


def hbm_in_use() -> int:
    return int(load().merf_hbm_in_use())


def scene_bytes(handle: int) -> int:
    return int(load().merf_scene_bytes(C.c_void_p(handle)))


def camera_array(cams):
    """merf_camera[n] from a synth.Cameras-like object."""
    n = len(cams)
    arr = (merf_camera * max(n, 1))()
    for i in range(n):
        c = arr[i]
        for k, v in enumerate(np.asarray(cams.c2w[i], np.float32).reshape(12)):
            c.c2w[k] = float(v)
        c.fx, c.fy, c.cx, c.cy = [float(v) for v in np.asarray(cams.intr[i], np.float32)]
        c.width, c.height = int(cams.size[i, 0]), int(cams.size[i, 1])
    return arr


SKIP = {"distance": 0, "levels": 1}
ORDER = {"heavy_first": 0, "plain": 1}


def render_params(step: float = 0.0, t_min: float = 2e-4, delta_mode: int = 0, mlp_prec="f32",
                  feat_prec="f32", skip="distance", order="heavy_first",
                  stats_ptr: Optional[int] = None) -> merf_render_params:
    p = merf_render_params()
    p.struct_size = C.sizeof(merf_render_params)
    p.step, p.t_min, p.delta_mode = float(step), float(t_min), int(delta_mode)
    p.mlp_prec = PREC[mlp_prec] if isinstance(mlp_prec, str) else int(mlp_prec)
    p.feat_prec = FEAT[feat_prec] if isinstance(feat_prec, str) else int(feat_prec)
    p.skip_mode = SKIP[skip] if isinstance(skip, str) else int(skip)
    p.tile_order = ORDER[order] if isinstance(order, str) else int(order)
    p.stats_dev = stats_ptr
    return p


def merf_render(handle: int, cam_arr, n_cams: int, params: merf_render_params, out_ptr: int, stream_ptr: int = 0):
    """Raw merf_render: cam_arr from camera_array(), out_ptr a device pointer."""
    _check(load().merf_render(C.c_void_p(handle), cam_arr, int(n_cams), C.byref(params), C.c_void_p(out_ptr),
                              C.c_void_p(stream_ptr)))


def merf_render_noalloc(handle: int, cam_arr, n_cams: int, params: merf_render_params, out_ptr: int,
                        stream_ptr: int = 0):
    """Raw merf_render_noalloc (same arguments as merf_render)."""
    _check(load().merf_render_noalloc(C.c_void_p(handle), cam_arr, int(n_cams), C.byref(params),
                                      C.c_void_p(out_ptr), C.c_void_p(stream_ptr)))


def merf_dequantize(codes_ptr: int, n: int, m: float, prec: int, out_ptr: int, stream_ptr: int = 0):
    _check(load().merf_dequantize(C.c_void_p(codes_ptr), int(n), float(m), int(prec), C.c_void_p(out_ptr),
                                  C.c_void_p(stream_ptr)))


def occupancy_pyramid(mask, factors, stream=None):
    """Max-pool a cubic device mask (torch uint8 [r, r, r]) by each factor; returns
    a list of torch uint8 tensors [r/f, r/f, r/f] (merf_occupancy_pyramid)."""
    import torch
    r = int(mask.shape[0])
    assert mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous() and tuple(mask.shape) == (r, r, r)
    outs = [torch.empty((r // f,) * 3, dtype=torch.uint8, device=mask.device) for f in factors]
    fac = (C.c_int32 * len(factors))(*[int(f) for f in factors])
    ptrs = (C.c_void_p * len(factors))(*[o.data_ptr() for o in outs])
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().merf_occupancy_pyramid(C.c_void_p(mask.data_ptr()), r, fac, len(factors), ptrs,
                                         C.c_void_p(st.cuda_stream)))
    return outs


def distance_grid(levels, stream=None, octants=False):
    """Empty-space grid of an occupancy hierarchy: the Chebyshev distance grid
    (merf_distance_grid; torch uint8 [r, r, r]) or, with octants=True, the
    eight forward-extent grids (merf_octant_extent_grid; [8, r, r, r]).
    levels: torch uint8 cubes [r_l, r_l, r_l] on the GPU, coarse to fine."""
    import torch
    for o in levels:
        assert o.is_cuda and o.dtype == torch.uint8 and o.is_contiguous() and o.dim() == 3
    r = int(levels[-1].shape[0])
    shape = (8, r, r, r) if octants else (r, r, r)
    out = torch.empty(shape, dtype=torch.uint8, device=levels[-1].device)
    ptrs = (C.c_void_p * len(levels))(*[o.data_ptr() for o in levels])
    res = (C.c_int32 * len(levels))(*[int(o.shape[0]) for o in levels])
    st = stream if stream is not None else torch.cuda.current_stream()
    fn = load().merf_octant_extent_grid if octants else load().merf_distance_grid
    _check(fn(ptrs, res, len(levels), C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))
    return out


class Renderer:
    """Convenience wrapper: one resident scene rendered into torch tensors."""

    def __init__(self, scene):
        self.scene = scene
        self.handle = scene_upload(scene)

    def close(self):
        if self.handle:
            merf_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def render(self, cams, out=None, stream=None, stats=None, **kw):
        """Render cams into a [pixels, 4] float32 cuda tensor (allocated if out is None)."""
        import torch
        n = cams.num_pixels()
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= 4 * n
        st = stream if stream is not None else torch.cuda.current_stream()
        p = render_params(stats_ptr=stats.data_ptr() if stats is not None else None, **kw)
        merf_render(self.handle, camera_array(cams), len(cams), p, out.data_ptr(), st.cuda_stream)
        return out


# ---------------------------------------------------------------------------
# serving runtime (include/merf_serve.h)
# ---------------------------------------------------------------------------

class merf_server_config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("slots", C.c_int32), ("max_batch", C.c_int32),
                ("use_graphs", C.c_int32), ("evict_idle", C.c_int32), ("pad", C.c_int32),
                ("hbm_budget", C.c_size_t)]


class merf_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("launches", C.c_uint64),
                ("graph_launches", C.c_uint64), ("mixed_launches", C.c_uint64), ("evictions", C.c_uint64),
                ("admissions", C.c_uint64), ("admission_us", C.c_uint64), ("image_admissions", C.c_uint64),
                ("resident_bytes", C.c_size_t), ("resident_scenes", C.c_int32), ("registered", C.c_int32),
                ("max_inflight", C.c_int32), ("pad", C.c_int32)]


SERVE_EXPORTS = ["merf_server_create", "merf_server_destroy", "merf_server_add_scene", "merf_server_remove_scene",
                 "merf_server_submit", "merf_server_poll", "merf_server_wait", "merf_server_drain",
                 "merf_server_get_stats"]


def _serve_lib():
    lib = load()
    if getattr(lib, "_serve_ready", False):
        return lib
    vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
    lib.merf_server_create.argtypes = [C.POINTER(merf_server_config), C.POINTER(vp)]
    lib.merf_server_destroy.argtypes = [vp]
    lib.merf_server_add_scene.argtypes = [vp, C.POINTER(merf_scene_desc), C.POINTER(i32)]
    lib.merf_server_remove_scene.argtypes = [vp, i32]
    lib.merf_server_submit.argtypes = [vp, i32, C.POINTER(merf_camera), C.POINTER(merf_render_params), vp,
                                       C.POINTER(u64)]
    lib.merf_server_poll.argtypes = [vp, u64]
    lib.merf_server_wait.argtypes = [vp, u64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.merf_server_drain.argtypes = [vp]
    lib.merf_server_get_stats.argtypes = [vp, C.POINTER(merf_server_stats)]
    for n in SERVE_EXPORTS:
        getattr(lib, n).restype = C.c_int
    lib._serve_ready = True
    return lib


MEASURE_EXPORTS = ["merf_gather_slots", "merf_record_gathers", "merf_render_phases", "merf_render_timed",
                   "merf_replay_gathers"]
# slots of the phase profile, in the kernel's order (enum PhaseSlot)
PHASE_FIELDS = ["setup_cycles", "march_cycles", "open_cycles", "shade_cycles", "composite_cycles", "mlp_cycles",
                "waves", "march_passes", "open_passes", "open_lanes", "shade_passes", "shade_lanes", "rounds"]


def _measure_lib():
    lib = load()
    if getattr(lib, "_measure_ready", False):
        return lib
    vp, i32 = C.c_void_p, C.c_int32
    lib.merf_gather_slots.argtypes = [C.POINTER(merf_camera), i32, C.POINTER(i32)]
    lib.merf_record_gathers.argtypes = [vp, C.POINTER(merf_camera), i32, C.POINTER(merf_render_params), vp, i32, vp,
                                        vp, vp, vp]
    lib.merf_replay_gathers.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp]
    lib.merf_render_timed.argtypes = [vp, C.POINTER(merf_camera), i32, C.POINTER(merf_render_params), vp, vp, vp, vp]
    lib.merf_render_phases.argtypes = [vp, C.POINTER(merf_camera), i32, C.POINTER(merf_render_params), vp, vp, vp]
    for n in MEASURE_EXPORTS:
        getattr(lib, n).restype = C.c_int
    lib._measure_ready = True
    return lib


def _event_handle(e) -> int:
    """Raw hipEvent_t of a torch.cuda.Event (recorded once, so that it exists),
    a ctypes.c_void_p or an int."""
    if hasattr(e, "cuda_event"):
        assert e.cuda_event, "record the torch event once first"
        return int(e.cuda_event)
    return int(e.value) if isinstance(e, C.c_void_p) else int(e)


def render_timed(handle: int, cams, out, ev_start, ev_end, stream=None, **params):
    """merf_render_timed: render cams (one launch) into the cuda tensor out and
    record the events ev_start / ev_end (timing enabled) right around the
    render kernel."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    p = render_params(**params)
    _check(_measure_lib().merf_render_timed(C.c_void_p(handle), camera_array(cams), len(cams), C.byref(p),
                                            C.c_void_p(out.data_ptr()), C.c_void_p(_event_handle(ev_start)),
                                            C.c_void_p(_event_handle(ev_end)), C.c_void_p(st.cuda_stream)))


def render_phases(handle: int, cams, out, stream=None, **params) -> dict:
    """merf_render_phases: render cams (one launch) into the cuda tensor out
    and return the phase profile summed over the launch's waves (a dict of
    PHASE_FIELDS) and the statistics counters."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    ph = torch.zeros(16, dtype=torch.int64, device="cuda")
    p = render_params(stats_ptr=stats.data_ptr(), **params)
    _check(_measure_lib().merf_render_phases(C.c_void_p(handle), camera_array(cams), len(cams), C.byref(p),
                                             C.c_void_p(out.data_ptr()), C.c_void_p(ph.data_ptr()),
                                             C.c_void_p(st.cuda_stream)))
    st.synchronize()
    v = ph.cpu().numpy()
    res = {n: int(v[i]) for i, n in enumerate(PHASE_FIELDS)}
    res["stats"] = {n: int(x) for n, x in zip(STATS_FIELDS, stats.cpu().numpy())}
    return res


class GatherRecord:
    """Record the texel gathers of one launch (merf_record_gathers) and replay
    them without arithmetic (merf_replay_gathers).  Buffers are torch tensors."""

    def __init__(self, handle: int, cams, cap: int = 64, **params):
        import torch
        lib = _measure_lib()
        self.handle, self.cap = handle, int(cap)
        arr = camera_array(cams)
        n = C.c_int32()
        _check(lib.merf_gather_slots(arr, len(cams), C.byref(n)))
        self.n_slots = n.value
        self.rec = torch.empty((self.cap, self.n_slots, 4), dtype=torch.int32, device="cuda")
        self.count = torch.empty(self.n_slots, dtype=torch.int32, device="cuda")
        self.order = torch.empty(self.n_slots // 64, dtype=torch.int32, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        self.image = torch.empty((cams.num_pixels(), 4), dtype=torch.float32, device="cuda")
        self.out = torch.empty((self.n_slots, 4), dtype=torch.float32, device="cuda")
        p = render_params(stats_ptr=self.stats.data_ptr(), **params)
        st = torch.cuda.current_stream().cuda_stream
        _check(lib.merf_record_gathers(C.c_void_p(handle), arr, len(cams), C.byref(p), C.c_void_p(self.rec.data_ptr()),
                                       self.cap, C.c_void_p(self.count.data_ptr()), C.c_void_p(self.order.data_ptr()),
                                       C.c_void_p(self.image.data_ptr()), C.c_void_p(st)))

    def replay(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(_measure_lib().merf_replay_gathers(C.c_void_p(self.handle), C.c_void_p(self.rec.data_ptr()),
                                                   C.c_void_p(self.count.data_ptr()), self.cap,
                                                   C.c_void_p(self.order.data_ptr()), self.n_slots,
                                                   C.c_void_p(self.out.data_ptr()), C.c_void_p(st.cuda_stream)))
        return self.out


def server_config(slots=4, max_batch=16, use_graphs=True, evict_idle=False, hbm_budget=0) -> merf_server_config:
    c = merf_server_config()
    c.struct_size = C.sizeof(merf_server_config)
    c.slots, c.max_batch, c.use_graphs, c.evict_idle = int(slots), int(max_batch), int(bool(use_graphs)), int(bool(evict_idle))
    c.hbm_budget = int(hbm_budget)
    return c


class Server:
    """Resident scenes + continuous batching of single-view requests."""

    def __init__(self, **cfg):
        self.lib = _serve_lib()
        h = C.c_void_p()
        c = server_config(**cfg)
        _check(self.lib.merf_server_create(C.byref(c), C.byref(h)))
        self.h = h.value

    def close(self):
        if self.h:
            rc = self.lib.merf_server_destroy(C.c_void_p(self.h))
            self.h = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_scene(self, scene) -> int:
        d, keep = scene_desc(scene)
        sid = C.c_int32()
        _check(self.lib.merf_server_add_scene(C.c_void_p(self.h), C.byref(d), C.byref(sid)))
        del keep
        return sid.value

    def remove_scene(self, sid: int):
        _check(self.lib.merf_server_remove_scene(C.c_void_p(self.h), int(sid)))

    def submit(self, sid: int, cam_arr, index: int, out_ptr: int, params: merf_render_params) -> int:
        """Queue camera cam_arr[index] (from camera_array) of scene sid into device memory out_ptr."""
        t = C.c_uint64()
        _check(self.lib.merf_server_submit(C.c_void_p(self.h), int(sid), C.byref(cam_arr[index]), C.byref(params),
                                           C.c_void_p(out_ptr), C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        rc = self.lib.merf_server_poll(C.c_void_p(self.h), C.c_uint64(ticket))
        if rc < 0:
            _check(rc)
        return rc == 1

    def wait(self, ticket: int):
        """Block until done; returns (latency_ms, queue_ms)."""
        lat, q = C.c_double(), C.c_double()
        _check(self.lib.merf_server_wait(C.c_void_p(self.h), C.c_uint64(ticket), C.byref(lat), C.byref(q)))
        return lat.value, q.value

    def drain(self):
        _check(self.lib.merf_server_drain(C.c_void_p(self.h)))

    def stats(self) -> dict:
        s = merf_server_stats()
        _check(self.lib.merf_server_get_stats(C.c_void_p(self.h), C.byref(s)))
        return {n: getattr(s, n) for n, _ in merf_server_stats._fields_}
