"""ctypes binding of ``libprobestream.so`` (argument marshalling only).

Names follow the C ABI: ``Context`` (pv_ctx), ``Scene`` (pv_scene),
``Volume`` (pv_volume: ``update_probes``, ``blend_rays``, ``get_maps`` ...),
``Client`` (pv_client: ``pack_delta``, ``packet_download`` ...).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libprobestream.so")

PV_OK = 0
PV_MAP_FP32 = 0
PV_MAP_FP16 = 1
PV_FIRST_FRAME_NO_HISTORY = 1
PV_KEEP_HITS = 2
PV_MULTI_BOUNCE = 4
PV_CLASSIFY = 8
# blend paths (pv_volume_set_blend_mode)
PV_BLEND_AUTO, PV_BLEND_BF16X3, PV_BLEND_F32, PV_BLEND_TILES, PV_BLEND_VALU = 0, 1, 2, 3, 4
BLEND_MODES = {"auto": 0, "bf16x3": 1, "f32": 2, "tiles": 3, "valu": 4, "bf16x6": 5}
# pv_measure_ceiling kinds
PV_CEIL_COPY, PV_CEIL_FMA_F32, PV_CEIL_MFMA_F32 = 0, 1, 2
PV_MAX_LIGHTS = 8

# every symbol include/probestream.h declares
EXPORTED_SYMBOLS = [
    "pv_last_error", "pv_version", "pv_ctx_create", "pv_ctx_destroy", "pv_scene_create",
    "pv_scene_set_dynamic", "pv_scene_destroy", "pv_create_volume", "pv_volume_destroy",
    "pv_volume_footprint", "pv_set_scene", "pv_update_probes", "pv_update_probes_after", "pv_update_probes_batched",
    "pv_blend_rays", "pv_get_maps", "pv_get_rays", "pv_set_maps", "pv_read_maps",
    "pv_client_create", "pv_client_destroy", "pv_client_reset", "pv_client_footprint",
    "pv_pack_delta", "pv_packet_device", "pv_packet_download", "pv_get_masks", "pv_sync",
    "pv_trace_counts", "pv_measure_ceiling", "pv_packet_stage", "pv_ctx_set_timing", "pv_ctx_stage_times",
    "pv_client_read_state", "pv_client_set_state", "pv_volume_set_trace_config", "pv_volume_get_trace_config",
    "pv_batch_graph_create", "pv_batch_graph_launch", "pv_batch_graph_destroy", "pv_probe_query",
    "pv_receiver_create", "pv_receiver_destroy", "pv_receiver_apply", "pv_receiver_status",
    "pv_receiver_get_maps", "pv_receiver_read_maps", "pv_yuv_dims", "pv_encode_yuv", "pv_decode_yuv",
    "pv_get_active", "pv_client_set_view", "pv_client_clear_view", "pv_client_get_view",
    "pv_entropy_encode", "pv_entropy_download", "pv_receiver_apply_compressed", "pv_pack_delta_noalloc",
    "pv_scene_read_bvh", "pv_volume_set_blend_mode", "pv_volume_get_blend_mode",
]

STAGES = ["raydirs", "trace", "blend", "pack_mask", "pack_scan", "pack_compact", "batched", "shadow", "shade",
          "pack_finish", "bounce", "unpack", "codec", "select", "entropy"]


class NativeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"probestream status {status}: {msg}")
        self.status = status


class VolumeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3),
                ("rays_per_probe", ctypes.c_int), ("irr_res", ctypes.c_int), ("vis_res", ctypes.c_int),
                ("hysteresis", ctypes.c_float), ("max_distance", ctypes.c_float),
                ("vis_sharpness", ctypes.c_int), ("format", ctypes.c_int),
                ("sky", ctypes.c_float * 3), ("flags", ctypes.c_uint32)]


class PointLight(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("intensity", ctypes.c_float * 3)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int), ("positions", ctypes.c_void_p),
                ("n_triangles", ctypes.c_int), ("indices", ctypes.c_void_p),
                ("albedo", ctypes.c_void_p), ("emission", ctypes.c_void_p),
                ("n_dynamic_triangles", ctypes.c_int), ("n_lights", ctypes.c_int),
                ("lights", ctypes.c_void_p)]


class TraceConfig(ctypes.Structure):
    _fields_ = [("brick", ctypes.c_int * 3), ("persistent", ctypes.c_int), ("top_nodes", ctypes.c_int),
                ("block_threads", ctypes.c_int), ("split_shadows", ctypes.c_int)]


class Frame(ctypes.Structure):
    _fields_ = [("rotation", ctypes.c_float * 9), ("n_lights", ctypes.c_int),
                ("lights", ctypes.POINTER(PointLight))]


_lib = None


def lib_path() -> str:
    return _SO


def build(verbose: bool = False) -> str:
    from . import native_build as _b
    return _b.build(verbose=verbose)


def lib():
    """Load the native library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise ImportError(f"native library {_SO} is missing: build it first "
                          "(paper_2103_05875_amd.native_build.build())")
    L = ctypes.CDLL(_SO)
    vp, i32, u32, u64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "pv_last_error": ([], ctypes.c_char_p),
        "pv_version": ([], ctypes.c_char_p),
        "pv_ctx_create": ([i32, P(vp)], i32),
        "pv_ctx_destroy": ([vp], i32),
        "pv_scene_create": ([vp, P(SceneDesc), P(vp)], i32),
        "pv_scene_set_dynamic": ([vp, vp, vp], i32),
        "pv_scene_destroy": ([vp], i32),
        "pv_scene_read_bvh": ([vp, i32, vp, u64, vp, u64, P(ctypes.c_int64), P(f32)], i32),
        "pv_create_volume": ([vp, P(VolumeDesc), P(vp)], i32),
        "pv_volume_destroy": ([vp], i32),
        "pv_volume_footprint": ([P(VolumeDesc), P(u64)], i32),
        "pv_set_scene": ([vp, vp], i32),
        "pv_update_probes": ([vp, P(Frame), vp], i32),
        "pv_update_probes_after": ([vp, P(Frame), vp, vp], i32),
        "pv_update_probes_batched": ([P(vp), P(Frame), i32, vp], i32),
        "pv_blend_rays": ([vp, P(Frame), vp, vp], i32),
        "pv_get_maps": ([vp, P(vp), P(vp)], i32),
        "pv_get_rays": ([vp, P(vp), P(vp), P(vp)], i32),
        "pv_set_maps": ([vp, vp, vp, ctypes.c_int64], i32),
        "pv_probe_query": ([vp, vp, vp, ctypes.c_int64, vp, vp], i32),
        "pv_receiver_create": ([vp, i32, P(vp)], i32),
        "pv_receiver_destroy": ([vp], i32),
        "pv_receiver_apply": ([vp, vp, u64, vp], i32),
        "pv_receiver_status": ([vp, P(i32), P(u32)], i32),
        "pv_receiver_get_maps": ([vp, P(vp), P(vp)], i32),
        "pv_receiver_read_maps": ([vp, vp, vp], i32),
        "pv_yuv_dims": ([i32, i32, P(ctypes.c_int64)], i32),
        "pv_get_active": ([vp, P(vp)], i32),
        "pv_client_set_view": ([vp, P(f32), i32, vp], i32),
        "pv_client_clear_view": ([vp], i32),
        "pv_client_get_view": ([vp, P(vp)], i32),
        "pv_entropy_encode": ([vp, vp], i32),
        "pv_entropy_download": ([vp, vp, u64, P(u64), vp], i32),
        "pv_receiver_apply_compressed": ([vp, vp, u64, vp], i32),
        "pv_encode_yuv": ([vp, f32, i32, vp, vp, vp], i32),
        "pv_decode_yuv": ([vp, i32, i32, vp, vp, vp, vp, vp], i32),
        "pv_read_maps": ([vp, vp, vp, P(ctypes.c_int64)], i32),
        "pv_client_create": ([vp, u32, P(vp)], i32),
        "pv_client_destroy": ([vp], i32),
        "pv_client_reset": ([vp, vp], i32),
        "pv_client_footprint": ([P(VolumeDesc), P(u64)], i32),
        "pv_pack_delta": ([vp, f32, f32, vp], i32),
        "pv_pack_delta_noalloc": ([vp, vp, vp, vp, vp, i32, f32, f32, u32, u32, vp, u64, vp], i32),
        "pv_packet_device": ([vp, P(vp), P(u64)], i32),
        "pv_packet_download": ([vp, vp, u64, P(u64), vp], i32),
        "pv_get_masks": ([vp, P(vp), P(vp)], i32),
        "pv_sync": ([vp], i32),
        "pv_trace_counts": ([vp, P(Frame), P(u64)], i32),
        "pv_measure_ceiling": ([vp, i32, i32, P(ctypes.c_double)], i32),
        "pv_packet_stage": ([vp, P(ctypes.c_void_p), P(u64), vp], i32),
        "pv_ctx_set_timing": ([vp, i32], i32),
        "pv_client_read_state": ([vp, vp, vp, P(u32)], i32),
        "pv_volume_set_trace_config": ([vp, P(TraceConfig)], i32),
        "pv_batch_graph_create": ([P(vp), i32, P(vp)], i32),
        "pv_batch_graph_launch": ([vp, P(Frame), vp], i32),
        "pv_batch_graph_destroy": ([vp], i32),
        "pv_volume_get_trace_config": ([vp, P(TraceConfig)], i32),
        "pv_volume_set_blend_mode": ([vp, i32], i32),
        "pv_volume_get_blend_mode": ([vp, P(i32)], i32),
        "pv_client_set_state": ([vp, vp, vp, u32], i32),
        "pv_ctx_stage_times": ([vp, P(ctypes.c_double), P(u64)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(st: int):
    if st != PV_OK:
        raise NativeError(st, lib().pv_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    """None or 0 -> HIP's default stream; a torch.cuda.Stream or a raw
    hipStream_t value is passed through."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


# --------------------------------------------------------------------------
# device buffer views (torch plumbing)
# --------------------------------------------------------------------------
class _DevArray:
    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(shape),
                                         "typestr": typestr, "version": 2, "strides": None}


_TYPESTR = {"float32": "<f4", "float16": "<f2", "int32": "<i4", "uint8": "|u1", "uint16": "<u2", "int16": "<i2"}


def device_view(ptr: int, shape, dtype: str):
    """Zero-copy torch view of library-owned device memory."""
    import torch
    return torch.as_tensor(_DevArray(ptr, shape, _TYPESTR[dtype]), device="cuda")


_hip = None


def device_to_host(ptr: int, shape, dtype: str) -> np.ndarray:
    """Copy library-owned device memory to a new numpy array."""
    try:
        return device_view(ptr, shape, dtype).cpu().numpy()
    except Exception:
        global _hip
        if _hip is None:
            _hip = ctypes.CDLL("libamdhip64.so")
            _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        out = np.empty(shape, np.dtype(_TYPESTR[dtype]))
        if _hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), out.nbytes, 2) != 0:  # device to host
            raise RuntimeError("hipMemcpy failed")
        return out


# --------------------------------------------------------------------------
# handles
# --------------------------------------------------------------------------
class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().pv_ctx_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def set_timing(self, enable: bool):
        _check(lib().pv_ctx_set_timing(self.h, 1 if enable else 0))

    def stage_times(self) -> dict:
        """{stage: (total ms, launches)} since the previous call."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_uint64 * len(STAGES))()
        _check(lib().pv_ctx_stage_times(self.h, ms, cnt))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}

    def measure_ceiling(self, kind: int, reps: int = 5) -> float:
        """Attainable rate of a plain kernel on this device: bytes/s for
        PV_CEIL_COPY, FLOP/s for PV_CEIL_FMA_F32 and PV_CEIL_MFMA_F32."""
        r = ctypes.c_double(0.0)
        _check(lib().pv_measure_ceiling(self.h, int(kind), int(reps), ctypes.byref(r)))
        return r.value

    def close(self):
        if getattr(self, "h", None):
            lib().pv_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _lights_array(lights) -> tuple:
    lights = np.ascontiguousarray(lights, np.float32).reshape(-1, 6)
    arr = (PointLight * max(len(lights), 1))()
    for i, l in enumerate(lights):
        arr[i].pos[:] = [float(x) for x in l[:3]]
        arr[i].intensity[:] = [float(x) for x in l[3:]]
    return arr, len(lights)


class Scene:
    def __init__(self, ctx: Context, positions, indices, albedo, emission=None, lights=None,
                 n_dynamic: int = 0):
        self.ctx = ctx
        self._pos = np.ascontiguousarray(positions, np.float32).reshape(-1, 3)
        self._idx = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
        self._alb = np.ascontiguousarray(albedo, np.float32).reshape(-1, 3)
        self._emi = None if emission is None else np.ascontiguousarray(emission, np.float32).reshape(-1, 3)
        self._lights, nl = _lights_array(np.zeros((0, 6)) if lights is None else lights)
        d = SceneDesc()
        d.n_vertices = self._pos.shape[0]
        d.positions = self._pos.ctypes.data
        d.n_triangles = self._idx.shape[0]
        d.indices = self._idx.ctypes.data
        d.albedo = self._alb.ctypes.data
        d.emission = None if self._emi is None else self._emi.ctypes.data
        d.n_dynamic_triangles = int(n_dynamic)
        d.n_lights = nl
        d.lights = ctypes.cast(self._lights, ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(lib().pv_scene_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.n_dynamic = int(n_dynamic)

    @classmethod
    def from_synth(cls, ctx: Context, scene):
        return cls(ctx, scene.positions, scene.indices, scene.albedo, scene.emission, scene.lights,
                   n_dynamic=scene.n_dynamic)

    def set_dynamic(self, positions, stream=None):
        pos = np.ascontiguousarray(positions, np.float32).reshape(-1)
        _check(lib().pv_scene_set_dynamic(self.h, pos.ctypes.data, _stream_handle(stream)))

    def read_bvh(self, dynamic: bool = False):
        """(nodes uint32 [N, 16], triangle slots float32 [T, 12], shadow-ray
        offset) of the device BVH (layout in the header)."""
        cnt = (ctypes.c_int64 * 2)()
        eps = ctypes.c_float(0.0)
        _check(lib().pv_scene_read_bvh(self.h, int(dynamic), None, 0, None, 0, cnt, ctypes.byref(eps)))
        nodes = np.zeros((cnt[0], 16), np.uint32)
        tris = np.zeros((cnt[1], 12), np.float32)
        _check(lib().pv_scene_read_bvh(self.h, int(dynamic), nodes.ctypes.data, nodes.nbytes, tris.ctypes.data,
                                       tris.nbytes, cnt, ctypes.byref(eps)))
        return nodes, tris, eps.value

    def close(self):
        if getattr(self, "h", None):
            lib().pv_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc(cfg, flags: Optional[int] = None) -> VolumeDesc:
    """pv_volume_desc from a volume description object with the fields of
    synth.VolumeConfig."""
    d = VolumeDesc()
    d.nx, d.ny, d.nz = cfg.nx, cfg.ny, cfg.nz
    d.origin[:] = [float(v) for v in cfg.origin]
    d.spacing[:] = [float(v) for v in cfg.spacing]
    d.rays_per_probe = cfg.rays_per_probe
    d.irr_res, d.vis_res = cfg.irr_res, cfg.vis_res
    d.hysteresis = cfg.hysteresis
    d.max_distance = cfg.max_distance
    d.vis_sharpness = cfg.vis_sharpness
    d.format = PV_MAP_FP16 if cfg.fp16 else PV_MAP_FP32
    d.sky[:] = [float(v) for v in cfg.sky]
    if flags is None:
        flags = desc_flags(cfg)
    d.flags = flags
    return d


def make_frame(rotation, lights=None):
    f = Frame()
    f.rotation[:] = [float(v) for v in np.asarray(rotation, np.float32).reshape(9)]
    keep = None
    if lights is not None and len(np.asarray(lights).reshape(-1, 6)) > 0:
        keep, nl = _lights_array(lights)
        f.n_lights = nl
        f.lights = ctypes.cast(keep, ctypes.POINTER(PointLight))
    else:
        f.n_lights = 0
        f.lights = None
    return f, keep


def volume_footprint(cfg, flags: Optional[int] = None) -> int:
    b = ctypes.c_uint64(0)
    _check(lib().pv_volume_footprint(ctypes.byref(make_desc(cfg, flags)), ctypes.byref(b)))
    return b.value


def client_footprint(cfg) -> int:
    b = ctypes.c_uint64(0)
    _check(lib().pv_client_footprint(ctypes.byref(make_desc(cfg)), ctypes.byref(b)))
    return b.value


def desc_flags(cfg, keep_hits: bool = False) -> int:
    return ((PV_FIRST_FRAME_NO_HISTORY if cfg.first_frame_no_history else 0) |
            (PV_KEEP_HITS if keep_hits else 0) |
            (PV_MULTI_BOUNCE if getattr(cfg, "multi_bounce", False) else 0) |
            (PV_CLASSIFY if getattr(cfg, "classify", False) else 0))


class Volume:
    def __init__(self, ctx: Context, cfg, keep_hits: bool = False):
        self.ctx = ctx
        self.cfg = cfg
        self._desc = make_desc(cfg, desc_flags(cfg, keep_hits))
        h = ctypes.c_void_p()
        _check(lib().pv_create_volume(ctx.h, ctypes.byref(self._desc), ctypes.byref(h)))
        self.h = h
        self.P = cfg.nx * cfg.ny * cfg.nz
        self.n = cfg.rays_per_probe
        self.fp16 = bool(cfg.fp16)
        self.keep_hits = keep_hits
        self.scene = None

    def set_scene(self, scene: Scene):
        _check(lib().pv_set_scene(self.h, scene.h))
        self.scene = scene

    def update_probes(self, rotation, lights=None, stream=None, after=None):
        """One update on 'stream'. after: an event (torch.cuda.Event or a raw
        hipEvent_t) that the kernels after the trace wait for (the packs of
        the previous frame), or None."""
        f, keep = make_frame(rotation, lights)
        if after is None:
            _check(lib().pv_update_probes(self.h, ctypes.byref(f), _stream_handle(stream)))
        else:
            ev = after.cuda_event if hasattr(after, "cuda_event") else after
            _check(lib().pv_update_probes_after(self.h, ctypes.byref(f), _stream_handle(stream), ctypes.c_void_p(ev)))
        del keep

    def set_trace_config(self, brick=(4, 4, 4), persistent=2, top_nodes=21, block_threads=256,
                         split_shadows=False):
        c = TraceConfig()
        c.brick[:] = [int(b) for b in brick]
        c.persistent = int(persistent)
        c.top_nodes = int(top_nodes)
        c.block_threads = int(block_threads)
        c.split_shadows = 1 if split_shadows else 0
        _check(lib().pv_volume_set_trace_config(self.h, ctypes.byref(c)))

    def set_blend_mode(self, mode):
        """Blend path: "auto", "bf16x3", "f32", "tiles", "valu", "bf16x6" or its number."""
        _check(lib().pv_volume_set_blend_mode(self.h, BLEND_MODES.get(mode, mode) if isinstance(mode, str)
                                              else int(mode)))

    def get_blend_mode(self) -> str:
        m = ctypes.c_int(0)
        _check(lib().pv_volume_get_blend_mode(self.h, ctypes.byref(m)))
        return {v: k for k, v in BLEND_MODES.items()}[m.value]

    def get_trace_config(self) -> dict:
        c = TraceConfig()
        _check(lib().pv_volume_get_trace_config(self.h, ctypes.byref(c)))
        return {"brick": tuple(c.brick), "persistent": int(c.persistent), "top_nodes": c.top_nodes,
                "block_threads": c.block_threads, "split_shadows": bool(c.split_shadows)}

    def trace_counts(self, rotation, lights=None):
        f, keep = make_frame(rotation, lights)
        out = (ctypes.c_uint64 * 3)()
        _check(lib().pv_trace_counts(self.h, ctypes.byref(f), out))
        return {"node_visits": out[0], "tri_tests": out[1], "shadow_rays": out[2]}

    def blend_rays(self, rotation, rays_dev_ptr: int, stream=None):
        f, keep = make_frame(rotation)
        _check(lib().pv_blend_rays(self.h, ctypes.byref(f), ctypes.c_void_p(rays_dev_ptr), _stream_handle(stream)))

    def get_maps(self):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().pv_get_maps(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def get_rays(self):
        r, h, d = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().pv_get_rays(self.h, ctypes.byref(r), ctypes.byref(h), ctypes.byref(d)))
        return r.value, h.value, d.value

    def read_maps(self):
        """Synchronous copy of the maps: (irr [P,3,10,10], vis [P,2,18,18],
        frame); float32, or uint16 bit patterns for FP16 maps."""
        dt = np.uint16 if self.fp16 else np.float32
        irr = np.zeros((self.P, 3, 10, 10), dt)
        vis = np.zeros((self.P, 2, 18, 18), dt)
        fr = ctypes.c_int64(0)
        _check(lib().pv_read_maps(self.h, irr.ctypes.data, vis.ctypes.data, ctypes.byref(fr)))
        return irr, vis, fr.value

    def set_maps(self, irr, vis, frame: int):
        dt = np.uint16 if self.fp16 else np.float32
        irr = np.ascontiguousarray(irr, dt)
        vis = np.ascontiguousarray(vis, dt)
        assert irr.shape == (self.P, 3, 10, 10) and vis.shape == (self.P, 2, 18, 18)
        _check(lib().pv_set_maps(self.h, irr.ctypes.data, vis.ctypes.data, int(frame)))

    def probe_query(self, points, normals, stream=None):
        """Shading query of the current maps at points [m,3] around normals
        [m,3] (float32 torch tensors on the device, or arrays copied there);
        returns the [m,3] float32 device tensor (asynchronous on ``stream``)."""
        import torch
        pts = torch.as_tensor(points, dtype=torch.float32, device="cuda").contiguous()
        nrm = torch.as_tensor(normals, dtype=torch.float32, device="cuda").contiguous()
        if pts.dim() != 2 or pts.shape[1] != 3 or nrm.shape != pts.shape:
            raise ValueError("points and normals must both be [m, 3]")
        out = torch.empty_like(pts)
        _check(lib().pv_probe_query(self.h, pts.data_ptr(), nrm.data_ptr(), pts.shape[0], out.data_ptr(),
                                    _stream_handle(stream)))
        return out

    def read_active(self) -> np.ndarray:
        """Probe activity of the last update, bool [P] (volumes created with
        cfg.classify)."""
        sync()
        a = ctypes.c_void_p()
        _check(lib().pv_get_active(self.h, ctypes.byref(a)))
        return device_to_host(a.value, (self.P,), "uint8").astype(bool)

    def encode_yuv(self, irr_scale: float, tiles_per_row: int, stream=None, out=None):
        """Codec surfaces of the current maps: (irradiance planes [3, h, w]
        uint16 as int16 bits, visibility planes [3, hv, wv] uint8), torch
        device tensors (asynchronous on ``stream``); ``out`` may hold two
        contiguous tensors of those shapes and sizes to write into."""
        import torch
        w, h, wv, hv = yuv_dims(self.P, tiles_per_row)
        if out is None:
            ip = torch.empty((3, h, w), dtype=torch.int16, device="cuda")
            vp = torch.empty((3, hv, wv), dtype=torch.uint8, device="cuda")
        else:
            ip, vp = out
            if tuple(ip.shape) != (3, h, w) or tuple(vp.shape) != (3, hv, wv) or ip.element_size() != 2 \
                    or vp.element_size() != 1 or not (ip.is_contiguous() and vp.is_contiguous()):
                raise ValueError("output planes do not match the layout")
        _check(lib().pv_encode_yuv(self.h, float(irr_scale), int(tiles_per_row), ip.data_ptr(), vp.data_ptr(),
                                   _stream_handle(stream)))
        return ip, vp

    def read_rays(self):
        """Ray records [P,n,4] float32 (L rgb, distance), hit ids [P,n]
        (None unless keep_hits) and directions [n,4], copied to the host."""
        sync()
        r, h, d = self.get_rays()
        rays = device_to_host(r, (self.P, self.n, 4), "float32")
        dirs = device_to_host(d, (self.n, 4), "float32")
        hits = device_to_host(h, (self.P, self.n), "int32") if h else None
        return rays, hits, dirs

    def close(self):
        if getattr(self, "h", None):
            lib().pv_volume_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def update_probes_batched(volumes: Sequence[Volume], rotations, lights=None, stream=None):
    n = len(volumes)
    arr = (ctypes.c_void_p * n)(*[v.h.value for v in volumes])
    frames = (Frame * n)()
    keeps = []
    for i in range(n):
        f, keep = make_frame(rotations[i], None if lights is None else lights[i])
        frames[i] = f
        keeps.append(keep)
    _check(lib().pv_update_probes_batched(arr, frames, n, _stream_handle(stream)))


class BatchGraph:
    """Captured HIP graph of the batched update of a fixed set of volumes."""

    def __init__(self, volumes: Sequence[Volume]):
        self.volumes = list(volumes)
        arr = (ctypes.c_void_p * len(volumes))(*[v.h.value for v in volumes])
        h = ctypes.c_void_p()
        _check(lib().pv_batch_graph_create(arr, len(volumes), ctypes.byref(h)))
        self.h = h

    def launch(self, rotations, lights=None, stream=None):
        n = len(self.volumes)
        frames = (Frame * n)()
        keeps = []
        for i in range(n):
            f, keep = make_frame(rotations[i], None if lights is None else lights[i])
            frames[i] = f
            keeps.append(keep)
        _check(lib().pv_batch_graph_launch(self.h, frames, _stream_handle(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().pv_batch_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Client:
    def __init__(self, volume: Volume, client_id: int = 0):
        self.volume = volume
        h = ctypes.c_void_p()
        _check(lib().pv_client_create(volume.h, int(client_id), ctypes.byref(h)))
        self.h = h
        self.client_id = client_id

    def pack_delta(self, tau_irr: float = 0.0, tau_vis: float = 0.0, stream=None):
        _check(lib().pv_pack_delta(self.h, float(tau_irr), float(tau_vis), _stream_handle(stream)))

    def reset(self, stream=None):
        _check(lib().pv_client_reset(self.h, _stream_handle(stream)))

    def packet_device(self):
        p, cap = ctypes.c_void_p(), ctypes.c_uint64()
        _check(lib().pv_packet_device(self.h, ctypes.byref(p), ctypes.byref(cap)))
        return p.value, cap.value

    def packet_stage(self, stream=None):
        """Waits for the pack on 'stream' and stages the packet in the
        client's pinned host buffer: (address, size), borrowed until the next
        stage or download on this client."""
        ptr, nb = ctypes.c_void_p(), ctypes.c_uint64(0)
        _check(lib().pv_packet_stage(self.h, ctypes.byref(ptr), ctypes.byref(nb), _stream_handle(stream)))
        return ptr.value, nb.value

    def packet_download(self, stream=None) -> bytes:
        """The last packet as bytes (waits for the pack on 'stream'): staged
        in the client's pinned host buffer, then copied once into the
        returned object."""
        ptr, nb = ctypes.c_void_p(), ctypes.c_uint64(0)
        _check(lib().pv_packet_stage(self.h, ctypes.byref(ptr), ctypes.byref(nb), _stream_handle(stream)))
        return ctypes.string_at(ptr.value, nb.value)

    def read_state(self):
        P = self.volume.P
        ri = np.zeros((P, 3, 64), np.uint16)
        rv = np.zeros((P, 2, 256), np.uint16)
        seq = ctypes.c_uint32(0)
        _check(lib().pv_client_read_state(self.h, ri.ctypes.data, rv.ctypes.data, ctypes.byref(seq)))
        return ri, rv, seq.value

    def set_state(self, ref_irr, ref_vis, seq: int):
        ri = np.ascontiguousarray(ref_irr, np.uint16)
        rv = np.ascontiguousarray(ref_vis, np.uint16)
        assert ri.size == self.volume.P * 192 and rv.size == self.volume.P * 512
        _check(lib().pv_client_set_state(self.h, ri.ctypes.data, rv.ctypes.data, int(seq)))

    def entropy_encode(self, stream=None):
        """Entropy-code the last packet on the device (asynchronous)."""
        _check(lib().pv_entropy_encode(self.h, _stream_handle(stream)))

    def entropy_download(self, stream=None) -> bytes:
        nb = ctypes.c_uint64(0)
        st = lib().pv_entropy_download(self.h, None, 0, ctypes.byref(nb), _stream_handle(stream))
        if st not in (0, -5):
            _check(st)
        buf = np.zeros(max(nb.value, 1), np.uint8)
        _check(lib().pv_entropy_download(self.h, buf.ctypes.data, buf.size, ctypes.byref(nb), _stream_handle(stream)))
        return buf[:nb.value].tobytes()

    def set_view(self, eye, n_rays: int = 4096, stream=None):
        """Cull to the probes a spherical view from ``eye`` can see."""
        e = (ctypes.c_float * 3)(*[float(v) for v in eye])
        _check(lib().pv_client_set_view(self.h, e, int(n_rays), _stream_handle(stream)))

    def clear_view(self):
        _check(lib().pv_client_clear_view(self.h))

    def read_view(self):
        """The view mask, bool [P], or None when no view is set."""
        sync()
        a = ctypes.c_void_p()
        _check(lib().pv_client_get_view(self.h, ctypes.byref(a)))
        return None if not a.value else device_to_host(a.value, (self.volume.P,), "uint8").astype(bool)

    def read_masks(self):
        sync()
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().pv_get_masks(self.h, ctypes.byref(a), ctypes.byref(b)))
        P = self.volume.P
        return (device_to_host(a.value, (P,), "uint8").astype(bool),
                device_to_host(b.value, (P,), "uint8").astype(bool))

    def close(self):
        if getattr(self, "h", None):
            lib().pv_client_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def packet_capacity(n_probes: int) -> int:
    """Bytes of a full-resend packet of n_probes probes."""
    idx = (2 * 2 * n_probes + 15) // 16 * 16
    return 32 + idx + n_probes * 6 * 64 + n_probes * 4 * 256


def pack_delta_noalloc(ctx: Context, cur_irr: int, cur_vis: int, ref_irr: int, ref_vis: int, n_probes: int,
                       tau_irr: float, tau_vis: float, client_id: int, seq: int, packet: int, packet_cap: int,
                       stream=None):
    """pv_pack_delta_noalloc on device addresses (caller-owned buffers)."""
    _check(lib().pv_pack_delta_noalloc(ctx.h, ctypes.c_void_p(cur_irr), ctypes.c_void_p(cur_vis),
                                       ctypes.c_void_p(ref_irr), ctypes.c_void_p(ref_vis), int(n_probes),
                                       float(tau_irr), float(tau_vis), int(client_id), int(seq),
                                       ctypes.c_void_p(packet), int(packet_cap), _stream_handle(stream)))


def yuv_dims(n_probes: int, tiles_per_row: int):
    """(irradiance plane width, height, visibility plane width, height)."""
    d = (ctypes.c_int64 * 4)()
    _check(lib().pv_yuv_dims(int(n_probes), int(tiles_per_row), d))
    return tuple(int(x) for x in d)


def decode_yuv(ctx: "Context", n_probes: int, tiles_per_row: int, irr_planes, vis_planes, stream=None, out=None):
    """Codec surfaces (torch device tensors) back to A2RGB10 codes [P, 64]
    (int32 bits) and visibility binary16 patterns [P, 2, 256] (int16 bits);
    ``out`` may hold two contiguous tensors of those shapes to write into."""
    import torch
    w, h, wv, hv = yuv_dims(n_probes, tiles_per_row)
    if tuple(irr_planes.shape) != (3, h, w) or tuple(vis_planes.shape) != (3, hv, wv):
        raise ValueError("plane shapes do not match the layout")
    if irr_planes.element_size() != 2 or vis_planes.element_size() != 1:
        raise ValueError("irradiance planes are 16-bit, visibility planes 8-bit")
    ip, vp = irr_planes.contiguous(), vis_planes.contiguous()
    if out is None:
        codes = torch.empty((n_probes, 64), dtype=torch.int32, device="cuda")
        vis = torch.empty((n_probes, 2, 256), dtype=torch.int16, device="cuda")
    else:
        codes, vis = out
        if tuple(codes.shape) != (n_probes, 64) or codes.element_size() != 4 or tuple(vis.shape) != (n_probes, 2, 256) \
                or vis.element_size() != 2 or not (codes.is_contiguous() and vis.is_contiguous()):
            raise ValueError("output buffers do not match the layout")
    _check(lib().pv_decode_yuv(ctx.h, int(n_probes), int(tiles_per_row), ip.data_ptr(), vp.data_ptr(),
                               codes.data_ptr(), vis.data_ptr(), _stream_handle(stream)))
    return codes, vis


class Receiver:
    """Client-side state of one volume: FP16 tiles (guard bands included)
    updated from delta packets on the device."""

    def __init__(self, ctx: Context, n_probes: int):
        self.ctx = ctx
        self.P = int(n_probes)
        h = ctypes.c_void_p()
        _check(lib().pv_receiver_create(ctx.h, self.P, ctypes.byref(h)))
        self.h = h

    def apply(self, packet: bytes, stream=None):
        buf = np.frombuffer(packet, np.uint8)
        _check(lib().pv_receiver_apply(self.h, buf.ctypes.data, buf.size, _stream_handle(stream)))

    def apply_compressed(self, container: bytes, stream=None):
        buf = np.frombuffer(container, np.uint8)
        _check(lib().pv_receiver_apply_compressed(self.h, buf.ctypes.data, buf.size, _stream_handle(stream)))

    def status(self):
        """(result, seq): 0 applied, -2 checksum mismatch, -4 invalid index."""
        rc, seq = ctypes.c_int(0), ctypes.c_uint32(0)
        _check(lib().pv_receiver_status(self.h, ctypes.byref(rc), ctypes.byref(seq)))
        return rc.value, seq.value

    def read_maps(self):
        irr = np.zeros((self.P, 3, 10, 10), np.uint16)
        vis = np.zeros((self.P, 2, 18, 18), np.uint16)
        _check(lib().pv_receiver_read_maps(self.h, irr.ctypes.data, vis.ctypes.data))
        return irr, vis

    def close(self):
        if getattr(self, "h", None):
            lib().pv_receiver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sync(stream=None):
    _check(lib().pv_sync(_stream_handle(stream)))
