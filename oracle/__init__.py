"""FP64 CPU oracle (ctypes front end of ``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark. The product library never imports,
links or calls anything here, and nothing here imports the product package.

Functions follow the paper's Section 3.2 (octahedral irradiance and
visibility maps with guard bands), Section 3.3 (FP16 values split into two
bytes) and Section 3.4 (repacking without guard bands, delta-coded 2-byte
probe index buffer, per-client last-transmitted textures, change
thresholding). The probe update itself is the irradiance-volume method the
paper adopts (Section 3.2) but does not restate; the oracle takes its steps
in order: ray directions, closest hit, shading, weighted means, hysteresis,
guard-band copy.

Parity pins: every function here is pinned by ``tests/test_oracle_pins.py``
against closed forms, special cases, brute force, library routines or the
paper's worked numbers; the shading of fully shadowed scenes at scale is
covered only through those small-scene pins (see the test module docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PV_ORACLE_SANITIZE=1 builds and loads a copy with AddressSanitizer and
# UndefinedBehaviorSanitizer (for a test run with the ASan runtime preloaded)
_SANITIZE = os.environ.get("PV_ORACLE_SANITIZE") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
# oracle.c: the method in FP64; bvh4_replay.c: the GPU trace's traversal work
# replayed on the host from the library's exported BVH (counts only)
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "bvh4_replay.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction beyond the explicit
    fmaf calls, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", *(_SAN_FLAGS if _SANITIZE else []), "-o", tmp, *_SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U16 = ctypes.POINTER(ctypes.c_uint16)
_U8 = ctypes.POINTER(ctypes.c_uint8)


class _Volume(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n", ctypes.c_int), ("irr_res", ctypes.c_int), ("vis_res", ctypes.c_int),
                ("vis_sharpness", ctypes.c_int), ("first_frame_no_history", ctypes.c_int),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("hysteresis", ctypes.c_double), ("max_distance", ctypes.c_double),
                ("sky", ctypes.c_double * 3)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.or_half_to_double.restype = ctypes.c_double
        L.or_half_to_double.argtypes = [ctypes.c_uint16]
        L.or_double_to_half.restype = ctypes.c_uint16
        L.or_double_to_half.argtypes = [ctypes.c_double]
        L.or_round_half_array.argtypes = [_D, _D, ctypes.c_int64]
        L.or_oct_decode.argtypes = [ctypes.c_double, ctypes.c_double, _D]
        L.or_oct_encode.argtypes = [_D, _D]
        L.or_texel_dirs.argtypes = [ctypes.c_int, _D]
        L.or_ray_dirs.argtypes = [ctypes.c_int, _F, _D]
        L.or_scene_create.restype = ctypes.c_void_p
        L.or_scene_create.argtypes = [ctypes.c_int, _F, _F, _F, ctypes.c_int]
        L.or_scene_destroy.argtypes = [ctypes.c_void_p]
        L.or_scene_eps.restype = ctypes.c_double
        L.or_scene_eps.argtypes = [ctypes.c_void_p]
        L.or_scene_diag.restype = ctypes.c_double
        L.or_scene_diag.argtypes = [ctypes.c_void_p]
        L.or_trace_shade.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Volume), _F, ctypes.c_int, _F,
                                     ctypes.c_double, _D, _D, _D, _D, _D, _D, _I32, _D, _I32, _I32,
                                     ctypes.c_int, ctypes.c_int, ctypes.POINTER(_D), ctypes.c_double]
        L.or_probe_lookup.argtypes = [_D, ctypes.c_int, ctypes.c_int, _D, _D]
        L.or_yuv_dims.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.or_huf_lengths.argtypes = [ctypes.POINTER(ctypes.c_uint64), _U8]
        L.or_huf_codes.argtypes = [_U8, ctypes.POINTER(ctypes.c_uint32)]
        L.or_huf_encode.argtypes = [_U8, _U8, ctypes.c_int64]
        L.or_huf_encode.restype = ctypes.c_int64
        L.or_huf_decode.argtypes = [_U8, ctypes.c_int64, _U8, ctypes.c_int64]
        L.or_huf_decode.restype = ctypes.c_int64
        L.or_irr_code.argtypes = [ctypes.c_float, ctypes.c_float]
        L.or_irr_code.restype = ctypes.c_uint16
        L.or_yuv_encode.argtypes = [ctypes.c_int, ctypes.c_int, _D, _U16, ctypes.c_float, _U16, _U8]
        L.or_yuv_decode.argtypes = [ctypes.c_int, ctypes.c_int, _U16, _U8, ctypes.POINTER(ctypes.c_uint32), _U16]
        L.or_probe_query.argtypes = [ctypes.POINTER(_Volume), _D, _D, _D, _D, _D]
        L.or_closest_hits.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, _I32, _D, _I32, ctypes.c_double]
        L.or_closest_hits_brute.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, _I32, _D]
        L.or_border.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.or_blend_update.argtypes = [ctypes.POINTER(_Volume), _D, _D, _D, ctypes.c_int, ctypes.c_int,
                                      _D, _D, ctypes.c_int]
        L.or_payload_checksum.restype = ctypes.c_uint32
        L.or_payload_checksum.argtypes = [_U8, ctypes.c_int64]
        L.or_packet_bytes.restype = ctypes.c_int64
        L.or_packet_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_pack.restype = ctypes.c_int64
        L.or_pack.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _U16, _U16, _U16, _U16,
                              ctypes.c_double, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                              _U8, ctypes.c_int64, _U8, _U8, _U8]
        L.or_client_apply.restype = ctypes.c_int
        L.or_client_apply.argtypes = [_U8, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      _U16, _U16, ctypes.POINTER(ctypes.c_uint32)]
        L.or_max_threads.restype = ctypes.c_int
        L.rp_trace_counts.restype = ctypes.c_int
        L.rp_trace_counts.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F, _F,
                                      ctypes.c_int, _F, ctypes.c_int, _F, ctypes.c_float,
                                      ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# scalar helpers
# --------------------------------------------------------------------------
def half_to_double(bits: int) -> float:
    return lib().or_half_to_double(int(bits))


def double_to_half(x: float) -> int:
    return lib().or_double_to_half(float(x))


def round_half(a: np.ndarray) -> np.ndarray:
    a = _c(a, np.float64)
    out = np.empty_like(a)
    lib().or_round_half_array(_p(a, _D), _p(out, _D), a.size)
    return out


def oct_decode(u: float, w: float) -> np.ndarray:
    out = np.zeros(3)
    lib().or_oct_decode(float(u), float(w), _p(out, _D))
    return out


def oct_encode(v) -> np.ndarray:
    v = _c(v, np.float64)
    out = np.zeros(2)
    lib().or_oct_encode(_p(v, _D), _p(out, _D))
    return out


def texel_dirs(N: int) -> np.ndarray:
    out = np.zeros((N * N, 3))
    lib().or_texel_dirs(N, _p(out, _D))
    return out


def ray_dirs(n: int, R) -> np.ndarray:
    R = _c(R, np.float32).reshape(9)
    out = np.zeros((n, 3))
    lib().or_ray_dirs(n, _p(R, _F), _p(out, _D))
    return out


# --------------------------------------------------------------------------
# scene
# --------------------------------------------------------------------------
class OracleScene:
    """Triangles (float32 [T,3,3]) with per-triangle albedo/emission and the
    oracle's own median-split BVH. ``n_static`` leading triangles define the
    scene extent (and the shadow-ray offset)."""

    def __init__(self, tris, albedo, emission=None, n_static: Optional[int] = None):
        tris = _c(tris, np.float32).reshape(-1, 9)
        self.ntri = tris.shape[0]
        self._tris = tris
        self._alb = _c(albedo, np.float32).reshape(-1, 3)
        self._emi = _c(emission if emission is not None else np.zeros_like(self._alb), np.float32).reshape(-1, 3)
        ns = self.ntri if n_static is None else int(n_static)
        self.h = lib().or_scene_create(self.ntri, _p(self._tris, _F), _p(self._alb, _F), _p(self._emi, _F), ns)

    @classmethod
    def from_scene(cls, scene, n_static: Optional[int] = None):
        if n_static is None:
            n_static = scene.n_triangles - scene.n_dynamic
        return cls(scene.triangles(), scene.albedo, scene.emission, n_static=n_static)

    @property
    def eps(self) -> float:
        return lib().or_scene_eps(self.h)

    @property
    def diag(self) -> float:
        return lib().or_scene_diag(self.h)

    def closest_hits(self, o, d, margin: float = 0.0):
        o = _c(o, np.float64).reshape(-1, 3)
        d = _c(d, np.float64).reshape(-1, 3)
        n = o.shape[0]
        tri = np.zeros(n, np.int32)
        t = np.zeros(n)
        near = np.zeros(n, np.int32)
        lib().or_closest_hits(self.h, n, _p(o, _D), _p(d, _D), _p(tri, _I32), _p(t, _D), _p(near, _I32), margin)
        return tri, t, near

    def closest_hits_brute(self, o, d):
        o = _c(o, np.float64).reshape(-1, 3)
        d = _c(d, np.float64).reshape(-1, 3)
        n = o.shape[0]
        tri = np.zeros(n, np.int32)
        t = np.zeros(n)
        lib().or_closest_hits_brute(self.h, n, _p(o, _D), _p(d, _D), _p(tri, _I32), _p(t, _D))
        return tri, t

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_scene_destroy(self.h)
                self.h = None
        except Exception:
            pass


def _volume_struct(cfg) -> _Volume:
    v = _Volume()
    v.nx, v.ny, v.nz = cfg.nx, cfg.ny, cfg.nz
    v.n = cfg.rays_per_probe
    v.irr_res, v.vis_res = cfg.irr_res, cfg.vis_res
    v.vis_sharpness = cfg.vis_sharpness
    v.first_frame_no_history = 1 if cfg.first_frame_no_history else 0
    for k in range(3):
        # the volume description is FP32 data on both sides
        v.origin[k] = float(np.float32(cfg.origin[k]))
        v.spacing[k] = float(np.float32(cfg.spacing[k]))
        v.sky[k] = float(np.float32(cfg.sky[k]))
    v.hysteresis = float(np.float32(cfg.hysteresis))
    v.max_distance = float(np.float32(cfg.max_distance))
    return v


def trace_shade(scene: OracleScene, cfg, R, lights, delta_rel: float = 1e-6, maxc: int = 8,
                nthreads: int = 0, bounds: bool = True, prev=None, ind_rel: float = 0.0):
    """Trace and shade every (probe, ray). Returns a dict of arrays shaped
    [P, n(, 3)]: L, r (nominal), L_lo, L_hi, r_lo, r_hi (tie bounds),
    hit, hit_t, cand [P, n, maxc], ncand. With ``prev`` = (irr, vis) maps
    (float64 tiles), or (irr, vis, irr_lo, vis_lo, irr_hi, vis_hi) with the
    tie-bound trajectories, every hit also receives the second bounce from
    them; its lo/hi span the three trajectories, widened by ``ind_rel`` of
    the term."""
    v = _volume_struct(cfg)
    P, n = cfg.n_probes, cfg.rays_per_probe
    R = _c(R, np.float32).reshape(9)
    lights = _c(lights, np.float32).reshape(-1, 6)
    prev_ptrs, keep = None, []
    if prev is not None:
        keep = [_c(m, np.float64) for m in prev]
        prev_ptrs = (_D * 6)(*[_p(m, _D) for m in keep], *([None] * (6 - len(keep))))
    L = np.zeros((P, n, 3))
    r = np.zeros((P, n))
    Llo = np.zeros((P, n, 3)) if bounds else None
    Lhi = np.zeros((P, n, 3)) if bounds else None
    rlo = np.zeros((P, n)) if bounds else None
    rhi = np.zeros((P, n)) if bounds else None
    hit = np.zeros((P, n), np.int32)
    hit_t = np.zeros((P, n))
    cand = np.zeros((P, n, maxc), np.int32)
    ncand = np.zeros((P, n), np.int32)
    lib().or_trace_shade(scene.h, ctypes.byref(v), _p(R, _F), lights.shape[0], _p(lights, _F), delta_rel,
                         _p(L, _D), _p(Llo, _D), _p(Lhi, _D), _p(r, _D), _p(rlo, _D), _p(rhi, _D),
                         _p(hit, _I32), _p(hit_t, _D), _p(cand, _I32), _p(ncand, _I32), maxc, nthreads,
                         prev_ptrs, float(ind_rel))
    out = dict(L=L, r=r, hit=hit, hit_t=hit_t, cand=cand, ncand=ncand)
    if bounds:
        out.update(L_lo=Llo, L_hi=Lhi, r_lo=rlo, r_hi=rhi)
    return out


def probe_lookup(tile: np.ndarray, d) -> np.ndarray:
    """Bilinear lookup of one probe's tile [C, N+2, N+2] in direction d."""
    t = _c(tile, np.float64)
    C, S, _ = t.shape
    out = np.zeros(C)
    lib().or_probe_lookup(_p(t, _D), S - 2, C, _p(_c(d, np.float64), _D), _p(out, _D))
    return out


def probe_query(cfg, irr, vis, x, n) -> np.ndarray:
    """Mean radiance at point x around normal n from the maps (irr, vis)."""
    v = _volume_struct(cfg)
    out = np.zeros(3)
    lib().or_probe_query(ctypes.byref(v), _p(_c(irr, np.float64), _D), _p(_c(vis, np.float64), _D),
                         _p(_c(x, np.float64), _D), _p(_c(n, np.float64), _D), _p(out, _D))
    return out


def irr_scale_factor(scale: float) -> np.float32:
    """k of the irradiance code: the FP32 value nearest 1023 / scale."""
    return np.float32(1023.0 / float(scale))


def yuv_dims(P: int, C: int):
    """(irradiance plane width, height, visibility plane width x', height)."""
    out = (ctypes.c_int64 * 4)()
    lib().or_yuv_dims(P, C, out)
    return tuple(int(v) for v in out)


def irr_code(v: float, scale: float) -> int:
    return int(lib().or_irr_code(float(np.float32(v)), float(irr_scale_factor(scale))))


def yuv_encode(irr_tiles, vis_bits, scale: float, C: int):
    """Codec surfaces of a volume: irradiance YUV444 planes [3, H, W] uint16
    and visibility planes [3, Hv, x'] uint8."""
    irr = _c(irr_tiles, np.float64)
    vis = _c(vis_bits, np.uint16)
    P = irr.shape[0]
    W, H, Wv, Hv = yuv_dims(P, C)
    ip = np.zeros((3, H, W), np.uint16)
    vp = np.zeros((3, Hv, Wv), np.uint8)
    lib().or_yuv_encode(P, C, _p(irr, _D), _p(vis, _U16), float(irr_scale_factor(scale)), _p(ip, _U16), _p(vp, _U8))
    return ip, vp


def yuv_decode(irr_planes, vis_planes, P: int, C: int):
    """Inverse of yuv_encode: A2RGB10 codes [P, 64] uint32 and visibility
    binary16 interiors [P, 2, 256] uint16."""
    ip = _c(irr_planes, np.uint16)
    vp = _c(vis_planes, np.uint8)
    codes = np.zeros((P, 64), np.uint32)
    vis = np.zeros((P, 2, 256), np.uint16)
    lib().or_yuv_decode(P, C, _p(ip, _U16), _p(vp, _U8), codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                        _p(vis, _U16))
    return codes, vis


# --------------------------------------------------------------------------
# probe selection (Sec. 3.4): active probes, the client's visible set
# --------------------------------------------------------------------------
def _unit_normals(scene: "OracleScene") -> np.ndarray:
    t = scene._tris.reshape(-1, 3, 3).astype(np.float64)
    n = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def probe_activity(scene: "OracleScene", cfg, R, rays, graze: float = 1e-6, tol: float = 1e-5):
    """Which probes are active after a frame whose trace gave ``rays``
    (trace_shade output). A probe is inactive when more than a quarter of
    its rays hit a triangle from behind (the side its normal (v1 - v0) x
    (v2 - v0) points away from: the probe sits inside a solid), or when none
    of its rays hits anything closer than the cell diagonal |spacing| (no
    surface near enough to be shaded by it). Returns (nominal, lo, hi) bool
    [P]: lo = active whatever the accepted hits and rounding, hi = active for
    some of them (a ray with a grazing hit counts both ways, a hit within
    ``tol`` relative of the diagonal both ways)."""
    P, n = cfg.n_probes, cfg.rays_per_probe
    d = ray_dirs(n, R)
    un = _unit_normals(scene) if scene.ntri else np.zeros((0, 3))
    sp = np.array([float(np.float32(s)) for s in cfg.spacing])
    diag = float(np.sqrt((sp * sp).sum()))
    cand, ncand, hit, t = rays["cand"], rays["ncand"], rays["hit"], rays["hit_t"]
    maxc = cand.shape[2]
    valid = np.arange(maxc)[None, None, :] < ncand[..., None]
    cc = np.where(valid, cand, -2)                     # -2: no candidate in this slot
    is_hit = cc >= 0
    cosv = np.where(is_hit, np.einsum("pnck,nk->pnc", un[np.clip(cc, 0, None)] if scene.ntri else
                                      np.zeros(cc.shape + (3,)), d), 0.0)
    back_c = is_hit & (cosv > graze)
    front_c = (cc == -1) | (is_hit & (cosv < -graze))
    back_nom = (hit >= 0) & (np.where(hit >= 0, np.einsum("pnk,nk->pn", un[np.clip(hit, 0, None)] if scene.ntri
                                                          else np.zeros(hit.shape + (3,)), d), 0.0) > 0)
    back_lo = (back_c | ~valid).all(axis=2) & back_c.any(axis=2)     # every candidate surely from behind
    back_hi = (~(front_c | ~valid)).any(axis=2)                        # some candidate possibly from behind
    near_nom = (hit >= 0) & (t < diag)
    all_hit = (is_hit | ~valid).all(axis=2)
    near_lo = all_hit & (hit >= 0) & (t < diag * (1 - tol))
    near_hi = (is_hit.any(axis=2) & ((hit < 0) | (t < diag * (1 + tol))))

    nom = (4 * back_nom.sum(axis=1) <= n) & near_nom.any(axis=1)
    lo = (4 * back_hi.sum(axis=1) <= n) & near_lo.any(axis=1)
    hi = (4 * back_lo.sum(axis=1) <= n) & near_hi.any(axis=1)
    return nom, lo, hi


def _cell_range(g, dim, tol):
    """Cells an axis coordinate g (grid units) may fall in: the clamped
    floor, and its neighbour when g lies within tol of a cell plane."""
    if dim == 1:
        return {0}
    out = set()
    for x in (g - tol, g, g + tol):
        out.add(int(min(max(np.floor(x), 0), dim - 2)))
    return out


def client_pvs(scene: "OracleScene", cfg, eye, n_rays: int, tol: float = 1e-5, delta_rel: float = 1e-6):
    """The client's potentially visible set (Sec. 3.4: a spherical view from
    the client's position): n_rays spherical-Fibonacci directions (no
    rotation) from ``eye``; every probe at a corner of the grid cell (clamped
    to the grid) holding a hit point. Returns (nominal, lo, hi) bool [P]: hi
    adds, for rays near a tie, every corner of the cells around the hit and,
    for points within tol of a cell plane, both cells; lo keeps only the rays
    whose cell is certain. For a ray near a tie the hits of the ray started
    +-delta along each axis are taken as well (as the trace's accepted set
    does)."""
    P = cfg.n_probes
    dims = (cfg.nx, cfg.ny, cfg.nz)
    o = np.array([float(np.float32(v)) for v in cfg.origin])
    s = np.array([float(np.float32(v)) for v in cfg.spacing])
    eye = np.array([float(np.float32(v)) for v in eye])
    d = ray_dirs(n_rays, np.eye(3, dtype=np.float32))
    m = 2.0 * delta_rel * scene.diag
    tri, t, near = scene.closest_hits(np.repeat(eye[None], n_rays, 0), d, margin=m)
    nom = np.zeros(P, bool)
    lo = np.zeros(P, bool)
    hi = np.zeros(P, bool)

    def mark(mask, cells):
        for cx in cells[0]:
            for cy in cells[1]:
                for cz in cells[2]:
                    for bz in range(2 if dims[2] > 1 else 1):
                        for by in range(2 if dims[1] > 1 else 1):
                            for bx in range(2 if dims[0] > 1 else 1):
                                mask[(cx + bx) + dims[0] * ((cy + by) + dims[1] * (cz + bz))] = True
    def cells(x, widen):
        g = (x - o) / s
        w = [_cell_range(g[a], dims[a], tol) for a in range(3)]
        if widen:
            w = [set(range(max(min(c) - 1, 0), min(max(c) + 1, max(dims[a] - 2, 0)) + 1)) for a, c in enumerate(w)]
        return w

    near_rays = np.nonzero(near)[0]
    alt = {}
    if near_rays.size:
        delta = delta_rel * scene.diag
        for a in range(3):
            for sg in (-1.0, 1.0):
                e2 = eye.copy()
                e2[a] += sg * delta
                tr, tt, _ = scene.closest_hits(np.repeat(e2[None], near_rays.size, 0), d[near_rays])
                for k, r in enumerate(near_rays):
                    if tr[k] >= 0:
                        alt.setdefault(r, []).append(e2 + tt[k] * d[r])
    for r in range(n_rays):
        if tri[r] >= 0:
            x = eye + t[r] * d[r]
            g = (x - o) / s
            mark(nom, [_cell_range(g[a], dims[a], 0.0) for a in range(3)])
            w = cells(x, near[r])
            if not near[r] and all(len(c) == 1 for c in w):
                mark(lo, w)
            mark(hi, w)
        for x in alt.get(r, []):
            mark(hi, cells(x, True))
    return nom, lo, hi


# --------------------------------------------------------------------------
# entropy stage
# --------------------------------------------------------------------------
HUF_MAX_BITS = 12
HUF_CHUNK = 1024


def huf_lengths(hist) -> np.ndarray:
    h = _c(hist, np.uint64)
    assert h.size == 256
    out = np.zeros(256, np.uint8)
    lib().or_huf_lengths(h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _p(out, _U8))
    return out


def huf_codes(lengths) -> np.ndarray:
    ln = _c(lengths, np.uint8)
    out = np.zeros(256, np.uint32)
    lib().or_huf_codes(_p(ln, _U8), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def huf_encode(packet: bytes) -> bytes:
    a = np.frombuffer(packet, np.uint8).copy()
    cap = 64 + 2 * len(packet) + 11 * (132 + 4 * (len(packet) // HUF_CHUNK + 2))
    out = np.zeros(cap, np.uint8)
    n = lib().or_huf_encode(_p(a, _U8), _p(out, _U8), cap)
    assert n > 0
    return out[:n].tobytes()


def huf_decode(container: bytes, cap: int) -> bytes:
    a = np.frombuffer(container, np.uint8).copy()
    out = np.zeros(cap, np.uint8)
    n = lib().or_huf_decode(_p(a, _U8), a.size, _p(out, _U8), cap)
    if n < 0:
        raise ValueError("malformed container")
    return out[:n].tobytes()


def border(tiles: np.ndarray) -> np.ndarray:
    """Guard-band copy of a float tile set [P, C, N+2, N+2] (returns a copy)."""
    t = _c(tiles, np.float64).copy()
    P, C, S, _ = t.shape
    lib().or_border(P, C, S - 2, _p(t, _D))
    return t


def empty_maps(cfg):
    """Zero-initialised float64 maps: irradiance [P,3,Ni+2,Ni+2], visibility
    [P,2,Nv+2,Nv+2]."""
    P = cfg.n_probes
    return (np.zeros((P, 3, cfg.irr_res + 2, cfg.irr_res + 2)),
            np.zeros((P, 2, cfg.vis_res + 2, cfg.vis_res + 2)))


def blend_update(cfg, dirs, L, r, irr, vis, first: bool, fp16: Optional[bool] = None, nthreads: int = 0):
    """One blend + hysteresis + guard-band step on float64 maps (in place,
    also returned). ``dirs``: [n,3] ray directions of the frame."""
    v = _volume_struct(cfg)
    fp16 = cfg.fp16 if fp16 is None else fp16
    dirs = _c(dirs, np.float64)
    L = _c(L, np.float64)
    r = _c(r, np.float64)
    assert irr.dtype == np.float64 and irr.flags.c_contiguous
    assert vis.dtype == np.float64 and vis.flags.c_contiguous
    lib().or_blend_update(ctypes.byref(v), _p(dirs, _D), _p(L, _D), _p(r, _D), 1 if first else 0,
                          1 if fp16 else 0, _p(irr, _D), _p(vis, _D), nthreads)
    return irr, vis


class OracleVolume:
    """Oracle state of one probe volume over frames: nominal maps plus the
    lower/upper tie-bound maps (all float64; FP16-valued when cfg.fp16)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.irr, self.vis = empty_maps(cfg)
        self.irr_lo, self.vis_lo = empty_maps(cfg)
        self.irr_hi, self.vis_hi = empty_maps(cfg)
        self.frame = 0
        self.last = None

    def update(self, scene: OracleScene, R, lights, nthreads: int = 0, delta_rel: float = 1e-6,
               ind_rel: float = 0.0):
        cfg = self.cfg
        prev = None
        if getattr(cfg, "multi_bounce", False):
            prev = tuple(m.copy() for m in (self.irr, self.vis, self.irr_lo, self.vis_lo, self.irr_hi, self.vis_hi))
        rays = trace_shade(scene, cfg, R, lights, delta_rel=delta_rel, nthreads=nthreads, prev=prev,
                           ind_rel=ind_rel)
        dirs = ray_dirs(cfg.rays_per_probe, R)
        first = self.frame == 0
        blend_update(cfg, dirs, rays["L"], rays["r"], self.irr, self.vis, first, nthreads=nthreads)
        blend_update(cfg, dirs, rays["L_lo"], rays["r_lo"], self.irr_lo, self.vis_lo, first, nthreads=nthreads)
        blend_update(cfg, dirs, rays["L_hi"], rays["r_hi"], self.irr_hi, self.vis_hi, first, nthreads=nthreads)
        self.frame += 1
        self.last = rays
        return rays


# --------------------------------------------------------------------------
# traversal work of the GPU trace, replayed on the host
# --------------------------------------------------------------------------
def replay_trace_counts(static_bvh, dynamic_bvh, cfg, dirs, lights, eps: float) -> dict:
    """Node visits, triangle tests and shadow rays of tracing every (probe,
    ray) of ``cfg`` through the library's own BVHs (``(nodes, tris)`` as
    Scene.read_bvh returns them) with directions ``dirs`` [n, 4] float32 as
    the device computed them; see bvh4_replay.c."""
    sn, st = (np.ascontiguousarray(a) for a in static_bvh)
    dn, dt = (np.ascontiguousarray(a) for a in dynamic_bvh)
    f = lambda v: np.array([float(np.float32(x)) for x in v], np.float32)
    o, sp = f(cfg.origin), f(cfg.spacing)
    dirs = _c(dirs, np.float32).reshape(-1, 4)
    lights = _c(lights, np.float32).reshape(-1, 6)
    out = (ctypes.c_uint64 * 3)()
    rc = lib().rp_trace_counts(sn.ctypes.data, sn.shape[0], st.ctypes.data, dn.ctypes.data, dn.shape[0],
                               dt.ctypes.data, cfg.nx, cfg.ny, cfg.nz, _p(o, _F), _p(sp, _F), dirs.shape[0],
                               _p(dirs, _F), lights.shape[0], _p(lights, _F), float(eps), out)
    assert rc == 0, "traversal stack overflow in the replay"
    return {"node_visits": int(out[0]), "tri_tests": int(out[1]), "shadow_rays": int(out[2])}


# --------------------------------------------------------------------------
# packing
# --------------------------------------------------------------------------
def packet_bytes(K_irr: int, K_vis: int, irr_res: int = 8, vis_res: int = 16) -> int:
    return int(lib().or_packet_bytes(K_irr, K_vis, irr_res, vis_res))


def payload_checksum(payload: bytes) -> int:
    a = np.frombuffer(payload, np.uint8).copy()
    return int(lib().or_payload_checksum(_p(a, _U8), a.size))


class OracleClientState:
    """Server-side per-client last-transmitted interiors (uint16)."""

    def __init__(self, n_probes: int, irr_res: int = 8, vis_res: int = 16, client: int = 0):
        self.P, self.Ni, self.Nv = n_probes, irr_res, vis_res
        self.ref_irr = np.zeros((n_probes, 3, irr_res * irr_res), np.uint16)
        self.ref_vis = np.zeros((n_probes, 2, vis_res * vis_res), np.uint16)
        self.client = client
        self.seq = 0

    def pack(self, cur_irr: np.ndarray, cur_vis: np.ndarray, tau_irr: float = 0.0, tau_vis: float = 0.0,
             eligible=None):
        """Pack FP16 tiles (uint16 [P,3,Ni+2,Ni+2] / [P,2,Nv+2,Nv+2]); only
        ``eligible`` probes (bool [P], None = all) may be sent.
        Returns (packet bytes, mask_irr, mask_vis)."""
        cur_irr = _c(cur_irr, np.uint16)
        cur_vis = _c(cur_vis, np.uint16)
        assert cur_irr.shape == (self.P, 3, self.Ni + 2, self.Ni + 2)
        assert cur_vis.shape == (self.P, 2, self.Nv + 2, self.Nv + 2)
        cap = packet_bytes(self.P, self.P, self.Ni, self.Nv)
        out = np.zeros(cap, np.uint8)
        mi = np.zeros(self.P, np.uint8)
        mv = np.zeros(self.P, np.uint8)
        n = lib().or_pack(self.P, self.Ni, self.Nv, _p(cur_irr, _U16), _p(cur_vis, _U16),
                          _p(self.ref_irr, _U16), _p(self.ref_vis, _U16), float(tau_irr), float(tau_vis),
                          self.client, self.seq, _p(out, _U8), cap, _p(mi, _U8), _p(mv, _U8),
                          None if eligible is None else _p(_c(eligible, np.uint8), _U8))
        assert n > 0
        self.seq += 1
        return out[:n].tobytes(), mi.astype(bool), mv.astype(bool)

    def reset(self):
        self.ref_irr[:] = 0
        self.ref_vis[:] = 0


class OracleClientDecoder:
    """The receiving client: FP16 tiles updated from packets."""

    def __init__(self, n_probes: int, irr_res: int = 8, vis_res: int = 16):
        self.P, self.Ni, self.Nv = n_probes, irr_res, vis_res
        self.irr = np.zeros((n_probes, 3, irr_res + 2, irr_res + 2), np.uint16)
        self.vis = np.zeros((n_probes, 2, vis_res + 2, vis_res + 2), np.uint16)
        self.seq = None

    def apply(self, packet: bytes) -> int:
        a = np.frombuffer(packet, np.uint8).copy()
        seq = ctypes.c_uint32(0)
        rc = lib().or_client_apply(_p(a, _U8), a.size, self.P, self.Ni, self.Nv, _p(self.irr, _U16),
                                   _p(self.vis, _U16), ctypes.byref(seq))
        if rc == 0:
            self.seq = seq.value
        return rc

    def reset(self):
        self.irr[:] = 0
        self.vis[:] = 0
        self.seq = None


def max_threads() -> int:
    return int(lib().or_max_threads())
