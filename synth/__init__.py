"""Seeded synthetic inputs for the probe-volume workloads.

This module only *generates data*: triangle scenes, point lights, per-frame
random rotations, light paths, moving occluders, volume descriptions and
random FP16 probe maps / ray records for stage-level tests. It holds none of
the method's arithmetic (no ray directions, intersection, shading, blending,
border copy or packing) and imports neither the GPU library nor the oracle,
so both sides can consume exactly the same inputs.

The paper's scenes (Tomb Buddha, Greek Villa, Night Street; scene-statistics
table in Section 4) are not available, so procedural box scenes with the
paper's grid shapes and 256 rays/probe (Section 4, latency discussion) stand
in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Scene", "VolumeConfig", "box_room", "box_city", "box_field",
    "emissive_box", "cube_shell", "empty_scene", "random_triangle_soup",
    "rotation", "light_path", "moving_occluders", "random_fp16_maps",
    "perturb_fp16_maps", "synthetic_rays", "CONFIGS", "config",
]


@dataclasses.dataclass
class Scene:
    positions: np.ndarray          # float32 [V, 3]
    indices: np.ndarray            # uint32  [T, 3]
    albedo: np.ndarray             # float32 [T, 3]
    emission: np.ndarray           # float32 [T, 3]
    lights: np.ndarray             # float32 [L, 6]  (position xyz, intensity rgb)
    n_dynamic: int = 0             # trailing triangles that move per frame
    dynamic_seed: int = 0

    @property
    def n_triangles(self) -> int:
        return int(self.indices.shape[0])

    def triangles(self) -> np.ndarray:
        """Per-triangle vertex positions, float32 [T, 3, 3] (pure gather)."""
        return self.positions[self.indices.astype(np.int64)]

    def with_dynamic(self, dyn_positions: Optional[np.ndarray]) -> "Scene":
        """Copy whose trailing dynamic triangles take ``dyn_positions``
        (float32 [n_dynamic, 3, 3]); the copy stores them as a flat soup."""
        if dyn_positions is None or self.n_dynamic == 0:
            return self
        tris = self.triangles().copy()
        tris[-self.n_dynamic:] = dyn_positions
        return soup_scene(tris, self.albedo, self.emission, self.lights,
                          n_dynamic=self.n_dynamic)


def soup_scene(tris, albedo, emission, lights, n_dynamic=0) -> Scene:
    tris = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 3, 3)
    t = tris.shape[0]
    return Scene(tris.reshape(-1, 3).copy(),
                 np.arange(3 * t, dtype=np.uint32).reshape(t, 3),
                 np.ascontiguousarray(albedo, np.float32).reshape(t, 3),
                 np.ascontiguousarray(emission, np.float32).reshape(t, 3),
                 np.ascontiguousarray(lights, np.float32).reshape(-1, 6),
                 n_dynamic=n_dynamic)


# --------------------------------------------------------------------------
# geometry helpers (data construction only)
# --------------------------------------------------------------------------
_BOX_FACES = (
    # each face as 4 corner ids into the 8 corners (bit0=x, bit1=y, bit2=z)
    (0, 2, 6, 4), (1, 5, 7, 3),    # -x, +x
    (0, 4, 5, 1), (2, 3, 7, 6),    # -y, +y
    (0, 1, 3, 2), (4, 6, 7, 5),    # -z, +z
)


def _box_triangles(lo, hi, inward: bool = False) -> np.ndarray:
    """12 triangles (2 per face) of an axis-aligned box, float64 [12,3,3].
    Wound so that (v1 - v0) x (v2 - v0) points out of the box (a solid), or
    into it with ``inward`` (a room whose inside is open space)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    corners = np.array([[hi[0] if (c & 1) else lo[0],
                         hi[1] if (c & 2) else lo[1],
                         hi[2] if (c & 4) else lo[2]] for c in range(8)])
    out = []
    for a, b, c, d in _BOX_FACES:
        if inward:
            out.append([corners[a], corners[b], corners[c]])
            out.append([corners[a], corners[c], corners[d]])
        else:
            out.append([corners[a], corners[c], corners[b]])
            out.append([corners[a], corners[d], corners[c]])
    return np.array(out)


def empty_scene(lights=None) -> Scene:
    lights = np.zeros((0, 6), np.float32) if lights is None else lights
    return Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.uint32),
                 np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                 np.asarray(lights, np.float32).reshape(-1, 6))


def box_room(seed: int = 1) -> Scene:
    """Closed room [-1,4]^3 plus a floating cube [1.25,1.75]^3: 12 axis-aligned
    quads = 24 triangles, per-quad albedo U(0.2,0.8)^3, one point light at
    (0.4, 3.6, 0.4) with intensity (20, 20, 20)."""
    rng = np.random.default_rng(seed)
    room = _box_triangles([-1, -1, -1], [4, 4, 4], inward=True)
    cube = _box_triangles([1.25, 1.25, 1.25], [1.75, 1.75, 1.75])
    tris = np.concatenate([room, cube])
    quad_alb = rng.uniform(0.2, 0.8, size=(12, 3))
    albedo = np.repeat(quad_alb, 2, axis=0)
    emission = np.zeros_like(albedo)
    lights = np.array([[0.4, 3.6, 0.4, 20.0, 20.0, 20.0]])
    return soup_scene(tris, albedo, emission, lights)


def emissive_box(half_width: float = 1.0, center=(0.0, 0.0, 0.0),
                 emission=(0.7, 0.4, 0.2)) -> Scene:
    """Closed box whose walls all emit the same radiance and reflect nothing."""
    c = np.asarray(center, np.float64)
    tris = _box_triangles(c - half_width, c + half_width, inward=True)
    e = np.tile(np.asarray(emission, np.float64), (12, 1))
    return soup_scene(tris, np.zeros((12, 3)), e, np.zeros((0, 6)))


def cube_shell(half_width: float, center=(0.0, 0.0, 0.0), albedo=0.5,
               lights=None) -> Scene:
    c = np.asarray(center, np.float64)
    tris = _box_triangles(c - half_width, c + half_width, inward=True)
    lights = np.zeros((0, 6)) if lights is None else lights
    return soup_scene(tris, np.full((12, 3), albedo), np.zeros((12, 3)), lights)


def random_triangle_soup(n_tris: int, seed: int, extent: float = 10.0,
                         size: float = 1.0) -> Scene:
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, extent, size=(n_tris, 1, 3))
    offs = rng.normal(0.0, size, size=(n_tris, 3, 3))
    tris = centers + offs
    alb = rng.uniform(0.2, 0.8, size=(n_tris, 3))
    return soup_scene(tris, alb, np.zeros_like(alb), np.zeros((0, 6)))


def box_city(n_tris: int = 50_000, seed_layout: int = 10,
             seed_heights: int = 11, extent: float = 64.0,
             light_intensity: float = 400.0) -> Scene:
    """Procedural city: one ground quad plus (n_tris-2)//12 boxes whose
    footprints are jittered on a regular grid of cells covering
    [0, extent]^2 (seed_layout) and whose heights are log-normal with
    median 3 and sigma 0.6 (seed_heights). Y is up."""
    n_boxes = (n_tris - 2) // 12
    rng = np.random.default_rng(seed_layout)
    hrng = np.random.default_rng(seed_heights)
    cells = int(math.ceil(math.sqrt(n_boxes)))
    cell = extent / cells
    chosen = rng.permutation(cells * cells)[:n_boxes]
    cx = (chosen % cells).astype(np.float64)
    cz = (chosen // cells).astype(np.float64)
    fx = rng.uniform(0.3, 0.9, n_boxes) * cell
    fz = rng.uniform(0.3, 0.9, n_boxes) * cell
    ox = rng.uniform(0.0, 1.0, n_boxes) * (cell - fx)
    oz = rng.uniform(0.0, 1.0, n_boxes) * (cell - fz)
    heights = np.exp(math.log(3.0) + 0.6 * hrng.standard_normal(n_boxes))
    x0 = cx * cell + ox
    z0 = cz * cell + oz
    # the ground faces up (+y)
    tris = [np.array([[[-1.0, 0.0, -1.0], [extent + 1, 0.0, extent + 1], [extent + 1, 0.0, -1.0]],
                      [[-1.0, 0.0, -1.0], [-1.0, 0.0, extent + 1], [extent + 1, 0.0, extent + 1]]])]
    # box bottoms sit just below the ground plane, so no face is coplanar
    # with the ground (no overlapping surfaces)
    for b in range(n_boxes):
        tris.append(_box_triangles([x0[b], -0.05, z0[b]],
                                   [x0[b] + fx[b], heights[b], z0[b] + fz[b]]))
    tris = np.concatenate(tris)
    t = tris.shape[0]
    arng = np.random.default_rng(seed_layout + 1000)
    box_alb = arng.uniform(0.2, 0.8, size=(n_boxes, 3))
    albedo = np.concatenate([np.full((2, 3), 0.5), np.repeat(box_alb, 12, axis=0)])
    emission = np.zeros((t, 3))
    lights = np.array([[extent * 0.5, 12.0, extent * 0.5,
                        light_intensity, light_intensity * 0.9, light_intensity * 0.8]])
    return soup_scene(tris, albedo, emission, lights)


def box_field(n_tris: int, seed: int, extent: float = 64.0,
              n_moving: int = 0, light_intensity: float = 400.0) -> Scene:
    """Box scene for the batched / encode / served workloads: a city-like
    field with ``n_tris`` static triangles, plus ``n_moving`` occluder boxes
    (12 triangles each) appended as dynamic triangles."""
    base = box_city(n_tris=n_tris, seed_layout=seed, seed_heights=seed + 1,
                    extent=extent, light_intensity=light_intensity)
    if n_moving == 0:
        return base
    dyn = moving_occluders(seed, 0, n_moving, extent)
    tris = np.concatenate([base.triangles(), dyn])
    alb = np.concatenate([base.albedo, np.full((12 * n_moving, 3), 0.6, np.float32)])
    emi = np.concatenate([base.emission, np.zeros((12 * n_moving, 3), np.float32)])
    sc = soup_scene(tris, alb, emi, base.lights, n_dynamic=12 * n_moving)
    sc.dynamic_seed = seed
    return sc


def moving_occluders(seed: int, frame: int, n_boxes: int = 4,
                     extent: float = 64.0) -> np.ndarray:
    """Triangles of ``n_boxes`` occluder boxes at ``frame`` on seeded
    sinusoidal paths, float32 [12*n_boxes, 3, 3]."""
    rng = np.random.default_rng([seed, 777])
    out = []
    for _ in range(n_boxes):
        c0 = rng.uniform(0.2 * extent, 0.8 * extent, 3)
        c0[1] = rng.uniform(4.0, 9.0)
        amp = rng.uniform(2.0, 6.0, 3)
        freq = rng.uniform(0.02, 0.08, 3)
        phase = rng.uniform(0.0, 2 * math.pi, 3)
        half = rng.uniform(0.8, 2.0, 3)
        c = c0 + amp * np.sin(2 * math.pi * freq * frame + phase)
        out.append(_box_triangles(c - half, c + half))
    return np.concatenate(out).astype(np.float32)


# --------------------------------------------------------------------------
# per-frame inputs
# --------------------------------------------------------------------------
def rotation(seed: int, frame: int) -> np.ndarray:
    """Uniform random rotation for (seed, frame) from a uniform random unit
    quaternion (Shoemake's subgroup method), as a row-major float32 3x3."""
    u1, u2, u3 = np.random.default_rng([seed, frame]).uniform(0.0, 1.0, 3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    m = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
    return m.astype(np.float32).reshape(9)


def light_path(seed: int, n_frames: int, extent: float = 64.0,
               n_ctrl: int = 8, y_range=(8.0, 14.0)) -> np.ndarray:
    """Light positions for ``n_frames`` frames along a closed Catmull-Rom
    spline through ``n_ctrl`` seeded control points, float32 [F, 3]."""
    rng = np.random.default_rng(seed)
    ctrl = np.stack([rng.uniform(0.15 * extent, 0.85 * extent, n_ctrl),
                     rng.uniform(y_range[0], y_range[1], n_ctrl),
                     rng.uniform(0.15 * extent, 0.85 * extent, n_ctrl)], axis=1)
    out = np.zeros((n_frames, 3))
    for f in range(n_frames):
        s = f / max(n_frames, 1) * n_ctrl
        i = int(s)
        u = s - i
        p0, p1, p2, p3 = (ctrl[(i - 1) % n_ctrl], ctrl[i % n_ctrl],
                          ctrl[(i + 1) % n_ctrl], ctrl[(i + 2) % n_ctrl])
        out[f] = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                        + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# stage-level synthetic data
# --------------------------------------------------------------------------
def random_fp16_maps(n_probes: int, irr_res: int, vis_res: int, seed: int,
                     scale: float = 4.0):
    """Random FP16 probe tiles as uint16 bit patterns:
    irradiance [P, 3, irr_res+2, irr_res+2], visibility [P, 2, vis_res+2, vis_res+2].
    Values are non-negative with a spread of exponents (including some
    denormals and exact zeros)."""
    rng = np.random.default_rng(seed)

    def draw(shape):
        mag = np.exp(rng.uniform(math.log(1e-6), math.log(scale), size=shape))
        mag[rng.uniform(size=shape) < 0.02] = 0.0
        return mag.astype(np.float16).view(np.uint16)

    irr = draw((n_probes, 3, irr_res + 2, irr_res + 2))
    vis = draw((n_probes, 2, vis_res + 2, vis_res + 2))
    return irr, vis


def perturb_fp16_maps(irr: np.ndarray, vis: np.ndarray, seed: int,
                      p_probe: float = 0.3, p_texel: float = 0.05,
                      rel: float = 2e-3):
    """Copy of FP16 tiles where a random subset of probes (p_probe) have a
    random subset of texels (p_texel) multiplied by (1 + U(-rel, rel)), with
    values re-rounded to FP16. Borders are perturbed too (they are not part
    of what is compared). Returns (irr, vis) uint16."""
    rng = np.random.default_rng(seed)
    out = []
    for m in (irr, vis):
        f = m.view(np.float16).astype(np.float64)
        probe_sel = rng.uniform(size=(m.shape[0], 1, 1, 1)) < p_probe
        tex_sel = rng.uniform(size=m.shape) < p_texel
        fac = 1.0 + rng.uniform(-rel, rel, size=m.shape)
        f = np.where(probe_sel & tex_sel, f * fac, f)
        out.append(f.astype(np.float16).view(np.uint16))
    return out[0], out[1]


def query_maps(cfg, seed: int, var_lo: float = 0.02):
    """Stored maps for shading-query tests: full tiles (guard texels drawn
    like the interior) with irradiance in [0, 2] per channel, visibility mean
    mu in [0.3, 3] and mean square mu^2 + var, var in [var_lo, 0.5]. Float64
    arrays holding values of the volume's storage format (binary16 values
    when cfg.fp16): irradiance [P, 3, 10, 10], visibility [P, 2, 18, 18]."""
    rng = np.random.default_rng(seed)
    P = cfg.n_probes
    si, sv = cfg.irr_res + 2, cfg.vis_res + 2
    irr = rng.uniform(0.0, 2.0, size=(P, 3, si, si))
    mu = rng.uniform(0.3, 3.0, size=(P, sv, sv))
    var = rng.uniform(var_lo, 0.5, size=mu.shape)
    vis = np.stack([mu, mu * mu + var], axis=1)
    dt = np.float16 if cfg.fp16 else np.float32
    return irr.astype(dt).astype(np.float64), vis.astype(dt).astype(np.float64)


def query_points(cfg, n_points: int, seed: int):
    """Query points and normals (float32 [m, 3] each): uniform over the probe
    grid's box grown by one spacing on every side (clamped cells), then every
    probe position; normals uniform on the sphere, then the six axis
    directions in turn (octahedral poles and fold lines)."""
    rng = np.random.default_rng(seed)
    o = np.asarray(cfg.origin, np.float64)
    s = np.asarray(cfg.spacing, np.float64)
    dims = np.array([cfg.nx, cfg.ny, cfg.nz])
    lo, hi = o - s, o + s * dims
    pts = rng.uniform(lo, hi, size=(n_points, 3))
    idx = np.arange(cfg.n_probes)
    grid = np.stack([idx % cfg.nx, (idx // cfg.nx) % cfg.ny, idx // (cfg.nx * cfg.ny)], axis=1)
    pts = np.concatenate([pts, o + s * grid])
    nrm = rng.normal(size=pts.shape)
    axes = np.concatenate([np.eye(3), -np.eye(3)])
    nrm[n_points:] = axes[np.arange(len(pts) - n_points) % 6]
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts.astype(np.float32), nrm.astype(np.float32)


def synthetic_rays(n_probes: int, n_rays: int, seed: int, max_distance: float = 4.0):
    """Random ray records for blend-only tests: radiance rgb >= 0 (float32
    [P, n, 3]) and distance in [0, max_distance] (float32 [P, n])."""
    rng = np.random.default_rng(seed)
    L = rng.gamma(2.0, 0.5, size=(n_probes, n_rays, 3)).astype(np.float32)
    r = rng.uniform(0.0, max_distance, size=(n_probes, n_rays)).astype(np.float32)
    r[rng.uniform(size=r.shape) < 0.1] = max_distance
    return L, r


# --------------------------------------------------------------------------
# volume descriptions of the workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class VolumeConfig:
    nx: int
    ny: int
    nz: int
    origin: tuple
    spacing: tuple
    rays_per_probe: int
    irr_res: int = 8
    vis_res: int = 16
    hysteresis: float = 0.97
    max_distance: float = 4.0
    vis_sharpness: int = 50
    fp16: bool = True
    sky: tuple = (0.0, 0.0, 0.0)
    first_frame_no_history: bool = True
    multi_bounce: bool = False
    classify: bool = False

    @property
    def n_probes(self) -> int:
        return self.nx * self.ny * self.nz


def _c1():
    return VolumeConfig(4, 4, 4, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 128,
                        max_distance=4.0, fp16=False)


def _c2():
    # 16 x 8 x 16 probes over the 64 x 64 city, y is up.
    return VolumeConfig(16, 8, 16, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), 256,
                        max_distance=6.0, fp16=True, sky=(0.10, 0.15, 0.25))


def _c4():
    return VolumeConfig(32, 16, 32, (1.0, 0.25, 1.0), (2.0, 1.0, 2.0), 256,
                        max_distance=3.0, fp16=True, sky=(0.10, 0.15, 0.25))


CONFIGS = {"box_room": _c1, "city": _c2, "encode": _c4}


def config(name: str) -> VolumeConfig:
    return CONFIGS[name]()


def served_clients(n_clients: int = 64, seed: int = 30) -> List[VolumeConfig]:
    """The served workload's clients: probes log-uniform in [512, 16384]
    (multiple of 256, grid 16 x P/256 x 16) and rays/probe uniform in
    {64, 128, 256}, over one shared 64 x 64 scene."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_clients):
        p = int(round(math.exp(rng.uniform(math.log(512), math.log(16384))) / 256)) * 256
        p = min(max(p, 512), 16384)
        n = int(rng.choice([64, 128, 256]))
        ny = p // 256
        out.append(VolumeConfig(16, ny, 16, (2.0, 0.25, 2.0), (4.0, 14.0 / max(ny - 1, 1), 4.0), n,
                                max_distance=6.0, fp16=True, sky=(0.10, 0.15, 0.25)))
    return out


def poisson_arrivals(rate_hz: float, duration_s: float, n_clients: int, seed: int = 30):
    """Arrival times (s) and uniformly chosen client ids of a Poisson
    request stream."""
    rng = np.random.default_rng([seed, 1])
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append((t, int(rng.integers(0, n_clients))))
    return out


def batched_volumes(n_volumes: int = 32, seed: int = 20) -> List[dict]:
    """The batched workload: per volume a probe count log-uniform in
    [256, 8192] (multiple of 256, grid 16 x P/256 x 16), rays/probe uniform in
    {64,128,256,512}, and its own box scene of log-uniform [5k, 100k]
    triangles (seed 21+v)."""
    rng = np.random.default_rng(seed)
    out = []
    for v in range(n_volumes):
        p = int(round(math.exp(rng.uniform(math.log(256), math.log(8192))) / 256)) * 256
        p = min(max(p, 256), 8192)
        n = int(rng.choice([64, 128, 256, 512]))
        t = int(math.exp(rng.uniform(math.log(5000), math.log(100000))))
        ny = p // 256
        cfg = VolumeConfig(16, ny, 16, (2.0, 0.25, 2.0), (4.0, 12.0 / max(ny, 1), 4.0), n,
                           max_distance=6.0, fp16=True, sky=(0.10, 0.15, 0.25))
        out.append({"config": cfg, "n_tris": t, "scene_seed": 21 + v})
    return out
