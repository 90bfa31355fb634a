"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test ties one oracle function to a closed form, a special case that
reduces to a known answer, brute force on tiny inputs, a library routine
(numpy), an invariant of the mathematics, or the paper's printed numbers.
Absolute radiance of shadowed scenes at scale is not pinned beyond these
small-scene cases ("parity unpinned" for that part; the GPU is compared with
the oracle, which is trusted through these pins).
"""
import json
import math
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.usefixtures("oracle_lib")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


# ---------------------------------------------------------------- binary16
def test_half_to_double_all_patterns_match_numpy(O):
    bits = np.arange(65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = np.array([O.half_to_double(int(b)) for b in bits])
    finite = np.isfinite(ref)
    assert np.array_equal(got[finite], ref[finite])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[np.isinf(ref)], ref[np.isinf(ref)])


def test_double_to_half_rounding_matches_numpy(O):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.uniform(-70000, 70000, 20000),
        np.exp(rng.uniform(-20, 11.5, 20000)) * rng.choice([-1, 1], 20000),
        np.ldexp(rng.integers(0, 4096, 5000).astype(np.float64), -26),   # subnormal region
        [0.0, -0.0, 65504.0, 65519.99, 65520.0, 1e9, 2.0 ** -25, 3 * 2.0 ** -26],
    ])
    # exact ties between binary16 neighbours
    h = rng.integers(0, 0x7bff, 5000).astype(np.uint16)
    a = h.view(np.float16).astype(np.float64)
    b = (h + 1).astype(np.uint16).view(np.float16).astype(np.float64)
    x = np.concatenate([x, (a + b) / 2])
    got = np.array([O.double_to_half(v) for v in x], dtype=np.uint16)
    with np.errstate(over="ignore"):   # values past 65520 round to infinity on purpose
        ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- octahedral
def test_octahedral_round_trip(O):
    rng = np.random.default_rng(1)
    v = rng.normal(size=(3000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for d in v:
        uw = O.oct_encode(d)
        assert np.all(np.abs(uw) <= 1.0 + 1e-15)
        assert np.allclose(O.oct_decode(*uw), d, atol=1e-12)
    for u, w in rng.uniform(-1, 1, size=(3000, 2)):
        assert np.allclose(O.oct_encode(O.oct_decode(u, w)), (u, w), atol=1e-12)


def test_octahedral_landmarks(O):
    assert np.allclose(O.oct_decode(0.0, 0.0), (0, 0, 1))
    for cu, cw in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        assert np.allclose(O.oct_decode(cu, cw), (0, 0, -1))
    # the diamond |u|+|w| = 1 is the equator
    for a in np.linspace(0, 1, 7):
        assert abs(O.oct_decode(a, 1 - a)[2]) < 1e-15
    # edge points (1, w) and (1, -w) are the same direction (the fold)
    for w in np.linspace(-1, 1, 9):
        assert np.allclose(O.oct_decode(1.0, w), O.oct_decode(1.0, -w), atol=1e-15)
        assert np.allclose(O.oct_decode(w, 1.0), O.oct_decode(-w, 1.0), atol=1e-15)


@pytest.mark.parametrize("N", [8, 16])
def test_texel_centres_round_trip_to_their_texel(O, N):
    dirs = O.texel_dirs(N)
    assert np.allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-14)
    for t, d in enumerate(dirs):
        u, w = O.oct_encode(d)
        i = int(math.floor((u + 1) * 0.5 * N))
        j = int(math.floor((w + 1) * 0.5 * N))
        assert j * N + i == t


# ---------------------------------------------------------------- ray directions
@pytest.mark.parametrize("n", [64, 128, 256, 1000])
def test_spherical_fibonacci_properties(O, n):
    I = np.eye(3, dtype=np.float32).reshape(9)
    d = O.ray_dirs(n, I)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    z = np.sort(d[:, 2])
    assert np.allclose(np.diff(z), 2.0 / n, atol=1e-12)          # equal-area bands
    assert np.allclose(z, -z[::-1], atol=1e-12)                   # symmetric about the equator
    phi = np.arctan2(d[:, 1], d[:, 0])
    golden_angle = 2 * math.pi * (2 - (1 + math.sqrt(5)) / 2)     # 137.5 degrees
    step = np.mod(phi[:-1] - phi[1:], 2 * math.pi)               # clockwise steps
    assert np.allclose(step, golden_angle, atol=1e-9)
    # near-uniform: first moment ~0, second moment ~I/3
    assert np.linalg.norm(d.mean(axis=0)) < 2.0 / n
    assert np.abs(d.T @ d / n - np.eye(3) / 3).max() < 4.0 / n


def test_ray_dirs_rotate_with_R(O):
    I = np.eye(3, dtype=np.float32).reshape(9)
    for f in range(5):
        R = synth.rotation(2, f)
        Rm = R.reshape(3, 3).astype(np.float64)
        assert abs(np.linalg.det(Rm) - 1) < 1e-6
        assert np.allclose(Rm @ Rm.T, np.eye(3), atol=1e-6)
        assert np.allclose(O.ray_dirs(128, R), O.ray_dirs(128, I) @ Rm.T, atol=1e-14)


# ---------------------------------------------------------------- intersection
@pytest.mark.parametrize("n_tris,seed", [(1, 0), (7, 1), (60, 2), (500, 3), (2000, 4)])
def test_bvh_matches_brute_force(O, n_tris, seed):
    sc = synth.random_triangle_soup(n_tris, seed, extent=10.0, size=1.5)
    osc = O.OracleScene.from_scene(sc)
    rng = np.random.default_rng(100 + seed)
    o = rng.uniform(-2, 12, size=(4000, 3))
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tb, tt, _ = osc.closest_hits(o, d)
    bb, bt = osc.closest_hits_brute(o, d)
    assert np.array_equal(tb, bb)
    hit = bb >= 0
    assert np.array_equal(tt[hit], bt[hit])
    if n_tris >= 60:
        assert hit.mean() > 0.05


def test_tie_flag_on_shared_edge(O):
    sc = synth.box_room()
    osc = O.OracleScene.from_scene(sc)
    # wall x = -1 is split along its diagonal from (-1,-1,-1) to (-1,4,4)
    o = np.array([[1.0, 0.5, 0.7]])
    target = np.array([-1.0, 1.3, 1.3])               # on that diagonal
    d = (target - o) / np.linalg.norm(target - o)
    _, _, near = osc.closest_hits(o, d, margin=1e-5)
    assert near[0] == 1
    target2 = np.array([-1.0, 0.2, 2.9])              # well inside one triangle
    d2 = (target2 - o) / np.linalg.norm(target2 - o)
    tri, t, near2 = osc.closest_hits(o, d2, margin=1e-5)
    assert near2[0] == 0 and tri[0] >= 0
    assert np.isclose(t[0], np.linalg.norm(target2 - o[0]), rtol=1e-12)


def test_ray_on_box_edge_accepts_both_faces(O):
    """A ray that runs into a box edge (to FP32 rounding of the box data) can
    hit either face that meets there, or graze past; the accepted set holds a
    triangle of each face (the reading of the closest-hit margin)."""
    cfg = synth.VolumeConfig(1, 1, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 64, max_distance=8.0, fp16=False)
    R = synth.rotation(5, 0)
    d = O.ray_dirs(64, R)
    found = 0
    for j in (0, 17, 40):
        dj = d[j]
        X = 2.0 * dj                                   # the ray meets the edge at t = 2
        # box whose edge along the axis of least |d| passes through X; the
        # ray comes from outside, towards the two faces that meet there
        ax = int(np.argmin(np.abs(dj)))
        a, b_ = [k for k in range(3) if k != ax]
        lo, hi = X.copy(), X.copy()
        for k in (a, b_):
            if dj[k] > 0:
                hi[k] = X[k] + 1.0                     # the ray enters through the face at X[k]
            else:
                lo[k] = X[k] - 1.0
        lo[ax], hi[ax] = X[ax] - 0.5, X[ax] + 0.5
        tris = synth._box_triangles(lo, hi).astype(np.float32)
        osc = O.OracleScene(tris, np.full((12, 3), 0.5, np.float32))
        rays = O.trace_shade(osc, cfg, R, np.zeros((0, 6), np.float32))
        cand = [c for c in rays["cand"][0, j][: rays["ncand"][0, j]] if c >= 0]
        # which face each candidate lies on: the axis its plane is normal to
        axes = set()
        for c in cand:
            t = tris[c].astype(np.float64)
            nrm = np.cross(t[1] - t[0], t[2] - t[0])
            axes.add(int(np.argmax(np.abs(nrm))))
        assert {a, b_} <= axes, (j, cand, axes)
        found += 1
    assert found == 3


# ---------------------------------------------------------------- trace + shade special cases
def _cfg(**kw):
    base = dict(nx=2, ny=2, nz=2, origin=(0.0, 0.0, 0.0), spacing=(0.5, 0.5, 0.5), rays_per_probe=256,
                max_distance=4.0, fp16=False)
    base.update(kw)
    return synth.VolumeConfig(**base)


def test_empty_scene_uniform_sky_gives_constant_maps(O):
    """Uniform radiance environment: irradiance equals the sky radiance and
    visibility equals (D_max, D_max^2) in every texel."""
    sky = (0.3, 0.6, 1.2)
    cfg = _cfg(sky=sky, max_distance=2.5)
    sc = O.OracleScene(np.zeros((0, 3, 3), np.float32), np.zeros((0, 3), np.float32))
    vol = O.OracleVolume(cfg)
    vol.update(sc, synth.rotation(5, 0), np.zeros((0, 6), np.float32))
    irr = vol.irr[:, :, 1:-1, 1:-1]
    skyf = np.array(sky, np.float32).astype(np.float64)
    for c in range(3):
        assert np.allclose(irr[:, c], skyf[c], rtol=1e-13)
    dm = float(np.float32(2.5))
    assert np.allclose(vol.vis[:, 0, 1:-1, 1:-1], dm, rtol=1e-13)
    assert np.allclose(vol.vis[:, 1, 1:-1, 1:-1], dm * dm, rtol=1e-13)


def test_closed_emissive_box_gives_its_emission(O):
    E = (0.7, 0.4, 0.2)
    sc = synth.emissive_box(half_width=3.0, center=(0.5, 0.5, 0.5), emission=E)
    cfg = _cfg(rays_per_probe=128)
    vol = O.OracleVolume(cfg)
    vol.update(O.OracleScene.from_scene(sc), synth.rotation(6, 0), sc.lights)
    Ef = np.array(E, np.float32).astype(np.float64)
    for c in range(3):
        assert np.allclose(vol.irr[:, c, 1:-1, 1:-1], Ef[c], rtol=1e-13)


def test_distance_in_centred_cube_closed_form(O):
    a = 1.25
    for dmax in (5.0, 1.5):
        sc = synth.cube_shell(a, center=(0.0, 0.0, 0.0))
        cfg = _cfg(nx=1, ny=1, nz=1, origin=(0.0, 0.0, 0.0), rays_per_probe=300, max_distance=dmax)
        R = synth.rotation(7, 1)
        rays = O.trace_shade(O.OracleScene.from_scene(sc), cfg, R, np.zeros((0, 6), np.float32))
        d = O.ray_dirs(300, R)
        expect = np.minimum(a / np.abs(d).max(axis=1), float(np.float32(dmax)))
        assert np.allclose(rays["r"][0], expect, rtol=1e-12)


def test_convex_room_direct_light_closed_form(O):
    """Room without occluder: each ray's radiance is rho/pi * I cos / d^2 at
    the wall point found by the slab method (no shadowing possible)."""
    room = synth.box_room()
    tris = room.triangles()[:12]                        # the 6 walls only
    alb = room.albedo[:12]
    light = np.array([[1.1, 2.9, 0.3, 15.0, 12.0, 9.0]], np.float32)
    osc = O.OracleScene(tris, alb)
    cfg = _cfg(nx=2, ny=2, nz=2, origin=(0.2, 0.3, 0.4), spacing=(1.7, 1.9, 2.1), rays_per_probe=128)
    R = synth.rotation(8, 0)
    rays = O.trace_shade(osc, cfg, R, light)
    d = O.ray_dirs(128, R)
    lo, hi = -1.0, 4.0
    Lp = light[0, :3].astype(np.float64)
    I = light[0, 3:].astype(np.float64)
    for p in range(8):
        x, y, z = p % 2, (p // 2) % 2, p // 4
        f = lambda v: float(np.float32(v))                 # the description is FP32 data
        o = np.array([f(0.2) + f(1.7) * x, f(0.3) + f(1.9) * y, f(0.4) + f(2.1) * z])
        for j in range(128):
            dj = d[j]
            ts = [((hi if dj[k] > 0 else lo) - o[k]) / dj[k] for k in range(3)]
            k = int(np.argmin(ts))
            t = ts[k]
            xh = o + t * dj
            nrm = np.zeros(3)
            nrm[k] = -np.sign(dj[k])
            face = 2 * k + (1 if dj[k] > 0 else 0)
            rho = alb[2 * face].astype(np.float64)
            lv = Lp - xh
            dist = np.linalg.norm(lv)
            cos = max(0.0, nrm @ lv / dist)
            expect = rho / math.pi * I * cos / dist ** 2
            assert np.allclose(rays["L"][p, j], expect, rtol=1e-9, atol=1e-12), (p, j)
            assert np.isclose(rays["r"][p, j], min(t, 4.0), rtol=1e-12)


def test_square_occluder_shadow_closed_form(O):
    """A floor, a floating two-sided square and a light above it: a floor
    point is lit exactly when its segment to the light misses the square
    (checked where that segment crosses the square's plane); points on the
    square's underside face away from the light; misses see the sky."""
    f32 = lambda v: np.float32(v)
    floor = np.array([[[-60, 0, -60], [60, 0, -60], [60, 0, 60]], [[-60, 0, -60], [60, 0, 60], [-60, 0, 60]]],
                     np.float32)
    a0, a1, hy = 0.0, 1.5, 2.0                               # square [a0,a1]^2 at height hy
    square = np.array([[[a0, hy, a0], [a1, hy, a0], [a1, hy, a1]], [[a0, hy, a0], [a1, hy, a1], [a0, hy, a1]]],
                      np.float32)
    tris = np.concatenate([floor, square])
    alb = np.array([[0.5, 0.6, 0.7]] * 2 + [[0.3, 0.3, 0.3]] * 2, np.float32)
    Lp = np.array([0.7, 6.0, 0.8])
    I = np.array([40.0, 30.0, 20.0])
    light = np.array([[*Lp, *I]], np.float32)
    sky = (0.05, 0.1, 0.2)
    cfg = _cfg(nx=3, ny=1, nz=3, origin=(-0.5, 1.0, -0.5), spacing=(1.0, 1.0, 1.0), rays_per_probe=256,
               max_distance=8.0, sky=sky)
    osc = O.OracleScene(tris, alb)
    R = synth.rotation(21, 0)
    rays = O.trace_shade(osc, cfg, R, light)
    d = O.ray_dirs(256, R)
    Lp64, I64 = Lp.astype(np.float32).astype(np.float64), I.astype(np.float32).astype(np.float64)
    n_lit = n_shadow = n_under = n_clean = 0
    for p in range(cfg.n_probes):
        x, z = p % 3, p // 3
        o = np.array([f32(-0.5) + f32(1.0) * x, f32(1.0), f32(-0.5) + f32(1.0) * z], np.float64)
        for j in range(256):
            dj = d[j]
            L = rays["L"][p, j]
            t_sq = (hy - o[1]) / dj[1] if dj[1] > 0 else np.inf
            if np.isfinite(t_sq):
                h = o + t_sq * dj
                if a0 < h[0] < a1 and a0 < h[2] < a1:
                    if min(h[0] - a0, a1 - h[0], h[2] - a0, a1 - h[2]) < 1e-6:
                        continue                              # grazing an edge: a tie
                    assert np.allclose(L, 0.0, atol=1e-15), (p, j)   # underside faces away from the light
                    n_under += 1
                    continue
            if dj[1] >= 0:
                assert np.allclose(L, sky, rtol=1e-12), (p, j)
                continue
            t = -o[1] / dj[1]
            xh = o + t * dj
            if max(abs(xh[0]), abs(xh[2])) > 60.0 - 1e-6:
                if max(abs(xh[0]), abs(xh[2])) > 60.0 + 1e-6:
                    assert np.allclose(L, sky, rtol=1e-12), (p, j)   # beyond the floor's edge
                continue
            lv = Lp64 - xh
            s = (hy - xh[1]) / lv[1]                          # where the segment to the light crosses y = hy
            c = xh + s * lv
            m = min(c[0] - a0, a1 - c[0], c[2] - a0, a1 - c[2])
            if abs(m) < 1e-6:
                continue                                      # shadow-ray edge tie
            dist = np.linalg.norm(lv)
            lit = rays["L"][p, j]
            expect = alb[0].astype(np.float64) / math.pi * I64 * (lv[1] / dist) / dist ** 2
            if m > 0:
                assert np.allclose(lit, 0.0, atol=1e-15), (p, j)
                n_shadow += 1
            else:
                assert np.allclose(lit, expect, rtol=1e-9), (p, j)
                n_lit += 1
            if abs(m) > 1e-3:
                # a shadow ray far from the square's edges decides alone: one
                # accepted answer, bounds equal to it
                assert rays["ncand"][p, j] == 1, (p, j)
                assert np.array_equal(rays["L_lo"][p, j], lit) and np.array_equal(rays["L_hi"][p, j], lit), (p, j)
                n_clean += 1
    assert n_lit > 100 and n_shadow > 20 and n_under > 20, (n_lit, n_shadow, n_under)
    assert n_clean > 100


def test_box_room_invariants_and_bounds(O):
    cfg = synth.config("box_room")
    sc = synth.box_room()
    vol = O.OracleVolume(cfg)
    rays = vol.update(O.OracleScene.from_scene(sc), synth.rotation(2, 0), sc.lights)
    dmax = float(np.float32(cfg.max_distance))
    m1 = vol.vis[:, 0, 1:-1, 1:-1]
    m2 = vol.vis[:, 1, 1:-1, 1:-1]
    assert np.all(m1 <= dmax * (1 + 1e-15)) and np.all(m1 > 0)
    assert np.all(m2 >= m1 * m1 * (1 - 1e-12))                    # Jensen
    assert np.all(vol.irr >= 0)
    assert np.all(rays["L_lo"] <= rays["L"] + 1e-15) and np.all(rays["L"] <= rays["L_hi"] + 1e-15)
    assert np.all(rays["r_lo"] <= rays["r"]) and np.all(rays["r"] <= rays["r_hi"])
    assert np.all(vol.irr_lo <= vol.irr + 1e-12) and np.all(vol.irr <= vol.irr_hi + 1e-12)
    # the floating cube casts shadows: some lit-side rays see occluded points
    assert (rays["L"] == 0).any() and (rays["L"] > 0).any()


def test_box_room_bounds_collapse_to_the_nominal_answer(O):
    """The box room has no ray within the tie margin of an edge and no
    shadow ray grazing the cube: every ray has one accepted answer and its
    radiance and distance bounds equal the nominal values, so the bound maps
    equal the nominal maps."""
    cfg = synth.config("box_room")
    sc = synth.box_room()
    vol = O.OracleVolume(cfg)
    rays = vol.update(O.OracleScene.from_scene(sc), synth.rotation(2, 0), sc.lights)
    assert (rays["ncand"] == 1).all()
    for k in ("L", "r"):
        assert np.array_equal(rays[k + "_lo"], rays[k]) and np.array_equal(rays[k + "_hi"], rays[k])
    assert np.array_equal(vol.irr_lo, vol.irr) and np.array_equal(vol.irr_hi, vol.irr)
    assert np.array_equal(vol.vis_lo, vol.vis) and np.array_equal(vol.vis_hi, vol.vis)
    assert (rays["L"] == 0).any()          # shadowed rays are among them


def test_tie_bounds_are_narrow_on_the_city(O):
    """How wide the accepted sets are on the city's first frame (524,288
    rays): a ray has more than one accepted answer only within the tie
    margin of an edge or of another surface, so few rays and few texels may
    differ from the nominal answer. Bounds about twice the measured values
    (ncand > 1: 1.2e-3 of rays; radiance bounds apart: 3.0e-4; distance
    bounds apart: 7.3e-4; irradiance texels wider than 1% of their value:
    1.8%, visibility 0.28%; each such ray reaches about half the texels of
    its probe's irradiance map). A shadow decision widened on every shadow
    ray, or a tie set that always holds more than the nominal hit, breaks
    them by orders of magnitude."""
    cfg = synth.config("city")
    sc = synth.box_city()
    lights = sc.lights.copy()
    lights[0, :3] = synth.light_path(12, 60)[0]
    vol = O.OracleVolume(cfg)
    rays = vol.update(O.OracleScene.from_scene(sc), synth.rotation(13, 0), lights)
    assert (rays["ncand"] > 1).mean() <= 2.5e-3
    assert np.any(rays["L_lo"] != rays["L_hi"], axis=-1).mean() <= 6e-4
    assert (rays["r_lo"] != rays["r_hi"]).mean() <= 1.5e-3
    for lo, hi, nom, frac, mean in ((vol.irr_lo, vol.irr_hi, vol.irr, 3.6e-2, 1.2e-2),
                                    (vol.vis_lo, vol.vis_hi, vol.vis, 6e-3, 1e-3)):
        rel = (hi - lo) / np.maximum(np.abs(nom), 1e-3 * np.abs(nom).max())
        assert (rel > 1e-2).mean() <= frac
        assert rel.mean() <= mean
    # the shadows are real: many rays are dark, many lit
    assert (rays["L"].max(axis=-1) < 1e-3).mean() > 0.05 and (rays["L"].max(axis=-1) > 0.05).mean() > 0.3


# ---------------------------------------------------------------- blend
def _blend_linear(O, n, s, a, c):
    """Blend ray radiance L_j = c + a.d_j (and distance r_j the same) with
    the oracle; compare with the exact integrals of the weighted means."""
    cfg = _cfg(nx=1, ny=1, nz=1, rays_per_probe=n, vis_sharpness=s, fp16=False)
    R = synth.rotation(9, 0)
    d = O.ray_dirs(n, R)
    val = c + d @ a
    L = np.repeat(val[None, :, None], 3, axis=2)
    r = val[None, :]
    irr, vis = O.empty_maps(cfg)
    O.blend_update(cfg, d, L, r, irr, vis, first=True)
    wi = O.texel_dirs(cfg.irr_res)
    wv = O.texel_dirs(cfg.vis_res)
    # cosine lobe: E[d] = (2/3) omega; cosine^s lobe: E[d] = (s+1)/(s+2) omega
    exp_irr = c + (2.0 / 3.0) * (wi @ a)
    exp_vis = c + (s + 1.0) / (s + 2.0) * (wv @ a)
    got_irr = irr[0, 0, 1:-1, 1:-1].reshape(-1)
    got_vis = vis[0, 0, 1:-1, 1:-1].reshape(-1)
    return np.abs(got_irr - exp_irr).max(), np.abs(got_vis - exp_vis).max()


def test_blend_weighted_means_match_lobe_integrals(O):
    a = np.array([0.3, -0.5, 0.8])
    e_irr, e_vis = _blend_linear(O, 8192, 50, a, 2.0)
    assert e_irr < 2e-3 and e_vis < 1e-2
    # a wrong exponent would move the visibility mean by >= 0.08 |a| here
    e_irr2, e_vis2 = _blend_linear(O, 8192, 2, a, 2.0)
    assert e_vis2 < 2e-3
    # convergence with n
    e_small, _ = _blend_linear(O, 256, 50, a, 2.0)
    assert e_irr < e_small


def test_single_ray_blend_is_that_ray_or_the_old_value(O):
    """One ray: every texel whose lobe holds the ray takes that ray's value
    exactly (the weighted mean of one sample); texels whose weight sum is
    at most the floor (1e-20) keep their old value."""
    cfg = _cfg(nx=1, ny=1, nz=1, rays_per_probe=1, fp16=False)
    R = synth.rotation(12, 3)
    d = O.ray_dirs(1, R)
    L = np.array([[[0.25, 0.5, 0.75]]])
    r = np.array([[1.5]])
    irr, vis = O.empty_maps(cfg)
    irr[:] = 9.0
    vis[:] = 9.0
    O.blend_update(cfg, d, L, r, irr, vis, first=True)
    ci = O.texel_dirs(8) @ d[0]
    cv = O.texel_dirs(16) @ d[0]
    gi = irr[0, :, 1:-1, 1:-1].reshape(3, -1)
    gv = vis[0, :, 1:-1, 1:-1].reshape(2, -1)
    for c in range(3):
        assert np.allclose(gi[c][ci > 1e-20], L[0, 0, c], rtol=1e-14)
        assert np.all(gi[c][ci <= 0] == 9.0)
    lobe = np.maximum(cv, 0) ** 50 > 1e-20
    assert lobe.any() and (~lobe).any()
    assert np.allclose(gv[0][lobe], 1.5, rtol=1e-14) and np.allclose(gv[1][lobe], 2.25, rtol=1e-14)
    assert np.all(gv[:, ~lobe] == 9.0)


def test_hysteresis_constant_estimate(O):
    """Constant estimate e from zero-initialised maps: map_k = e (1 - h^k)
    without the first-frame rule, and e from the first frame with it."""
    sky = (0.5, 1.0, 2.0)
    sc = O.OracleScene(np.zeros((0, 3, 3), np.float32), np.zeros((0, 3), np.float32))
    h = float(np.float32(0.97))
    skyf = np.array(sky, np.float32).astype(np.float64)
    for flag in (False, True):
        cfg = _cfg(sky=sky, first_frame_no_history=flag, rays_per_probe=64, hysteresis=0.97)
        vol = O.OracleVolume(cfg)
        for k in range(1, 6):
            vol.update(sc, synth.rotation(10, k), np.zeros((0, 6), np.float32))
            for c in range(3):
                expect = skyf[c] if flag else skyf[c] * (1 - h ** k)
                assert np.allclose(vol.irr[:, c, 1:-1, 1:-1], expect, rtol=1e-12)


def test_fp16_maps_are_binary16_values(O):
    cfg = synth.config("box_room")
    cfg.fp16 = True
    sc = synth.box_room()
    vol = O.OracleVolume(cfg)
    vol.update(O.OracleScene.from_scene(sc), synth.rotation(2, 0), sc.lights)
    for m in (vol.irr, vol.vis):
        assert np.array_equal(m, m.astype(np.float16).astype(np.float64))


# ---------------------------------------------------------------- border
def _bilinear(tile, N, u, w):
    """Bilinear lookup of a guard-banded tile at octahedral coords (u, w),
    as a texture unit would sample it."""
    # continuous tile coordinate: tile column c spans [c, c+1); interior
    # texel i sits in column i+1 with its centre at u = 2(i+1/2)/N - 1
    x = (u + 1) * 0.5 * N + 1.0
    y = (w + 1) * 0.5 * N + 1.0
    x0, y0 = int(math.floor(x - 0.5)), int(math.floor(y - 0.5))
    fx, fy = x - 0.5 - x0, y - 0.5 - y0
    v00, v10 = tile[y0, x0], tile[y0, x0 + 1]
    v01, v11 = tile[y0 + 1, x0], tile[y0 + 1, x0 + 1]
    return (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11)


@pytest.mark.parametrize("N", [8, 16])
def test_border_makes_bilinear_lookup_continuous_across_the_fold(O, N):
    rng = np.random.default_rng(N)
    tiles = np.zeros((3, 1, N + 2, N + 2))
    tiles[:, :, 1:-1, 1:-1] = rng.uniform(0, 1, size=(3, 1, N, N))
    tiles = O.border(tiles)
    for p in range(3):
        T = tiles[p, 0]
        for w in rng.uniform(-1, 1, 50):
            # (1, w) and (1, -w) are one direction; so are (w, 1) and (-w, 1)
            assert math.isclose(_bilinear(T, N, 1.0, w), _bilinear(T, N, 1.0, -w), abs_tol=1e-12)
            assert math.isclose(_bilinear(T, N, -1.0, w), _bilinear(T, N, -1.0, -w), abs_tol=1e-12)
            assert math.isclose(_bilinear(T, N, w, 1.0), _bilinear(T, N, -w, 1.0), abs_tol=1e-12)
            assert math.isclose(_bilinear(T, N, w, -1.0), _bilinear(T, N, -w, -1.0), abs_tol=1e-12)
        corners = [_bilinear(T, N, cu, cw) for cu in (-1.0, 1.0) for cw in (-1.0, 1.0)]
        assert np.allclose(corners, corners[0], atol=1e-12)
        # interior untouched
        assert np.array_equal(T[1:-1, 1:-1], tiles[p, 0, 1:-1, 1:-1])


# ---------------------------------------------------------------- probe query (second bounce)
def _random_tiles(O, rng, P, C, N, lo=0.0, hi=1.0):
    t = np.zeros((P, C, N + 2, N + 2))
    t[:, :, 1:-1, 1:-1] = rng.uniform(lo, hi, size=(P, C, N, N))
    return O.border(t)


@pytest.mark.parametrize("N", [8, 16])
def test_probe_lookup_at_texel_centres_returns_the_texel(O, N):
    """Looking up the direction of an interior texel's centre returns that
    texel exactly (the lookup's texel convention is the blend's)."""
    rng = np.random.default_rng(40 + N)
    tile = _random_tiles(O, rng, 1, 2, N)[0]
    dirs = O.texel_dirs(N)
    for t in rng.choice(N * N, 40, replace=False):
        j, i = divmod(int(t), N)
        got = O.probe_lookup(tile, dirs[t])
        assert np.allclose(got, tile[:, j + 1, i + 1], rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [8, 16])
def test_probe_lookup_continuous_across_the_fold(O, N):
    """Directions just either side of the lower hemisphere's fold lines
    (x = 0 or y = 0 with z < 0) land on opposite edges of the square; with
    the guard bands the bilinear lookups agree in the limit."""
    rng = np.random.default_rng(50 + N)
    tile = _random_tiles(O, rng, 1, 1, N)[0]
    eps = 1e-10
    for _ in range(60):
        a, zc = rng.uniform(-1, 1), -rng.uniform(0.05, 1.0)
        for d0, d1 in (((a, eps, zc), (a, -eps, zc)), ((eps, a, zc), (-eps, a, zc))):
            u = O.probe_lookup(tile, np.array(d0) / np.linalg.norm(d0))
            w = O.probe_lookup(tile, np.array(d1) / np.linalg.norm(d1))
            assert np.allclose(u, w, atol=1e-7)
    # the bottom pole (all four corners of the square) is one value
    poles = [O.probe_lookup(tile, np.array([sx * 1e-9, sy * 1e-9, -1.0])) for sx in (-1, 1) for sy in (-1, 1)]
    assert np.allclose(poles, poles[0], atol=1e-7)


def _query_cfg(nx, ny, nz, spacing=(1.0, 1.0, 1.0)):
    return _cfg(nx=nx, ny=ny, nz=nz, spacing=spacing, origin=(0.0, 0.0, 0.0))


def _const_maps(O, cfg, irr_vals, mean, var):
    """Maps with probe p's irradiance the constant RGB irr_vals[p] and its
    visibility moments (mean[p], mean[p]^2 + var[p]) in every texel."""
    irr, vis = O.empty_maps(cfg)
    for p in range(cfg.n_probes):
        irr[p] = np.asarray(irr_vals[p], np.float64)[:, None, None]
        vis[p, 0] = mean[p]
        vis[p, 1] = mean[p] ** 2 + var[p]
    return irr, vis


def test_probe_query_at_a_probe_is_that_probes_lookup(O):
    """At a probe's own position the trilinear weight is 1 for that probe
    (grid indexing p = x + nx (y + ny z), including the last plane of each
    axis), so the query is its lookup in the normal's direction."""
    cfg = _query_cfg(3, 2, 4, spacing=(0.5, 1.25, 0.75))
    rng = np.random.default_rng(7)
    irr = _random_tiles(O, rng, cfg.n_probes, 3, cfg.irr_res, 0.1, 2.0)
    vis = np.zeros((cfg.n_probes, 2, cfg.vis_res + 2, cfg.vis_res + 2))
    for p in range(cfg.n_probes):
        x, y, z = p % 3, (p // 3) % 2, p // 6
        pos = np.array([0.5 * x, 1.25 * y, 0.75 * z])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        got = O.probe_query(cfg, irr, vis, pos, n)
        assert np.allclose(got, O.probe_lookup(irr[p], n), rtol=1e-12, atol=0)


def test_probe_query_trilinear_without_occlusion(O):
    """Probes whose recorded distances lie beyond the point: weights are the
    trilinear ones, so the query of per-probe constants is their trilinear
    interpolation (exact fractions chosen so the weights are known)."""
    cfg = _query_cfg(2, 2, 2)
    vals = [(float(p), 2.0 * p, 1.0) for p in range(8)]
    irr, vis = _const_maps(O, cfg, vals, [100.0] * 8, [1.0] * 8)
    fx, fy, fz = 0.25, 0.5, 0.75
    want = np.zeros(3)
    for p in range(8):
        bx, by, bz = p & 1, (p >> 1) & 1, p >> 2
        w = (fx if bx else 1 - fx) * (fy if by else 1 - fy) * (fz if bz else 1 - fz)
        want += w * np.array(vals[p])
    got = O.probe_query(cfg, irr, vis, np.array([fx, fy, fz]), np.array([0.0, 0.0, 1.0]))
    assert np.allclose(got, want, rtol=1e-12)
    # outside the grid the edge cell is used with its weights clamped
    got = O.probe_query(cfg, irr, vis, np.array([-3.0, 0.5, 9.0]), np.array([0.0, 1.0, 0.0]))
    assert np.allclose(got, 0.5 * (np.array(vals[4]) + np.array(vals[6])), rtol=1e-12)


@pytest.mark.parametrize("var, want", [(0.09, 3.0), (0.0, 4.0), (0.01, (0.5 * 0.1 * 1 + 0.5 * 4) / (0.5 * 0.1 + 0.5))])
def test_probe_query_chebyshev_weight(O, var, want):
    """Two probes 1 apart, the point halfway. Probe A recorded mean distance
    0.2 towards it (occluder nearer than the point, 0.3 short), probe B 10.
    A's weight is 1/2 * var / (var + 0.3^2): with var = 0.09 that is 1/4 and
    the query (1/4 * 1 + 1/2 * 4) / (3/4) = 3; with var = 0 A is excluded."""
    cfg = _query_cfg(2, 1, 1)
    irr, vis = _const_maps(O, cfg, [(1.0, 1.0, 1.0), (4.0, 4.0, 4.0)], [0.2, 10.0], [var, 1.0])
    got = O.probe_query(cfg, irr, vis, np.array([0.5, 0.0, 0.0]), np.array([0.0, 0.0, 1.0]))
    assert np.allclose(got, want, rtol=1e-12)


def test_probe_query_of_empty_maps_is_zero(O):
    cfg = _query_cfg(2, 2, 2)
    irr, vis = O.empty_maps(cfg)
    assert np.array_equal(O.probe_query(cfg, irr, vis, np.array([0.3, 0.4, 0.5]), np.array([1.0, 0, 0])),
                          np.zeros(3))


@pytest.mark.parametrize("h", [0.0, 0.6])
def test_second_bounce_in_closed_box_closed_form(O, h):
    """Closed box, every wall emitting E with albedo rho, no lights. Frame 0
    reads empty maps, so the map is E. From then on every hit adds rho times
    the (uniform) stored radiance: m_k = h m_(k-1) + (1 - h)(E + rho m_(k-1)),
    the geometric series E (1 + rho + ... + rho^k) when h = 0, converging to
    E / (1 - rho)."""
    E = np.array([0.7, 0.4, 0.2])
    rho = np.array([0.5, 0.25, 0.8])
    tris = synth._box_triangles(np.array([-1.5, -1.0, -1.25]), np.array([2.0, 1.75, 1.5]))
    sc = O.OracleScene(tris.astype(np.float32), np.tile(rho, (12, 1)).astype(np.float32),
                       np.tile(E, (12, 1)).astype(np.float32))
    cfg = _cfg(nx=3, ny=2, nz=2, spacing=(0.5, 0.75, 0.6), origin=(-0.4, -0.3, -0.2), rays_per_probe=128,
               hysteresis=h, multi_bounce=True)
    vol = O.OracleVolume(cfg)
    Ef = E.astype(np.float32).astype(np.float64)
    rf = rho.astype(np.float32).astype(np.float64)
    hf = float(np.float32(h))
    m = Ef.copy()
    for k in range(5):
        vol.update(sc, synth.rotation(8, k), np.zeros((0, 6), np.float32))
        if k > 0:
            m = hf * m + (1 - hf) * (Ef + rf * m)
        for c in range(3):
            assert np.allclose(vol.irr[:, c, 1:-1, 1:-1], m[c], rtol=1e-12), (k, c)
    if h == 0.0:
        assert np.allclose(m, Ef * (1 - rf ** 5) / (1 - rf), rtol=1e-12)


def test_second_bounce_off_leaves_the_update_unchanged(O):
    """Without the flag the maps do not depend on the stored ones: a box
    whose walls reflect gives the emission alone every frame."""
    E = np.array([0.3, 0.6, 0.9])
    tris = synth._box_triangles(np.array([-2.0, -2.0, -2.0]), np.array([2.0, 2.0, 2.0]))
    sc = O.OracleScene(tris.astype(np.float32), np.full((12, 3), 0.5, np.float32),
                       np.tile(E, (12, 1)).astype(np.float32))
    cfg = _cfg(rays_per_probe=64, hysteresis=0.0)
    vol = O.OracleVolume(cfg)
    for k in range(3):
        vol.update(sc, synth.rotation(9, k), np.zeros((0, 6), np.float32))
        for c in range(3):
            assert np.allclose(vol.irr[:, c, 1:-1, 1:-1], np.float32(E[c]), rtol=1e-12)


# ---------------------------------------------------------------- packing
def _np_masks(cur_irr, cur_vis, ref_irr, ref_vis, tau_irr, tau_vis):
    ci = cur_irr[:, :, 1:-1, 1:-1].reshape(cur_irr.shape[0], 3, -1)
    cv = cur_vis[:, :, 1:-1, 1:-1].reshape(cur_vis.shape[0], 2, -1)

    def changed(c, r, tau):
        if tau == 0:
            return (c != r).any(axis=(1, 2))
        diff = np.abs(c.view(np.float16).astype(np.float64) - r.view(np.float16).astype(np.float64))
        return (diff > tau).any(axis=(1, 2))
    return changed(ci, ref_irr, tau_irr), changed(cv, ref_vis, tau_vis)


def _parse(pkt, Ni=8, Nv=16):
    hdr = np.frombuffer(pkt[:32], np.uint32)
    magic, _, client, seq, P, Ki, Kv, chk = hdr
    idx = np.frombuffer(pkt[32:32 + 2 * (Ki + Kv)], np.uint16)
    off = 32 + ((2 * (Ki + Kv) + 15) // 16) * 16
    pi = np.frombuffer(pkt[off:off + Ki * 6 * Ni * Ni], np.uint8).reshape(6, Ki, Ni * Ni)
    off += Ki * 6 * Ni * Ni
    pv = np.frombuffer(pkt[off:off + Kv * 4 * Nv * Nv], np.uint8).reshape(4, Kv, Nv * Nv)
    assert off + Kv * 4 * Nv * Nv == len(pkt)
    return dict(magic=magic, client=client, seq=seq, P=P, Ki=Ki, Kv=Kv, chk=chk,
                idx_irr=np.cumsum(idx[:Ki].astype(np.int64)), idx_vis=np.cumsum(idx[Ki:].astype(np.int64)),
                planes_irr=pi, planes_vis=pv)


@pytest.mark.parametrize("tau", [0.0, 1.0 / 1024])
def test_pack_matches_numpy_definition(O, tau):
    P = 300
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=3)
    ref_i0, ref_v0 = synth.perturb_fp16_maps(cur_i, cur_v, seed=4, p_probe=0.4, p_texel=0.02, rel=2e-3)
    st = O.OracleClientState(P)
    st.ref_irr[:] = ref_i0[:, :, 1:-1, 1:-1].reshape(P, 3, -1)
    st.ref_vis[:] = ref_v0[:, :, 1:-1, 1:-1].reshape(P, 2, -1)
    ref_i, ref_v = st.ref_irr.copy(), st.ref_vis.copy()
    pkt, mi, mv = st.pack(cur_i, cur_v, tau, tau)
    ei, ev = _np_masks(cur_i, cur_v, ref_i, ref_v, tau, tau)
    assert np.array_equal(mi, ei) and np.array_equal(mv, ev)
    assert 0 < ei.sum() < P and 0 < ev.sum() < P
    d = _parse(pkt)
    assert d["magic"] == 0x4B505650 and d["P"] == P and d["Ki"] == ei.sum() and d["Kv"] == ev.sum()
    assert np.array_equal(d["idx_irr"], np.nonzero(ei)[0]) and np.array_equal(d["idx_vis"], np.nonzero(ev)[0])
    ci = cur_i[:, :, 1:-1, 1:-1].reshape(P, 3, -1)
    cv = cur_v[:, :, 1:-1, 1:-1].reshape(P, 2, -1)
    xi = (ci[ei] ^ ref_i[ei])                 # [Ki, 3, 64]
    xv = (cv[ev] ^ ref_v[ev])
    for c in range(3):
        assert np.array_equal(d["planes_irr"][2 * c], (xi[:, c] & 0xff).astype(np.uint8))
        assert np.array_equal(d["planes_irr"][2 * c + 1], (xi[:, c] >> 8).astype(np.uint8))
    for c in range(2):
        assert np.array_equal(d["planes_vis"][2 * c], (xv[:, c] & 0xff).astype(np.uint8))
        assert np.array_equal(d["planes_vis"][2 * c + 1], (xv[:, c] >> 8).astype(np.uint8))
    # reference: sent probes take the current interior, others keep theirs
    assert np.array_equal(st.ref_irr[ei], ci[ei]) and np.array_equal(st.ref_irr[~ei], ref_i[~ei])
    assert np.array_equal(st.ref_vis[ev], cv[ev]) and np.array_equal(st.ref_vis[~ev], ref_v[~ev])


def test_threshold_compare_exhaustive_pairs(O):
    """The tau > 0 decision equals the exact real comparison |a - b| > tau for
    every finite binary16 a against sampled b (one probe per pair)."""
    rng = np.random.default_rng(11)
    a_bits = np.arange(0, 0x7c00, dtype=np.uint16)                # all finite non-negative
    a_bits = np.concatenate([a_bits, a_bits | 0x8000])
    tau = 1.0 / 1024
    fa = a_bits.view(np.float16).astype(np.float64)
    # partners: exactly at +-tau, one ulp around it, and random nearby values
    cand = np.stack([fa + tau, fa - tau, fa + rng.uniform(-3, 3, fa.size) * tau,
                     fa * (1 + rng.uniform(-1e-3, 1e-3, fa.size))], axis=1)
    b_bits = cand[np.arange(fa.size), rng.integers(0, 4, fa.size)].astype(np.float16).view(np.uint16)
    B = 4096
    for s in range(0, a_bits.size, B):
        a = a_bits[s:s + B]
        b = b_bits[s:s + B]
        P = a.size
        cur_i = np.zeros((P, 3, 10, 10), np.uint16)
        cur_v = np.zeros((P, 2, 18, 18), np.uint16)
        cur_i[:, 1, 4, 6] = a
        st = O.OracleClientState(P)
        st.ref_irr[:, 1, 3 * 8 + 5] = b
        _, mi, mv = st.pack(cur_i, cur_v, tau, tau)
        exact = np.abs(a.view(np.float16).astype(np.float64) - b.view(np.float16).astype(np.float64)) > tau
        assert np.array_equal(mi, exact)
        assert not mv.any()


def test_pack_round_trip_replay_and_checksum(O):
    """120-frame replay: after every packet the client's interiors equal the
    server's last-transmitted state, and with tau = 0 also the current maps;
    guard bands are rebuilt from the interiors. A corrupted packet is refused."""
    P = 64
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=20)
    st0 = O.OracleClientState(P)
    st1 = O.OracleClientState(P)
    cl0 = O.OracleClientDecoder(P)
    cl1 = O.OracleClientDecoder(P)
    for f in range(120):
        cur_i, cur_v = synth.perturb_fp16_maps(cur_i, cur_v, seed=1000 + f, p_probe=0.2, p_texel=0.1, rel=4e-3)
        for st, cl, tau in ((st0, cl0, 0.0), (st1, cl1, 1.0 / 1024)):
            pkt, _, _ = st.pack(cur_i, cur_v, tau, tau)
            assert cl.apply(pkt) == 0 and cl.seq == st.seq - 1
            assert np.array_equal(cl.irr[:, :, 1:-1, 1:-1].reshape(P, 3, -1), st.ref_irr)
            assert np.array_equal(cl.vis[:, :, 1:-1, 1:-1].reshape(P, 2, -1), st.ref_vis)
        assert np.array_equal(cl0.irr[:, :, 1:-1, 1:-1], cur_i[:, :, 1:-1, 1:-1])
        assert np.array_equal(cl0.vis[:, :, 1:-1, 1:-1], cur_v[:, :, 1:-1, 1:-1])
    # guard bands of the client tiles equal the fold copy of their interiors
    b = O.border(cl0.irr.view(np.float16).astype(np.float64)).astype(np.float16).view(np.uint16)
    assert np.array_equal(b, cl0.irr)
    # XOR is an involution: applying the same packet twice restores the state
    cur_i2, cur_v2 = synth.perturb_fp16_maps(cur_i, cur_v, seed=5, p_probe=0.5, p_texel=0.5)
    pkt, _, _ = st0.pack(cur_i2, cur_v2)
    before = cl0.irr.copy()
    assert cl0.apply(pkt) == 0
    assert cl0.apply(pkt) == 0
    assert np.array_equal(cl0.irr[:, :, 1:-1, 1:-1], before[:, :, 1:-1, 1:-1])
    bad = bytearray(pkt)
    bad[-5] ^= 0x10
    assert cl0.apply(bytes(bad)) == -2


def test_unchanged_state_sends_empty_packet(O):
    P = 40
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=7)
    st = O.OracleClientState(P)
    pkt, mi, mv = st.pack(cur_i, cur_v)
    assert mi.all() and mv.all() and len(pkt) == O.packet_bytes(P, P)
    pkt2, mi2, mv2 = st.pack(cur_i, cur_v)
    assert not mi2.any() and not mv2.any() and len(pkt2) == 32
    # -0 versus +0: bit patterns differ (tau = 0) but values are equal (tau > 0)
    z_i = cur_i.copy()
    z_i[3, 0, 1, 1] = 0x8000
    st.ref_irr[3, 0, 0] = 0x0000
    _, mi3, _ = st.pack(z_i, cur_v, 1.0 / 1024, 1.0 / 1024)
    assert not mi3[3]
    st.ref_irr[3, 0, 0] = 0x0000
    _, mi4, _ = st.pack(z_i, cur_v, 0.0, 0.0)
    assert mi4[3]


# ---------------------------------------------------------------- the paper's sizes
def _r(x, nd=0):
    """Round half away from zero, as printed numbers are rounded."""
    return math.floor(x * 10 ** nd + 0.5) / 10 ** nd


def test_paper_worked_sizes():
    g = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))
    ni, nv, b = g["irr_texels_per_probe_side"]["value"], g["vis_texels_per_probe_side"]["value"], g["bits_per_texel"]["value"]
    kb = 1024.0
    irr_kb = ni * ni * b / kb
    vis_kb = nv * nv * b / kb
    assert irr_kb == g["irr_kb_per_probe"]["value"]
    assert vis_kb == g["vis_kb_per_probe"]["value"]
    assert 2048 * irr_kb / 1024 == g["irr_Mb_2048"]["value"]
    assert _r(2048 * ni * ni * b / 8 / 2 ** 20, 2) == g["irr_MB_2048"]["value"]
    assert 10 * 2048 * irr_kb / 1024 == g["irr_Mbps_2048_10Hz"]["value"]
    assert _r(vis_kb / irr_kb, 2) == g["vis_over_irr_ratio"]["value"]
    assert _r(2048 * vis_kb / 1024, 1) == g["vis_Mb_2048"]["value"]
    assert _r(2048 * nv * nv * b / 8 / 2 ** 20, 1) == g["vis_MB_2048"]["value"]
    assert 10 * 2048 * vis_kb / 1024 == g["vis_Mbps_2048_10Hz"]["value"]
    assert _r(10 * 2048 * (irr_kb + vis_kb) / 1024) == g["total_Mbps_2048_10Hz"]["value"]
    for P, mb in zip(g["uncompressed_color_MB"]["probes"], g["uncompressed_color_MB"]["value"]):
        assert _r(P * ni * ni * b / 8 / 2 ** 20, 2) == mb
    for P, mb in zip(g["uncompressed_vis_MB"]["probes"], g["uncompressed_vis_MB"]["value"]):
        assert _r(P * nv * nv * b / 8 / 2 ** 20, 2) == mb
    # guard-band removal: the interiors (8x8, 16x16) are what the packet carries
    assert _r(100 * (1 - 8 * 8 / (ni * ni))) == g["guard_band_drop_irr_pct"]["value"]
    assert _r(100 * (1 - 16 * 16 / (nv * nv))) == g["guard_band_drop_vis_pct"]["value"]


def test_packet_sizes_follow_the_layout(O):
    g = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))
    ib = g["index_bytes_per_probe"]["value"]
    for Ki, Kv in ((0, 0), (1, 0), (0, 1), (7, 3), (2048, 2048)):
        idx = ((ib * (Ki + Kv) + 15) // 16) * 16
        assert O.packet_bytes(Ki, Kv) == 32 + idx + Ki * 8 * 8 * 3 * 2 + Kv * 16 * 16 * 2 * 2


# ---------------------------------------------------------------- codec surfaces (Sec. 3.3)
def test_visibility_interleave_is_yuvy_uvyu_vyuv(O):
    """Three RG16F texels (12 bytes) fill four YUV samples in the order the
    paper gives: YUVY, UVYU, VYUV; a 16-texel row (64 bytes) needs
    ceil(4 * 16 / 3) = 22 samples, the last holding one byte."""
    P, C = 1, 1
    vis = np.zeros((P, 2, 18, 18), np.uint16)
    b = np.arange(1, 65, dtype=np.uint16)           # bytes 1..64 of the first row, in texel order
    for i in range(16):
        vis[0, 0, 1, i + 1] = b[4 * i] | (b[4 * i + 1] << 8)       # mean: lo, hi
        vis[0, 1, 1, i + 1] = b[4 * i + 2] | (b[4 * i + 3] << 8)   # mean^2: lo, hi
    irr = np.zeros((P, 3, 10, 10))
    ip, vp = O.yuv_encode(irr, vis, 1.0, C)
    assert O.yuv_dims(P, C) == (8, 8, 22, 16) and vp.shape == (3, 16, 22)
    Y, U, V = vp[0, 0], vp[1, 0], vp[2, 0]
    # texel 0 -> Y0 U0 V0 Y1, texel 1 -> U1 V1 Y2 U2, texel 2 -> V2 Y3 U3 V3
    assert [Y[0], U[0], V[0], Y[1]] == [1, 2, 3, 4]
    assert [U[1], V[1], Y[2], U[2]] == [5, 6, 7, 8]
    assert [V[2], Y[3], U[3], V[3]] == [9, 10, 11, 12]
    assert (Y[21], U[21], V[21]) == (64, 0, 0)
    assert not vp[:, 1:].any()                       # the other rows of the first probe are zero here


def test_irradiance_code_examples(O):
    """10-bit codes of normalised values, shifted into the top of 16 bits:
    ties go to even, values clamp to [0, 1023]."""
    assert O.irr_code(0.5, 1.0) == 512                # 511.5 -> 512
    assert O.irr_code(0.25, 1.0) == 256               # 255.75
    assert O.irr_code(510.5, 1023.0) == 510           # k = 1: an exact tie, to even
    assert O.irr_code(511.5, 1023.0) == 512
    assert O.irr_code(2.0, 1.0) == 1023 and O.irr_code(-1.0, 1.0) == 0 and O.irr_code(0.0, 1.0) == 0
    irr = np.zeros((1, 3, 10, 10))
    irr[0, 0, 1, 1], irr[0, 1, 1, 1], irr[0, 2, 1, 1] = 1.0, 0.5, 0.0
    ip, _ = O.yuv_encode(irr, np.zeros((1, 2, 18, 18), np.uint16), 1.0, 1)
    assert (ip[0, 0, 0], ip[1, 0, 0], ip[2, 0, 0]) == (0xFFC0, 512 << 6, 0)


@pytest.mark.parametrize("P, C", [(1, 1), (7, 3), (48, 16), (100, 7)])
def test_codec_surfaces_layout_and_round_trip(O, P, C):
    """Probe p sits in atlas tile (p % C, p / C); decoding the surfaces gives
    back every visibility bit pattern and the A2RGB10 codes of every texel."""
    rng = np.random.default_rng(P * 31 + C)
    irr16, vis = synth.random_fp16_maps(P, 8, 16, seed=P + C, scale=3.0)
    irr = irr16.view(np.float16).astype(np.float64)
    scale = 2.5
    ip, vp = O.yuv_encode(irr, vis, scale, C)
    W, H, Wv, Hv = O.yuv_dims(P, C)
    assert (W, H) == (8 * C, 8 * -(-P // C)) and (Wv, Hv) == (-(-64 * C // 3), 16 * -(-P // C))
    assert not (ip & 0x3F).any()                      # low 6 bits of every sample are zero
    codes, vback = O.yuv_decode(ip, vp, P, C)
    assert np.array_equal(vback, vis[:, :, 1:-1, 1:-1].reshape(P, 2, 256))
    k = np.float32(1023.0 / scale)
    want = np.clip(np.rint(irr[:, :, 1:-1, 1:-1].astype(np.float32) * k), 0, 1023).astype(np.uint32)
    want = want.reshape(P, 3, 64)
    assert np.array_equal(codes, want[:, 0] | (want[:, 1] << 10) | (want[:, 2] << 20))
    p = int(rng.integers(P))
    tx, ty = p % C, p // C
    assert np.array_equal(ip[1, ty * 8:(ty + 1) * 8, tx * 8:(tx + 1) * 8] >> 6, want[p, 1].reshape(8, 8))
    # tiles past the last probe are zero
    if P % C:
        assert not ip[:, -8:, (P % C) * 8:].any()


# ---------------------------------------------------------------- probe selection (Sec. 3.4)
def test_pack_sends_only_eligible_probes(O):
    """With an eligibility mask (active probes in the client's view) the sent
    set is changed AND eligible; ineligible probes keep their reference."""
    P = 200
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=13)
    st = O.OracleClientState(P)
    elig = np.random.default_rng(5).uniform(size=P) < 0.6
    pkt, mi, mv = st.pack(cur_i, cur_v, eligible=elig)
    full_i, full_v = _np_masks(cur_i, cur_v, np.zeros((P, 3, 64), np.uint16), np.zeros((P, 2, 256), np.uint16), 0, 0)
    assert np.array_equal(mi, full_i & elig) and np.array_equal(mv, full_v & elig)
    d = _parse(pkt)
    assert np.array_equal(d["idx_irr"], np.nonzero(full_i & elig)[0])
    assert not st.ref_irr[~elig].any() and not st.ref_vis[~elig].any()
    # the same probes become sendable once eligible
    pkt2, mi2, _ = st.pack(cur_i, cur_v)
    assert np.array_equal(mi2, full_i & ~elig)


def _solid_box_scene(O):
    tris = synth._box_triangles([-0.5, -0.5, -0.5], [0.5, 0.5, 0.5]).astype(np.float32)   # outward: a solid
    return O.OracleScene(tris, np.full((12, 3), 0.5, np.float32))


def test_activity_inside_near_and_far(O):
    """Probes 1 apart on a line from the centre of a solid unit box: inside
    it (every ray hits a face from behind) inactive; at 1 and 2 (the face
    within the cell diagonal sqrt 3) active; at 3 (nothing within sqrt 3)
    inactive."""
    cfg = _cfg(nx=4, ny=1, nz=1, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), rays_per_probe=256)
    sc = _solid_box_scene(O)
    R = synth.rotation(3, 0)
    rays = O.trace_shade(sc, cfg, R, np.zeros((0, 6), np.float32))
    nom, lo, hi = O.probe_activity(sc, cfg, R, rays)
    assert nom.tolist() == [False, True, True, False]
    assert np.array_equal(lo, nom) and np.array_equal(hi, nom)


def test_activity_below_a_ground_plane(O):
    """Half the rays of a probe below an upward-facing ground hit it from
    behind (> 1/4): inactive; above it: active."""
    ground = synth.box_city(n_tris=14).triangles()[:2].astype(np.float32)
    sc = O.OracleScene(ground, np.full((2, 3), 0.5, np.float32))
    cfg = _cfg(nx=2, ny=2, nz=1, spacing=(1.0, 1.0, 1.0), origin=(10.0, -0.5, 10.0), rays_per_probe=256)
    R = synth.rotation(3, 0)
    nom, lo, hi = O.probe_activity(sc, cfg, R, O.trace_shade(sc, cfg, R, np.zeros((0, 6), np.float32)))
    assert nom.tolist() == [False, False, True, True] and np.array_equal(lo, hi)


def test_client_view_marks_the_cells_of_visible_points(O):
    """A wall at z = 2.5 in front of the eye, nothing else: the visible
    points all lie in cells with z index 2, so exactly the probes with
    z in {2, 3} are in the view; an empty scene marks nothing."""
    cfg = _cfg(nx=4, ny=4, nz=4, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0))
    wall = np.array([[[-5, -5, 2.5], [5, 5, 2.5], [5, -5, 2.5]], [[-5, -5, 2.5], [-5, 5, 2.5], [5, 5, 2.5]]],
                    np.float32)
    sc = O.OracleScene(wall, np.full((2, 3), 0.5, np.float32))
    nom, lo, hi = O.client_pvs(sc, cfg, (1.5, 1.5, 0.2), 4096)
    z = np.arange(64) // 16
    assert np.array_equal(nom, z >= 2) and np.array_equal(lo, nom) and np.array_equal(hi, nom)
    empty = O.OracleScene(np.zeros((0, 3, 3), np.float32), np.zeros((0, 3), np.float32))
    assert not any(m.any() for m in O.client_pvs(empty, cfg, (1.5, 1.5, 0.2), 512))


# ---------------------------------------------------------------- entropy stage
def test_huffman_lengths_textbook_example(O):
    """Frequencies 45, 13, 12, 16, 9, 5 (a-f) give the textbook optimal
    code lengths 1, 3, 3, 3, 4, 4 (224 bits in all)."""
    h = np.zeros(256, np.uint64)
    h[[0, 1, 2, 3, 4, 5]] = [45, 13, 12, 16, 9, 5]
    ln = O.huf_lengths(h)
    assert ln[:6].tolist() == [1, 3, 3, 3, 4, 4] and not ln[6:].any()
    assert int((ln.astype(np.int64) * h.astype(np.int64)).sum()) == 224


def test_huffman_codes_are_canonical_and_prefix_free(O):
    rng = np.random.default_rng(8)
    h = np.zeros(256, np.uint64)
    h[rng.choice(256, 40, replace=False)] = rng.integers(1, 10_000, 40)
    ln = O.huf_lengths(h)
    cd = O.huf_codes(ln)
    used = np.nonzero(ln)[0]
    assert abs(sum(2.0 ** -int(ln[s]) for s in used) - 1.0) < 1e-12      # complete code (Kraft equality)
    words = [format(int(cd[s]), f"0{int(ln[s])}b") for s in used]
    for i, a in enumerate(words):
        for j, c in enumerate(words):
            assert i == j or not c.startswith(a)
    order = sorted(used, key=lambda s: (ln[s], s))                        # canonical: consecutive in (length, symbol)
    for a, c in zip(order, order[1:]):
        assert int(cd[c]) == (int(cd[a]) + 1) << (int(ln[c]) - int(ln[a]))
    one = np.zeros(256, np.uint64)
    one[7] = 3
    assert O.huf_lengths(one)[7] == 1


def test_huffman_length_limit(O):
    """Fibonacci frequencies force a 30-level tree; the counts are halved
    until the longest code fits 12 bits, and the code stays complete."""
    h = np.zeros(256, np.uint64)
    f = [1, 1]
    while len(f) < 30:
        f.append(f[-1] + f[-2])
    h[:30] = f
    ln = O.huf_lengths(h)
    assert ln.max() == 12 and (ln[:30] > 0).all()
    assert abs(sum(2.0 ** -int(ln[s]) for s in range(30)) - 1.0) < 1e-12


def test_entropy_round_trip_and_size(O):
    """A real packet: decode(encode) gives it back byte for byte, and the
    container size follows the layout: 40 bytes + per stream 132 bytes + 4
    per 1,024-byte chunk + each chunk's sum of code lengths rounded up to 32
    bits."""
    P = 300
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=3)
    ref_i, ref_v = synth.perturb_fp16_maps(cur_i, cur_v, seed=4, p_probe=0.5, p_texel=0.1, rel=2e-3)
    st = O.OracleClientState(P)
    st.ref_irr[:] = ref_i[:, :, 1:-1, 1:-1].reshape(P, 3, -1)
    st.ref_vis[:] = ref_v[:, :, 1:-1, 1:-1].reshape(P, 2, -1)
    pkt, mi, mv = st.pack(cur_i, cur_v)
    enc = O.huf_encode(pkt)
    assert O.huf_decode(enc, len(pkt) + 64) == pkt
    d = _parse(pkt)
    Ki, Kv = int(d["Ki"]), int(d["Kv"])
    buf = np.frombuffer(pkt, np.uint8)
    idx_pad = -(-2 * (Ki + Kv) // 16) * 16
    streams = [buf[32:32 + 2 * (Ki + Kv)]]
    off = 32 + idx_pad
    streams += [buf[off + k * Ki * 64: off + (k + 1) * Ki * 64] for k in range(6)]
    off += 6 * Ki * 64
    streams += [buf[off + k * Kv * 256: off + (k + 1) * Kv * 256] for k in range(4)]
    size = 40
    for s in streams:
        ln = O.huf_lengths(np.bincount(s, minlength=256).astype(np.uint64)).astype(np.int64)
        nch = -(-s.size // 1024)
        size += 132 + 4 * nch
        for c in range(nch):
            size += -(-int(ln[s[c * 1024:(c + 1) * 1024]].sum()) // 32) * 4
    assert len(enc) == size
    assert len(enc) < len(pkt)            # XOR planes of small changes are mostly zero bytes
