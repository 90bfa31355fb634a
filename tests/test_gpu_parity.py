"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (see the module helpers for the exact measures):
  - packing, deltas, masks, index buffers: bit-exact;
  - hit triangle per ray: inside the oracle's accepted set (the nominal hit,
    or another triangle a tiny perturbation of the ray reaches) for every
    ray, and equal to the nominal hit for >= 99.99% of rays;
  - per-ray radiance and distance: inside the oracle's tie bounds with
    relative slack 1e-4 for every ray, and within 1e-4 of the nominal answer
    for >= 99.9% of rays;
  - FP32 maps: inside the oracle's tie bounds with relative slack 1e-4
    (dark texels: 1e-3 of the map maximum), and >= 99.9% of texels within
    1e-4 of the nominal map;
  - FP16 maps: inside the oracle's FP16 tie bounds with 2 binary16 ulps of
    slack, and >= 99.9% of texels within 1 ulp of the nominal trajectory;
  - every map also against the oracle's FP64 blend of the GPU's own ray
    records (no tie can enter there): FP32 within 1e-4 everywhere, FP16
    within 2 ulps everywhere and 1 ulp for >= 99.9% of texels.
"""
import math

import numpy as np
import pytest

import synth
from helpers import (excess_fp16_ulps, excess_fp32, f16, fold_consistent, hit_agreement, ulps_from)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_05875_amd as ps
    ps.lib()
    return ps


@pytest.fixture(scope="module")
def ctx(ps):
    c = ps.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def _say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ a1
@pytest.mark.parametrize("n", [1, 7, 128, 256, 1000, 4096])
def test_ray_directions(ps, ctx, O, n):
    _say(f"ray directions n={n}")
    cfg = synth.VolumeConfig(1, 1, 1, (0, 0, 0), (1, 1, 1), n, fp16=False)
    vol = ps.Volume(ctx, cfg)
    sc = ps.Scene.from_synth(ctx, synth.empty_scene())
    vol.set_scene(sc)
    R = synth.rotation(3, n)
    vol.update_probes(R)
    _, _, dirs = vol.read_rays()
    want = O.ray_dirs(n, R)
    assert np.abs(dirs[:, :3] - want).max() < 1e-6


# ------------------------------------------------------------------ a2..a6 on the box room
def _update_both(ps, ctx, O, cfg, scene, frames, keep_hits=True, dyn=None, lights_per_frame=None):
    """Run ``frames`` updates on the GPU and in the oracle; yields per frame
    (gpu maps, oracle volume, gpu rays, gpu hits, oracle rays)."""
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg, keep_hits=keep_hits)
    vol.set_scene(sc)
    ov = O.OracleVolume(cfg)
    ov.g_irr, ov.g_vis = O.empty_maps(cfg)     # the oracle's blend of the GPU's rays
    n_static = scene.n_triangles - scene.n_dynamic
    osc = O.OracleScene.from_scene(scene, n_static=n_static)
    for f, R in enumerate(frames):
        lights = scene.lights if lights_per_frame is None else lights_per_frame[f]
        if dyn is not None:
            d = dyn(f)
            sc.set_dynamic(d)
            osc = O.OracleScene(np.concatenate([scene.triangles()[:n_static], d]), scene.albedo, scene.emission,
                                n_static=n_static)
        vol.update_probes(R, lights)
        rays = ov.update(osc, R, lights)
        irr, vis, fr = vol.read_maps()
        grays, ghits, _ = vol.read_rays()
        assert fr == f + 1
        O.blend_update(cfg, O.ray_dirs(cfg.rays_per_probe, R), grays[..., :3], grays[..., 3], ov.g_irr, ov.g_vis,
                       first=(f == 0))
        _check_reblend(irr, vis, ov, cfg.fp16)
        yield irr, vis, ov, grays, ghits, rays
    sc.close()
    vol.close()


def _check_reblend(irr, vis, ov, fp16):
    """The GPU maps against the oracle's FP64 blend of the GPU's own ray
    records: the blend, hysteresis and guard bands alone, with no tie."""
    for name, g, o in (("irr", irr, ov.g_irr), ("vis", vis, ov.g_vis)):
        if fp16:
            d = ulps_from(g, o)
            _say(f"  re-blend {name}: max {d.max():.2f} ulp, within 1 ulp {(d <= 1.0).mean():.5f}")
            assert d.max() <= 2.0 and (d <= 1.0).mean() >= 0.999
        else:
            e = excess_fp32(g, o, o)[0]
            _say(f"  re-blend {name}: max relative difference {e:.2e}")
            assert e <= 1e-4


def _check_fp32_maps(irr, vis, ov):
    for name, g, lo, hi, nom in (("irr", irr, ov.irr_lo, ov.irr_hi, ov.irr), ("vis", vis, ov.vis_lo, ov.vis_hi, ov.vis)):
        ex, _ = excess_fp32(g, lo, hi)
        _, dn = excess_fp32(g, nom, nom)
        near = float((dn <= 1e-4).mean())
        _say(f"  {name}: bound excess {ex:.2e}, within 1e-4 of nominal {near:.5f}")
        assert ex <= 1e-4 and near >= 0.999
        assert fold_consistent(g)


def _check_rays(grays, ghits, rays, min_equal=0.9999):
    eq, ok = hit_agreement(ghits, rays)
    if ok != 1.0:
        bad = np.argwhere(~np.any(rays["cand"] == ghits[..., None], axis=-1) & (ghits != rays["hit"]))
        for p, j in bad[:10]:
            _say(f"  ray ({p},{j}): gpu {ghits[p, j]} nominal {rays['hit'][p, j]} t {rays['hit_t'][p, j]:.6f} "
                 f"cand {rays['cand'][p, j].tolist()} L {grays[p, j].tolist()}")
    assert ok == 1.0, f"hits outside the accepted set: {1 - ok:.2e}"
    assert eq >= min_equal, f"nominal hit agreement {eq:.6f}"
    L = grays[..., :3].astype(np.float64)
    r = grays[..., 3].astype(np.float64)
    scale = max(float(np.abs(rays["L_hi"]).max()), 1e-30)
    tolL = 1e-4 * np.maximum(np.maximum(np.abs(rays["L_lo"]), np.abs(rays["L_hi"])), 1e-2 * scale)
    assert np.all(L >= rays["L_lo"] - tolL) and np.all(L <= rays["L_hi"] + tolL)
    tolr = 1e-4 * np.maximum(rays["r_hi"], 1e-3)
    assert np.all(r >= rays["r_lo"] - tolr) and np.all(r <= rays["r_hi"] + tolr)
    # the nominal answer itself, for all but the rays near a tie
    dL = np.abs(L - rays["L"]) / np.maximum(np.abs(rays["L"]), 1e-2 * scale)
    dr = np.abs(r - rays["r"]) / np.maximum(rays["r"], 1e-3)
    close = float(((dL.max(axis=-1) <= 1e-4) & (dr <= 1e-4)).mean())
    _say(f"  hits: nominal {eq:.6f}, accepted {ok:.6f}; rays within 1e-4 of nominal {close:.6f}")
    assert close >= 0.999


def test_box_room_update_fp32(ps, ctx, O):
    """The box-room workload: 4x4x4 probes, 24 triangles, 128 rays, FP32
    maps, one frame."""
    _say("box room, FP32 maps, 1 frame")
    cfg = synth.config("box_room")
    scene = synth.box_room()
    for irr, vis, ov, grays, ghits, rays in _update_both(ps, ctx, O, cfg, scene, [synth.rotation(2, 0)]):
        _check_rays(grays, ghits, rays)
        _check_fp32_maps(irr, vis, ov)
        assert (rays["L"] == 0).any()  # the cube casts shadows into the record


def _fp16_checks(irr, vis, ov, label):
    for name, g, lo, hi, nom in (("irr", irr, ov.irr_lo, ov.irr_hi, ov.irr), ("vis", vis, ov.vis_lo, ov.vis_hi, ov.vis)):
        ex, _ = excess_fp16_ulps(g, lo, hi)
        within1 = float((ulps_from(g, nom) <= 1.0).mean())
        _say(f"  {label} {name}: bound excess {ex:.2f} ulp, within 1 ulp of nominal {within1:.5f}")
        assert ex <= 2.0
        assert within1 >= 0.999
        assert fold_consistent(g)


def test_box_room_fp16_moving_light(ps, ctx, O):
    _say("box room, FP16 maps, 12 frames, moving light, hysteresis")
    cfg = synth.config("box_room")
    cfg.fp16 = True
    scene = synth.box_room()
    frames = [synth.rotation(2, f) for f in range(12)]
    lights = []
    for f in range(12):
        l = scene.lights.copy()
        l[0, :3] = [0.4 + 0.2 * f, 3.6 - 0.1 * f, 0.4 + 0.15 * f]
        lights.append(l)
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(
            _update_both(ps, ctx, O, cfg, scene, frames, lights_per_frame=lights)):
        _check_rays(grays, ghits, rays)
        _fp16_checks(irr, vis, ov, f"frame {f}")


@pytest.mark.parametrize("grid,n", [((5, 3, 7), 64), ((1, 1, 1), 1), ((2, 9, 1), 300)])
def test_ragged_grids_and_ray_counts(ps, ctx, O, grid, n):
    """Grids that do not fill 4x4x4 bricks, a single ray, ray counts that
    straddle the blend's chunk of 256."""
    _say(f"ragged grid {grid}, n={n}")
    cfg = synth.VolumeConfig(*grid, (-0.3, -0.2, -0.1), (0.7, 0.45, 0.6), n, fp16=False, max_distance=3.0,
                             sky=(0.2, 0.1, 0.05))
    scene = synth.box_room()
    for irr, vis, ov, grays, ghits, rays in _update_both(ps, ctx, O, cfg, scene,
                                                          [synth.rotation(4, 0), synth.rotation(4, 1)]):
        _check_rays(grays, ghits, rays)
        _check_fp32_maps(irr, vis, ov)


def test_empty_scene_and_emissive_box(ps, ctx, O):
    _say("empty scene (sky) and closed emissive box")
    cfg = synth.VolumeConfig(2, 3, 2, (0, 0, 0), (0.4, 0.4, 0.4), 128, fp16=False, max_distance=2.5,
                             sky=(0.3, 0.6, 1.2))
    for irr, vis, ov, grays, ghits, rays in _update_both(ps, ctx, O, cfg, synth.empty_scene(), [synth.rotation(5, 0)]):
        sky = np.array(cfg.sky, np.float32)
        for c in range(3):
            assert np.allclose(irr[:, c], sky[c], rtol=2e-6)
        assert np.allclose(vis[:, 0], np.float32(2.5), rtol=2e-6)
        assert np.allclose(vis[:, 1], np.float32(2.5) ** 2, rtol=2e-6)
    E = (0.7, 0.4, 0.2)
    box = synth.emissive_box(half_width=3.0, center=(0.5, 0.5, 0.5), emission=E)
    for irr, vis, ov, grays, ghits, rays in _update_both(ps, ctx, O, cfg, box, [synth.rotation(6, 0)]):
        for c in range(3):
            assert np.allclose(irr[:, c], np.float32(E[c]), rtol=2e-6)
        _check_rays(grays, ghits, rays)


# ------------------------------------------------------------------ the city at full size
def test_city_full_size_frames(ps, ctx, O):
    """The at-scale workload: 16x8x16 probes, 256 rays, 50k-triangle city,
    FP16 maps; three frames with the light moving on its spline."""
    cfg = synth.config("city")
    scene = synth.box_city()
    path = synth.light_path(12, 60)
    frames, lights = [], []
    for f in range(3):
        frames.append(synth.rotation(13, f))
        l = scene.lights.copy()
        l[0, :3] = path[f]
        lights.append(l)
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(
            _update_both(ps, ctx, O, cfg, scene, frames, lights_per_frame=lights)):
        _say(f"city frame {f}")
        _check_rays(grays, ghits, rays)
        _fp16_checks(irr, vis, ov, f"city frame {f}")


def test_encode_full_size_frames(ps, ctx, O):
    """The encode workload at full size: 32x16x32 = 16,384 probes, 256 rays,
    200k-triangle field with 4 moving occluders (dynamic BVH rebuilt per
    frame) and a moving light; two frames against the oracle."""
    cfg = synth.config("encode")
    scene = synth.box_field(200_000, seed=40, n_moving=4)
    path = synth.light_path(12, 120)
    frames, lights = [], []
    for f in range(2):
        frames.append(synth.rotation(41, f))
        l = scene.lights.copy()
        l[0, :3] = path[f]
        lights.append(l)
    dyn = lambda f: synth.moving_occluders(40, f, 4)
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(
            _update_both(ps, ctx, O, cfg, scene, frames, dyn=dyn, lights_per_frame=lights)):
        _say(f"encode frame {f}")
        _check_rays(grays, ghits, rays)
        _fp16_checks(irr, vis, ov, f"encode frame {f}")


def test_dynamic_occluders(ps, ctx, O):
    """Moving occluder boxes (dynamic triangles) over a small box field."""
    _say("moving occluders, 4 frames")
    scene = synth.box_field(3000, seed=40, extent=24.0, n_moving=3)
    cfg = synth.VolumeConfig(8, 4, 8, (1.0, 0.3, 1.0), (3.0, 2.0, 3.0), 64, max_distance=5.0, fp16=True,
                             sky=(0.1, 0.15, 0.25))
    dyn = lambda f: synth.moving_occluders(40, f * 7, 3, 24.0)
    frames = [synth.rotation(41, f) for f in range(4)]
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(_update_both(ps, ctx, O, cfg, scene, frames, dyn=dyn)):
        _check_rays(grays, ghits, rays)
        _fp16_checks(irr, vis, ov, f"dyn frame {f}")
        # the occluders are actually hit
        if f == 0:
            assert (ghits >= scene.n_triangles - scene.n_dynamic).any()


# ------------------------------------------------------------------ traversal work counts
@pytest.mark.parametrize("workload", ["city", "encode"])
def test_trace_counts_equal_host_replay(ps, ctx, O, workload):
    """The device's instrumented counts (node visits, triangle tests, shadow
    rays: the roofline's FLOP per launch is built from them) against a host
    replay of the same traversal over the BVH the library built (read back
    from the device), for every ray of a full-size frame. The replay's
    reciprocals are correctly rounded where the device's are approximate,
    so a few boundary decisions may differ: totals within 1e-5 (measured: the
    city frame equal to one node visit in 9.3 M)."""
    if workload == "city":
        cfg, scene = synth.config("city"), synth.box_city()
        R, dyn = synth.rotation(13, 0), None
        path = synth.light_path(12, 60)
    else:
        cfg, scene = synth.config("encode"), synth.box_field(200_000, seed=40, n_moving=4)
        R, dyn = synth.rotation(41, 0), synth.moving_occluders(40, 0, 4)
        path = synth.light_path(12, 120)
    lights = scene.lights.copy()
    lights[0, :3] = path[0]
    _say(f"trace counts vs host replay: {workload}")
    sc = ps.Scene.from_synth(ctx, scene)
    if dyn is not None:
        sc.set_dynamic(dyn)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    vol.update_probes(R, lights)
    _, _, dirs = vol.read_rays()
    got = vol.trace_counts(R, lights)
    rep = O.replay_trace_counts(sc.read_bvh(False)[:2], sc.read_bvh(True)[:2], cfg, dirs, lights, sc.read_bvh()[2])
    rays = cfg.n_probes * cfg.rays_per_probe
    _say(f"  device {got}; replay {rep}; per ray {rep['node_visits'] / rays:.3f} nodes, "
         f"{rep['tri_tests'] / rays:.3f} triangles, {rep['shadow_rays'] / rays:.3f} shadow rays")
    for k in ("node_visits", "tri_tests", "shadow_rays"):
        assert abs(got[k] - rep[k]) <= 1e-5 * rep[k], k
    assert rep["node_visits"] > 10 * rays and rep["shadow_rays"] > 0.1 * rays
    vol.close()
    sc.close()


# ------------------------------------------------------------------ blend from given rays
@pytest.mark.parametrize("fp16,n,grid,sharp", [(False, 64, (37, 1, 1), 50), (False, 300, (3, 2, 2), 50),
                                               (True, 256, (9, 5, 3), 50), (True, 513, (2, 1, 3), 50),
                                               (False, 96, (3, 1, 2), 7), (True, 4096, (2, 1, 1), 1),
                                               (False, 130, (11, 1, 1), 128)])
def test_blend_from_given_rays(ps, ctx, O, fp16, n, grid, sharp):
    """a4-a6 alone: both sides blend the same seeded ray records over five
    frames of hysteresis; visibility exponents other than 50 take the
    blend's generic power, 4,096 rays its longest chunk loop."""
    import torch
    _say(f"blend from given rays fp16={fp16} n={n} grid={grid} sharpness={sharp}")
    cfg = synth.VolumeConfig(*grid, (0, 0, 0), (1, 1, 1), n, fp16=fp16, max_distance=4.0, vis_sharpness=sharp)
    vol = ps.Volume(ctx, cfg)
    irr_o, vis_o = O.empty_maps(cfg)
    for f in range(5):
        R = synth.rotation(60 + n, f)
        L, r = synth.synthetic_rays(cfg.n_probes, n, seed=100 * f + n)
        rec = np.concatenate([L, r[..., None]], axis=-1).astype(np.float32)
        dev = torch.from_numpy(rec).cuda()
        torch.cuda.synchronize()
        vol.blend_rays(R, dev.data_ptr())
        ps.native.sync()
        O.blend_update(cfg, O.ray_dirs(n, R), L, r, irr_o, vis_o, first=(f == 0))
        irr, vis, _ = vol.read_maps()
        if fp16:
            for g, o in ((irr, irr_o), (vis, vis_o)):
                d = ulps_from(g, o)
                assert d.max() <= 2.0 and (d <= 1.0).mean() >= 0.999
        else:
            # x^s carries about s times the FP32 rounding of its base, so the
            # visibility bound grows with s up to the FP32 map bound (1e-4)
            assert excess_fp32(irr, irr_o, irr_o)[0] <= 1e-5
            assert excess_fp32(vis, vis_o, vis_o)[0] <= (1e-5 if sharp <= 50 else 1e-4)
        assert fold_consistent(irr) and fold_consistent(vis)
        del dev
    vol.close()


@pytest.mark.parametrize("mode", ["bf16x3", "f32", "tiles", "valu", "bf16x6"])
@pytest.mark.parametrize("fp16,n,grid", [(False, 96, (19, 1, 1)), (True, 256, (9, 5, 3)), (True, 300, (3, 2, 2)),
                                          (False, 33, (2, 1, 1)), (True, 1, (3, 1, 1)), (False, 4096, (2, 1, 1)),
                                          (True, 224, (5, 3, 2)), (False, 1, (17, 1, 1))])
def test_blend_paths_against_oracle(ps, ctx, O, mode, fp16, n, grid):
    """Every blend path (weight table with split-BF16, FP32 or vector-FMA
    products, or the per-tile weights) on the same seeded ray records over
    four frames of hysteresis: FP16 maps within 2 ulps (1 ulp for 99.9%) of
    the oracle's FP16 trajectory; FP32 maps within 1e-5 (the BF16x3
    products, whose terms carry about 2^-16 of relative error, within
    1e-4; BF16x6, about 2^-25, within 1e-5). Ray counts give one, two,
    three, seven and ten 32-ray steps (odd and even counts, ragged last
    steps) and 128; with one ray most texels have no weight and keep their
    stored value (FP16 and FP32 maps)."""
    import torch
    _say(f"blend path {mode} fp16={fp16} n={n} grid={grid}")
    cfg = synth.VolumeConfig(*grid, (0, 0, 0), (1, 1, 1), n, fp16=fp16, max_distance=4.0)
    vol = ps.Volume(ctx, cfg)
    vol.set_blend_mode(mode)
    assert vol.get_blend_mode() == mode
    irr_o, vis_o = O.empty_maps(cfg)
    for f in range(4):
        R = synth.rotation(70 + n, f)
        L, r = synth.synthetic_rays(cfg.n_probes, n, seed=10 * f + n)
        rec = np.concatenate([L, r[..., None]], axis=-1).astype(np.float32)
        dev = torch.from_numpy(rec).cuda()
        torch.cuda.synchronize()
        vol.blend_rays(R, dev.data_ptr())
        ps.native.sync()
        O.blend_update(cfg, O.ray_dirs(n, R), L, r, irr_o, vis_o, first=(f == 0))
        irr, vis, _ = vol.read_maps()
        for name, g, o in (("irr", irr, irr_o), ("vis", vis, vis_o)):
            if fp16:
                d = ulps_from(g, o)
                assert d.max() <= 2.0 and (d <= 1.0).mean() >= 0.999, (name, f, d.max())
            else:
                e = excess_fp32(g, o, o)[0]
                assert e <= (1e-4 if mode == "bf16x3" else 1e-5), (name, f, e)
        assert fold_consistent(irr) and fold_consistent(vis)
        del dev
    vol.close()


def test_tuner_over_frames_and_batched_buckets(ps, ctx):
    """The autotuner timed over several frames leaves a candidate shape on
    the volume; the batched tuner leaves one shape per probe-count bucket,
    and the batched update at the tuned shapes equals the per-volume
    updates bit for bit."""
    from paper_2103_05875_amd import autotune
    scene = synth.box_field(3000, seed=12, extent=24.0)
    sc = ps.Scene.from_synth(ctx, scene)
    cfgs = [synth.VolumeConfig(4, 4, 4, (1.0, 0.3, 1.0), (3.0, 2.0, 3.0), 32, fp16=True, max_distance=5.0),
            synth.VolumeConfig(8, 4, 8, (1.0, 0.3, 1.0), (1.5, 2.0, 1.5), 32, fp16=True, max_distance=5.0),
            synth.VolumeConfig(8, 8, 8, (1.0, 0.3, 1.0), (1.5, 1.0, 1.5), 16, fp16=True, max_distance=5.0)]
    frames = [(synth.rotation(5, f), None) for f in range(3)]
    v = ps.Volume(ctx, cfgs[0])
    v.set_scene(sc)
    r = autotune.tune(v, *frames[0], n_triangles=scene.n_triangles, reps=1, cache=None, shipped=False,
                      frames=frames, space="batched")
    got = v.get_trace_config()
    assert r["tried"] == len(autotune.candidates("batched"))
    assert tuple(got["brick"]) == tuple(r["config"]["brick"]) and got["top_nodes"] == r["config"]["top_nodes"]
    v.close()
    plain, batched = [], []
    for c in cfgs:
        a, b = ps.Volume(ctx, c), ps.Volume(ctx, c)
        a.set_scene(sc)
        b.set_scene(sc)
        plain.append(a)
        batched.append(b)
    rots = [synth.rotation(6 + i, 0) for i in range(len(cfgs))]
    tb = autotune.tune_batched(batched, rots, reps=1)
    assert set(tb["choices"]) == {autotune.probe_bucket(b) for b in batched}
    for b in batched:
        c = tb["choices"][autotune.probe_bucket(b)]
        got = b.get_trace_config()
        assert tuple(got["brick"]) == tuple(c["brick"]) and got["top_nodes"] == c["top_nodes"]
    for a, b in zip(plain, batched):
        a.set_maps(*b.read_maps()[:2], b.read_maps()[2])
    for f in range(2):
        rots = [synth.rotation(9 + i, f) for i in range(len(cfgs))]
        for a, R in zip(plain, rots):
            a.update_probes(R)
        ps.update_probes_batched(batched, rots)
        ps.native.sync()
        for a, b in zip(plain, batched):
            ia, va, _ = a.read_maps()
            ib, vb, _ = b.read_maps()
            assert np.array_equal(ia, ib) and np.array_equal(va, vb)
    for h in plain + batched + [sc]:
        h.close()


def test_blend_mode_default_follows_volume_size(ps, ctx):
    """A new volume takes the per-tile weights below 2,048 probes and the
    three-part BF16 table product from there; AUTO restores that choice."""
    for grid, want in (((4, 4, 4), "tiles"), ((16, 8, 15), "tiles"), ((16, 8, 16), "bf16x6"), ((16, 16, 16), "bf16x6")):
        vol = ps.Volume(ctx, synth.VolumeConfig(*grid, (0, 0, 0), (1, 1, 1), 64, fp16=True))
        assert vol.get_blend_mode() == want
        vol.set_blend_mode("valu")
        assert vol.get_blend_mode() == "valu"
        vol.set_blend_mode("auto")
        assert vol.get_blend_mode() == want
        vol.close()


# ------------------------------------------------------------------ pack (bit-exact)
def _grid_for(P):
    for nx in range(min(P, 64), 0, -1):
        if P % nx == 0 and P // nx <= 1024:
            return nx, P // nx, 1
    return P, 1, 1


# 16,377 probes: 2,048 tiles, the last with one probe (the largest scan-free
# pack); 16,392 probes: 2,049 tiles (the one-block scan runs); 256 and 257
# probes: 32 and 33 tiles, one and two checksum shares in a group word (32
# groups); 8,191 probes: 1,024 tiles, 32 shares per group, the last ragged
@pytest.mark.parametrize("P,taus", [(1, (0.0, 0.0)), (37, (1.0 / 1024, 0.0)), (2048, (0.0, 1.0 / 1024)),
                                    (16384, (1.0 / 1024, 1.0 / 1024)), (1000, (0.01, 0.003)),
                                    (16377, (0.0, 1.0 / 1024)), (16392, (1.0 / 1024, 0.0)),
                                    (256, (0.0, 0.0)), (257, (1.0 / 1024, 0.0)), (8191, (0.0, 1.0 / 1024))])
def test_pack_bit_exact(ps, ctx, O, P, taus):
    _say(f"pack P={P} taus={taus}")
    nx, ny, nz = _grid_for(P)
    if ny > 1024:
        nx, ny, nz = 64, P // 64, 1
    cfg = synth.VolumeConfig(nx, ny, nz, (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol, client_id=P)
    st = O.OracleClientState(P, client=P)
    dec = O.OracleClientDecoder(P)
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=P)
    for f in range(8):
        vol.set_maps(cur_i, cur_v, f)
        cl.pack_delta(*taus)
        got = cl.packet_download()
        want, mi, mv = st.pack(cur_i, cur_v, *taus)
        gmi, gmv = cl.read_masks()
        assert np.array_equal(gmi, mi) and np.array_equal(gmv, mv)
        assert got == want, f"frame {f}: packet differs ({len(got)} vs {len(want)} bytes)"
        assert dec.apply(got) == 0
        assert np.array_equal(dec.irr[:, :, 1:-1, 1:-1].reshape(P, 3, -1), st.ref_irr)
        cur_i, cur_v = synth.perturb_fp16_maps(cur_i, cur_v, seed=1000 * P + f, p_probe=0.3, p_texel=0.05)
    # forced resend after a reset: every non-zero probe again
    cl.reset()
    st.reset()
    vol.set_maps(cur_i, cur_v, 9)
    cl.pack_delta(*taus)
    assert cl.packet_download() == st.pack(cur_i, cur_v, *taus)[0]
    cl.close()
    vol.close()


def _straddling_pairs(tau, rng, n):
    """n pairs of binary16 values (bit patterns) whose difference lies within
    a few binary16 steps of tau on either side, led by a pair whose binary32
    difference rounds onto tau although the exact one exceeds it (3 against
    3 * 2^-24 when tau = 3 - 2^-22)."""
    pairs = [(np.float16(3.0), np.float16(3 * 2.0 ** -24))]
    while len(pairs) < n:
        a = np.float16(rng.uniform(tau, tau + 8.0))
        b = np.float16(float(a) - tau)
        for k in range(-2, 3):
            bb = np.uint16(int(b.view(np.uint16)) + k).view(np.float16)
            if np.isfinite(bb):
                pairs.append((a, bb) if rng.uniform() < 0.5 else (bb, a))
    return [(x.view(np.uint16), y.view(np.uint16)) for x, y in pairs[:n]]


@pytest.mark.parametrize("tau", [3.0 - 2.0 ** -22, 1.0 / 1024, 0.75, 1.0, 1.5])
def test_pack_threshold_boundaries(ps, ctx, O, tau):
    """The change test |cur - ref| > tau is exact (Sec. 3.4's threshold, strict):
    one texel per probe steps across a difference within a few binary16 steps
    of tau; the masks and the packet equal the oracle's, which compares in
    binary64. A binary32 difference would miss the leading pair."""
    tau = float(np.float32(tau))
    P = 512
    _say(f"pack threshold boundaries tau={tau!r}")
    cfg = synth.VolumeConfig(8, 8, 8, (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol, client_id=9)
    st = O.OracleClientState(P, client=9)
    rng = np.random.default_rng(int(tau * 1e6) % 1000)
    pairs = _straddling_pairs(tau, rng, 2 * P)
    a_i = np.zeros((P, 3, 10, 10), np.uint16)
    a_v = np.zeros((P, 2, 18, 18), np.uint16)
    b_i, b_v = a_i.copy(), a_v.copy()
    for p in range(P):
        (x0, y0), (x1, y1) = pairs[p], pairs[P + p]
        c, r, q = p % 3, 1 + p % 8, 1 + (p // 8) % 8
        a_i[p, c, r, q], b_i[p, c, r, q] = x0, y0
        a_v[p, p % 2, 1 + p % 16, 1 + (p // 16) % 16], b_v[p, p % 2, 1 + p % 16, 1 + (p // 16) % 16] = x1, y1
    for f, (mi_, mv_) in enumerate(((a_i, a_v), (b_i, b_v))):
        vol.set_maps(mi_, mv_, f)
        t = 0.0 if f == 0 else tau
        cl.pack_delta(t, t)
        got = cl.packet_download()
        want, mi, mv = st.pack(mi_, mv_, t, t)
        gmi, gmv = cl.read_masks()
        assert np.array_equal(gmi, mi) and np.array_equal(gmv, mv), f"frame {f}: masks differ"
        assert got == want
    # both outcomes occur, and the leading pair counts as changed
    assert 0 < mi.sum() < P and 0 < mv.sum() < P
    if tau == float(np.float32(3.0 - 2.0 ** -22)):
        assert mi[0] == 1
    cl.close()
    vol.close()


def test_pack_maximum_probe_count(ps, ctx, O):
    P = 65536
    _say("pack P=65536")
    cfg = synth.VolumeConfig(64, 32, 32, (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol, client_id=3)
    st = O.OracleClientState(P, client=3)
    cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=5)
    for f in range(2):
        vol.set_maps(cur_i, cur_v, f)
        cl.pack_delta(0.0, 0.0)
        assert cl.packet_download() == st.pack(cur_i, cur_v)[0]
        cur_i, cur_v = synth.perturb_fp16_maps(cur_i, cur_v, seed=77, p_probe=0.1)
    cl.close()
    vol.close()


def test_update_then_pack_round_trip(ps, ctx, O):
    """GPU update + GPU pack over 20 frames; a client applying the packets
    holds exactly the server's current interiors (tau = 0) every frame."""
    _say("update + pack round trip, 20 frames")
    scene = synth.box_city(n_tris=6000, extent=32.0)
    cfg = synth.VolumeConfig(8, 4, 8, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), 64, fp16=True, max_distance=6.0,
                             sky=(0.1, 0.15, 0.25))
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    cl = ps.Client(vol, client_id=11)
    dec = O.OracleClientDecoder(cfg.n_probes)
    path = synth.light_path(12, 20, extent=32.0)
    sent = []
    for f in range(20):
        l = scene.lights.copy()
        l[0, :3] = path[f]
        vol.update_probes(synth.rotation(13, f), l)
        cl.pack_delta(0.0, 0.0)
        pkt = cl.packet_download()
        assert dec.apply(pkt) == 0 and dec.seq == f
        irr, vis, _ = vol.read_maps()
        assert np.array_equal(dec.irr[:, :, 1:-1, 1:-1], irr[:, :, 1:-1, 1:-1])
        assert np.array_equal(dec.vis[:, :, 1:-1, 1:-1], vis[:, :, 1:-1, 1:-1])
        assert np.array_equal(dec.irr, irr) and np.array_equal(dec.vis, vis)   # guard bands rebuilt
        sent.append(len(pkt))
    assert sent[0] >= sent[-1]
    cl.close()
    vol.close()
    sc.close()


# ------------------------------------------------------------------ batched = plain
@pytest.mark.parametrize("maps", ["mixed", "fp16", "fp32", "fp16_bf16x3"])
def test_batched_matches_plain_bitwise(ps, ctx, O, maps):
    """Six uneven volumes, three frames: the batched update equals the
    per-volume updates bit for bit; the batched volumes take different trace
    shapes (probe bricks, staged top nodes) of their own, the plain ones
    other schedules. Map types and blend paths select the batched blend
    kernel: mixed map types (every path compiled in), one map type with the
    per-tile, FP32-table (third volume) and BF16x6-table (fifth volume)
    paths, or a BF16x3 volume among them (every path again)."""
    _say(f"batched vs plain, 6 uneven volumes, 3 frames, maps {maps}")
    specs = [((4, 4, 4), 64, True, 2000), ((5, 3, 7), 128, True, 800), ((16, 2, 16), 256, True, 5000),
             ((1, 1, 1), 512, False, 300), ((8, 8, 4), 64, False, 1200), ((3, 3, 3), 1, True, 100)]
    shapes_b = [((8, 8, 1), 85), ((2, 4, 8), 0), ((16, 4, 1), 21), ((4, 4, 4), 85), ((8, 4, 2), 0), ((4, 4, 4), 21)]
    shapes_p = [((4, 4, 4), 1), ((8, 4, 2), 0), ((2, 4, 8), 2), ((8, 8, 1), 1), ((16, 4, 1), 0), ((4, 4, 4), 2)]
    plain, batched, scenes = [], [], []
    for i, (g, n, fp16, nt) in enumerate(specs):
        sc_syn = synth.box_city(n_tris=nt, seed_layout=70 + i, seed_heights=80 + i, extent=16.0)
        sc = ps.Scene.from_synth(ctx, sc_syn)
        scenes.append(sc)
        if maps != "mixed":
            fp16 = maps != "fp32"
        cfg = synth.VolumeConfig(*g, (1.0, 0.3, 1.0), (2.0, 1.0, 2.0), n, fp16=fp16, max_distance=5.0,
                                 sky=(0.1, 0.15, 0.25))
        a, b = ps.Volume(ctx, cfg), ps.Volume(ctx, cfg)
        a.set_scene(sc)
        b.set_scene(sc)
        a.set_trace_config(shapes_p[i][0], shapes_p[i][1], 21, 256, False)
        b.set_trace_config(shapes_b[i][0], 2, shapes_b[i][1], 256, False)
        if i in (2, 4) and maps != "mixed":
            for v in (a, b):
                v.set_blend_mode("bf16x3" if maps == "fp16_bf16x3" else "f32" if i == 2 else "bf16x6")
        plain.append(a)
        batched.append(b)
    for f in range(3):
        rots = [synth.rotation(90 + i, f) for i in range(len(specs))]
        for v, R in zip(plain, rots):
            v.update_probes(R)
        ps.update_probes_batched(batched, rots)
        ps.native.sync()
        for a, b in zip(plain, batched):
            ia, va, fa = a.read_maps()
            ib, vb, fb = b.read_maps()
            assert fa == fb == f + 1
            assert np.array_equal(ia.view(np.uint8), ib.view(np.uint8))
            assert np.array_equal(va.view(np.uint8), vb.view(np.uint8))
    for h in plain + batched + scenes:
        h.close()


def test_pipelined_update_and_pack_match_serial(ps, ctx, O):
    """Frames pipelined over two streams (each pack on a second stream,
    overlapping the next frame's directions and trace; the next blend waits
    for it through pv_update_probes_after) give the serial maps and packets
    bit for bit, with the BF16x6 table and the per-tile blend."""
    import torch
    _say("pipelined update + pack over two streams vs serial")
    scene = synth.box_city(n_tris=6000, seed_layout=5, seed_heights=6, extent=16.0)
    sc = ps.Scene.from_synth(ctx, scene)
    for mode in ("bf16x6", "tiles"):
        cfg = synth.VolumeConfig(16, 8, 16, (1.0, 0.3, 1.0), (1.0, 1.0, 1.0), 64, fp16=True, max_distance=4.0,
                                 sky=(0.1, 0.15, 0.25))
        a, b = ps.Volume(ctx, cfg), ps.Volume(ctx, cfg)
        for v in (a, b):
            v.set_scene(sc)
            v.set_blend_mode(mode)
        ca, cb = ps.Client(a, client_id=1), ps.Client(b, client_id=1)
        frames = 6
        want = []
        for f in range(frames):
            a.update_probes(synth.rotation(40, f))
            ca.pack_delta(0.0, 0.0)
            want.append(ca.packet_download())
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        evs = [torch.cuda.Event() for _ in range(2)]
        got = []
        b.update_probes(synth.rotation(40, 0), stream=s1)
        for f in range(frames):
            s2.wait_stream(s1)
            cb.pack_delta(0.0, 0.0, stream=s2)
            evs[f % 2].record(s2)
            # the next frame's update is enqueued before this frame's packet
            # is read: its directions and trace may run beside the pack
            if f + 1 < frames:
                b.update_probes(synth.rotation(40, f + 1), stream=s1, after=evs[f % 2])
            got.append(cb.packet_download(stream=s2))
        torch.cuda.synchronize()
        assert got == want
        ia, va, _ = a.read_maps()
        ib, vb, _ = b.read_maps()
        assert np.array_equal(ia.view(np.uint16), ib.view(np.uint16))
        assert np.array_equal(va.view(np.uint16), vb.view(np.uint16))
        for h in (ca, cb, a, b):
            h.close()
    sc.close()


def test_checkpoint_export_import_continues_identically(ps, ctx, O):
    _say("checkpoint export/import")
    scene = synth.box_room()
    cfg = synth.config("box_room")
    cfg.fp16 = True
    sc = ps.Scene.from_synth(ctx, scene)
    a = ps.Volume(ctx, cfg)
    a.set_scene(sc)
    for f in range(3):
        a.update_probes(synth.rotation(2, f))
    irr, vis, fr = a.read_maps()
    b = ps.Volume(ctx, cfg)
    b.set_scene(sc)
    b.set_maps(irr, vis, fr)
    for f in range(3, 6):
        a.update_probes(synth.rotation(2, f))
        b.update_probes(synth.rotation(2, f))
    ia, va, _ = a.read_maps()
    ib, vb, _ = b.read_maps()
    assert np.array_equal(ia, ib) and np.array_equal(va, vb)
    for h in (a, b, sc):
        h.close()


def test_invalid_arguments_are_refused(ps, ctx):
    cfg = synth.config("box_room")
    v = ps.Volume(ctx, cfg)
    with pytest.raises(ps.NativeError) as e:
        v.update_probes(synth.rotation(1, 0))      # no scene set
    assert e.value.status == -4
    sc = ps.Scene.from_synth(ctx, synth.box_room())
    v.set_scene(sc)
    with pytest.raises(ps.NativeError):
        v.update_probes(np.full(9, 2.0, np.float32))   # not a rotation
    with pytest.raises(ps.NativeError) as e:
        ps.Client(v)                                 # FP32 maps cannot be packed
    assert e.value.status == -6
    bad = synth.box_room()
    bad.indices = bad.indices.copy()
    bad.indices[0, 0] = 10 ** 6
    with pytest.raises(ps.NativeError):
        ps.Scene.from_synth(ctx, bad)
    v.close()
    sc.close()


# ------------------------------------------------------------------ served: alone = in the mix
def test_served_results_equal_alone_results(ps, ctx, O):
    """Requests of 8 clients arrive as a Poisson trace and are served with
    continuous batching under an HBM budget that forces evictions; every
    client's packets equal the packets of the same requests served alone."""
    from paper_2103_05875_amd import serve
    _say("served vs alone, 8 clients, 64 requests, budget forcing evictions")
    scene_syn = synth.box_city(n_tris=8000, extent=32.0)
    scene = ps.Scene.from_synth(ctx, scene_syn)
    rng = np.random.default_rng(31)
    cfgs = []
    for c in range(8):
        ny = int(rng.integers(1, 4))
        cfgs.append(synth.VolumeConfig(8, ny, 8, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), int(rng.choice([32, 64, 128])),
                                       fp16=True, max_distance=6.0, sky=(0.1, 0.15, 0.25)))
    path = synth.light_path(12, 64, extent=32.0)
    t = np.cumsum(rng.exponential(1.0 / 800.0, 64))
    frame_of = [0] * 8

    def make():
        reqs, fo = [], [0] * 8
        for i in range(64):
            c = int(rng_c[i])
            l = scene_syn.lights.copy()
            l[0, :3] = path[fo[c] % 64]
            reqs.append(serve.Request(c, synth.rotation(200 + c, fo[c]), l, float(t[i])))
            fo[c] += 1
        return reqs
    rng_c = rng.integers(0, 8, 64)
    fps = [ps.volume_footprint(c) + ps.client_footprint(c) for c in cfgs]
    budget = int(sum(sorted(fps)[-4:]) * 1.05)       # about half the clients fit at once
    srv = serve.Server(ctx, scene, cfgs, hbm_budget=budget, n_streams=3, max_batch=8)
    served = srv.run(make())
    srv.close()
    assert srv.evictions > 0 and max(r.batch_size for r in served) > 1
    alone = serve.serve_plain(ctx, scene, cfgs, make())
    by_client = lambda rs: {c: [r.packet for r in sorted((r for r in rs if r.client == c), key=lambda r: r.arrival)]
                            for c in range(8)}
    a, b = by_client(served), by_client(alone)
    for c in range(8):
        assert a[c] == b[c], f"client {c} differs"
    _say(f"  evictions {srv.evictions}, largest batch {max(r.batch_size for r in served)}, "
         f"latency {serve.latency_stats(served)}")
    # delivery at the pinned staging, headers kept: the same headers and sizes
    srv2 = serve.Server(ctx, scene, cfgs, hbm_budget=budget, n_streams=3, max_batch=8, keep_packets=False)
    staged = srv2.run(make())
    srv2.close()
    hdr = lambda rs: {c: [(r.header, r.nbytes) for r in sorted((r for r in rs if r.client == c),
                                                              key=lambda r: r.arrival)] for c in range(8)}
    h2 = hdr(staged)
    for c in range(8):
        assert all(r.packet is None for r in staged)
        assert h2[c] == [(p[:32], len(p)) for p in b[c]], f"client {c}: staged headers differ"
    scene.close()


def test_trace_launch_shapes_are_bit_identical(ps, ctx, O):
    """Every trace launch shape the autotuner may pick (brick, persistent
    queues, LDS-staged top nodes, block size) gives the same bits."""
    from paper_2103_05875_amd import autotune
    _say("trace launch shapes: identical bits")
    scene = ps.Scene.from_synth(ctx, synth.box_city(n_tris=12000, extent=32.0))
    cfg = synth.VolumeConfig(7, 5, 9, (2.0, 0.25, 2.0), (4.0, 1.5, 3.5), 96, fp16=True, max_distance=6.0,
                             sky=(0.1, 0.15, 0.25))
    ref = None
    for c in autotune.candidates()[::7] + [autotune.candidates()[-1]]:
        v = ps.Volume(ctx, cfg, keep_hits=True)
        v.set_scene(scene)
        v.set_trace_config(c["brick"], c["persistent"], c["top_nodes"], c["block_threads"], c["split_shadows"])
        for f in range(2):
            v.update_probes(synth.rotation(77, f))
        irr, vis, _ = v.read_maps()
        rays, hits, _ = v.read_rays()
        got = (irr.tobytes(), vis.tobytes(), rays.tobytes(), hits.tobytes())
        if ref is None:
            ref = got
        assert got == ref, f"launch shape {c} differs"
        v.close()
    scene.close()


def _three_lights(extent):
    return np.array([[0.3 * extent, 9.0, 0.4 * extent, 300.0, 280.0, 260.0],
                     [0.8 * extent, 6.0, 0.7 * extent, 120.0, 90.0, 60.0],
                     [0.5 * extent, 1.2, 0.1 * extent, 30.0, 40.0, 50.0]], np.float32)


@pytest.mark.parametrize("case", ["dynamic_3_lights", "one_triangle", "empty", "emissive"])
def test_refill_trace_equals_packet_trace(ps, ctx, case):
    """The stepped traces (separate node and triangle steps; with and without
    per-lane ray refill) write the same bits as the one-wave-per-packet
    trace: static and moving triangles, several lights, a ragged grid,
    degenerate scenes."""
    _say(f"refill trace vs packet trace: {case}")
    cfg = synth.VolumeConfig(7, 5, 9, (1.0, 0.3, 1.0), (3.0, 1.7, 2.5), 80, fp16=True, max_distance=6.0,
                             sky=(0.1, 0.15, 0.25))
    dyn = None
    if case == "dynamic_3_lights":
        scene = synth.box_field(3000, seed=41, extent=24.0, n_moving=3)
        scene.lights = _three_lights(24.0)
        dyn = lambda f: synth.moving_occluders(41, f * 5, 3, 24.0)
    elif case == "one_triangle":
        tri = np.array([[[0.0, 0.5, 0.0], [20.0, 0.5, 0.0], [0.0, 0.5, 20.0]]], np.float32)
        scene = synth.soup_scene(tri, np.full((1, 3), 0.6, np.float32), np.zeros((1, 3), np.float32),
                                 _three_lights(20.0)[:1])
    elif case == "empty":
        scene = synth.empty_scene()
    else:
        scene = synth.emissive_box(half_width=3.0, center=(10.0, 4.0, 10.0))
    sc = ps.Scene.from_synth(ctx, scene)
    out = {}
    for persistent, brick in ((0, (4, 4, 4)), (1, (4, 4, 4)), (1, (8, 4, 2)), (1, (16, 4, 1)), (2, (4, 4, 4)),
                              (2, (8, 8, 1))):
        v = ps.Volume(ctx, cfg, keep_hits=True)
        v.set_scene(sc)
        v.set_trace_config(brick, persistent, 21 if persistent else 0, 128, False)
        got = []
        for f in range(3):
            if dyn is not None:
                sc.set_dynamic(dyn(f))
            v.update_probes(synth.rotation(91, f), scene.lights)
            rays, hits, _ = v.read_rays()
            got.append((rays.tobytes(), hits.tobytes()))
        irr, vis, _ = v.read_maps()
        got.append((irr.tobytes(), vis.tobytes()))
        out[(persistent, brick)] = got
        c = v.trace_counts(synth.rotation(91, 3), scene.lights)
        _say(f"  persistent={persistent} brick={brick}: counts {c}")
        v.close()
    ref = out[(0, (4, 4, 4))]
    for k, got in out.items():
        for f, (a, b) in enumerate(zip(got, ref)):
            assert a == b, f"{k} differs from the packet trace at step {f}"
    sc.close()


def test_batch_graph_replays_match_eager(ps, ctx, O):
    """The captured batched frame, replayed 6 times with eager work and
    synchronizations in between, equals the eager plain path every frame."""
    import torch
    _say("captured batched graph: 6 replays against eager")
    specs = [((4, 4, 4), 64, True, 2000), ((5, 3, 7), 128, True, 900), ((2, 2, 2), 256, False, 400)]
    plain, graphed, scenes = [], [], []
    for i, (g, n, fp16, nt) in enumerate(specs):
        sc = ps.Scene.from_synth(ctx, synth.box_city(n_tris=nt, seed_layout=50 + i, seed_heights=60 + i, extent=16.0))
        scenes.append(sc)
        cfg = synth.VolumeConfig(*g, (1.0, 0.3, 1.0), (2.0, 1.0, 2.0), n, fp16=fp16, max_distance=5.0)
        a, b = ps.Volume(ctx, cfg), ps.Volume(ctx, cfg)
        a.set_scene(sc)
        b.set_scene(sc)
        plain.append(a)
        graphed.append(b)
    graph = ps.BatchGraph(graphed)
    stream = torch.cuda.Stream()
    for f in range(6):
        rots = [synth.rotation(400 + i, f) for i in range(len(specs))]
        for v, R in zip(plain, rots):
            v.update_probes(R, stream=stream)
        graph.launch(rots, stream=stream)
        x = torch.ones(1 << 20, device="cuda")            # unrelated eager work between replays
        x.mul_(2.0)
        torch.cuda.synchronize()
        for a, b in zip(plain, graphed):
            ia, va, fa = a.read_maps()
            ib, vb, fb = b.read_maps()
            assert fa == fb == f + 1
            assert np.array_equal(ia.view(np.uint8), ib.view(np.uint8)), f"replay {f}"
            assert np.array_equal(va.view(np.uint8), vb.view(np.uint8)), f"replay {f}"
    graph.close()
    for h in plain + graphed + scenes:
        h.close()
