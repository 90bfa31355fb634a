"""GPU parity of the shading query (pv_probe_query) and of the second bounce
(PV_MULTI_BOUNCE) against the FP64 oracle.

Bars:
  - query on given maps: relative error <= 1e-4 (floor 1e-2 of the value
    scale) at every point, FP32 and FP16 maps;
  - closed emissive, reflecting box: the maps follow the geometric series the
    oracle pin derives, to FP32 rounding;
  - updates with the second bounce: the same bars as without it (ray records
    inside the oracle's bounds, FP32 maps within 1e-4, FP16 maps within
    2 ulp and 99.9% within 1 ulp), where the oracle's bounds span the bounce
    term on its nominal and tie-bound maps, widened by 1e-3 (FP32) or 4e-3
    (FP16) of the term for the rounding of the stored maps;
  - batched and graphed updates: bit-identical to the plain ones.
"""
import numpy as np
import pytest

import synth
from helpers import excess_fp16_ulps, excess_fp32, fold_consistent, hit_agreement, ulps_from

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


def _upload(vol, cfg, irr, vis):
    if cfg.fp16:
        vol.set_maps(irr.astype(np.float16).view(np.uint16), vis.astype(np.float16).view(np.uint16), 1)
    else:
        vol.set_maps(irr.astype(np.float32), vis.astype(np.float32), 1)


# ------------------------------------------------------------------ query
@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("grid", [(4, 4, 4), (5, 3, 2), (1, 6, 1), (1, 1, 1)])
def test_probe_query_matches_oracle(ps, ctx, O, fp16, grid):
    _say(f"probe query grid={grid} fp16={fp16}")
    cfg = synth.VolumeConfig(*grid, (-1.0, 0.5, 2.0), (0.7, 1.3, 0.9), 64, fp16=fp16)
    irr, vis = synth.query_maps(cfg, seed=sum(grid) + 7 * fp16)
    pts, nrm = synth.query_points(cfg, 1500, seed=3 + sum(grid))
    vol = ps.Volume(ctx, cfg)
    _upload(vol, cfg, irr, vis)
    got = vol.probe_query(pts, nrm).cpu().numpy().astype(np.float64)
    want = np.array([O.probe_query(cfg, irr, vis, p.astype(np.float64), n.astype(np.float64))
                     for p, n in zip(pts, nrm)])
    tol = 1e-4 * np.maximum(np.abs(want), 1e-2 * np.abs(want).max())
    err = np.abs(got - want)
    _say(f"  max relative error {float((err / np.maximum(np.abs(want), 1e-30)).max()):.2e}")
    assert np.all(err <= tol)
    vol.close()


def test_probe_query_edge_cases(ps, ctx, O):
    import torch
    _say("probe query: empty maps, no points")
    cfg = synth.VolumeConfig(3, 2, 2, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 64, fp16=True)
    vol = ps.Volume(ctx, cfg)
    pts, nrm = synth.query_points(cfg, 100, seed=11)
    assert not torch.any(vol.probe_query(pts, nrm))          # zero maps: every weight vanishes
    assert vol.probe_query(np.zeros((0, 3)), np.zeros((0, 3))).shape == (0, 3)
    with pytest.raises(ValueError):
        vol.probe_query(np.zeros((4, 2)), np.zeros((4, 2)))
    vol.close()


# ------------------------------------------------------------------ second bounce
def _closed_box(E, rho):
    tris = synth._box_triangles(np.array([-1.5, -1.0, -1.25]), np.array([2.0, 1.75, 1.5]))
    return synth.soup_scene(tris, np.tile(rho, (12, 1)), np.tile(E, (12, 1)), np.zeros((0, 6)))


@pytest.mark.parametrize("h", [0.0, 0.6])
def test_second_bounce_closed_box_geometric_series(ps, ctx, O, h):
    """Every wall emits E and reflects rho: map_k = h map_(k-1) +
    (1 - h)(E + rho map_(k-1)), map_0 = E."""
    _say(f"second bounce, closed box, h={h}")
    E, rho = np.array([0.7, 0.4, 0.2]), np.array([0.5, 0.25, 0.8])
    cfg = synth.VolumeConfig(3, 2, 2, (-0.4, -0.3, -0.2), (0.5, 0.75, 0.6), 128, fp16=False, hysteresis=h,
                             multi_bounce=True)
    sc = ps.Scene.from_synth(ctx, _closed_box(E, rho))
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    Ef, rf, hf = E.astype(np.float32).astype(np.float64), rho.astype(np.float32).astype(np.float64), float(np.float32(h))
    m = Ef.copy()
    for k in range(5):
        vol.update_probes(synth.rotation(8, k), np.zeros((0, 6), np.float32))
        if k > 0:
            m = hf * m + (1 - hf) * (Ef + rf * m)
        irr = vol.read_maps()[0][:, :, 1:-1, 1:-1].astype(np.float64)
        for c in range(3):
            assert np.allclose(irr[:, c], m[c], rtol=1e-5, atol=0), (k, c)
    vol.close()
    sc.close()


def _update_both(ps, ctx, O, cfg, scene, frames, ind_rel):
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg, keep_hits=True)
    vol.set_scene(sc)
    ov = O.OracleVolume(cfg)
    osc = O.OracleScene.from_scene(scene)
    g_irr, g_vis = O.empty_maps(cfg)   # the oracle's blend of the GPU's own ray records
    for f, R in enumerate(frames):
        vol.update_probes(R, scene.lights)
        rays = ov.update(osc, R, scene.lights, ind_rel=ind_rel)
        irr, vis, fr = vol.read_maps()
        grays, ghits, _ = vol.read_rays()
        assert fr == f + 1
        O.blend_update(cfg, O.ray_dirs(cfg.rays_per_probe, R), grays[..., :3], grays[..., 3], g_irr, g_vis,
                       first=(f == 0))
        for name, g, o in (("irr", irr, g_irr), ("vis", vis, g_vis)):
            if cfg.fp16:
                d = ulps_from(g, o)
                _say(f"  re-blend {name}: max {d.max():.2f} ulp, within 1 ulp {(d <= 1.0).mean():.5f}")
                assert d.max() <= 2.0 and (d <= 1.0).mean() >= 0.999
            else:
                e = excess_fp32(g, o, o)[0]
                _say(f"  re-blend {name}: max relative difference {e:.2e}")
                assert e <= 1e-4
        yield irr, vis, ov, grays, ghits, rays
    vol.close()
    sc.close()


def _check_rays(grays, ghits, rays, min_equal=0.9999):
    eq, ok = hit_agreement(ghits, rays)
    assert ok == 1.0, f"hits outside the accepted set: {1 - ok:.2e}"
    assert eq >= min_equal, f"nominal hit agreement {eq:.6f}"
    L = grays[..., :3].astype(np.float64)
    scale = max(float(np.abs(rays["L_hi"]).max()), 1e-30)
    tolL = 1e-4 * np.maximum(np.maximum(np.abs(rays["L_lo"]), np.abs(rays["L_hi"])), 1e-2 * scale)
    below = rays["L_lo"] - tolL - L
    above = L - rays["L_hi"] - tolL
    _say(f"  ray radiance: worst excess below {below.max():.2e}, above {above.max():.2e}")
    assert np.all(below <= 0) and np.all(above <= 0)


def test_second_bounce_box_room_fp32(ps, ctx, O):
    """The box room with its light, FP32 maps, h = 0.5, 4 frames."""
    _say("second bounce, box room, FP32 maps, 4 frames")
    cfg = synth.config("box_room")
    cfg.hysteresis = 0.5
    cfg.multi_bounce = True
    frames = [synth.rotation(12, f) for f in range(4)]
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(_update_both(ps, ctx, O, cfg, synth.box_room(), frames,
                                                                        ind_rel=1e-3)):
        _check_rays(grays, ghits, rays)
        e1, _ = excess_fp32(irr, ov.irr_lo, ov.irr_hi)
        e2, _ = excess_fp32(vis, ov.vis_lo, ov.vis_hi)
        _say(f"  frame {f}: irradiance excess {e1:.2e}, visibility excess {e2:.2e}")
        assert e1 <= 1e-4 and e2 <= 1e-4
        assert fold_consistent(irr) and fold_consistent(vis)
    # the case exercises the bounce: it adds light over the direct-only update
    direct = synth.config("box_room")
    direct.hysteresis = 0.5
    od = O.OracleVolume(direct)
    osc = O.OracleScene.from_scene(synth.box_room())
    for R in frames:
        od.update(osc, R, synth.box_room().lights)
    assert ov.irr[:, :, 1:-1, 1:-1].sum() > 1.01 * od.irr[:, :, 1:-1, 1:-1].sum()


def test_second_bounce_box_room_fp16(ps, ctx, O):
    _say("second bounce, box room, FP16 maps, 4 frames")
    cfg = synth.config("box_room")
    cfg.hysteresis = 0.5
    cfg.fp16 = True
    cfg.multi_bounce = True
    frames = [synth.rotation(13, f) for f in range(4)]
    for f, (irr, vis, ov, grays, ghits, rays) in enumerate(_update_both(ps, ctx, O, cfg, synth.box_room(), frames,
                                                                        ind_rel=4e-3)):
        _check_rays(grays, ghits, rays)
        for name, g, lo, hi, nom in (("irr", irr, ov.irr_lo, ov.irr_hi, ov.irr),
                                     ("vis", vis, ov.vis_lo, ov.vis_hi, ov.vis)):
            ex, _ = excess_fp16_ulps(g, lo, hi)
            within1 = float((ulps_from(g, nom) <= 1.0).mean())
            _say(f"  frame {f} {name}: bound excess {ex:.2f} ulp, within 1 ulp of nominal {within1:.5f}")
            assert ex <= 2.0
            assert within1 >= 0.999


def test_second_bounce_batched_and_graph_bitwise(ps, ctx, O):
    """Volumes with and without the second bounce in one batch: batched and
    graphed updates equal the plain ones bit for bit."""
    _say("second bounce: batched and graph vs plain")
    specs = [((4, 4, 4), 64, True, True), ((5, 3, 7), 128, False, False), ((3, 2, 5), 96, True, False),
             ((2, 2, 2), 256, False, True)]
    sc = ps.Scene.from_synth(ctx, synth.box_city(n_tris=1500, seed_layout=31, seed_heights=32, extent=16.0))
    plain, batched, graphed = [], [], []
    for g, n, fp16, mb in specs:
        cfg = synth.VolumeConfig(*g, (1.0, 0.3, 1.0), (2.0, 1.0, 2.0), n, fp16=fp16, max_distance=5.0,
                                 hysteresis=0.5, multi_bounce=mb, sky=(0.1, 0.15, 0.25))
        for lst in (plain, batched, graphed):
            v = ps.Volume(ctx, cfg)
            v.set_scene(sc)
            lst.append(v)
    graph = ps.BatchGraph(graphed)
    for f in range(3):
        rots = [synth.rotation(500 + i, f) for i in range(len(specs))]
        for v, R in zip(plain, rots):
            v.update_probes(R)
        ps.update_probes_batched(batched, rots)
        graph.launch(rots)
        ps.native.sync()
        for a, b, c in zip(plain, batched, graphed):
            ia, va, _ = a.read_maps()
            for other in (b, c):
                io, vo, _ = other.read_maps()
                assert np.array_equal(ia.view(np.uint8), io.view(np.uint8)), f"frame {f}"
                assert np.array_equal(va.view(np.uint8), vo.view(np.uint8)), f"frame {f}"
    graph.close()
    for v in plain + batched + graphed:
        v.close()
    sc.close()
