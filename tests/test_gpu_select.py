"""GPU parity of probe selection (PV_CLASSIFY, pv_client_set_view) against
the oracle: activity and view masks inside the oracle's bound masks (equal
where the bounds coincide), packets bit-exact with the oracle's
eligible-only pack, batched activity equal to plain."""
import numpy as np
import pytest

import synth

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


def _within(g, lo, hi):
    return bool(np.all(g >= lo) and np.all(g <= hi))


def _scenes():
    solid = synth.soup_scene(synth._box_triangles([-0.5, -0.5, -0.5], [0.5, 0.5, 0.5]), np.full((12, 3), 0.5),
                             np.zeros((12, 3)), np.zeros((0, 6)))
    ground = synth.box_city(n_tris=14).triangles()[:2]
    ground = synth.soup_scene(ground, np.full((2, 3), 0.5), np.zeros((2, 3)), np.zeros((0, 6)))
    city = synth.box_city(n_tris=6000, extent=32.0)
    return [
        ("solid box", solid, synth.VolumeConfig(4, 1, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 256, fp16=False,
                                                classify=True)),
        ("ground", ground, synth.VolumeConfig(2, 2, 1, (10.0, -0.5, 10.0), (1.0, 1.0, 1.0), 256, fp16=False,
                                              classify=True)),
        ("city", city, synth.VolumeConfig(8, 4, 8, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), 64, fp16=True,
                                          max_distance=6.0, classify=True)),
    ]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_activity_matches_oracle(ps, ctx, O, case):
    name, scene, cfg = _scenes()[case]
    _say(f"activity: {name}")
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    assert vol.read_active().all()                    # before any update every probe counts as active
    R = synth.rotation(3, 0)
    vol.update_probes(R, scene.lights)
    got = vol.read_active()
    osc = O.OracleScene.from_scene(scene)
    nom, lo, hi = O.probe_activity(osc, cfg, R, O.trace_shade(osc, cfg, R, scene.lights))
    _say(f"  active {got.sum()} of {got.size}; oracle nominal {nom.sum()}, bounds {lo.sum()}..{hi.sum()}")
    assert _within(got, lo, hi)
    if case < 2:
        assert np.array_equal(got, nom)
    else:
        assert 0 < got.sum() < got.size
    vol.close()
    sc.close()


def test_client_view_matches_oracle(ps, ctx, O):
    _say("client view: wall and city")
    wall = np.array([[[-5, -5, 2.5], [5, 5, 2.5], [5, -5, 2.5]], [[-5, -5, 2.5], [-5, 5, 2.5], [5, 5, 2.5]]])
    wall_scene = synth.soup_scene(wall, np.full((2, 3), 0.5), np.zeros((2, 3)), np.zeros((0, 6)))
    city = synth.box_city(n_tris=6000, extent=32.0)
    cases = [(wall_scene, synth.VolumeConfig(4, 4, 4, (0, 0, 0), (1, 1, 1), 64, fp16=True), (1.5, 1.5, 0.2), 4096),
             (city, synth.VolumeConfig(8, 4, 8, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), 64, fp16=True), (13.1, 1.7, 17.3),
              8192)]
    for k, (scene, cfg, eye, n_rays) in enumerate(cases):
        sc = ps.Scene.from_synth(ctx, scene)
        vol = ps.Volume(ctx, cfg)
        vol.set_scene(sc)
        cl = ps.Client(vol)
        assert cl.read_view() is None
        cl.set_view(eye, n_rays)
        got = cl.read_view()
        nom, lo, hi = O.client_pvs(O.OracleScene.from_scene(scene), cfg, eye, n_rays)
        _say(f"  case {k}: view {got.sum()} of {got.size}; oracle {nom.sum()}, bounds {lo.sum()}..{hi.sum()}")
        assert _within(got, lo, hi)
        if k == 0:
            assert np.array_equal(got, nom) and np.array_equal(got, np.arange(64) // 16 >= 2)
        cl.clear_view()
        assert cl.read_view() is None
        for h in (cl, vol, sc):
            h.close()


def test_pack_sends_only_selected_probes(ps, ctx, O):
    """Activity from an update, a view from the client's position, then
    synthetic maps packed: the packet equals the oracle's pack of the same
    maps with eligible = active and in view (bounds coinciding)."""
    _say("pack with activity and view")
    tris = np.concatenate([
        np.array([[[-5, -5, 3.5], [5, 5, 3.5], [5, -5, 3.5]], [[-5, -5, 3.5], [-5, 5, 3.5], [5, 5, 3.5]]]),  # faces -z
        synth._box_triangles([0.6, 0.6, 0.6], [1.4, 1.4, 1.4]),                                          # solid around probe (1,1,1)
    ])
    scene = synth.soup_scene(tris, np.full((14, 3), 0.5), np.zeros((14, 3)), np.zeros((0, 6)))
    cfg = synth.VolumeConfig(4, 4, 4, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 128, fp16=True, classify=True)
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    R = synth.rotation(9, 0)
    vol.update_probes(R)
    osc = O.OracleScene.from_scene(scene)
    anom, alo, ahi = O.probe_activity(osc, cfg, R, O.trace_shade(osc, cfg, R, np.zeros((0, 6), np.float32)))
    eye = (2.2, 2.7, 0.4)
    vnom, vlo, vhi = O.client_pvs(osc, cfg, eye, 4096)
    assert np.array_equal(alo, ahi) and np.array_equal(vlo, vhi)
    elig = anom & vnom
    _say(f"  active {anom.sum()}, in view {vnom.sum()}, eligible {elig.sum()} of 64")
    assert 0 < elig.sum() < 64 and not anom[1 + 4 + 16]      # the probe inside the solid is inactive
    cl = ps.Client(vol, client_id=4)
    cl.set_view(eye, 4096)
    assert np.array_equal(vol.read_active(), anom) and np.array_equal(cl.read_view(), vnom)
    irr, vis = synth.random_fp16_maps(64, 8, 16, seed=21)
    vol.set_maps(irr, vis, 1)
    cl.pack_delta()
    st = O.OracleClientState(64, client=4)
    want, wi, wv = st.pack(irr, vis, eligible=elig)
    assert cl.packet_download() == want
    mi, mv = cl.read_masks()
    assert np.array_equal(mi, wi) and np.array_equal(mv, wv)
    ri, rv, _ = cl.read_state()
    assert np.array_equal(ri, st.ref_irr) and np.array_equal(rv, st.ref_vis)
    # without the view every active changed probe goes
    cl.clear_view()
    cl.pack_delta()
    want2, _, _ = st.pack(irr, vis, eligible=anom)
    assert cl.packet_download() == want2
    for h in (cl, vol, sc):
        h.close()


def test_batched_activity_equals_plain(ps, ctx, O):
    _say("batched and graphed activity vs plain")
    city = synth.box_city(n_tris=4000, extent=32.0)
    sc = ps.Scene.from_synth(ctx, city)
    specs = [((8, 4, 8), 64, True), ((5, 3, 7), 128, False), ((4, 4, 4), 96, True)]
    plain, batched, graphed = [], [], []
    for g, n, cls in specs:
        cfg = synth.VolumeConfig(*g, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), n, fp16=True, classify=cls,
                                 multi_bounce=not cls)
        for lst in (plain, batched, graphed):
            v = ps.Volume(ctx, cfg)
            v.set_scene(sc)
            lst.append(v)
    graph = ps.BatchGraph(graphed)
    for f in range(2):
        rots = [synth.rotation(70 + i, f) for i in range(len(specs))]
        for v, R in zip(plain, rots):
            v.update_probes(R)
        ps.update_probes_batched(batched, rots)
        graph.launch(rots)
        ps.native.sync()
        for (g, n, cls), a, b, c in zip(specs, plain, batched, graphed):
            ia, va, _ = a.read_maps()
            for other in (b, c):
                io, vo, _ = other.read_maps()
                assert np.array_equal(ia.view(np.uint8), io.view(np.uint8))
                assert np.array_equal(va.view(np.uint8), vo.view(np.uint8))
                if cls:
                    assert np.array_equal(a.read_active(), other.read_active())
    graph.close()
    for v in plain + batched + graphed:
        v.close()
    sc.close()
