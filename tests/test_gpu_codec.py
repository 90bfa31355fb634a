"""GPU parity of the codec surfaces (pv_encode_yuv / pv_decode_yuv) against
the oracle's: every plane sample and every decoded code and bit pattern
bit-exact, over ragged atlas shapes and at 65,536 probes."""
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


def _grid(P):
    for nx in (64, 32, 16, 8, 4, 2, 1):
        if P % nx == 0:
            rest = P // nx
            for ny in (32, 16, 8, 4, 2, 1):
                if rest % ny == 0:
                    return nx, ny, rest // ny
    return P, 1, 1


@pytest.mark.parametrize("P, C, scale", [(1, 1, 1.0), (7, 3, 2.5), (100, 7, 0.75), (2048, 32, 2.5),
                                         (65536, 256, 3.0)])
def test_codec_surfaces_match_oracle(ps, ctx, O, P, C, scale):
    _say(f"codec surfaces P={P} C={C} scale={scale}")
    irr, vis = synth.random_fp16_maps(P, 8, 16, seed=P + 3 * C, scale=3.0)
    cfg = synth.VolumeConfig(*_grid(P), (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    vol.set_maps(irr, vis, 0)
    ip, vp = vol.encode_yuv(scale, C)
    want_i, want_v = O.yuv_encode(irr.view(np.float16).astype(np.float64), vis, scale, C)
    gi = ip.cpu().numpy().view(np.uint16)
    gv = vp.cpu().numpy()
    assert np.array_equal(gi, want_i)
    assert np.array_equal(gv, want_v)
    codes, vback = ps.decode_yuv(ctx, P, C, ip, vp)
    wc, wv = O.yuv_decode(want_i, want_v, P, C)
    assert np.array_equal(codes.cpu().numpy().view(np.uint32), wc)
    assert np.array_equal(vback.cpu().numpy().view(np.uint16), wv)
    assert np.array_equal(wv, vis[:, :, 1:-1, 1:-1].reshape(P, 2, 256))
    vol.close()


def test_codec_surfaces_after_an_update_and_errors(ps, ctx, O):
    _say("codec surfaces of an updated volume; argument errors")
    scene = synth.box_city(n_tris=3000, extent=32.0)
    cfg = synth.VolumeConfig(8, 4, 8, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), 64, fp16=True, max_distance=6.0)
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    vol.update_probes(synth.rotation(5, 0))
    irr, vis, _ = vol.read_maps()
    ip, vp = vol.encode_yuv(4.0, 20)
    wi, wvp = O.yuv_encode(irr.view(np.float16).astype(np.float64), vis, 4.0, 20)
    assert np.array_equal(ip.cpu().numpy().view(np.uint16), wi) and np.array_equal(vp.cpu().numpy(), wvp)
    _, vback = ps.decode_yuv(ctx, cfg.n_probes, 20, ip, vp)
    assert np.array_equal(vback.cpu().numpy().view(np.uint16), vis[:, :, 1:-1, 1:-1].reshape(-1, 2, 256))
    # caller-provided outputs (filled with garbage first) give the same bytes
    import torch
    ip2, vp2 = torch.full_like(ip, -1), torch.full_like(vp, 0xAB)
    codes2, vis2 = torch.full((cfg.n_probes, 64), -1, dtype=torch.int32, device="cuda"), \
        torch.full((cfg.n_probes, 2, 256), -1, dtype=torch.int16, device="cuda")
    vol.encode_yuv(4.0, 20, out=(ip2, vp2))
    ps.decode_yuv(ctx, cfg.n_probes, 20, ip2, vp2, out=(codes2, vis2))
    assert torch.equal(ip2, ip) and torch.equal(vp2, vp) and torch.equal(vis2, vback)
    with pytest.raises(ValueError):
        vol.encode_yuv(4.0, 21, out=(ip2, vp2))
    for bad in ((0.0, 20), (float("inf"), 20), (1.0, 0), (1.0, 70000)):
        with pytest.raises(ps.NativeError):
            vol.encode_yuv(*bad)
    f32 = ps.Volume(ctx, synth.VolumeConfig(2, 2, 2, (0, 0, 0), (1, 1, 1), 8, fp16=False))
    with pytest.raises(ps.NativeError):
        f32.encode_yuv(1.0, 2)
    for h in (f32, vol, sc):
        h.close()
