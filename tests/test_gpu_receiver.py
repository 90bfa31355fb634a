"""GPU parity of the client-side unpack (pv_receiver_*) against the oracle's
client decoder: tiles bit-exact (guard bands included) after every packet;
packets with a bad checksum or index are refused without touching the
tiles; header errors are reported at once."""
import struct

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


def _server(ps, ctx, nx=8, ny=4, nz=8, n=64, tris=5000):
    scene = synth.box_city(n_tris=tris, extent=32.0)
    cfg = synth.VolumeConfig(nx, ny, nz, (2.0, 0.25, 2.0), (4.0, 1.5, 4.0), n, fp16=True, max_distance=6.0,
                             sky=(0.1, 0.15, 0.25))
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    return scene, cfg, sc, vol


def test_receiver_matches_oracle_decoder_over_frames(ps, ctx, O):
    _say("receiver vs oracle decoder, 12 frames, tau 0 and 1/1024")
    scene, cfg, sc, vol = _server(ps, ctx)
    cl = ps.Client(vol, client_id=5)
    rx = ps.Receiver(ctx, cfg.n_probes)
    dec = O.OracleClientDecoder(cfg.n_probes)
    path = synth.light_path(21, 12, extent=32.0)
    for f in range(12):
        l = scene.lights.copy()
        l[0, :3] = path[f]
        vol.update_probes(synth.rotation(22, f), l)
        tau = 0.0 if f % 3 else 1.0 / 1024
        cl.pack_delta(tau, tau)
        pkt = cl.packet_download()
        rx.apply(pkt)
        assert rx.status() == (0, f)
        assert dec.apply(pkt) == 0
        irr, vis = rx.read_maps()
        assert np.array_equal(irr, dec.irr) and np.array_equal(vis, dec.vis), f"frame {f}"
        ri, rv, _ = cl.read_state()
        assert np.array_equal(irr[:, :, 1:-1, 1:-1].reshape(cfg.n_probes, 3, 64), ri)
        assert np.array_equal(vis[:, :, 1:-1, 1:-1].reshape(cfg.n_probes, 2, 256), rv)
    # nothing changed since the last pack: an empty packet
    cl.pack_delta(0.0, 0.0)
    pkt = cl.packet_download()
    assert struct.unpack_from("<II", pkt, 20) == (0, 0)
    before = rx.read_maps()
    rx.apply(pkt)
    assert rx.status()[0] == 0
    after = rx.read_maps()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    for h in (rx, cl, vol, sc):
        h.close()


def _with_checksum(O, pkt: bytearray) -> bytes:
    struct.pack_into("<I", pkt, 28, O.payload_checksum(bytes(pkt[32:])))
    return bytes(pkt)


def test_receiver_refuses_corrupt_packets(ps, ctx, O):
    _say("receiver: corrupt checksum, invalid index, header errors")
    scene, cfg, sc, vol = _server(ps, ctx, nx=4, ny=4, nz=4, n=64, tris=3000)
    P = cfg.n_probes
    cl = ps.Client(vol, client_id=1)
    rx = ps.Receiver(ctx, P)
    vol.update_probes(synth.rotation(30, 0))
    cl.pack_delta()
    first = cl.packet_download()
    rx.apply(first)
    assert rx.status() == (0, 0)
    good = rx.read_maps()
    vol.update_probes(synth.rotation(30, 1))
    cl.pack_delta()
    pkt = cl.packet_download()
    K_irr, K_vis = struct.unpack_from("<II", pkt, 20)
    assert K_irr >= 2

    def unchanged():
        now = rx.read_maps()
        return all(np.array_equal(a, b) for a, b in zip(good, now))

    bad = bytearray(pkt)
    bad[-1] ^= 0x40                                  # a payload byte: checksum no longer matches
    rx.apply(bytes(bad))
    assert rx.status() == (-2, 0) and unchanged()
    bad = bytearray(pkt)
    struct.pack_into("<H", bad, 34, 0)               # second irradiance entry: a zero delta (repeat)
    rx.apply(_with_checksum(O, bad))
    assert rx.status()[0] == -4 and unchanged()
    bad = bytearray(pkt)
    struct.pack_into("<H", bad, 32, P)               # first entry: probe P (out of range)
    rx.apply(_with_checksum(O, bad))
    assert rx.status()[0] == -4 and unchanged()
    for broken in (b"\0" * 16, b"XXXX" + pkt[4:], pkt[:-1], pkt + b"\0" * 16):
        with pytest.raises(ps.NativeError):
            rx.apply(broken)
    other = ps.Receiver(ctx, P + 1)
    with pytest.raises(ps.NativeError):
        other.apply(pkt)
    other.close()
    # the intact packet still applies on top of the unchanged state
    rx.apply(pkt)
    assert rx.status() == (0, 1)
    dec = O.OracleClientDecoder(P)
    assert dec.apply(first) == 0 and dec.apply(pkt) == 0
    irr, vis = rx.read_maps()
    assert np.array_equal(irr, dec.irr) and np.array_equal(vis, dec.vis)
    for h in (rx, cl, vol, sc):
        h.close()


def test_receiver_full_size_volume(ps, ctx, O):
    """65,536 probes (the index limit), every probe sent twice."""
    _say("receiver at 65,536 probes")
    P = 65536
    irr0, vis0 = synth.random_fp16_maps(P, 8, 16, seed=3)
    irr1, vis1 = synth.perturb_fp16_maps(irr0, vis0, seed=4, p_probe=0.5)
    cfg = synth.VolumeConfig(64, 32, 32, (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol, client_id=2)
    rx = ps.Receiver(ctx, P)
    dec = O.OracleClientDecoder(P)
    for f, (i, v) in enumerate(((irr0, vis0), (irr1, vis1))):
        vol.set_maps(i, v, f)
        cl.pack_delta()
        pkt = cl.packet_download()
        rx.apply(pkt)
        assert rx.status() == (0, f)
        assert dec.apply(pkt) == 0
        gi, gv = rx.read_maps()
        assert np.array_equal(gi, dec.irr) and np.array_equal(gv, dec.vis)
    for h in (rx, cl, vol):
        h.close()


def test_packet_download_entry_points_agree(ps, ctx):
    """pv_packet_download into a caller buffer and pv_packet_stage (the
    binding's path) return the same bytes; a short buffer is refused with
    the needed size."""
    import ctypes
    _say("packet download vs pinned staging")
    scene, cfg, sc, vol = _server(ps, ctx, nx=4, ny=4, nz=4, n=64, tris=3000)
    cl = ps.Client(vol, client_id=3)
    L = ps.lib()
    # before the first pack there is no packet to hand out
    ptr, nb = ctypes.c_void_p(), ctypes.c_uint64(0)
    assert L.pv_packet_stage(cl.h, ctypes.byref(ptr), ctypes.byref(nb), None) == -4   # PV_ERR_STATE
    assert L.pv_packet_download(cl.h, None, 0, ctypes.byref(nb), None) == -4
    for f in range(3):
        vol.update_probes(synth.rotation(31, f))
        cl.pack_delta(0.0, 1.0 / 1024)
        staged = cl.packet_download()
        nb = ctypes.c_uint64(0)
        assert L.pv_packet_download(cl.h, None, 0, ctypes.byref(nb), None) == -5   # PV_ERR_CAPACITY
        assert nb.value == len(staged)
        buf = (ctypes.c_uint8 * nb.value)()
        assert L.pv_packet_download(cl.h, buf, nb.value, ctypes.byref(nb), None) == 0
        assert bytes(buf) == staged
    for h in (cl, vol, sc):
        h.close()
