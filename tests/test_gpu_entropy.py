"""GPU parity of the entropy stage (pv_entropy_encode, pv_receiver_apply_
compressed) against the oracle's coder: containers byte-identical for the
same packets, and compressed packets applied on the device give the tiles
the oracle's decoder builds from the uncompressed ones."""
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


def _grid(P):
    for nx in (64, 32, 16, 8, 4, 2, 1):
        if P % nx == 0:
            rest = P // nx
            for ny in (32, 16, 8, 4, 2, 1):
                if rest % ny == 0:
                    return nx, ny, rest // ny
    return P, 1, 1


@pytest.mark.parametrize("P", [64, 300, 4096, 65536])
def test_entropy_containers_match_oracle(ps, ctx, O, P):
    """Three packets per size (full resend, a partial change, nothing
    changed): the GPU's packet equals the oracle's, its container equals the
    oracle's byte for byte, and a receiver fed the containers holds what the
    oracle's decoder holds."""
    _say(f"entropy P={P}")
    cfg = synth.VolumeConfig(*_grid(P), (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol, client_id=7)
    rx = ps.Receiver(ctx, P)
    st = O.OracleClientState(P, client=7)
    dec = O.OracleClientDecoder(P)
    irr, vis = synth.random_fp16_maps(P, 8, 16, seed=P)
    irr2, vis2 = synth.perturb_fp16_maps(irr, vis, seed=P + 1, p_probe=0.3)
    for f, (i, v) in enumerate(((irr, vis), (irr2, vis2), (irr2, vis2))):
        vol.set_maps(i, v, f)
        cl.pack_delta()
        pkt = cl.packet_download()
        want_pkt, _, _ = st.pack(i, v)
        assert pkt == want_pkt
        cl.entropy_encode()
        got = cl.entropy_download()
        want = O.huf_encode(want_pkt)
        _say(f"  frame {f}: packet {len(pkt)} B, container {len(got)} B")
        assert got == want
        rx.apply_compressed(got)
        assert rx.status() == (0, f)
        assert dec.apply(want_pkt) == 0
        gi, gv = rx.read_maps()
        assert np.array_equal(gi, dec.irr) and np.array_equal(gv, dec.vis)
    if P == 64:
        assert struct.unpack_from("<II", pkt, 20) == (0, 0) and len(got) == 40 + 11 * 132
    for h in (rx, cl, vol):
        h.close()


def test_compressed_apply_refuses_malformed_containers(ps, ctx, O):
    _say("entropy: malformed containers")
    P = 256
    cfg = synth.VolumeConfig(*_grid(P), (0, 0, 0), (1, 1, 1), 1, fp16=True)
    vol = ps.Volume(ctx, cfg)
    cl = ps.Client(vol)
    irr, vis = synth.random_fp16_maps(P, 8, 16, seed=9)
    vol.set_maps(irr, vis, 0)
    cl.pack_delta()
    cl.entropy_encode()
    good = cl.entropy_download()
    rx = ps.Receiver(ctx, P)
    for bad in (good[:39], b"XXXX" + good[4:], good[:-4], good + b"\0" * 4):
        with pytest.raises(ps.NativeError):
            rx.apply_compressed(bad)
    # a flipped bit in a chunk decodes to other bytes: the packet checksum refuses it
    flipped = bytearray(good)
    flipped[-5] ^= 0x10
    rx.apply_compressed(bytes(flipped))
    assert rx.status()[0] in (-2, -4)
    assert not rx.read_maps()[0].any()
    rx.apply_compressed(good)
    assert rx.status() == (0, 0)
    for h in (rx, cl, vol):
        h.close()
