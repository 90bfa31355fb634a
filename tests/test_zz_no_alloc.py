"""The delta pack's allocation-free entry point (pv_pack_delta_noalloc: caller
buffers in and out, intermediates in the library's static device array)
against the client pack (pv_pack_delta) on the same maps: packets and
reference states byte for byte equal over consecutive calls, the later ones
on a smaller volume, so the second size runs on what the first left in the
array."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_05875_amd as ps
    ps.lib()
    return ps


def _packet_size(hdr_words):
    k_irr, k_vis = int(hdr_words[5]), int(hdr_words[6])
    idx = (2 * (k_irr + k_vis) + 15) // 16 * 16
    return 32 + idx + k_irr * 6 * 64 + k_vis * 4 * 256


def test_noalloc_pack_equals_client_pack(ps):
    import torch
    ctx = ps.Context(0)
    # 16,392 probes: past the fused-summary limit (the scan launch runs);
    # then 37 probes (a ragged last tile of odd length) on the same array
    for P, tau, seed in ((16392, 1.0 / 1024, 3), (37, 0.0, 4)):
        _say(f"no-alloc pack: {P} probes, tau {tau}")
        cfg = synth.VolumeConfig(P, 1, 1, (0, 0, 0), (1, 1, 1), 64, fp16=True)
        vol = ps.Volume(ctx, cfg)
        cl = ps.Client(vol, client_id=9)
        ref_i = torch.zeros((P, 3, 64), dtype=torch.int16, device="cuda")
        ref_v = torch.zeros((P, 2, 256), dtype=torch.int16, device="cuda")
        cap = ps.packet_capacity(P)
        pkt = torch.zeros(cap, dtype=torch.uint8, device="cuda")
        cur_i, cur_v = synth.random_fp16_maps(P, 8, 16, seed=seed)
        for f in range(3):
            vol.set_maps(cur_i, cur_v, f)
            cl.pack_delta(tau, tau)
            want = cl.packet_download()
            irr_ptr, vis_ptr = vol.get_maps()
            torch.cuda.synchronize()
            ps.pack_delta_noalloc(ctx, irr_ptr, vis_ptr, ref_i.data_ptr(), ref_v.data_ptr(), P, tau, tau, 9, f,
                                  pkt.data_ptr(), cap)
            ps.native.sync()
            hdr = pkt[:32].cpu().numpy().view(np.uint32)
            got = pkt[:_packet_size(hdr)].cpu().numpy().tobytes()
            _say(f"  frame {f}: {len(got)} bytes (client pack {len(want)}), K = {int(hdr[5])}, {int(hdr[6])}")
            assert got == want
            ri, rv, _ = cl.read_state()
            assert np.array_equal(ref_i.cpu().numpy().view(np.uint16), ri)
            assert np.array_equal(ref_v.cpu().numpy().view(np.uint16), rv)
            cur_i, cur_v = synth.perturb_fp16_maps(cur_i, cur_v, seed=100 * seed + f)
        cl.close()
        vol.close()
    # sizes beyond the array's limit and a short packet buffer are refused
    # on the host (no kernel runs)
    with pytest.raises(ps.NativeError):
        ps.pack_delta_noalloc(ctx, pkt.data_ptr(), pkt.data_ptr(), pkt.data_ptr(), pkt.data_ptr(), 65537, 0.0, 0.0,
                              0, 0, pkt.data_ptr(), 1 << 40)
    with pytest.raises(ps.NativeError):
        ps.pack_delta_noalloc(ctx, pkt.data_ptr(), pkt.data_ptr(), pkt.data_ptr(), pkt.data_ptr(), 37, 0.0, 0.0,
                              0, 0, pkt.data_ptr(), 64)
    ctx.close()
