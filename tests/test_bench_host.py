"""Host-side logic of bench.py: the HBM byte counters of the trace kernel are
scaled by the copy kernel's reading and used only for the kernel source and
launch shape they were taken on."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, v) in enumerate(rows):
            f.write(f'{i},"{k}",{counter},{v}\n')


def test_counters_scale_and_staleness(tmp_path):
    b = _bench()
    tr = "void pv::k_trace<false, 128, 21, false, unsigned short>(pv::TraceGrid)"
    cnt = "void pv::k_trace<true, 128, 21, false, unsigned short>(pv::TraceGrid)"
    other = "void pv::k_trace<false, 256, 21, false, unsigned short>(pv::TraceGrid)"   # another launch shape
    # the copy reads 256 MiB but FETCH_SIZE shows half of it: scale 2
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0), (tr, 1000.0), (tr, 3000.0),
                                            (cnt, 99999.0), (other, 77777.0), ("__amd_rocclr_copyBuffer", 4.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (tr, 500.0)])
    out = tmp_path / "c.txt"
    t = b.write_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "8,4,2,0,21,128,0")
    assert t == 2000 * 1024 * 2 + 500 * 1024
    cfg = {"brick": [8, 4, 2], "persistent": False, "top_nodes": 21, "block_threads": 128, "split_shadows": False}
    v, src = b.read_counters(str(out), cfg)
    assert v == t and src == str(out)
    v, why = b.read_counters(str(out), {**cfg, "top_nodes": 0})
    assert v is None and "launch shape" in why
    txt = out.read_text().replace(b.kernel_source_hash(), "0" * 64)
    out.write_text(txt)
    v, why = b.read_counters(str(out), cfg)
    assert v is None and "changed" in why
    assert b.read_counters(str(tmp_path / "missing.txt"), cfg)[0] is None


def test_lane_utilisation_and_kernel_instance(tmp_path):
    """The counters file carries the trace instance's VALU lane utilisation
    from an SQ run; the bench names the template instance a shape runs."""
    b = _bench()
    tr = "void pv::k_trace_refill<false, 128, 21, unsigned short, false>(pv::VolumeParams)"
    refill = "void pv::k_trace_refill<false, 128, 21, unsigned short, true>(pv::VolumeParams)"
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0), (tr, 10.0), (refill, 9e9)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (tr, 20.0)])
    with open(tmp_path / "s.csv", "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value,Grid_Size\n")
        f.write(f'"{tr}",SQ_THREAD_CYCLES_VALU,3200,1\n"{tr}",SQ_ACTIVE_INST_VALU,100,1\n')
        f.write(f'"{refill}",SQ_THREAD_CYCLES_VALU,6400,1\n"{refill}",SQ_ACTIVE_INST_VALU,100,1\n')
    out = tmp_path / "c.txt"
    cfg_s = "16,4,1,2,21,128,0"
    t = b.write_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), cfg_s, sq_csv=str(tmp_path / "s.csv"))
    assert t == 10 * 1024 * 2 + 20 * 1024
    cfg = b.parse_trace_config(cfg_s)
    assert b.read_lane_utilisation(str(out), cfg) == 0.5
    assert b.read_lane_utilisation(str(out), {**cfg, "block_threads": 256}) is None
    assert b.trace_kernel_instance(cfg) == "k_trace_refill<false, 128, 21, unsigned short, false>"
    assert b.trace_kernel_instance({**cfg, "persistent": 0}) == "k_trace<false, 128, 21, false, unsigned short>"


def test_trace_config_string_round_trip():
    b = _bench()
    for s in ("4,4,4,0,21,256,0", "4,4,4,1,0,128,0", "4,4,4,2,21,256,0", "8,8,1,0,85,256,1"):
        c = b.parse_trace_config(s)
        assert b.config_string(c) == s
    assert b.parse_trace_config("4,4,4,2,21,256,0")["persistent"] == 2
