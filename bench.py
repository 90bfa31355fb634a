"""Benchmark of the probe-volume hot path on one MI355X.

One step = one pass of the whole path on the at-scale workload: the
16x8x16-probe volume (2048 probes, 256 rays per probe) over the procedural
50k-triangle city, FP16 maps with FP32 arithmetic, light moving on its
spline; the step updates the volume (ray directions, trace + shade, blend +
hysteresis + guard bands) and packs the delta for one client (change mask,
ordered compaction, XOR byte planes, index buffer, reference update), all on
the device. Inputs are resident in HBM before timing starts.

Prints one JSON line. ``value`` is primary probe-rays per second; the line
also carries probes/s, per-stage kernel times measured with HIP events on the
launch stream, the roofline of the dominant kernel (the trace), and the FP64
oracle timed on the host cores on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "probe-rays/s and probes updated/s at 1 GPU (plain vs batched/served); p50/p99 latency"

# Algorithmic FP32 work of the traversal, the method's own and not this
# kernel's instruction count: a ray/box slab test is about 20 FLOP (six plane
# distances, the entry max and exit min, the compare) and a node visit tests
# four child boxes; a ray/triangle test is about 30 FLOP. Decoding the
# quantized boxes, the watertight test's vertex rotation and the stack are
# this implementation's overhead and are not counted.
FLOP_PER_NODE_VISIT = 4 * 20
FLOP_PER_TRI_TEST = 30
PEAK_FP32_VECTOR = 157.3e12        # MI355X published FP32 vector peak (FLOP/s)
PEAK_HBM = 8.0e12                  # MI355X published HBM3E bandwidth (B/s)
PEAK_BF16_MFMA = 2.5e15            # MI355X published dense BF16 matrix peak (FLOP/s)


DEFAULT_LEGS = ("batched,served,served_below_capacity,served_tight_memory,served_sweep,encode,multi_bounce,codec,"
                "blend_paths,selection")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="oracle baseline budget: half on one thread, half on every core")
    ap.add_argument("--legs", default=DEFAULT_LEGS,
                    help="extra workloads reported in the same line (comma list, or 'none')")
    ap.add_argument("--served-seconds", type=float, default=10.0,
                    help="arrival window of the served leg (2000 requests/s)")
    ap.add_argument("--served-low-rate", type=float, default=300.0,
                    help="arrival rate of the second served run, below the measured capacity")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (tuned once, then reused)")
    ap.add_argument("--retune", action="store_true", help="measure every launch shape, ignoring caches")
    ap.add_argument("--trace-config", default=None,
                    help="pin the trace launch shape: bx,by,bz,persistent,top_nodes,block_threads,split_shadows")
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "k_trace_city_counters.txt"),
                    help="HBM byte counters of the trace kernel (rocprofv3 --pmc), used for roofline.traffic "
                         "when they were taken on the current kernel source and launch shape")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV", default=None,
                    help="no GPU work: print the mean per dispatch of every counter in rocprofv3 --pmc "
                         "counter_collection.csv files, per kernel")
    ap.add_argument("--write-kernel-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"), default=None,
                    help="per-kernel HBM bytes of an encode-leg run, scaled by its 1 GiB cache-flush copy")
    ap.add_argument("--sq-csv", default=None, help="with --write-counters: the SQ counter run's CSV")
    ap.add_argument("--write-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"), default=None,
                    help="no GPU work: turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, "
                         "WRITE_SIZE) of this bench run with --calibrate-copy into the counters file")
    ap.add_argument("--encode-frames", type=int, default=120)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default trace launch shape")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (reference kernel for HBM byte counters)")
    return ap.parse_args()


# sources of the trace kernel (its BVH layout included): the counters stay valid while these are unchanged
KERNEL_SOURCES = ("trace.hip", "trace_device.h", "device_common.h", "trace_layout.h", "bvh.cpp")
COPY_BYTES = 256 << 20             # the --calibrate-copy kernel reads and writes this many bytes


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_05875_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse_trace_config(s: str) -> dict:
    """bx,by,bz,persistent,top_nodes,block_threads,split_shadows -> trace launch config
    (persistent is the schedule number 0, 1 or 2, not a flag)."""
    v = [int(x) for x in s.split(",")]
    if len(v) != 7:
        raise ValueError(f"--trace-config needs 7 integers, got {s!r}")
    return {"brick": tuple(v[0:3]), "persistent": v[3], "top_nodes": v[4], "block_threads": v[5],
            "split_shadows": bool(v[6])}


def config_string(c) -> str:
    return ",".join(str(int(v)) for v in (*c["brick"], c["persistent"], c["top_nodes"], c["block_threads"],
                                          c["split_shadows"]))


def read_counters(path, trace_config):
    """roofline.traffic from the committed counters file: HBM bytes per
    trace launch, or None unless the file was made from the current kernel
    sources with the same launch shape."""
    try:
        kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None, "no counters file"
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    if kv.get("trace_config") != config_string(trace_config):
        return None, "counters were taken with another launch shape"
    ap = os.path.abspath(path)  # named relative to the repository when it lies inside it
    return float(kv["traffic_bytes_per_launch"]), os.path.relpath(ap, ROOT) if ap.startswith(ROOT + os.sep) else ap


def read_lane_utilisation(path, trace_config):
    """VALU lane utilisation of the trace kernel from the same counters file
    (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)), or None."""
    try:
        kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if (kv.get("source_sha256") != kernel_source_hash() or kv.get("trace_config") != config_string(trace_config)
            or "valu_lane_utilisation" not in kv):
        return None
    return float(kv["valu_lane_utilisation"])


def trace_kernel_instance(c) -> str:
    """The template instance a launch shape runs (16-bit stack entries)."""
    w, t = c["block_threads"], c["top_nodes"]
    if c["persistent"] == 0:
        return f"k_trace<false, {w}, {t}, false, unsigned short>"
    return f"k_trace_refill<false, {w}, {t}, unsigned short, {'true' if c['persistent'] == 1 else 'false'}>"




def is_trace_kernel(name: str, trace_config=None) -> bool:
    """The uninstrumented trace kernel of any schedule (not the counting
    variant, not the split-shadow passes); with a launch shape, only the
    template instance that shape runs (block size, staged nodes, schedule)."""
    k = name.replace("void ", "", 1)
    if trace_config is None:
        return k.startswith("pv::k_trace<false") or k.startswith("pv::k_trace_refill<false")
    c = parse_trace_config(trace_config) if isinstance(trace_config, str) else trace_config
    w, t = c["block_threads"], c["top_nodes"]
    if c["persistent"] == 0:
        return k.startswith(f"pv::k_trace<false, {w}, {t}, false,")
    refill = "true" if c["persistent"] == 1 else "false"
    return k.startswith(f"pv::k_trace_refill<false, {w}, {t},") and k.split("(")[0].endswith(f", {refill}>")


def write_counters(fetch_csv, write_csv, out, trace_config, legs: str = "none", sq_csv=None):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the trace kernel by
    what the same counters read for the run's largest device copy (the 256
    MiB calibration copy, or with the encode leg its 1 GiB cache flush), and
    write the counters file that read_counters() accepts."""
    copy_bytes = (1 << 30) if "encode" in legs else COPY_BYTES
    legs_args = "--legs none" if legs == "none" else f"--legs {legs} --encode-frames 4"
    import csv

    def load(path, counter):
        rows = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return rows

    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = load(path, counter)
        # the calibration copy is the runtime's blit kernel (the ceiling
        # kernels' own 1 GiB copy is not it)
        copy = max(v for k, v in rows if "copyBuffer" in k)
        trace = [v for k, v in rows if is_trace_kernel(k, trace_config)]
        res[counter] = {"copy_kib": copy, "scale": copy_bytes / (copy * 1024.0),
                        "trace_kib": sum(trace) / len(trace), "n": len(trace)}
    fetch = res["FETCH_SIZE"]["trace_kib"] * 1024 * res["FETCH_SIZE"]["scale"]
    write = res["WRITE_SIZE"]["trace_kib"] * 1024 * res["WRITE_SIZE"]["scale"]
    with open(out, "w") as f:
        f.write("# HBM traffic of the trace kernel (uninstrumented; k_trace or k_trace_refill by schedule) on the "
                "city workload\n")
        f.write("# counters per dispatch from rocprofv3 --pmc, one counter per run; each scaled by what the\n")
        f.write(f"# same counter reads for the run's largest device-to-device copy (reads and writes {copy_bytes} bytes)\n")
        f.write("# commands (MI355X host, repository root, TMPDIR=/tmp), then on any host:\n")
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            f.write(f"#   rocprofv3 --pmc {c} -f csv -d OUT_DIR/pmc_{c} -o pmc -- python3 bench.py --steps 3 "
                    f"--warmup 1 {legs_args} --no-cpu-baseline --calibrate-copy --trace-config {trace_config}\n")
        f.write("#   python3 bench.py --write-counters OUT_DIR/pmc_FETCH_SIZE/pmc_counter_collection.csv "
                f"OUT_DIR/pmc_WRITE_SIZE/pmc_counter_collection.csv OUT --trace-config {trace_config}"
                + ("" if legs == "none" else f" --legs {legs}") + "\n")
        for c, r in res.items():
            f.write(f"{c.lower()}_copy_kib: {r['copy_kib']:.1f}\n")
            f.write(f"{c.lower()}_scale: {r['scale']:.4f}\n")
            f.write(f"{c.lower()}_trace_kib_mean: {r['trace_kib']:.1f}\n")
            f.write(f"{c.lower()}_trace_dispatches: {r['n']}\n")
        if sq_csv:
            thr, act = [], []
            with open(sq_csv) as fs:
                for r in csv.DictReader(fs):
                    if is_trace_kernel(r["Kernel_Name"], trace_config):
                        if r["Counter_Name"] == "SQ_THREAD_CYCLES_VALU":
                            thr.append(float(r["Counter_Value"]))
                        elif r["Counter_Name"] == "SQ_ACTIVE_INST_VALU":
                            act.append(float(r["Counter_Value"]))
            f.write("#   lane utilisation from the SQ counter run: rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU "
                    "SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_INSTS_LDS "
                    "(same command), then --sq-csv OUT_DIR/pmc_SQ_WAVES/pmc_counter_collection.csv\n")
            f.write(f"valu_lane_utilisation: {sum(thr) / len(thr) / (64 * sum(act) / len(act)):.4f}\n")
        f.write(f"fetch_bytes_per_launch: {fetch:.0f}\n")
        f.write(f"write_bytes_per_launch: {write:.0f}\n")
        f.write(f"traffic_bytes_per_launch: {fetch + write:.0f}\n")
        f.write(f"trace_config: {trace_config}\n")
        f.write(f"source_sha256: {kernel_source_hash()}\n")
    return fetch + write


def write_kernel_counters(fetch_csv, write_csv, out, copy_bytes: int, title: str, commands):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every kernel, per launch
    grid, scaled by what the same counters read for the run's largest
    device copy (copy_bytes read and written), as bytes per launch."""
    import csv
    import collections
    res = {}
    scale = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        acc = collections.defaultdict(list)
        copy = 0.0
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if "copyBuffer" in r["Kernel_Name"]:
                    copy = max(copy, v)
                    continue
                acc[(r["Kernel_Name"].split("(")[0].replace("void ", ""), int(r["Grid_Size"]))].append(v)
        scale[counter] = (copy, copy_bytes / (copy * 1024.0))
        for k, v in acc.items():
            res.setdefault(k, {})[counter] = (len(v), sum(v) / len(v) * 1024 * scale[counter][1])
    with open(out, "w") as f:
        f.write(f"# {title}\n")
        f.write("# rocprofv3 --pmc, one counter per run, mean per dispatch; each counter scaled by what it\n")
        f.write(f"# reads for the run's largest device copy ({copy_bytes} bytes read and written)\n")
        f.write("# commands (MI355X host, repository root, TMPDIR=/tmp), then on any host:\n")
        for c in commands:
            f.write(f"#   {c}\n")
        for c, (kib, sc) in scale.items():
            f.write(f"# {c}: copy reads {kib:.1f} KiB, scale {sc:.4f}\n")
        f.write(f"# {'kernel':70s} {'grid':>9s} {'n':>4s} {'fetch_MB':>9s} {'write_MB':>9s} {'total_MB':>9s}\n")
        for (k, g) in sorted(res, key=lambda kg: -sum(x[1] for x in res[kg].values())):
            r = res[(k, g)]
            fe = r.get("FETCH_SIZE", (0, 0.0))
            wr = r.get("WRITE_SIZE", (0, 0.0))
            f.write(f"{k[:70]:70s} {g:9d} {max(fe[0], wr[0]):4d} {fe[1] / 1e6:9.2f} {wr[1] / 1e6:9.2f} "
                    f"{(fe[1] + wr[1]) / 1e6:9.2f}\n")
    return res


def summarize_counters(paths):
    """Mean per dispatch of each counter, per kernel (template arguments
    kept, parameters dropped) and launch grid, from rocprofv3 --pmc CSV
    files."""
    import csv
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                k = r["Kernel_Name"].split("(")[0].replace("void ", "") + f"  [grid {r['Grid_Size']}]"
                acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = []
    for k in sorted(acc):
        lines.append(k)
        for c in sorted(acc[k]):
            v = acc[k][c]
            lines.append(f"    {c:28s} dispatches {len(v):4d}  mean {sum(v) / len(v):.6g}")
    return "\n".join(lines)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, scene, path, budget_s: float):
    """The oracle as it stands on the host cores: full frames of the same
    workload (trace + shade, blend, pack), as many as fit half the budget
    (at least one), on one thread and then on every core."""

    import oracle
    import synth
    osc = oracle.OracleScene.from_scene(scene)

    def run(threads: int, budget: float):
        irr, vis = oracle.empty_maps(cfg)
        st = oracle.OracleClientState(cfg.n_probes)
        frames = 0
        t0 = time.perf_counter()
        while True:
            R = synth.rotation(13, frames)
            lights = scene.lights.copy()
            lights[0, :3] = path[frames % len(path)]
            rays = oracle.trace_shade(osc, cfg, R, lights, bounds=False, nthreads=threads)
            oracle.blend_update(cfg, oracle.ray_dirs(cfg.rays_per_probe, R), rays["L"], rays["r"], irr, vis,
                                first=(frames == 0), nthreads=threads)
            bi = irr.astype(np.float16).view(np.uint16)
            bv = vis.astype(np.float16).view(np.uint16)
            st.pack(bi, bv)
            frames += 1
            if time.perf_counter() - t0 > budget or frames >= 200:
                break
        dt = time.perf_counter() - t0
        return frames, dt, frames * cfg.n_probes * cfg.rays_per_probe / dt, frames * cfg.n_probes / dt

    cores = oracle.max_threads()
    f1, dt1, rays1, probes1 = run(1, budget_s / 2)
    fn, dtn, raysn, probesn = run(cores, budget_s / 2)
    return {"value": raysn, "unit": "probe-rays/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "probes_per_s": probesn,
            "sample": f"{fn} full frame(s) of the same workload (trace + shade, blend, pack), "
                      f"{dtn:.1f} s wall, OpenMP over probes on {cores} threads",
            "single_thread": {"value": rays1, "unit": "probe-rays/s", "cores": 1, "probes_per_s": probes1,
                              "sample": f"{f1} full frame(s), {dt1:.1f} s wall, one thread"}}


def leg_batched(ps, torch, reps: int):
    """Batched workload: 32 volumes (probes log-uniform 256-8192, rays from
    {64,128,256,512}, each over its own 5k-100k-triangle box scene), one
    batched update per frame (three launches for all volumes: directions,
    trace, blend), eager and as a captured graph, against the same volumes
    updated one by one on the plain path. Trace launch shapes are tuned: each
    plain volume on its own over every shape, the batched volumes per size
    bucket on the batched launch itself over the shapes the batched trace
    takes (probe brick and staged top nodes; stepped lanes in 256-thread
    blocks). Also timed: both
    paths at the default shape (4x4x4 bricks, 21 staged nodes), and the idle
    time between the three launches of a batched frame (what one persistent
    launch could remove at most)."""
    import synth
    from paper_2103_05875_amd import autotune
    specs = synth.batched_volumes(32, seed=20)
    ctx = ps.Context(0)
    scenes, plain, batched = [], [], []
    for s in specs:
        sc_syn = synth.box_field(s["n_tris"], seed=s["scene_seed"])
        sc = ps.Scene.from_synth(ctx, sc_syn)
        scenes.append(sc)
        a, b = ps.Volume(ctx, s["config"]), ps.Volume(ctx, s["config"])
        a.set_scene(sc)
        b.set_scene(sc)
        plain.append(a)
        batched.append(b)
    rays = sum(s["config"].n_probes * s["config"].rays_per_probe for s in specs)
    probes = sum(s["config"].n_probes for s in specs)
    stream = torch.cuda.current_stream()

    def run(f, which):
        rots = [synth.rotation(20 + i, f) for i in range(len(specs))]
        if which == "plain":
            for v, R in zip(plain, rots):
                v.update_probes(R, stream=stream)
        else:
            ps.update_probes_batched(batched, rots, stream=stream)

    def time_it(step):
        for f in range(2):
            step(f)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for f in range(2, 2 + reps):
            step(f)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return {"ms_per_frame": ms, "probe_rays_per_s": rays / (ms / 1e3), "probes_per_s": probes / (ms / 1e3)}

    out = {}
    # the default shape on both paths (the batched form before per-volume shapes)
    out["plain_default_shape"] = time_it(lambda f: run(f, "plain"))
    out["batched_default_shape"] = time_it(lambda f: run(f, "batched"))
    # per-volume tuned shapes
    t0 = time.perf_counter()
    shapes = []
    for s, a in zip(specs, plain):
        ta = autotune.tune(a, synth.rotation(99, 0), n_triangles=s["n_tris"], reps=2, cache=None, shipped=False)
        shapes.append({"probes": s["config"].n_probes, "rays": s["config"].rays_per_probe, "triangles": s["n_tris"],
                       "plain": {**ta["config"], "brick": list(ta["config"]["brick"])}})
    tb = autotune.tune_batched(batched, [synth.rotation(98 + i, 0) for i in range(len(specs))])
    for sh, b in zip(shapes, batched):
        c = b.get_trace_config()
        sh["batched"] = {"brick": list(c["brick"]), "top_nodes": c["top_nodes"]}
    batched_tuning = {"bucket": "log2 of the probe count", "timed_launches": tb["tried"],
                      "trace_ms_default_shape": tb["default_ms"], "trace_ms_tuned": tb["ms"],
                      "choices": {str(k): {"brick": list(c["brick"]), "top_nodes": c["top_nodes"]}
                                  for k, c in sorted(tb["choices"].items())}}
    tune_s = time.perf_counter() - t0
    # the trial runs advanced the two sets by different frame counts: start
    # both from the plain volume's maps
    for a, b in zip(plain, batched):
        irr, vis, fr = a.read_maps()
        b.set_maps(irr, vis, fr)
    for which in ("plain", "batched"):
        out[which] = time_it(lambda f, w=which: run(f, w))
    # same frames on both sets since the tuning
    same = all(np.array_equal(a.read_maps()[0], b.read_maps()[0]) and np.array_equal(a.read_maps()[1], b.read_maps()[1])
               for a, b in zip(plain, batched))
    graph = ps.BatchGraph(batched)
    out["graph"] = time_it(lambda f: graph.launch([synth.rotation(20 + i, f) for i in range(len(specs))],
                                                  stream=stream))
    graph.close()
    # the batched frame's three launches by events: their sum against the
    # frame (the gaps are what a single persistent launch could remove)
    ctx.set_timing(True)
    ctx.stage_times()
    for f in range(reps):
        run(100 + f, "batched")
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.set_timing(False)
    kern = sum(st[k][0] for k in ("raydirs", "batched", "blend")) / reps
    out.update({"volumes": len(specs), "probes": probes, "probe_rays": rays, "bit_identical_to_plain": bool(same),
                "shapes": shapes, "tuning_s": tune_s, "batched_tuning": batched_tuning,
                "speedup": out["plain"]["ms_per_frame"] / out["batched"]["ms_per_frame"],
                "graph_speedup": out["plain"]["ms_per_frame"] / out["graph"]["ms_per_frame"],
                "tuned_over_default_batched": out["batched_default_shape"]["ms_per_frame"]
                / out["batched"]["ms_per_frame"],
                "launches_ms": {"directions": st["raydirs"][0] / reps, "trace": st["batched"][0] / reps,
                                "blend": st["blend"][0] / reps},
                "gaps_ms": max(0.0, out["batched"]["ms_per_frame"] - kern)})
    for h in plain + batched + scenes:
        h.close()
    ctx.close()
    return out


def leg_served(ps, duration_s: float, rate_hz: float = 2000.0, budget_frac: float = 1.0, with_plain: bool = True):
    """Served workload: 64 clients (probes log-uniform 512-16384, rays from
    {64,128,256}) over one shared 200k-triangle scene, Poisson requests at
    2000/s, continuous batching with HBM admission; against the same trace
    served one request at a time."""
    import synth
    from paper_2103_05875_amd import serve
    cfgs = synth.served_clients(64, seed=30)
    scene_syn = synth.box_field(200_000, seed=31)
    arrivals = synth.poisson_arrivals(rate_hz, duration_s, len(cfgs), seed=30)
    path = synth.light_path(12, 240)

    def make():
        fo = [0] * len(cfgs)
        reqs = []
        for t, c in arrivals:
            l = scene_syn.lights.copy()
            l[0, :3] = path[fo[c] % 240]
            reqs.append(serve.Request(c, synth.rotation(300 + c, fo[c]), l, t))
            fo[c] += 1
        return reqs
    ctx = ps.Context(0)
    scene = ps.Scene.from_synth(ctx, scene_syn)
    total_fp = sum(ps.volume_footprint(c) + ps.client_footprint(c) for c in cfgs)
    budget = int(budget_frac * total_fp) + (1 << 20)
    # requests complete with the packet in pinned host memory; only headers
    # (sizes, sequence, payload checksum) are kept for the comparison
    srv = serve.Server(ctx, scene, cfgs, hbm_budget=budget, n_streams=3, max_batch=32, keep_packets=False)
    t0 = time.perf_counter()
    served = srv.run(make(), timeout_s=120.0)
    span = max(r.done for r in served)
    srv.close()
    plain = serve.serve_plain(ctx, scene, cfgs, make(), timeout_s=240.0, keep_packets=False) if with_plain else None
    span_p = max(r.done for r in plain) if plain else None
    probes = sum(cfgs[r.client].n_probes for r in served)
    rays = sum(cfgs[r.client].n_probes * cfgs[r.client].rays_per_probe for r in served)
    same = plain is None or all(a.header == b.header and a.nbytes == b.nbytes
                                for a, b in zip(sorted(served, key=lambda r: r.arrival),
                                                sorted(plain, key=lambda r: r.arrival)))
    out = {"clients": len(cfgs), "requests": len(served), "arrival_rate_hz": rate_hz, "duration_s": duration_s,
           "offered_probes_per_s": probes / duration_s, "hbm_budget_bytes": budget, "footprint_all_bytes": total_fp,
           "served": dict(serve.latency_stats(served), probes_per_s=probes / span, probe_rays_per_s=rays / span,
                          mean_batch=float(np.mean([r.batch_size for r in served])),
                          evictions=srv.evictions, admissions=srv.admissions),
           "plain": None if plain is None else dict(serve.latency_stats(plain), probes_per_s=probes / span_p,
                                                    probe_rays_per_s=rays / span_p),
           "packets_identical": bool(same)}
    if plain is not None and span_p > 1.1 * duration_s:
        # the plain path fell behind, so its rate is its capacity: offered
        # load as a fraction of it
        out["offered_over_plain_capacity"] = out["offered_probes_per_s"] / out["plain"]["probes_per_s"]
    scene.close()
    ctx.close()
    return out


def leg_served_sweep(ps, rates=(300.0, 600.0, 1000.0, 1400.0, 1800.0), duration_s: float = 1.5):
    """The served workload at several arrival rates (no plain run): latency
    percentiles against offered load, to place the knee of p99."""
    rows = []
    for r in rates:
        o = leg_served(ps, duration_s, rate_hz=r, with_plain=False)
        rows.append({"arrival_rate_hz": r, "offered_probes_per_s": o["offered_probes_per_s"],
                     "served_probes_per_s": o["served"]["probes_per_s"], "p50_ms": o["served"]["p50_ms"],
                     "p99_ms": o["served"]["p99_ms"], "mean_batch": o["served"]["mean_batch"]})
    return {"duration_s": duration_s, "rows": rows}


def leg_encode(ps, torch, frames: int):
    """Encode path: 32x16x32 = 16,384 probes, 256 rays, 200k-triangle field
    with 4 moving occluders and a moving light; each frame updates and packs
    with tau = 1/1024 for both textures, entropy-codes the packet on the
    device, and a receiver (the client side) decodes and applies every
    container on the device; the receiver's tiles equal the server's record
    of what the client holds at every 20th frame. Pack throughput against
    HBM; packet and coded sizes."""
    import synth
    cfg = synth.config("encode")
    scene_syn = synth.box_field(200_000, seed=40, n_moving=4)
    ctx = ps.Context(0)
    sc = ps.Scene.from_synth(ctx, scene_syn)
    path = synth.light_path(12, frames)
    # trace launch shape: the shipped table's entry for this workload, else
    # measured on a scratch volume of the same shape
    from paper_2103_05875_amd import autotune
    scratch = ps.Volume(ctx, cfg)
    scratch.set_scene(sc)
    l0 = scene_syn.lights.copy()
    l0[0, :3] = path[0]
    tuned = autotune.tune(scratch, synth.rotation(41, 0), l0, n_triangles=scene_syn.n_triangles, cache=None)
    scratch.close()
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    c = tuned["config"]
    vol.set_trace_config(c["brick"], c["persistent"], c["top_nodes"], c["block_threads"], c["split_shadows"])
    cl = ps.Client(vol, 0)
    rx = ps.Receiver(ctx, cfg.n_probes)   # the client side: applies each packet on the device
    stream = torch.cuda.current_stream()
    ctx.set_timing(True)
    ctx.stage_times()
    sent_bytes, coded_bytes, changed, ok = 0, 0, [], True
    for f in range(frames):
        sc.set_dynamic(synth.moving_occluders(40, f, 4), stream=stream)
        l = scene_syn.lights.copy()
        l[0, :3] = path[f]
        vol.update_probes(synth.rotation(41, f), l, stream=stream)
        if f == frames - 1:
            saved = cl.read_state()   # the client before the last pack (timed again below)
        cl.pack_delta(1.0 / 1024, 1.0 / 1024, stream=stream)
        pkt = cl.packet_download(stream=stream)
        sent_bytes += len(pkt)
        cl.entropy_encode(stream=stream)
        coded = cl.entropy_download(stream=stream)
        coded_bytes += len(coded)
        rx.apply_compressed(coded, stream=stream)
        if f % 20 == 19 or f == frames - 1:
            ok &= rx.status() == (0, f)
            ri, rv, _ = cl.read_state()
            gi, gv = rx.read_maps()
            ok &= bool(np.array_equal(gi[:, :, 1:-1, 1:-1].reshape(cfg.n_probes, 3, -1), ri))
            ok &= bool(np.array_equal(gv[:, :, 1:-1, 1:-1].reshape(cfg.n_probes, 2, -1), rv))
        mi, mv = cl.read_masks()
        changed.append((int(mi.sum()), int(mv.sum())))
    st = ctx.stage_times()
    ctx.set_timing(False)
    P = cfg.n_probes
    pack_keys = ("pack_mask", "pack_scan", "pack_compact", "pack_finish")
    pack_ms = sum(st[k][0] for k in pack_keys) / frames

    # the last frame's pack again, warm and cold (1 GiB streamed through the
    # caches first; the maps, reference and packet, about 80 MB, would
    # otherwise sit in the 256 MB last-level cache): the client's state before
    # that pack is restored before every repetition
    flush_a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    flush_b = torch.empty_like(flush_a)

    def pack_again(cold: bool) -> float:
        times = []
        for _ in range(6):
            cl.set_state(*saved)
            if cold:
                flush_b.copy_(flush_a)
            torch.cuda.synchronize()
            ctx.set_timing(True)
            ctx.stage_times()
            cl.pack_delta(1.0 / 1024, 1.0 / 1024, stream=stream)
            s2 = ctx.stage_times()
            ctx.set_timing(False)
            times.append(sum(s2[k][0] for k in pack_keys))
        return float(np.median(times[1:]))

    warm_ms, cold_ms = pack_again(False), pack_again(True)
    del flush_a, flush_b
    ci, cv = changed[-1]
    last_bytes = P * 1408 * 2 + (ci * 384 + cv * 1024) * 2 + P * 2
    ki = np.mean([c[0] for c in changed])
    kv = np.mean([c[1] for c in changed])
    pack_bytes = P * 1408 * 2 + (ki * 384 + kv * 1024) * 2 + P * 2
    upd_ms = (st["raydirs"][0] + st["trace"][0] + st["blend"][0]) / frames
    per_kernel = {k: st[k][0] / max(st[k][1], 1) for k in ("pack_mask", "pack_scan", "pack_compact", "pack_finish",
                                                            "trace", "blend")}
    out = {"probes": P, "frames": frames, "round_trip_bit_exact": bool(ok),
           "trace_config": {**c, "brick": list(c["brick"])}, "trace_config_source": tuned["source"],
           "entropy_encode_ms": st["entropy"][0] / frames,
           "client_decode_and_unpack_ms": st["unpack"][0] / frames,
           "coded_bytes_per_frame": coded_bytes / frames,
           "coded_Mbps_at_10Hz": coded_bytes / frames * 8 * 10 / 1e6,
           "entropy_ratio": sent_bytes / max(coded_bytes, 1), "mean_changed_irr": ki,
           "kernel_ms": per_kernel,
           "mean_changed_vis": kv, "packet_bytes_per_frame": sent_bytes / frames,
           "Mbps_at_10Hz": sent_bytes / frames * 8 * 10 / 1e6,
           "update_ms": upd_ms, "probe_rays_per_s": P * cfg.rays_per_probe / (upd_ms / 1e3),
           "pack_last_frame": {"bytes": last_bytes, "warm_ms": warm_ms, "cold_ms": cold_ms,
                               "warm_hbm_frac": last_bytes / (warm_ms / 1e3) / PEAK_HBM,
                               "cold_hbm_frac": last_bytes / (cold_ms / 1e3) / PEAK_HBM},
           "pack_ms": pack_ms, "pack_hbm_GBps": pack_bytes / (pack_ms / 1e3) / 1e9,
           "pack_hbm_frac": pack_bytes / (pack_ms / 1e3) / PEAK_HBM}
    for h in (rx, cl, vol, sc, ctx):
        h.close()
    return out


def leg_codec(ps, torch, reps: int = 20):
    """Codec surfaces (Sec. 3.3) of the encode-size volume (16,384 probes,
    FP16 maps, 128 tiles per atlas row): encode and decode times and their
    algorithmic bytes (interiors read, planes written; planes read, codes and
    bit patterns written) against HBM."""
    import synth
    P, C = 16384, 128
    irr, vis = synth.random_fp16_maps(P, 8, 16, seed=60, scale=3.0)
    cfg = synth.config("encode")
    ctx = ps.Context(0)
    vol = ps.Volume(ctx, cfg)
    vol.set_maps(irr, vis, 0)
    stream = torch.cuda.current_stream()
    w, h, wv, hv = ps.yuv_dims(P, C)
    ip, vp = vol.encode_yuv(2.0, C, stream=stream)
    codes, vb = ps.decode_yuv(ctx, P, C, ip, vp, stream=stream)
    torch.cuda.synchronize()
    ok = bool(np.array_equal(vb.cpu().numpy().view(np.uint16), vis[:, :, 1:-1, 1:-1].reshape(P, 2, 256)))
    # outputs reused, so that the loops time the kernels, not allocation
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(reps):
        vol.encode_yuv(2.0, C, stream=stream, out=(ip, vp))
    ev[1].record(stream)
    for _ in range(reps):
        ps.decode_yuv(ctx, P, C, ip, vp, stream=stream, out=(codes, vb))
    ev[2].record(stream)
    torch.cuda.synchronize()
    enc_ms = ev[0].elapsed_time(ev[1]) / reps
    dec_ms = ev[1].elapsed_time(ev[2]) / reps
    interiors = P * (192 + 512) * 2
    planes = 3 * w * h * 2 + 3 * wv * hv
    dec_out = P * 64 * 4 + P * 512 * 2
    out = {"probes": P, "tiles_per_row": C, "irr_planes": [3, h, w], "vis_planes": [3, hv, wv],
           "visibility_round_trip_bit_exact": ok,
           "encode_ms": enc_ms, "encode_GBps": (interiors + planes) / (enc_ms / 1e3) / 1e9,
           "decode_ms": dec_ms, "decode_GBps": (planes + dec_out) / (dec_ms / 1e3) / 1e9}
    out["encode_hbm_frac"] = out["encode_GBps"] * 1e9 / PEAK_HBM
    out["decode_hbm_frac"] = out["decode_GBps"] * 1e9 / PEAK_HBM
    for hnd in (vol, ctx):
        hnd.close()
    return out


def leg_blend_paths(ps, torch, reps: int = 20):
    """The blend (weighted means, hysteresis, guard bands) of volumes of
    512, 1,024, 2,048 (the city), 4,096, 8,192 and 16,384 (the encode
    workload) probes, 256 rays (and 64 rays at 1,024 and 2,048 probes),
    FP16 maps, on every blend path, from the same seeded ray
    records: event time of the blend kernel, its algorithmic bytes (ray
    records, stored interiors read, tiles written) against HBM and its FLOP
    (2 per weight x record term) against the peak of its unit (BF16x3
    counts its three products against the BF16 matrix peak; FP32 matrix
    and vector FMAs against the FP32 peak)."""
    import synth
    out = {}
    ctx = ps.Context(0)
    stream = torch.cuda.current_stream()
    for name, (grid, n) in (("512", ((8, 8, 8), 256)), ("1024", ((16, 8, 8), 256)), ("1024_n64", ((16, 8, 8), 64)),
                            ("city", ((16, 8, 16), 256)), ("city_n64", ((16, 8, 16), 64)),
                            ("4096", ((16, 16, 16), 256)), ("8192", ((32, 16, 16), 256)),
                            ("encode", ((32, 16, 32), 256))):
        cfg = synth.VolumeConfig(*grid, (0, 0, 0), (1, 1, 1), n, fp16=True, max_distance=3.0)
        P = cfg.n_probes
        vol = ps.Volume(ctx, cfg)
        L, r = synth.synthetic_rays(P, n, seed=7, max_distance=3.0)
        dev = torch.from_numpy(np.concatenate([L, r[..., None]], axis=-1).astype(np.float32)).cuda()
        torch.cuda.synchronize()
        R = synth.rotation(8, 0)
        row = {}
        for mode in ("tiles", "f32", "bf16x3", "valu", "bf16x6"):
            vol.set_blend_mode(mode)
            for _ in range(3):
                vol.blend_rays(R, dev.data_ptr(), stream=stream)
            torch.cuda.synchronize()
            ctx.set_timing(True)
            ctx.stage_times()
            for _ in range(reps):
                vol.blend_rays(R, dev.data_ptr(), stream=stream)
            torch.cuda.synchronize()
            st = ctx.stage_times()
            ctx.set_timing(False)
            ms = st["blend"][0] / max(st["blend"][1], 1)
            bytes_ = P * (16 * n + (192 + 512) * 2 + (300 + 648) * 2)
            flop = P * 1408 * n
            peak = (PEAK_BF16_MFMA / 3 if mode == "bf16x3" else PEAK_BF16_MFMA / 6 if mode == "bf16x6"
                    else PEAK_FP32_VECTOR)
            row[mode] = {"ms": ms, "table_ms": st["raydirs"][0] / max(st["raydirs"][1], 1),
                         "hbm_frac": bytes_ / (ms / 1e3) / PEAK_HBM, "mfma_frac": flop / (ms / 1e3) / peak}
        out[name] = {"probes": P, "rays_per_probe": n, "paths": row}
        del dev
        vol.close()
    ctx.close()
    return out


def street_eye(scene, height: float = 1.7):
    """A client position at street level in the box city: the first point of a
    coarse grid over the city that lies outside every box (boxes are the
    12-triangle groups after the 2 ground triangles)."""
    tris = scene.triangles()
    boxes = tris[2:].reshape(-1, 12, 3, 3)
    lo, hi = boxes.min(axis=(1, 2)), boxes.max(axis=(1, 2))
    for x in np.linspace(5.3, 58.7, 24):
        for z in np.linspace(5.1, 58.9, 24):
            pt = np.array([x, height, z])
            if not np.any(np.all((pt > lo - 0.5) & (pt < hi + 0.5), axis=1)):
                return tuple(float(v) for v in pt)
    return (32.0, 12.0, 32.0)


def leg_selection(ps, torch, cfg, scene, frames, trace_config):
    """Probe selection on the city workload (Sec. 3.4): the volume classifies
    its probes every update; client A culls to a spherical view from a street
    position, client B sends every active changed probe; per-frame sent
    probes of both (tau = 0) and the cost of classification and view."""
    import dataclasses
    scfg = dataclasses.replace(cfg, classify=True)
    ctx = ps.Context(0)
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, scfg)
    vol.set_scene(sc)
    if trace_config:
        c = trace_config
        vol.set_trace_config(c["brick"], c["persistent"], c["top_nodes"], c["block_threads"], c["split_shadows"])
    a, bcl = ps.Client(vol, client_id=1), ps.Client(vol, client_id=2)
    stream = torch.cuda.current_stream()
    eye = street_eye(scene)
    ctx.set_timing(True)
    ctx.stage_times()
    a.set_view(eye, 16384, stream=stream)
    view_ms = ctx.stage_times()["select"][0]
    sent_a, sent_b, bytes_a, coded_a = [], [], [], []
    for i, (R, l) in enumerate(frames):
        vol.update_probes(R, l, stream=stream)
        a.pack_delta(0.0, 0.0, stream=stream)
        ma = [m.sum() for m in a.read_masks()]
        if i > 0:
            bytes_a.append(len(a.packet_download(stream=stream)))
            a.entropy_encode(stream=stream)
            coded_a.append(len(a.entropy_download(stream=stream)))
        bcl.pack_delta(0.0, 0.0, stream=stream)
        mb = [m.sum() for m in bcl.read_masks()]
        if i > 0:   # frame 0 sends the initial state
            sent_a.append(ma)
            sent_b.append(mb)
    st = ctx.stage_times()
    ctx.set_timing(False)
    P = scfg.n_probes
    active = vol.read_active()
    view = a.read_view()
    sa, sb = np.mean(sent_a, axis=0), np.mean(sent_b, axis=0)
    out = {"eye": eye, "view_rays": 16384, "view_ms": view_ms, "probes": P,
           "active": int(active.sum()), "in_view": int(view.sum()), "active_in_view": int((active & view).sum()),
           "classify_ms": st["select"][0] / max(st["select"][1], 1),
           "sent_per_frame_view": {"irr": float(sa[0]), "vis": float(sa[1])},
           "sent_per_frame_all_active": {"irr": float(sb[0]), "vis": float(sb[1])},
           "reduction_vs_active": 1.0 - float((sa[0] + sa[1]) / max(2 * active.sum(), 1)),
           "view_packet_Mbps_at_10Hz": float(np.mean(bytes_a)) * 8 * 10 / 1e6,
           "view_coded_Mbps_at_10Hz": float(np.mean(coded_a)) * 8 * 10 / 1e6,
           "view_coded_Mbps_at_60Hz": float(np.mean(coded_a)) * 8 * 60 / 1e6}
    for h in (a, bcl, vol, sc, ctx):
        h.close()
    return out


def leg_multi_bounce(ps, torch, cfg, scene, frames, trace_config):
    """The headline city step with the second bounce on: each hit adds its
    albedo times the query of the stored maps (one more launch per update).
    Reports the bounce kernel's time and the step time beside the plain
    step's stage times."""
    import dataclasses
    mcfg = dataclasses.replace(cfg, multi_bounce=True)
    ctx = ps.Context(0)
    sc = ps.Scene.from_synth(ctx, scene)
    vol = ps.Volume(ctx, mcfg)
    vol.set_scene(sc)
    if trace_config:
        c = trace_config
        vol.set_trace_config(c["brick"], c["persistent"], c["top_nodes"], c["block_threads"], c["split_shadows"])
    cl = ps.Client(vol, client_id=0)
    stream = torch.cuda.current_stream()
    W = min(5, len(frames) // 2)
    for R, l in frames[:W]:
        vol.update_probes(R, l, stream=stream)
        cl.pack_delta(0.0, 0.0, stream=stream)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for R, l in frames[W:]:
        vol.update_probes(R, l, stream=stream)
        cl.pack_delta(0.0, 0.0, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    K = len(frames) - W
    ms = t0.elapsed_time(t1) / K
    ctx.set_timing(True)
    ctx.stage_times()
    for R, l in frames[W:]:
        vol.update_probes(R, l, stream=stream)
        cl.pack_delta(0.0, 0.0, stream=stream)
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.set_timing(False)
    rays = mcfg.n_probes * mcfg.rays_per_probe
    out = {"ms_per_step": ms, "probe_rays_per_s": rays / (ms / 1e3),
           "stage_ms": {k: v[0] / max(v[1], 1) for k, v in st.items() if v[1]}}
    for h in (cl, vol, sc, ctx):
        h.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library runs the update and pack on a single GPU and has no cross-GPU exchange)", file=sys.stderr)
        sys.exit(2)
    if args.write_kernel_counters:
        fc, wc, out = args.write_kernel_counters
        cmd = ("python3 bench.py --steps 3 --warmup 1 --legs encode --encode-frames 4 --no-cpu-baseline "
               "--calibrate-copy" + (f" --trace-config {args.trace_config}" if args.trace_config else ""))
        write_kernel_counters(fc, wc, out, 1 << 30,
                              "HBM traffic per launch of every kernel of the city step and the encode leg (4 frames)",
                              [f"rocprofv3 --pmc {c} -f csv -d OUT_DIR/pmc_{c} -o pmc -- {cmd}"
                               for c in ("FETCH_SIZE", "WRITE_SIZE")]
                              + ["python3 bench.py --write-kernel-counters OUT_DIR/pmc_FETCH_SIZE/pmc_counter_collection.csv "
                                 "OUT_DIR/pmc_WRITE_SIZE/pmc_counter_collection.csv OUT"
                                 + (f" --trace-config {args.trace_config}" if args.trace_config else "")])
        print(f"-> {out}")
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters))
        return
    if args.write_counters:
        if not args.trace_config:
            sys.exit("--write-counters needs the --trace-config the counters were taken with")
        t = write_counters(*args.write_counters, trace_config=args.trace_config,
                           legs="none" if args.legs == DEFAULT_LEGS else args.legs, sq_csv=args.sq_csv)
        print(f"trace kernel HBM traffic {t / 1e6:.2f} MB per launch -> {args.write_counters[2]}")
        return
    import numpy as np
    import torch

    import synth
    import paper_2103_05875_amd as ps

    cfg = synth.config("city")
    scene = synth.box_city()
    K, W = args.steps, args.warmup
    path = synth.light_path(12, 60)
    frames = []
    for f in range(K + W):
        l = scene.lights.copy()
        l[0, :3] = path[f % 60]
        frames.append((synth.rotation(13, f), l))

    print(f"bench: city workload, {cfg.n_probes} probes x {cfg.rays_per_probe} rays, "
          f"{scene.n_triangles} triangles; warmup {W}, steps {K}", file=sys.stderr, flush=True)
    ctx = ps.Context(0)
    sc = ps.Scene.from_synth(ctx, scene)
    tuned = None
    if args.trace_config:
        tuned = {"config": parse_trace_config(args.trace_config), "ms": float("nan"), "tried": 0,
                 "source": "pinned"}
    elif not args.no_autotune:
        from paper_2103_05875_amd import autotune
        scratch = ps.Volume(ctx, cfg)
        scratch.set_scene(sc)
        tuned = autotune.tune(scratch, *frames[0], n_triangles=scene.n_triangles, cache=args.tune_cache,
                              force=args.retune, frames=frames[:8], reps=2)
        scratch.close()
        print(f"bench: trace launch {tuned['config']} ({tuned['source']}, {tuned['ms']:.3f} ms)",
              file=sys.stderr, flush=True)
    vol = ps.Volume(ctx, cfg)
    vol.set_scene(sc)
    if tuned:
        c = tuned["config"]
        vol.set_trace_config(c["brick"], c["persistent"], c["top_nodes"], c["block_threads"], c["split_shadows"])
    cl = ps.Client(vol, client_id=0)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(i):
        R, l = frames[i]
        vol.update_probes(R, l, stream=stream)
        cl.pack_delta(0.0, 0.0, stream=stream)

    for i in range(W):
        step(i)
    torch.cuda.synchronize()

    # timed region (clean: no instrumentation)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for i in range(W, W + K):
        step(i)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = t_start.elapsed_time(t_end)
    ms_per_step = max(gpu_ms, wall * 1e3) / K
    rays = cfg.n_probes * cfg.rays_per_probe
    value = rays * K / (ms_per_step * K / 1e3)
    print(f"bench: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # per-step distribution: each step of the same frames bracketed by
    # events on the launch stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for i, (a, b) in zip(range(W, W + K), evs):
        a.record(stream)
        step(i)
        b.record(stream)
    torch.cuda.synchronize()
    per_step = np.array([a.elapsed_time(b) for a, b in evs])
    step_dist = {"p50_ms": float(np.percentile(per_step, 50)), "p90_ms": float(np.percentile(per_step, 90)),
                 "min_ms": float(per_step.min()), "max_ms": float(per_step.max())}

    # same steps again with every kernel bracketed by HIP events on its stream
    ctx.set_timing(True)
    ctx.stage_times()
    for i in range(W, W + K):
        step(i)
    torch.cuda.synchronize()
    stages = ctx.stage_times()
    ctx.set_timing(False)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}

    # the same steps with the packet handed to the host each step (the
    # boundary's host buffer: header, then payload over PCIe); reported
    # beside the value, never as it
    torch.cuda.synchronize()
    pkt_bytes = 0
    wall0 = time.perf_counter()
    for i in range(W, W + K):
        step(i)
        pkt_bytes += len(cl.packet_download(stream=stream))
    torch.cuda.synchronize()
    pcie_ms = (time.perf_counter() - wall0) * 1e3 / K
    pcie = {"ms_per_step": pcie_ms, "probe_rays_per_s": cfg.n_probes * cfg.rays_per_probe / (pcie_ms / 1e3),
            "packet_bytes_mean": pkt_bytes / K}

    # algorithmic traversal work of the same frames (instrumented trace)
    node_visits = tri_tests = shadow = 0
    for i in range(W, W + K):
        c = vol.trace_counts(*frames[i])
        node_visits += c["node_visits"]
        tri_tests += c["tri_tests"]
        shadow += c["shadow_rays"]
    flop_per_launch = (node_visits * FLOP_PER_NODE_VISIT + tri_tests * FLOP_PER_TRI_TEST) / K
    # the traversal is k_trace, plus k_shadow and k_shade when shadow rays are split out
    trace_s = (stage_ms["trace"] + stage_ms["shadow"] + stage_ms["shade"]) / 1e3
    achieved = flop_per_launch / trace_s if trace_s > 0 else 0.0

    traffic, traffic_src = read_counters(args.counters, vol.get_trace_config())

    # attainable ceilings of plain kernels on this device, beside the
    # data-sheet peaks the fractions are quoted against
    ceil = {"hbm_copy_GBps": ctx.measure_ceiling(ps.native.PV_CEIL_COPY) / 1e9,
            "fma_f32_TFLOPs": ctx.measure_ceiling(ps.native.PV_CEIL_FMA_F32) / 1e12,
            "mfma_f32_TFLOPs": ctx.measure_ceiling(ps.native.PV_CEIL_MFMA_F32) / 1e12}

    # HBM figures of the blend and pack kernels (algorithmic bytes)
    P, n = cfg.n_probes, cfg.rays_per_probe
    blend_bytes = P * (16 * n + (192 + 512) * 2 + (300 + 648) * 2)
    blend_flop = P * 1408 * n
    mi, mv = cl.read_masks()
    k_changed = (int(mi.sum()) + int(mv.sum())) / 2.0
    pack_bytes = P * 1408 * 2 + (int(mi.sum()) * 384 + int(mv.sum()) * 1024) * 2 + P * 2
    pack_ms = stage_ms["pack_mask"] + stage_ms["pack_scan"] + stage_ms["pack_compact"] + stage_ms["pack_finish"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "probe-rays/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "city: 16x8x16 probes, 256 rays/probe, 50k-triangle procedural city, FP16 maps, "
                               "moving light; step = full update + delta pack for one client (tau = 0)",
                   "probes": P, "rays_per_probe": n, "triangles": scene.n_triangles,
                   "blend_path": vol.get_blend_mode(),
                   "arithmetic": "trace and shading FP32; blend products of FP32 operands split into three BF16 "
                                 "parts (six products, FP32 accumulation, about 2^-25 relative per term, the "
                                 "FP32 parity bars) when blend_path is bf16x6; FP16 maps"},
        "probes_per_s": P * 1e3 / ms_per_step,
        "trace_config": vol.get_trace_config(),
        "autotune": None if tuned is None else {"source": tuned["source"], "tried": tuned["tried"],
                                                 "best_ms": tuned["ms"], "top5": tuned.get("ranking")},
        "stage_ms": stage_ms,
        "roofline": {"bound": "alu", "kernel": trace_kernel_instance(vol.get_trace_config()),
                     "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "traffic_source": traffic_src,
                     "valu_lane_utilisation": read_lane_utilisation(args.counters, vol.get_trace_config()),
                     "trace_ms": trace_s * 1e3,
                     "flop_per_launch": flop_per_launch, "node_visits_per_ray": node_visits / (K * rays),
                     "tri_tests_per_ray": tri_tests / (K * rays), "shadow_rays_per_ray": shadow / (K * rays),
                     "frac_of_attainable_fma": achieved / (ceil["fma_f32_TFLOPs"] * 1e12)},
        "ceilings": ceil,
        "pcie_inclusive": pcie,
        "step_ms_distribution": step_dist,
        "blend": {"ms": stage_ms["blend"], "hbm_GBps": blend_bytes / (stage_ms["blend"] / 1e3) / 1e9 if stage_ms["blend"] else None,
                  "hbm_frac": blend_bytes / (stage_ms["blend"] / 1e3) / PEAK_HBM if stage_ms["blend"] else None,
                  "alu_frac": blend_flop / (stage_ms["blend"] / 1e3) / PEAK_FP32_VECTOR if stage_ms["blend"] else None},
        "pack": {"ms": pack_ms, "changed_probes": k_changed,
                 "hbm_GBps": pack_bytes / (pack_ms / 1e3) / 1e9 if pack_ms else None,
                 "hbm_frac": pack_bytes / (pack_ms / 1e3) / PEAK_HBM if pack_ms else None},
        "paper_context": "5.63 ms per full-volume update (mean of 2048/4096/8192-probe scenes, 256 rays/probe) on a "
                         "Quadro RTX 8000 with RT cores, i.e. about 0.22 G probe-rays/s and 0.85 M probes/s; "
                         "different scenes and hardware, so not a ratio",
    }
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    for h in (cl, vol, sc, ctx):
        h.close()
    runners = {"batched": lambda: leg_batched(ps, torch, reps=5),
               "served": lambda: leg_served(ps, args.served_seconds),
               "served_below_capacity": lambda: leg_served(ps, 2.0, rate_hz=args.served_low_rate),
               "served_sweep": lambda: leg_served_sweep(ps),
               "served_tight_memory": lambda: leg_served(ps, 2.0, rate_hz=args.served_low_rate, budget_frac=0.6,
                                                         with_plain=False),
               "encode": lambda: leg_encode(ps, torch, args.encode_frames),
               "codec": lambda: leg_codec(ps, torch),
               "blend_paths": lambda: leg_blend_paths(ps, torch),
               "selection": lambda: leg_selection(ps, torch, cfg, scene, frames, tuned["config"] if tuned else None),
               "multi_bounce": lambda: leg_multi_bounce(ps, torch, cfg, scene, frames,
                                                        tuned["config"] if tuned else None)}
    for name in legs:
        print(f"bench: {name} leg", file=sys.stderr, flush=True)
        try:
            out[name] = runners[name]()
        except Exception as e:  # a failed leg is reported, the headline line is still printed
            import traceback
            traceback.print_exc()
            out[name] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, scene, path, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
