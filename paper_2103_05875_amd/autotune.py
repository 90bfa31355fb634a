"""Autotuner for the trace launch shape.

Every launch shape computes bit-identical results; only speed differs. The
tuner times each candidate (probe brick of a wavefront packet, persistent
grid with per-XCD work queues or not, BVH nodes staged in LDS, block size)
on the caller's own volume, scene and frame, with HIP events around the trace
kernels (the library's stage timing), and keeps the fastest. Results are
cached in a JSON file keyed by grid shape, rays per probe and scene size, so
later volumes of the same shape reuse the choice without measuring. The
package also ships a small table of launch shapes measured on MI355X for the
workloads it is benchmarked on (``tuning_gfx950.json``, same keys); it is
consulted after the caller's cache and before measuring.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional

BRICKS = [(4, 4, 4), (8, 8, 1), (8, 4, 2), (16, 4, 1), (2, 4, 8)]
PERSISTENT = [0, 1, 2]   # packet / persistent with ray refill / packet with node and triangle steps
TOP_NODES = [0, 21, 85]
BLOCKS = [128, 256]
SPLIT = [False, True]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "probestream", "autotune.json")
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def candidates(space: str = "full") -> List[dict]:
    """Launch shapes to time. "full": every schedule, brick, staging, block
    size and shadow split (the split-shadow trace always runs the plain
    packet kernel: no other schedule). "batched": the shapes a volume can take
    inside the batched launch, which runs the stepped lanes in 128-thread
    blocks: probe brick and staged top nodes."""
    if space == "batched":
        return [{"brick": b, "persistent": 2, "top_nodes": t, "block_threads": 128, "split_shadows": False}
                for b, t in itertools.product(BRICKS, TOP_NODES)]
    return [{"brick": b, "persistent": p, "top_nodes": t, "block_threads": w, "split_shadows": s}
            for b, p, t, w, s in itertools.product(BRICKS, PERSISTENT, TOP_NODES, BLOCKS, SPLIT)
            if not (p and s)]


def _apply(volume, c):
    volume.set_trace_config(tuple(c["brick"]), c["persistent"], c["top_nodes"], c["block_threads"],
                            c.get("split_shadows", False))


def key(cfg, n_triangles: int) -> str:
    bucket = 1 << max(0, int(n_triangles).bit_length() - 1)
    return f"{cfg.nx}x{cfg.ny}x{cfg.nz}:n{cfg.rays_per_probe}:t{bucket}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict[str, dict]):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(volume, rotation, lights=None, n_triangles: int = 0, reps: int = 3,
         cache: Optional[str] = DEFAULT_CACHE, force: bool = False, verbose: bool = False,
         shipped: bool = True, space: str = "full", frames=None) -> dict:
    """Pick and set the fastest trace launch shape for ``volume``.

    Looks the shape up in ``cache``, then (if ``shipped``) in the shipped
    table, and measures every candidate only when neither has it or when
    ``force`` is set. The volume's maps are updated by the trial runs
    (callers tune before their real frames, or on a scratch volume of the
    same shape). Returns {"config": ..., "ms": ..., "tried": n, "cached":
    bool, "source": "cache" | "shipped" | "measured"}. ``space`` picks the
    candidate set (see candidates()); its choices are cached apart.
    ``frames`` (a list of (rotation, lights)) times every candidate over
    those frames instead of repeating one: a shape that is fastest on one
    frame need not be over a moving light and changing rotations.
    """
    seq = list(frames) if frames else [(rotation, lights)]
    k = key(volume.cfg, n_triangles) + ("" if space == "full" else ":" + space)
    if not force:
        for source, path in (("cache", cache), ("shipped", SHIPPED if shipped else None)):
            entry = _load(path).get(k) if path else None
            if entry:
                c = {**entry["config"], "brick": tuple(entry["config"]["brick"])}
                _apply(volume, c)
                return {"config": c, "ms": entry["ms"], "tried": 0, "cached": True, "source": source}
    ctx = volume.ctx
    ctx.set_timing(True)
    results = []
    try:
        for c in candidates(space):
            _apply(volume, c)
            volume.update_probes(*seq[0])                    # warm-up
            ctx.stage_times()
            for _ in range(reps):
                for fr in seq:
                    volume.update_probes(*fr)
            st = ctx.stage_times()
            ms = sum(st[s][0] for s in ("trace", "shadow", "shade")) / max(st["trace"][1], 1)
            results.append((ms, c))
            if verbose:
                print(f"autotune {c} -> {ms:.4f} ms", flush=True)
    finally:
        ctx.set_timing(False)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    _apply(volume, best)
    if cache:
        data = _load(cache)
        data[k] = {"config": {**best, "brick": list(best["brick"])}, "ms": best_ms,
                   "default_ms": next((ms for ms, c in results if c["brick"] == (4, 4, 4) and c["persistent"] == 2
                                       and c["top_nodes"] == 21 and c["block_threads"] == 256
                                       and not c["split_shadows"]), None),
                   "all": [[round(ms, 4), {**c, "brick": list(c["brick"])}] for ms, c in results]}
        _save(cache, data)
    return {"config": best, "ms": best_ms, "tried": len(results), "cached": False, "source": "measured",
            "ranking": [(round(ms, 4), c) for ms, c in results[:5]]}


def probe_bucket(volume) -> int:
    """Size bucket of a volume for batched tuning: log2 of its probe count."""
    return max(0, int(volume.P).bit_length() - 1)


def tune_batched(volumes, rotations, lights=None, reps: int = 6, bucket=probe_bucket,
                 verbose: bool = False, margin: float = 0.01) -> dict:
    """Pick per size bucket the trace shape (probe brick, staged top nodes)
    that makes the batched trace of ``volumes`` fastest, timed on the batched
    launch itself: in a batch every volume shares the device with the others,
    so a shape chosen on a volume alone (where a small grid is latency-bound)
    need not help. One pass of coordinate descent over the buckets, largest
    first; every other volume keeps its current shape while a bucket is
    timed, and each bucket starts from a fresh timing of the current shapes;
    a candidate replaces the current shape only when it is faster by more
    than ``margin`` (a bucket is a small share of the launch, so smaller
    differences are within the timing noise). The volumes' maps are updated by the trial frames. Returns
    {"choices": {bucket: config}, "ms": trace ms of the last pass' best,
    "default_ms": trace ms at the default shape, "tried": launches timed}."""
    from . import native
    ctx = volumes[0].ctx
    groups: Dict[int, List[int]] = {}
    for i, v in enumerate(volumes):
        groups.setdefault(bucket(v), []).append(i)
    cands = candidates("batched")
    default = next(c for c in cands if c["brick"] == (4, 4, 4) and c["top_nodes"] == 21)

    def measure() -> float:
        native.update_probes_batched(volumes, rotations, lights)      # warm-up
        ctx.stage_times()
        for _ in range(reps):
            native.update_probes_batched(volumes, rotations, lights)
        st = ctx.stage_times()
        return st["batched"][0] / max(st["batched"][1], 1)

    choices = {k: default for k in groups}
    tried = 0
    ctx.set_timing(True)
    try:
        for v in volumes:
            _apply(v, default)
        default_ms = best_ms = measure()
        # buckets with the most probe-rays first
        order = sorted(groups, key=lambda k: -sum(volumes[i].P * volumes[i].n for i in groups[k]))
        for k in order:
            best = (measure(), choices[k])
            for c in cands:
                if c is choices[k]:
                    continue
                for i in groups[k]:
                    _apply(volumes[i], c)
                ms = measure()
                tried += 1
                if verbose:
                    print(f"batched autotune bucket {k}: {c} -> {ms:.4f} ms", flush=True)
                if ms < best[0] * (1.0 - margin):
                    best = (ms, c)
            choices[k] = best[1]
            best_ms = best[0]
            for i in groups[k]:
                _apply(volumes[i], best[1])
    finally:
        ctx.set_timing(False)
    return {"choices": choices, "ms": best_ms, "default_ms": default_ms, "tried": tried}
