"""Request loop with continuous batching for many clients.

Each client owns a probe volume over a shared scene plus its last-transmitted
reference state (the paper's per-client textures, Section 3.4), resident in
HBM while admitted. A request asks for one frame of that client: update its
volume, pack the delta, return the packet. Requests of one client are served
in arrival order; requests of different clients that are ready at the same
time are fused into one batched update (three launches covering all their
volumes), and up to ``n_streams`` batches are in flight at once, so requests
that arrive while others run join the next batch as soon as a stream slot and
memory are free. Admission is by device footprint against a budget; idle
clients are evicted to host memory (bit-exact) and brought back on demand.

All GPU work goes through the C ABI (``pv_update_probes_batched``,
``pv_pack_delta``, ``pv_packet_stage``); this module only schedules.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import native


@dataclasses.dataclass
class Request:
    client: int
    rotation: np.ndarray
    lights: np.ndarray
    arrival: float                 # seconds on the server clock
    done: Optional[float] = None
    packet: Optional[bytes] = None   # the packet (keep_packets), else None
    header: Optional[bytes] = None   # its 32-byte header (sizes, sequence, payload checksum)
    nbytes: int = 0
    batch_size: int = 0


class _ClientSlot:
    def __init__(self, cid: int, cfg, footprint: int):
        self.cid = cid
        self.cfg = cfg
        self.footprint = footprint
        self.volume: Optional[native.Volume] = None
        self.client: Optional[native.Client] = None
        self.saved = None          # host checkpoint while evicted
        self.busy = False
        self.last_use = 0.0
        self.queue: collections.deque = collections.deque()


class Server:
    def __init__(self, ctx: native.Context, scene: native.Scene, configs: List, hbm_budget: int,
                 n_streams: int = 3, max_batch: int = 32, tau_irr: float = 0.0, tau_vis: float = 0.0,
                 max_wait_s: float = 0.05, keep_packets: bool = True):
        import torch
        self.ctx = ctx
        self.scene = scene
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.tau = (tau_irr, tau_vis)
        self.slots: Dict[int, _ClientSlot] = {}
        for cid, cfg in enumerate(configs):
            fp = native.volume_footprint(cfg) + native.client_footprint(cfg)
            if fp > self.budget:
                raise native.NativeError(-5, f"client {cid} needs {fp} bytes, above the budget {self.budget}")
            self.slots[cid] = _ClientSlot(cid, cfg, fp)
        self.used = 0
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.inflight: List[Optional[tuple]] = [None] * n_streams
        self.evictions = 0
        self.admissions = 0
        # a request whose client is not resident waits at most this long before
        # it may evict others; until then resident clients go first
        self.max_wait_s = max_wait_s
        # False: a request completes when its packet is in (pinned) host
        # memory, and only its header is kept (a server hands the bytes on)
        self.keep_packets = keep_packets

    # -------------------------------------------------------------- memory
    def _make_resident(self, slot: _ClientSlot, now: float) -> bool:
        if slot.volume is not None:
            return True
        while self.used + slot.footprint > self.budget:
            idle = [s for s in self.slots.values()
                    if s.volume is not None and not s.busy and not s.queue]
            if not idle:
                idle = [s for s in self.slots.values() if s.volume is not None and not s.busy]
            if not idle:
                return False
            victim = min(idle, key=lambda s: s.last_use)
            self._evict(victim)
        vol = native.Volume(self.ctx, slot.cfg)
        vol.set_scene(self.scene)
        cl = native.Client(vol, client_id=slot.cid)
        if slot.saved is not None:
            irr, vis, frame, ri, rv, seq = slot.saved
            vol.set_maps(irr, vis, frame)
            cl.set_state(ri, rv, seq)
            slot.saved = None
        slot.volume, slot.client = vol, cl
        self.used += slot.footprint
        self.admissions += 1
        return True

    def _evict(self, slot: _ClientSlot):
        irr, vis, frame = slot.volume.read_maps()
        ri, rv, seq = slot.client.read_state()
        slot.saved = (irr, vis, frame, ri, rv, seq)
        slot.client.close()
        slot.volume.close()
        slot.volume = slot.client = None
        self.used -= slot.footprint
        self.evictions += 1

    # -------------------------------------------------------------- batches
    def _launch(self, k: int, reqs: List[Request], now: float):
        stream = self.streams[k]
        vols = [self.slots[r.client].volume for r in reqs]
        if len(reqs) == 1:   # a batch of one: the plain launches, no descriptor upload
            vols[0].update_probes(reqs[0].rotation, reqs[0].lights, stream=stream)
        else:
            native.update_probes_batched(vols, [r.rotation for r in reqs], [r.lights for r in reqs], stream=stream)
        for r in reqs:
            self.slots[r.client].client.pack_delta(*self.tau, stream=stream)
            self.slots[r.client].busy = True
            self.slots[r.client].last_use = now
        import torch
        ev = torch.cuda.Event()
        ev.record(stream)
        self.inflight[k] = (reqs, ev)

    def _complete(self, k: int, clock) -> List[Request]:
        reqs, ev = self.inflight[k]
        if not ev.query():
            return []
        out = []
        for r in reqs:
            _deliver(r, self.slots[r.client].client, self.streams[k], self.keep_packets)
            r.done = clock()
            r.batch_size = len(reqs)
            self.slots[r.client].busy = False
            out.append(r)
        self.inflight[k] = None
        return out

    def run(self, requests: List[Request], timeout_s: float = 600.0) -> List[Request]:
        """Serve a trace of requests (arrival times in seconds from start,
        ascending) in real time; returns them with completion times."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        finished: List[Request] = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        total = len(pending)
        while len(finished) < total:
            now = clock()
            if now > timeout_s:
                raise TimeoutError(f"served {len(finished)} of {total} requests in {timeout_s} s")
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                self.slots[r.client].queue.append(r)
            progressed = False
            for k in range(len(self.streams)):
                if self.inflight[k] is not None:
                    done = self._complete(k, clock)
                    if done:
                        finished.extend(done)
                        progressed = True
            for k in range(len(self.streams)):
                if self.inflight[k] is not None:
                    continue
                # one head-of-queue request per client: resident clients and
                # requests past their wait bound first, then by age
                heads = [s for s in self.slots.values() if s.queue and not s.busy]
                heads.sort(key=lambda s: (not (s.volume is not None or now - s.queue[0].arrival > self.max_wait_s),
                                          s.queue[0].arrival))
                batch = []
                for s in heads:
                    if len(batch) >= self.max_batch:
                        break
                    if s.volume is None and now - s.queue[0].arrival <= self.max_wait_s and \
                            self.used + s.footprint > self.budget:
                        continue              # would evict: wait for its bound or for free memory
                    if self._make_resident(s, now):
                        batch.append(s.queue.popleft())
                        s.busy = True          # reserved: not evictable while the batch forms
                if batch:
                    self._launch(k, batch, now)
                    progressed = True
            if not progressed:
                # with work on the device, poll again at once (a sleep adds
                # its own granularity, 50-100 us, to every completion);
                # otherwise wait for the next arrival, at most 0.2 ms
                if any(f is not None for f in self.inflight):
                    continue
                nxt = pending[0].arrival - clock() if pending else 0.0
                time.sleep(min(nxt, 2e-4) if nxt > 0 else 5e-5)
        return finished

    def close(self):
        for s in self.slots.values():
            if s.client is not None:
                s.client.close()
            if s.volume is not None:
                s.volume.close()
            s.client = s.volume = None


def _deliver(r: Request, client: native.Client, stream, keep: bool):
    if keep:
        r.packet = client.packet_download(stream=stream)
        r.header, r.nbytes = r.packet[:32], len(r.packet)
    else:
        ptr, r.nbytes = client.packet_stage(stream=stream)
        r.header = ctypes.string_at(ptr, 32)


def serve_plain(ctx: native.Context, scene: native.Scene, configs: List, requests: List[Request],
                tau_irr: float = 0.0, tau_vis: float = 0.0, timeout_s: float = 600.0,
                keep_packets: bool = True) -> List[Request]:
    """The same trace served one request at a time (update, pack, download),
    with every client's state resident: the per-request path that the
    batched server is compared against."""
    vols, cls = {}, {}
    for cid, cfg in enumerate(configs):
        v = native.Volume(ctx, cfg)
        v.set_scene(scene)
        vols[cid] = v
        cls[cid] = native.Client(v, client_id=cid)
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    t0 = time.perf_counter()
    out = []
    try:
        while pending:
            r = pending.popleft()
            now = time.perf_counter() - t0
            if now < r.arrival:
                time.sleep(r.arrival - now)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("plain path exceeded its time limit")
            vols[r.client].update_probes(r.rotation, r.lights)
            cls[r.client].pack_delta(tau_irr, tau_vis)
            _deliver(r, cls[r.client], None, keep_packets)
            r.done = time.perf_counter() - t0
            r.batch_size = 1
            out.append(r)
    finally:
        for c in cls.values():
            c.close()
        for v in vols.values():
            v.close()
    return out


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
