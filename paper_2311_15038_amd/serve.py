"""Preview request serving with continuous batching on one GPU.

A request asks for n turntable frames of one volume at one resolution.  The
server keeps volumes resident in HBM together with their reduced preview
level (threshold, 2x level in the brick layout), admits queued requests
whenever a slot (a HIP stream) is free and their device-memory footprint fits
the budget, and runs admitted requests concurrently on their streams: a
request that arrives while others are on the GPU starts as soon as a slot and
memory free up, and its kernels overlap with theirs.  Idle resident volumes
are evicted least recently used first when memory is needed; a request never
allocates past the budget, it waits.  Completion is observed by polling each
request's event, which also enforces per-request deadlines.

The scheduling logic is independent of the GPU: an executor supplies the
footprints and does the work.  GpuExecutor runs the library's kernels;
FakeExecutor simulates durations and failures on the CPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    vol_id: int
    n_views: int
    res: int
    deadline: float = math.inf      # seconds after arrival
    t_arrival: float = 0.0
    t_admit: float = -1.0
    t_done: float = -1.0
    status: str = "new"             # queued | running | done | failed | expired | cancelled
    error: str = ""
    result: object = None
    measured: bool = True           # counted in the latency statistics

    def finished(self):
        return self.status in ("done", "failed", "expired", "cancelled")


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    views: int = 0
    done: int = 0
    failed: int = 0
    expired: int = 0
    cancelled: int = 0
    evictions: int = 0
    loads: int = 0
    hits: int = 0
    wall: float = 0.0
    max_inflight: int = 0
    peak_bytes: int = 0

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"requests": self.done, "failed": self.failed, "expired": self.expired,
                "cancelled": self.cancelled, "views": self.views,
                "views_per_s": self.views / self.wall if self.wall > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "loads": self.loads, "hits": self.hits,
                "evictions": self.evictions, "max_inflight": self.max_inflight,
                "peak_bytes": self.peak_bytes, "wall_s": self.wall}


class Server:
    """Admission, residency and slot scheduling over an executor.

    budget_bytes bounds resident volumes plus the transient memory of running
    requests; slots bounds the requests on the GPU at once.  With
    resident=False a volume is dropped as soon as no running request uses it
    (the plain path: every request loads and reduces its volume again).
    """

    def __init__(self, executor, budget_bytes, slots=4, resident=True, clock=time.perf_counter,
                 sleep=time.sleep):
        self.ex = executor
        self.sleep = sleep
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.keep_resident = resident
        self.clock = clock
        self.queue = collections.deque()
        self.running = []                            # [request, handle, bytes, slot]
        self.free_slots = list(range(self.slots))
        self.resident = collections.OrderedDict()    # vol_id -> bytes, least recent first
        self.pins = collections.Counter()            # vol_id -> running requests using it
        self.reserved = 0                            # transient bytes of running requests
        self.stats = Stats()

    # memory accounting -------------------------------------------------
    def used(self):
        return sum(self.resident.values()) + self.reserved

    def _evict(self, vol_id):
        self.ex.evict(vol_id)
        del self.resident[vol_id]
        self.stats.evictions += 1

    def _evict_for(self, need):
        """Evict idle volumes (least recent first) until `need` more bytes fit."""
        while self.used() + need > self.budget:
            victim = next((v for v in self.resident if self.pins[v] == 0), None)
            if victim is None:
                return False
            self._evict(victim)
        return True

    # request flow --------------------------------------------------------
    def submit(self, req: Request, now=None):
        """Queue a request (rejects an invalid one at once); returns it as its own handle."""
        req.t_arrival = self.clock() if now is None else now
        err = self.ex.validate(req)
        if err:
            self._finish(req, "failed", err)
            return req
        req.status = "queued"
        self.queue.append(req)
        return req

    def cancel(self, req: Request):
        """Drop a queued request; a running one is marked and its result discarded."""
        if req.status == "queued":
            self.queue.remove(req)
            self._finish(req, "cancelled")
        elif req.status == "running":
            req.status = "cancelling"

    def _finish(self, req, status, error=""):
        req.t_done = self.clock()
        req.status, req.error = status, error
        if status == "done":
            self.stats.done += 1
            self.stats.views += req.n_views
            if req.measured:
                self.stats.latencies.append(req.t_done - req.t_arrival)
        elif status == "failed":
            self.stats.failed += 1
        elif status == "expired":
            self.stats.expired += 1
        else:
            self.stats.cancelled += 1

    def _try_admit(self):
        admitted = False
        while self.queue and self.free_slots:
            req = self.queue[0]
            if self.clock() - req.t_arrival > req.deadline:
                self.queue.popleft()
                self._finish(req, "expired", "deadline passed while queued")
                continue
            resident = req.vol_id in self.resident
            vol_bytes = 0 if resident else self.ex.volume_bytes(req)
            work = self.ex.work_bytes(req)
            if vol_bytes + work > self.budget:
                self.queue.popleft()
                self._finish(req, "failed", "request larger than the memory budget")
                continue
            self.pins[req.vol_id] += 1    # never evict the volume this request needs
            if not self._evict_for(vol_bytes + work):
                self.pins[req.vol_id] -= 1
                break                     # wait for running requests to release memory
            self.queue.popleft()
            if resident:
                self.resident.move_to_end(req.vol_id)
                self.stats.hits += 1
            else:
                self.resident[req.vol_id] = vol_bytes
                self.stats.loads += 1
            self.reserved += work
            self.stats.peak_bytes = max(self.stats.peak_bytes, self.used())
            slot = self.free_slots.pop(0)
            req.t_admit = self.clock()
            req.status = "running"
            try:
                handle = self.ex.start(req, slot=slot, load=not resident)
            except Exception as e:        # this request fails; the loop goes on
                self._release(req, work, slot)
                if not resident:
                    self._drop(req.vol_id)
                self._finish(req, "failed", f"{type(e).__name__}: {e}")
                continue
            self.running.append([req, handle, work, slot])
            admitted = True
        self.stats.max_inflight = max(self.stats.max_inflight, len(self.running))
        return admitted

    def _drop(self, vol_id):
        if vol_id in self.resident and self.pins[vol_id] == 0:
            self._evict(vol_id)

    def _release(self, req, work, slot):
        self.pins[req.vol_id] -= 1
        self.reserved -= work
        self.free_slots.append(slot)
        self.free_slots.sort()
        if not self.keep_resident:
            self._drop(req.vol_id)

    def _poll(self):
        still = []
        progressed = False
        now = self.clock()
        for entry in self.running:
            req, h, work, slot = entry
            try:
                fin = self.ex.done(h)
            except Exception as e:
                self._release(req, work, slot)
                if not req.finished():
                    self._finish(req, "failed", f"{type(e).__name__}: {e}")
                progressed = True
                continue
            if fin:
                res = self.ex.result(h)
                self._release(req, work, slot)
                if req.status == "cancelling":
                    self._finish(req, "cancelled")
                elif req.status == "running":
                    req.result = res
                    self._finish(req, "done")
                # an expired request was reported already; its slot frees only now
                progressed = True
            else:
                if req.status == "running" and now - req.t_arrival > req.deadline:
                    # reported at once; the GPU work cannot be recalled, so the slot
                    # and memory stay held until its event completes
                    self._finish(req, "expired", "deadline passed while running")
                still.append(entry)
        self.running = still
        return progressed

    def pump(self):
        """One scheduling pass: observe completions, then admit; True if anything moved."""
        progressed = self._poll()
        progressed |= self._try_admit()
        return progressed

    def idle(self):
        return not self.queue and not self.running

    def drain(self, idle_sleep=20e-6):
        while not self.idle():
            if not self.pump():
                self.sleep(idle_sleep)

    def run(self, trace, warmup=0.0, idle_sleep=20e-6):
        """Serve a trace of (arrival offset in s, Request) in real time.

        Requests arriving before `warmup` run but are not measured; views/s is
        taken over the measured requests, from the end of the warm-up (or the
        first measured arrival) to the last completion.  Returns the stats."""
        trace = sorted(trace, key=lambda x: x[0])
        t0 = self.clock()
        i = 0
        while i < len(trace) or not self.idle():
            now = self.clock()
            while i < len(trace) and t0 + trace[i][0] <= now:
                off, req = trace[i]
                req.measured = off >= warmup
                self.submit(req, now=t0 + off)
                i += 1
            if not self.pump():
                if self.running or self.queue or i >= len(trace):
                    self.sleep(idle_sleep)
                else:                     # idle until the next arrival
                    self.sleep(min(max(t0 + trace[i][0] - self.clock(), 0.0), 1e-3))
        measured = [r for off, r in trace if off >= warmup and r.status == "done"]
        start = t0 + min((off for off, _ in trace if off >= warmup), default=warmup)
        self.stats.wall = max((r.t_done for r in measured), default=start) - start
        self.stats.views = sum(r.n_views for r in measured)
        return self.stats


# ------------------------------------------------------------------ workload
def make_trace(rate=50.0, duration=65.0, pool=64, seed=5000, lo=128, hi=1024, max_views=36,
               resolutions=(256, 512)):
    """Poisson arrivals at `rate`/s over `duration` s on a pool of volume ids;
    each id has a fixed cubic edge, log-uniform in [lo, hi]; views uniform in
    1..max_views; resolution drawn uniformly from `resolutions`.
    Returns (trace, edges)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=pool))).astype(int)
    t, trace, rid = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        vid = int(rng.integers(0, pool))
        trace.append((t, Request(rid, vid, int(rng.integers(1, max_views + 1)),
                                 int(resolutions[int(rng.integers(0, len(resolutions)))]))))
        rid += 1
    return trace, edges


def copy_trace(trace, burst=False):
    """Fresh Request objects for the same arrivals (all at t=0 when `burst`)."""
    return [(0.0 if burst else t, Request(r.rid, r.vol_id, r.n_views, r.res, r.deadline))
            for t, r in trace]


# ------------------------------------------------------------------ executors
class FakeExecutor:
    """CPU stand-in: bytes from the volume edge, durations proportional to the
    views, injected failures at start, at completion, or as invalid requests."""

    def __init__(self, edges, clock=time.perf_counter, s_per_view=1e-3, s_load=0.0,
                 fail_start=(), fail_done=(), bad_ids=(), max_views=48):
        self.edges = edges
        self.clock = clock
        self.s_per_view = s_per_view
        self.s_load = s_load
        self.fail_start = set(fail_start)
        self.fail_done = set(fail_done)
        self.bad_ids = set(bad_ids)
        self.max_views = max_views
        self.evicted = []
        self.loaded = []
        self.resident = set()
        self.started = []

    def validate(self, req):
        if not (0 <= req.vol_id < len(self.edges)) or req.vol_id in self.bad_ids:
            return "VR_ERR_RANGE: unknown volume"
        if not 1 <= req.n_views <= self.max_views or req.res not in (256, 512):
            return "VR_ERR_RANGE: bad view request"
        return ""

    def volume_bytes(self, req):
        return int(self.edges[req.vol_id]) ** 3 * 2

    def work_bytes(self, req):
        return req.n_views * req.res * req.res * 16

    def start(self, req, slot, load):
        if req.rid in self.fail_start:
            raise RuntimeError("injected failure")
        if load:
            assert req.vol_id not in self.resident
            self.loaded.append(req.vol_id)
            self.resident.add(req.vol_id)
        assert req.vol_id in self.resident
        self.started.append((req.rid, slot))
        t = self.clock() + (self.s_load if load else 0.0) + self.s_per_view * req.n_views
        return (t, req)

    def done(self, h):
        if h[1].rid in self.fail_done and self.clock() >= h[0]:
            raise RuntimeError("injected device error")
        return self.clock() >= h[0]

    def result(self, h):
        return ("frames", h[1].rid)

    def evict(self, vol_id):
        self.resident.discard(vol_id)
        self.evicted.append(vol_id)


class GpuExecutor:
    """Runs requests with the library on one GPU.

    A volume's bytes come from a host store (pinned memory, standing in for
    the reconstruction's output).  Loading a volume copies it to HBM and runs
    histogram, threshold selection and the 2x level in the brick layout with
    occupancy; these stay resident.  A request renders its turntable views
    from that level on its slot's stream."""

    def __init__(self, edges, slots=4, device="cuda:0", seed_base=7000, tf=None, step=0.5,
                 rule=None, rule_param=32, top_slices=3, store=None):
        import torch
        from . import synth, vr
        self.torch, self.synth, self.vr = torch, synth, vr
        self.dev = torch.device(device)
        self.edges = edges
        self.seed_base = seed_base
        self.step = step
        self.rule = vr.RULE_VALLEY if rule is None else rule
        self.rule_param = rule_param
        self.top_slices = top_slices
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        tf_host = synth.default_tf() if tf is None else tf
        self.tf = torch.from_numpy(tf_host).to(self.dev)
        # resident levels are kept as 4^3 bricks overlapping in x, marked above the level
        # the (fixed) TF leaves at zero extinction
        self.mark_above = vr.tf_mark_level(tf_host)
        self.vols = {}               # vol_id -> dict of device tensors
        self.store = store if store is not None else {}

    def host_volume(self, vol_id):
        """The volume in pinned host memory (generated once from its seed)."""
        if vol_id not in self.store:
            torch = self.torch
            n = int(self.edges[vol_id])
            spec = self.synth.scaled_spec(n, n, n, seed=self.seed_base + vol_id)
            t = self.synth.make_volume(spec, self.dev)
            h = torch.empty(t.shape, dtype=torch.int16, pin_memory=True)
            h.copy_(t.view(torch.int16))
            del t
            self.store[vol_id] = h
        return self.store[vol_id]

    def validate(self, req):
        if not (0 <= req.vol_id < len(self.edges)):
            return "VR_ERR_RANGE: unknown volume"
        if not 1 <= req.n_views <= self.vr.MAX_VIEWS_PER_LAUNCH or req.res not in (256, 512):
            return "VR_ERR_RANGE: bad view request"
        return ""

    def volume_bytes(self, req):
        n = int(self.edges[req.vol_id])
        lv = self.vr.level_shape((n, n, n), 1)
        _, nel, nocc = self.vr.vr_brick_count_layout(self.vr.LAYOUT_BRICK4_OVERLAP, lv[2], lv[1], lv[0])
        return (n ** 3 * 2 + int(np.prod(lv)) * 2 + nel * 2 + nocc
                + 2 * self.vr.NBINS * 8 + self.vr.KEEP_WORDS * 4 + 16)

    def work_bytes(self, req):
        return req.n_views * req.res * req.res * 16

    def _load(self, vol_id, stream):
        torch, vr = self.torch, self.vr
        h = self.host_volume(vol_id)
        with torch.cuda.stream(stream):
            raw = torch.empty(h.shape, dtype=torch.int16, device=self.dev)
            raw.copy_(h, non_blocking=True)
            v = raw.view(torch.uint16)
            H, Ht = vr.vr_histogram_with_top(v, self.top_slices, stream=stream)
            res, bits = vr.vr_select_threshold(H, Ht, self.rule, self.rule_param, stream=stream)
            (L1,) = vr.vr_threshold_downsample(v, bits, 1, stream=stream)
            bv = vr.vr_brick_volume(L1, stream=stream, overlap=True, mark_above=self.mark_above)
            ready = torch.cuda.Event()
            ready.record(stream)
        self.vols[vol_id] = dict(vol=raw, H=H, Ht=Ht, res=res, bits=bits, L1=L1, bv=bv, ready=ready)

    def start(self, req, slot, load):
        torch, vr = self.torch, self.vr
        s = self.streams[slot % len(self.streams)]
        if load:
            self._load(req.vol_id, s)
        ent = self.vols[req.vol_id]
        s.wait_event(ent["ready"])        # the level may have been made on another slot
        lz, ly, lx = ent["L1"].shape
        cams = self.synth.turntable_cameras(lx, ly, lz, n_views=req.n_views)
        with torch.cuda.stream(s):
            frames = torch.empty((req.n_views, req.res, req.res, 4), dtype=torch.float32,
                                 device=self.dev)
            vr.vr_raycast(ent["bv"], self.tf, cams, req.res, req.res, self.step, out=frames,
                          stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, frames, ent)          # the entry keeps the volume alive while in use

    def done(self, h):
        return h[0].query()

    def result(self, h):
        return (h[1], h[2]["res"])

    def evict(self, vol_id):
        ent = self.vols.pop(vol_id, None)
        if ent is not None:
            ent["ready"].synchronize()
