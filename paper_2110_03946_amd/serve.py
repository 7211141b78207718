"""Serving loop: inpainting requests of mixed resolution on one GPU.

Requests arrive over time (a Poisson stream, or all at once to measure
saturation throughput). Each names an input frame f and mask c that are
already resident in device memory (a decoder's output) and asks for the
inpainted frame u back in host memory.

Device-resident state: the server owns a pool of slots per request class
(resolution and mask-density range). A slot holds a solver plan created
with the autotuned parameters of its class, and its own f, c and u buffers,
so every solve on a slot uses the same device pointers: with use_graph the
plan captures the solve -- the coarse-to-fine pyramid, the coarse levels and
the first batch of finest-level sweeps -- into a HIP graph once and replays
it for every later request on that slot.

Admission by HBM footprint: the slots are carved out of a device-memory
budget (plan bytes from ddi_plan_footprint plus the slot's f, c, u), in
proportion to the expected share of each class. A request is admitted when
a slot of its class is free; otherwise it waits in its class queue. A slot
is busy from the solve until its result has been copied to host memory.

Concurrency: the slots are spread over a few lanes, each a compute stream,
a copy stream and a host thread of its own. The dispatcher (the thread
that calls run) hands an admitted request to its slot's lane; the lane
copies the frame into the slot, solves (the library call releases the
interpreter lock) and starts the copy of the result to host memory on its
copy stream. Solves of different lanes run on the GPU at the same time, so
one frame's latency-bound coarse levels overlap another's sweeps.

Latency = time from a request's arrival to its result in host memory; the
completion times come from HIP events on the copy stream.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import autotune, ddi, synth

# request mix of the serving stream: (height, width) -> share
SERVE_MIX = {(1080, 1920): 0.5, (2160, 3840): 0.3, (720, 1280): 0.2}
SERVE_DENSITY = (0.02, 0.08)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the stream
    size: tuple             # (h, w)
    density: float
    frame: int              # index into the frame pool of its size
    cls: tuple = None       # slot class, set by the server
    done: float = None      # completion (seconds from the start)


def poisson_stream(rate: float, duration: float, seed: int = 4, mix=SERVE_MIX,
                   density=SERVE_DENSITY, frames_per_size: int = 4):
    """Requests of a Poisson stream of `rate` per second over `duration`
    seconds: sizes drawn from `mix`, densities uniform in `density`; each
    request uses one of `frames_per_size` pooled frames of its size whose
    density it takes."""
    rng = np.random.default_rng(seed)
    sizes = list(mix)
    p = np.array([mix[s] for s in sizes], dtype=np.float64)
    p /= p.sum()
    # pooled frames: per size, frames_per_size densities
    pool_dens = {s: rng.uniform(density[0], density[1], frames_per_size) for s in sizes}
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = sizes[rng.choice(len(sizes), p=p)]
        k = int(rng.integers(frames_per_size))
        out.append(Request(len(out), t, s, float(pool_dens[s][k]), k))
    return out, pool_dens


def frame_pool(pool_dens, channels: int = 3, workload: int = 4, workers: int = 0,
               keep_host: bool = False):
    """Device-resident input frames: {(h, w): [(f, c), ...]} (generated in
    `workers` processes when > 1); with keep_host also the host copies, as
    a second dict of the same shape."""
    import torch
    args = [(h, w, channels, float(d), "bernoulli", workload, 1000 * (h // 10) + k)
            for (h, w), dens in pool_dens.items() for k, d in enumerate(dens)]
    data = iter(synth.make_workloads(args, workers=workers))
    pool, host = {}, {}
    for (h, w), dens in pool_dens.items():
        pool[(h, w)], host[(h, w)] = [], []
        for _ in dens:
            f, c = next(data)
            pool[(h, w)].append((torch.from_numpy(f).cuda(), torch.from_numpy(c).cuda()))
            if keep_host:
                host[(h, w)].append((f, c))
    return (pool, host) if keep_host else pool


@dataclass
class Slot:
    cls: tuple
    plan: object
    f: object
    c: object
    u: object
    host: object            # pinned host buffer for the result
    bytes: int
    lane: object = None
    busy: bool = False
    req: Request = None
    ev_done: object = None  # set by the lane once the result copy is enqueued


class Lane:
    """A compute stream, a copy stream and a host thread that runs the
    solves of its slots in the order they were handed over."""

    def __init__(self, torch, download: bool):
        self.torch = torch
        self.download = download
        self.stream = torch.cuda.Stream()  # default priority
        self.copy = torch.cuda.Stream()
        self.q = queue.Queue()
        self.error = None
        self.thread = threading.Thread(target=self._work, daemon=True)
        self.thread.start()

    def _work(self):
        torch = self.torch
        while True:
            item = self.q.get()
            if item is None:
                return
            s, f, c = item
            try:
                with torch.cuda.stream(self.stream):
                    s.f.copy_(f)
                    s.c.copy_(c)
                s.plan.solve(s.f, s.c, s.u)  # synchronises the slot's streams
                ev = torch.cuda.Event(enable_timing=True)
                if self.download:
                    self.copy.wait_stream(self.stream)
                    with torch.cuda.stream(self.copy):
                        s.host.copy_(s.u, non_blocking=True)
                        ev.record(self.copy)
                else:
                    ev.record(self.stream)
                s.ev_done = ev
            except Exception as e:  # re-raised by the dispatcher
                self.error = e
                return

    def close(self):
        self.q.put(None)
        self.thread.join()


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    makespan_s: float = 0.0
    requests: int = 0
    slots: dict = field(default_factory=dict)
    budget_bytes: int = 0
    used_bytes: int = 0
    max_queue: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies_ms)
        return {"requests": self.requests, "frames_per_s": round(self.requests / self.makespan_s, 2),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "max_ms": round(float(lat.max()), 3), "max_queue": self.max_queue,
                "slots": {f"{h}x{w}/{lo:.2f}-{hi:.2f}": n for (h, w, lo, hi), n in self.slots.items()},
                "hbm_budget_gb": round(self.budget_bytes / 1e9, 2),
                "hbm_used_gb": round(self.used_bytes / 1e9, 2)}


class Server:
    """Slot pools per class under an HBM budget; see the module docstring."""

    def __init__(self, channels: int = 3, budget_bytes: int = 16 << 30, mix=SERVE_MIX,
                 use_graph: bool = True, download: bool = True, table=None, max_slots: int = 8,
                 on_result=None, lanes: int = 3):
        import torch
        self.torch = torch
        self.C = channels
        self.download = download
        self.on_result = on_result  # called as on_result(request, host or device result)
        self.table = table or autotune.load_table()
        self.stream = torch.cuda.current_stream()
        self.lanes = [Lane(torch, download) for _ in range(max(1, lanes))]
        buckets = autotune.DENSITY_BUCKETS
        classes = [(h, w, lo, hi) for (h, w) in mix for lo, hi in buckets]
        share = {k: mix[k[:2]] / len(buckets) for k in classes}
        self.params = {}
        foot = {}
        for k in classes:
            h, w, lo, hi = k
            prm = autotune.params_for(self.table, h, w, "bernoulli", 0.5 * (lo + hi))
            prm.update(use_graph=1 if use_graph else 0, final_residual=0)
            p = ddi.default_params(**prm)
            self.params[k] = p
            data = channels * h * w * 4 * 2 + h * w  # f, u, c
            foot[k] = ddi.plan_footprint(h, w, channels, p) + data
        # one slot per class first, then by share while the budget lasts
        counts = {k: 0 for k in classes}
        used = 0
        order = sorted(classes, key=lambda k: -share[k])
        for k in order:
            if used + foot[k] > budget_bytes:
                raise ValueError(f"HBM budget {budget_bytes} B cannot hold one slot of {k}")
            counts[k] += 1
            used += foot[k]
        while True:
            # the class with the lowest slots-per-share that still fits
            cand = [k for k in classes if counts[k] < max_slots and used + foot[k] <= budget_bytes]
            if not cand:
                break
            k = min(cand, key=lambda k: counts[k] / share[k])
            counts[k] += 1
            used += foot[k]
        self.slots = {k: [] for k in classes}
        nslot = 0
        for k, n in counts.items():
            h, w = k[:2]
            for _ in range(n):
                # consecutive slots of a class on different lanes
                lane = self.lanes[nslot % len(self.lanes)]
                nslot += 1
                f = torch.empty((channels, h, w), dtype=torch.float32, device="cuda")
                c = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
                u = torch.empty_like(f)
                host = torch.empty((channels, h, w), dtype=torch.float32, pin_memory=True)
                plan = ddi.Plan(h, w, channels, params=ddi.Params.from_buffer_copy(self.params[k]),
                                stream=lane.stream)
                self.slots[k].append(Slot(k, plan, f, c, u, host, foot[k], lane))
        self.stats = ServeStats(slots=counts, budget_bytes=budget_bytes, used_bytes=used)

    def class_of(self, req: Request) -> tuple:
        h, w = req.size
        for lo, hi in autotune.DENSITY_BUCKETS:
            if lo <= req.density <= hi:
                return (h, w, lo, hi)
        lo, hi = min(autotune.DENSITY_BUCKETS, key=lambda b: min(abs(req.density - b[0]),
                                                                abs(req.density - b[1])))
        return (h, w, lo, hi)

    def close(self):
        for lane in self.lanes:
            lane.close()
        self.torch.cuda.synchronize()
        for lst in self.slots.values():
            for s in lst:
                s.plan.close()

    def _check_lanes(self):
        for lane in self.lanes:
            if lane.error is not None:
                raise lane.error

    # -- the loop -------------------------------------------------------

    def _retire(self, t_ref_event, block: bool = False):
        """Free the slots whose results have reached host memory (block:
        wait for every busy slot)."""
        for lst in self.slots.values():
            for s in lst:
                if not s.busy:
                    continue
                if block:
                    while s.ev_done is None:
                        self._check_lanes()
                        time.sleep(5e-5)
                    s.ev_done.synchronize()
                elif s.ev_done is None or not s.ev_done.query():
                    continue
                s.req.done = t_ref_event.elapsed_time(s.ev_done) / 1e3
                self.stats.latencies_ms.append((s.req.done - s.req.arrival) * 1e3)
                if self.on_result is not None:
                    self.on_result(s.req, s.host if self.download else s.u)
                s.busy = False
                s.req = None

    def _dispatch(self, s: Slot, req: Request, pool):
        """Hand an admitted request to its slot's lane."""
        f, c = pool[req.size][req.frame]
        s.busy, s.req, s.ev_done = True, req, None
        s.lane.q.put((s, f, c))

    def warmup(self, pool):
        """One solve on every slot (captures its graphs), outside any stream."""
        for (h, w, lo, hi), lst in self.slots.items():
            for s in lst:
                k = 0
                self._dispatch(s, Request(-1, 0.0, (h, w), 0.5 * (lo + hi), k), pool)
        for lst in self.slots.values():
            for s in lst:
                while s.ev_done is None:
                    self._check_lanes()
                    time.sleep(1e-4)
                s.ev_done.synchronize()
                s.busy, s.req = False, None
        self.torch.cuda.synchronize()

    def run(self, requests, pool, realtime: bool = True) -> ServeStats:
        """Serve `requests` (sorted by arrival). realtime: arrivals follow
        the wall clock; otherwise every request is present at time 0 (its
        arrival is taken as 0)."""
        torch = self.torch
        self.stats = ServeStats(slots=self.stats.slots, budget_bytes=self.stats.budget_bytes,
                                used_bytes=self.stats.used_bytes)
        queues = collections.defaultdict(collections.deque)
        for r in requests:
            r.cls = self.class_of(r)
            if not realtime:
                r.arrival = 0.0
        torch.cuda.synchronize()
        t_ref = torch.cuda.Event(enable_timing=True)
        t_ref.record(self.stream)
        t_ref.synchronize()
        t0 = time.perf_counter()
        nxt = 0
        n = len(requests)
        served = 0
        while served < n or any(s.busy for lst in self.slots.values() for s in lst):
            now = time.perf_counter() - t0
            while nxt < n and requests[nxt].arrival <= now:
                queues[requests[nxt].cls].append(requests[nxt])
                nxt += 1
            self.stats.max_queue = max(self.stats.max_queue, sum(len(q) for q in queues.values()))
            self._check_lanes()
            self._retire(t_ref)
            # oldest admissible request first
            best = None
            for k, q in queues.items():
                if q and any(not s.busy for s in self.slots[k]):
                    if best is None or q[0].arrival < queues[best][0].arrival:
                        best = k
            if best is not None:
                req = queues[best].popleft()
                slot = next(s for s in self.slots[best] if not s.busy)
                self._dispatch(slot, req, pool)
                served += 1
                continue
            if nxt < n:
                wait = requests[nxt].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 2e-4))
            else:
                time.sleep(5e-5)
        self._retire(t_ref, block=True)
        last = max(r.done for r in requests)
        first = min(r.arrival for r in requests)
        self.stats.makespan_s = last - first
        self.stats.requests = n
        return self.stats


def plain_path(requests, pool, channels: int = 3, table=None, download: bool = True):
    """The plain single-image path on the same requests, back to back: one
    eager plan per class (no graphs, no slots), solve straight from the
    pooled frames, result copied to host memory."""
    import torch
    table = table or autotune.load_table()
    plans, outs = {}, {}
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in requests:
        h, w = r.size
        key = (h, w, r.density >= 0.05)
        if key not in plans:
            prm = autotune.params_for(table, h, w, "bernoulli", r.density)
            prm.update(final_residual=0)
            plans[key] = ddi.Plan(h, w, channels, **prm)
            outs[key] = (torch.empty((channels, h, w), dtype=torch.float32, device="cuda"),
                         torch.empty((channels, h, w), dtype=torch.float32, pin_memory=True))
        f, c = pool[r.size][r.frame]
        u, hb = outs[key]
        ts = time.perf_counter()
        plans[key].solve(f, c, u)
        if download:
            hb.copy_(u)
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    lat = np.array(lat)
    return {"requests": len(requests), "frames_per_s": round(len(requests) / el, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3)}
