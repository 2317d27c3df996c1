"""Served form: continuous batching of calorimeter events.

Events arrive over time (for instance a Poisson stream). The scheduler

* makes an event visible at its arrival time and queues it (FIFO);
* admits queued events while the HBM they hold (inputs and outputs of every
  admitted, unfinished event) fits the budget left after the slots' arenas;
* whenever a slot (one library context with its own stream) is free, launches
  every admitted, not yet launched event as one batch (a contiguous run of
  the device pool, clustered by clue_run_batch_range with no copy);
* polls the slots' completion events, stamps each event's completion time,
  releases its budget and re-queues the events of a batch whose slot failed.

Slots run concurrently on separate streams, so batches overlap on the GPU
while new events keep arriving. Latency is completion minus arrival.

The scheduling logic is backend-independent: ``GpuPoolBackend`` drives the
HIP library on a device-resident event pool; ``GpuStagedBackend`` keeps the
events in pinned host memory and admission copies each one into a bounded
device staging ring sized from the HBM budget (the host-resident serving
variant: an event that finds no room waits in the queue); tests also drive the
scheduler with a CPU backend and a virtual clock.

``Server`` is the online form of the same loop: callers ``submit`` events as
they come and receive futures of their cluster ids.
"""
from __future__ import annotations

import gc
import threading
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

# HBM an in-flight event holds per hit in the pool: x, y, energy (float32),
# layer and event id (int32) in, cluster id (int32) and seed flag (uint8) out.
POOL_BYTES_PER_HIT = 5 * 4 + 4 + 1


@dataclass
class EventRecord:
    idx: int
    n_hits: int
    t_arrival: float
    t_admit: float = float("nan")
    t_launch: float = float("nan")
    t_done: float = float("nan")
    batch: int = -1
    attempts: int = 0


@dataclass
class RunStats:
    records: list
    batches: list = field(default_factory=list)  # (slot, first, count, hits, t_launch, t_done)
    wall_s: float = 0.0
    max_inflight_bytes: int = 0
    failures: int = 0

    def latencies(self):
        return np.array([r.t_done - r.t_arrival for r in self.records], dtype=float)

    def admission_waits(self):
        return np.array([r.t_admit - r.t_arrival for r in self.records], dtype=float)

    def summary(self):
        lat = self.latencies()
        wait = self.admission_waits()
        hits = sum(r.n_hits for r in self.records)
        t0 = min(r.t_arrival for r in self.records)
        t1 = max(r.t_done for r in self.records)
        sizes = [b[2] for b in self.batches]
        return dict(events=len(self.records), hits=int(hits), wall_s=round(t1 - t0, 6),
                    hits_per_s=hits / max(t1 - t0, 1e-12), events_per_s=len(self.records) / max(t1 - t0, 1e-12),
                    p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), batches=len(self.batches),
                    mean_batch_events=float(np.mean(sizes)) if sizes else 0.0,
                    max_batch_events=int(max(sizes)) if sizes else 0,
                    max_inflight_bytes=int(self.max_inflight_bytes), failures=self.failures,
                    admit_wait_p50_ms=float(np.percentile(wait, 50) * 1e3),
                    admit_wait_p99_ms=float(np.percentile(wait, 99) * 1e3))


class StagingRing:
    """Contiguous hit ranges of a fixed-capacity device region, given out in
    admission (FIFO) order and freed in any order: a freed range is reused once
    every older range is free too. A range that does not fit before the end
    of the region starts again at offset 0, so every range is contiguous."""

    def __init__(self, capacity_hits):
        self.capacity = int(capacity_hits)
        self.live = deque()   # [event, offset, hits, done] in admission order
        self.where = {}       # event -> its entry

    def allocate(self, event, n_hits):
        n = int(n_hits)
        if n > self.capacity:
            raise ValueError(f"event of {n} hits exceeds the staging capacity ({self.capacity})")
        if not self.live:
            off = 0
        else:
            tail = self.live[0][1]
            last = self.live[-1]
            head = last[1] + last[2]
            if last[1] >= tail:  # in use: [tail, head)
                if head + n <= self.capacity:
                    off = head
                elif n <= tail:
                    off = 0
                else:
                    return None
            elif head + n <= tail:  # wrapped: in use [tail, capacity) and [0, head)
                off = head
            else:
                return None
        ent = [event, off, n, False]
        self.live.append(ent)
        self.where[event] = ent
        return off

    def offset(self, event):
        return self.where[event][1]

    def adjacent(self, a, b):
        ea, eb = self.where.get(a), self.where.get(b)
        return ea is not None and eb is not None and eb[1] == ea[1] + ea[2]

    def release(self, event):
        self.where.pop(event)[3] = True
        while self.live and self.live[0][3]:
            self.live.popleft()

    def used_hits(self):
        """Hits of the region held by live ranges and the gaps between them."""
        if not self.live:
            return 0
        tail, last = self.live[0][1], self.live[-1]
        head = last[1] + last[2]
        return head - tail if last[1] >= tail else self.capacity - tail + head


class Scheduler:
    """Admission by HBM budget and continuous batching over backend slots.

    A backend may provide ``admit(i, n_hits)`` (reserve device room for
    event i and start its copy in; False while there is none), ``adjacent(i,
    j)`` (events i and j sit back to back in device memory, so one batch can
    take both) and ``release(events)`` (their room may be reused); without
    them every event is admitted at once and consecutive events are adjacent."""

    def __init__(self, backend, *, hbm_budget_bytes=0, max_batch_hits, max_batch_events):
        self.backend = backend
        self.max_batch_hits = int(max_batch_hits)
        self.max_batch_events = int(max_batch_events)
        arenas = backend.n_slots * backend.slot_bytes()
        if hbm_budget_bytes and hbm_budget_bytes <= arenas:
            raise ValueError(f"HBM budget {hbm_budget_bytes} B does not cover the slot arenas ({arenas} B)")
        self.event_budget = (hbm_budget_bytes - arenas) if hbm_budget_bytes else None

    def footprint(self, n_hits):
        return int(n_hits) * POOL_BYTES_PER_HIT

    def run(self, arrivals, n_hits):
        """Serves events 0..N-1 (pool order) arriving at ``arrivals`` seconds
        after the start. Returns RunStats. The cyclic garbage collector is
        paused for the duration (a full collection can stall the loop for
        milliseconds)."""
        enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(arrivals, n_hits)
        finally:
            if enabled:
                gc.enable()

    def _run(self, arrivals, n_hits):
        be = self.backend
        N = len(arrivals)
        for i in range(N):
            fp = self.footprint(n_hits[i])
            if self.event_budget is not None and fp > self.event_budget:
                raise ValueError(f"event {i} needs {fp} B, more than the HBM budget left for events")
            if n_hits[i] > self.max_batch_hits:
                raise ValueError(f"event {i} has {n_hits[i]} hits, more than a slot holds ({self.max_batch_hits})")
        admit = getattr(be, "admit", lambda i, n: True)
        adjacent = getattr(be, "adjacent", lambda i, j: j == i + 1)
        release = getattr(be, "release", lambda run: None)
        recs = [EventRecord(i, int(n_hits[i]), float(arrivals[i])) for i in range(N)]
        stats = RunStats(records=recs)
        queued = []        # arrived, not admitted (FIFO)
        admitted = []      # admitted, not launched (FIFO, consecutive pool indices)
        busy = {}          # slot -> (handle, [event indices], batch id)
        free = list(range(be.n_slots))
        inflight = 0
        nxt = 0            # next arrival
        done = 0
        t_start = be.start()
        while done < N:
            now = be.now()
            while nxt < N and recs[nxt].t_arrival <= now:
                queued.append(nxt)
                nxt += 1
            admitted_now = False
            while queued and (self.event_budget is None or
                              inflight + self.footprint(recs[queued[0]].n_hits) <= self.event_budget):
                if not admit(queued[0], recs[queued[0]].n_hits):
                    break  # no device room yet: the event waits for a completion
                i = queued.pop(0)
                admitted_now = True
                recs[i].t_admit = now
                inflight += self.footprint(recs[i].n_hits)
                admitted.append(i)
            stats.max_inflight_bytes = max(stats.max_inflight_bytes, inflight)
            # launch: one batch per free slot, a maximal run of consecutive events
            while free and admitted:
                run = [admitted[0]]
                hits = recs[admitted[0]].n_hits
                k = 1
                while (k < len(admitted) and admitted[k] == run[-1] + 1 and adjacent(run[-1], admitted[k])
                       and len(run) < self.max_batch_events
                       and hits + recs[admitted[k]].n_hits <= self.max_batch_hits):
                    run.append(admitted[k])
                    hits += recs[admitted[k]].n_hits
                    k += 1
                del admitted[:k]
                slot = free.pop(0)
                handle = be.launch(slot, run[0], len(run))
                bid = len(stats.batches)
                stats.batches.append([slot, run[0], len(run), hits, be.now(), float("nan")])
                for i in run:
                    recs[i].t_launch = stats.batches[-1][4]
                    recs[i].batch = bid
                    recs[i].attempts += 1
                busy[slot] = (handle, run, bid)
            # completions
            progressed = False
            for slot in list(busy):
                handle, run, bid = busy[slot]
                st = be.poll(slot, handle)
                if st is None:
                    continue
                progressed = True
                t = be.now()
                del busy[slot]
                free.append(slot)
                if st == "failed":  # the batch did not complete: run its events again, in order
                    stats.failures += 1
                    admitted = sorted(run + admitted)
                    continue
                stats.batches[bid][5] = t
                for i in run:
                    recs[i].t_done = t
                    inflight -= self.footprint(recs[i].n_hits)
                    done += 1
                release(run)
            if not progressed and not (free and admitted) and not admitted_now:
                be.idle(recs[nxt].t_arrival if nxt < N else None, bool(busy))
        stats.wall_s = be.now() - t_start if t_start is not None else 0.0
        return stats


class GpuPoolBackend:
    """Slots over the HIP library; events live in one device-resident pool.

    ``pool``: dict of contiguous device tensors x, y, energy (float32), layer,
    event (int32; pool event index of each hit), cluster_id (int32) and
    is_seed (uint8) outputs, and ``offsets`` (host, int64[N+1]) giving each
    event's hit range."""

    def __init__(self, params, pool, *, slots=2, max_batch_hits, max_batch_events, tuning=None, flags=0):
        import torch

        import paper_2001_09761_amd as clue
        self.torch = torch
        self.pool = pool
        self.offsets = np.asarray(pool["offsets"], dtype=np.int64)
        self.n_slots = int(slots)
        self.ctxs = []
        self.streams = []
        for _ in range(self.n_slots):
            ctx = clue.Context(params["dc"], params["rho_c"], params["delta_c"], params["delta_o"],
                               max_hits=max_batch_hits, max_events=max_batch_events,
                               extent=params.get("extent"), bounds=params.get("bounds"),
                               n_layers=params["n_layers"], flags=flags)
            if tuning:
                ctx.set_tuning(**tuning)
            self.ctxs.append(ctx)
            self.streams.append(torch.cuda.Stream())  # default priority
        self._slot_bytes = clue.footprint_bytes(params["dc"], params["rho_c"], params["delta_c"], params["delta_o"],
                                                max_batch_hits, max_batch_events, extent=params.get("extent"),
                                                bounds=params.get("bounds"), n_layers=params["n_layers"],
                                                flags=flags)
        self.t0 = None

    def slot_bytes(self):
        return self._slot_bytes

    def start(self):
        # one launch per slot before the clock starts: the first batched run
        # of a context captures its HIP graph
        for slot in range(self.n_slots):
            self.launch(slot, 0, 1)
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        return 0.0

    def now(self):
        return time.perf_counter() - self.t0

    def launch(self, slot, first, count):
        p = self.pool
        a, b = int(self.offsets[first]), int(self.offsets[first + count])
        s = self.streams[slot]
        self.ctxs[slot].run_batch_range(first, count, p["event"][a:b], p["x"][a:b], p["y"][a:b], p["layer"][a:b],
                                        p["energy"][a:b], p["cluster_id"][a:b], p["is_seed"][a:b], stream=s)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return ev

    def poll(self, slot, handle):
        return "ok" if handle.query() else None

    def idle(self, next_arrival, busy):
        # short spin: the GPU is running batches or nothing has arrived yet
        if next_arrival is not None and not busy:
            dt = next_arrival - self.now()
            if dt > 2e-4:
                # short sleeps: a long one can overshoot by milliseconds
                time.sleep(min(dt - 1e-4, 1e-3))
                return
        time.sleep(2e-5)

    def close(self):
        for c in self.ctxs:
            c.close()


class GpuStagedBackend:
    """Slots over the HIP library for events held in pinned host memory: the
    host-resident served variant. Admitting event i reserves a contiguous range
    of a device staging ring (inputs, event ids and outputs, POOL_BYTES_PER_HIT
    per hit) and copies the event's inputs into it on a copy stream; a batch is
    a run of events that sit back to back in the ring, clustered in place by
    clue_run_batch_range once their copies are done. Outputs stay in device
    memory; the ring range is reused after the batch completes. The ring holds
    ``ring_hits`` hits, normally sized from the HBM budget left after the
    slots' arenas, so admission gates real device memory.

    ``host_events`` are the distinct events; arrival i carries event
    ``i % len(host_events)``. Arrivals listed in ``keep`` also have their
    outputs copied back to host memory after their batch, for checking."""

    def __init__(self, params, host_events, *, ring_hits, slots=2, max_batch_hits, max_batch_events, tuning=None,
                 flags=0, keep=()):
        import torch

        import paper_2001_09761_amd as clue
        from .gen import concat_events
        self.torch = torch
        dev = torch.device("cuda", torch.cuda.current_device())
        b = concat_events(host_events)
        self.host = {k: torch.from_numpy(b[k]).pin_memory() for k in ("x", "y", "layer", "energy")}
        self.host_offsets = np.concatenate([[0], np.cumsum([e["x"].size for e in host_events])]).astype(np.int64)
        self.m = len(host_events)
        self.ring = StagingRing(ring_hits)
        C = int(ring_hits)
        self.dev = {k: torch.empty(C, dtype=dt, device=dev) for k, dt in
                    (("x", torch.float32), ("y", torch.float32), ("energy", torch.float32), ("layer", torch.int32),
                     ("event", torch.int32), ("cluster_id", torch.int32), ("is_seed", torch.uint8))}
        self.copy_stream = torch.cuda.Stream()  # default priority
        self.ready = {}
        self.n_hits = {}
        self.keep = set(int(i) for i in keep)
        self.kept = {}
        self.n_slots = int(slots)
        self.ctxs, self.streams = [], []
        for _ in range(self.n_slots):
            ctx = clue.Context(params["dc"], params["rho_c"], params["delta_c"], params["delta_o"],
                               max_hits=max_batch_hits, max_events=max_batch_events,
                               extent=params.get("extent"), bounds=params.get("bounds"),
                               n_layers=params["n_layers"], flags=flags)
            if tuning:
                ctx.set_tuning(**tuning)
            self.ctxs.append(ctx)
            self.streams.append(torch.cuda.Stream())  # default priority
        self._slot_bytes = clue.footprint_bytes(params["dc"], params["rho_c"], params["delta_c"], params["delta_o"],
                                                max_batch_hits, max_batch_events, extent=params.get("extent"),
                                                bounds=params.get("bounds"), n_layers=params["n_layers"],
                                                flags=flags)
        self.t0 = None

    @staticmethod
    def ring_hits_for(budget_bytes, slots, slot_bytes):
        """Ring capacity that the HBM budget leaves after the slots' arenas."""
        return max(0, (int(budget_bytes) - int(slots) * int(slot_bytes)) // POOL_BYTES_PER_HIT)

    def staging_bytes(self):
        return self.ring.capacity * POOL_BYTES_PER_HIT

    def slot_bytes(self):
        return self._slot_bytes

    def _src(self, i):
        k = i % self.m
        return int(self.host_offsets[k]), int(self.host_offsets[k + 1])

    def admit(self, i, n_hits):
        a, b = self._src(i)
        off = self.ring.allocate(i, b - a)
        if off is None:
            return False
        d, h, n = self.dev, self.host, b - a
        with self.torch.cuda.stream(self.copy_stream):
            for k in ("x", "y", "layer", "energy"):
                d[k][off:off + n].copy_(h[k][a:b], non_blocking=True)
            d["event"][off:off + n].fill_(i)
            ev = self.torch.cuda.Event()
            ev.record(self.copy_stream)
        self.ready[i] = ev
        self.n_hits[i] = n
        return True

    def adjacent(self, i, j):
        return self.ring.adjacent(i, j)

    def release(self, run):
        for i in run:
            self.ring.release(i)
            self.ready.pop(i, None)
            self.n_hits.pop(i, None)

    def start(self):
        # admit, run and release arrival 0 on every slot before the clock
        # starts (graph capture), then clear the ring
        for slot in range(self.n_slots):
            assert self.admit(0, None)
            self.launch(slot, 0, 1)
            self.torch.cuda.synchronize()
            self.release([0])
        self.kept.clear()
        self.t0 = time.perf_counter()
        return 0.0

    def now(self):
        return time.perf_counter() - self.t0

    def launch(self, slot, first, count):
        d = self.dev
        off = self.ring.offset(first)
        n = sum(self.n_hits[i] for i in range(first, first + count))
        s = self.streams[slot]
        s.wait_event(self.ready[first + count - 1])  # the copy stream is in order
        z = off + n
        self.ctxs[slot].run_batch_range(first, count, d["event"][off:z], d["x"][off:z], d["y"][off:z],
                                        d["layer"][off:z], d["energy"][off:z], d["cluster_id"][off:z],
                                        d["is_seed"][off:z], stream=s)
        with self.torch.cuda.stream(s):
            a = off
            for i in range(first, first + count):
                if i in self.keep:
                    m = self.n_hits[i]
                    self.kept[i] = (d["cluster_id"][a:a + m].to("cpu", non_blocking=True),
                                    d["is_seed"][a:a + m].to("cpu", non_blocking=True))
                a += self.n_hits[i]
        ev = self.torch.cuda.Event()
        ev.record(s)
        return ev

    def poll(self, slot, handle):
        return "ok" if handle.query() else None

    def idle(self, next_arrival, busy):
        GpuPoolBackend.idle(self, next_arrival, busy)

    def close(self):
        for c in self.ctxs:
            c.close()


def make_pool(events, device):
    """Concatenates host events into a device pool (inputs and outputs)."""
    import torch
    from .gen import concat_events
    b = concat_events(events)
    pool = {k: torch.from_numpy(v).to(device) for k, v in b.items() if isinstance(v, np.ndarray)}
    n = int(b["x"].size)
    pool["cluster_id"] = torch.empty(n, dtype=torch.int32, device=device)
    pool["is_seed"] = torch.empty(n, dtype=torch.uint8, device=device)
    pool["offsets"] = np.concatenate([[0], np.cumsum([e["x"].size for e in events])]).astype(np.int64)
    return pool


def plan_batch(sizes, max_hits, max_events):
    """How many events from the front of a FIFO form the next batch: as many
    as fit ``max_hits`` hits and ``max_events`` events (each event alone
    fits, so a non-empty queue always gives at least one)."""
    k = hits = 0
    for n in sizes:
        if k >= max_events or hits + n > max_hits:
            break
        hits += n
        k += 1
    return k


class _Slot:
    """One context, its stream, and its batch input columns (allocated once,
    max_batch_hits long): events are copied into them at their offsets."""

    def __init__(self, ctx, stream, max_hits, device):
        import torch
        self.ctx = ctx
        self.stream = stream
        self.inputs = {k: torch.empty(max_hits, dtype=dt, device=device) for k, dt in
                       (("x", torch.float32), ("y", torch.float32), ("layer", torch.int32),
                        ("energy", torch.float32), ("event", torch.int32))}


class Server:
    """Online served form: ``submit(x, y, layer, energy)`` queues one event and
    returns a ``concurrent.futures.Future`` of its ``(cluster_id, is_seed)``
    (int32 and uint8 device tensors, event-local as from ``Context.run``).

    A worker thread takes queued events in arrival order and, whenever one of
    the ``slots`` is free, copies a batch of them (up to ``max_batch_hits``
    hits and ``max_batch_events`` events) into the slot's input columns and
    runs the batched form on the slot's own stream; slots overlap on the GPU. Each
    event's result is a view of its batch's output tensors. The device memory
    the server works in is bounded when it is built (per slot: the context
    arena, the slot's batch input columns, allocated once, into which events
    are copied at their offsets, and one batch of outputs) and must fit
    ``hbm_budget`` bytes (0: no limit); events wait in the queue until a slot
    takes them.

    Inputs may be torch tensors on the server's device or on the host, or
    numpy arrays. Device inputs are read on the slot's stream after the work
    that the caller's current stream had queued when ``submit`` was called.
    An event with more than ``max_batch_hits`` hits fails its future with
    ValueError. With the VALIDATE flag every batch is checked when it
    completes and invalid input fails all futures of its batch; otherwise,
    as with ``Context``, device-side errors are deferred, here to ``close()``.
    Results are complete when their future resolves; they were allocated on
    the slot's stream, so work that a caller queues on another stream before
    dropping them should be covered by ``Tensor.record_stream``.
    """

    def __init__(self, dc, rho_c, delta_c, delta_o, *, max_batch_hits, max_batch_events=64, slots=2,
                 hbm_budget=0, extent=None, bounds=None, n_layers=100, tuning=None, flags=0, kernel="flat",
                 kernel_scale=0.0, device=None):
        import torch

        from . import Context, footprint_bytes
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
        self.max_batch_hits = int(max_batch_hits)
        self.max_batch_events = int(max_batch_events)
        per_slot = footprint_bytes(dc, rho_c, delta_c, delta_o, self.max_batch_hits, self.max_batch_events,
                                   extent=extent, bounds=bounds, n_layers=n_layers, flags=flags, kernel=kernel,
                                   kernel_scale=kernel_scale) + self.max_batch_hits * POOL_BYTES_PER_HIT
        self.device_bytes = int(slots) * per_slot
        if hbm_budget and self.device_bytes > hbm_budget:
            raise ValueError(f"{slots} slots need {self.device_bytes} B of device memory, more than the "
                             f"HBM budget of {hbm_budget} B")
        from . import VALIDATE
        self._validate = bool(flags & VALIDATE)
        self._slots = []
        try:
            for _ in range(int(slots)):
                ctx = Context(dc, rho_c, delta_c, delta_o, max_hits=self.max_batch_hits,
                              max_events=self.max_batch_events, extent=extent, bounds=bounds, n_layers=n_layers,
                              flags=flags, device=self.device.index, kernel=kernel, kernel_scale=kernel_scale)
                if tuning:
                    ctx.set_tuning(**tuning)
                sl = _Slot(ctx, torch.cuda.Stream(device=self.device), self.max_batch_hits, self.device)
                self._slots.append(sl)
                # one full batch of outputs, allocated and released on the slot's
                # stream, leaves its blocks in torch's cache for the batches to
                # come (the first batches then allocate nothing new)
                with torch.cuda.stream(sl.stream):
                    m = self.max_batch_hits
                    warm = [torch.empty(m, dtype=torch.int32, device=self.device),
                            torch.empty(m, dtype=torch.uint8, device=self.device)]
                    del warm
        except Exception:
            for sl in self._slots:
                sl.ctx.close()
            raise
        self._cv = threading.Condition()
        self._queue = deque()  # (n, inputs, ready event, future)
        self._closing = False
        self._thread = threading.Thread(target=self._serve, name="clue-server", daemon=True)
        self._thread.start()

    def _as_tensor(self, v, dtype, name, n):
        torch = self._torch
        t = v if isinstance(v, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(v))
        if t.dtype != dtype or t.dim() != 1 or t.numel() != n:
            raise TypeError(f"{name} must be a 1-D {dtype} array of {n} elements")
        if t.device.type != "cpu" and t.device != self.device:
            raise TypeError(f"{name} is on {t.device}, the server runs on {self.device}")
        return t

    def submit(self, x, y, layer, energy):
        """Queue one event; returns a Future of (cluster_id, is_seed)."""
        torch = self._torch
        fut = Future()
        n = int(x.numel()) if isinstance(x, torch.Tensor) else int(np.asarray(x).size)
        ins = (self._as_tensor(x, torch.float32, "x", n), self._as_tensor(y, torch.float32, "y", n),
               self._as_tensor(layer, torch.int32, "layer", n), self._as_tensor(energy, torch.float32, "energy", n))
        if n > self.max_batch_hits:
            fut.set_exception(ValueError(f"event of {n} hits exceeds max_batch_hits = {self.max_batch_hits}"))
            return fut
        ready = None
        if any(t.device.type != "cpu" for t in ins):
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(self.device))
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            self._queue.append((n, ins, ready, fut))
            self._cv.notify()
        return fut

    def _launch(self, slot, items):
        torch = self._torch
        sl = self._slots[slot]
        dev = self.device
        k = len(items)
        with torch.cuda.stream(sl.stream):
            for _, _, ready, _ in items:
                if ready is not None:
                    sl.stream.wait_event(ready)
            # each event's columns go straight into the slot's batch columns
            cols = sl.inputs
            a = 0
            for i, (n, ins, _, _) in enumerate(items):
                for name, t in zip(("x", "y", "layer", "energy"), ins):
                    cols[name][a:a + n].copy_(t, non_blocking=True)
                cols["event"][a:a + n].fill_(i)
                a += n
            total = a
            cid = torch.empty(total, dtype=torch.int32, device=dev)
            seed = torch.empty(total, dtype=torch.uint8, device=dev)
            sl.ctx.run_batch(cols["event"][:total], k, cols["x"][:total], cols["y"][:total], cols["layer"][:total],
                             cols["energy"][:total], cid, seed, stream=sl.stream)
            done = torch.cuda.Event()
            done.record(sl.stream)
        # each event's result is a view of the batch outputs
        outs, a = [], 0
        for n, _, _, fut in items:
            outs.append((fut, cid[a:a + n], seed[a:a + n]))
            a += n
        return done, outs, items

    def _finish(self, slot, outs, err=None):
        if err is None and self._validate:
            try:
                self._slots[slot].ctx.status(self._slots[slot].stream)
            except Exception as e:  # invalid input fails the whole batch
                err = e
        for fut, cid, seed in outs:
            if err is None:
                fut.set_result((cid, seed))
            else:
                fut.set_exception(err)

    def _serve(self):
        busy = {}  # slot -> (completion event, outputs, inputs held until done)
        try:
            self._loop(busy)
        except BaseException as e:  # the worker cannot go on: fail what it holds
            with self._cv:
                self._closing = True
                pending = [q[3] for q in self._queue]
                self._queue.clear()
            for _, outs, _ in busy.values():
                pending += [o[0] for o in outs]
            for fut in pending:
                if not fut.done():
                    fut.set_exception(RuntimeError(f"server worker stopped: {e!r}"))

    def _loop(self, busy):
        torch = self._torch
        torch.cuda.set_device(self.device)
        free = list(range(len(self._slots)))
        while True:
            launches = []
            with self._cv:
                while not self._queue and not busy and not self._closing:
                    self._cv.wait()
                if self._closing and not self._queue and not busy:
                    return
                while free and self._queue:
                    sizes = [q[0] for q in list(self._queue)[: self.max_batch_events]]
                    k = plan_batch(sizes, self.max_batch_hits, self.max_batch_events)
                    launches.append((free.pop(0), [self._queue.popleft() for _ in range(k)]))
            for slot, items in launches:
                try:
                    busy[slot] = self._launch(slot, items)
                except Exception as e:  # argument or launch error: fail this batch, keep serving
                    self._finish(slot, [(it[3], None, None) for it in items], err=e)
                    free.append(slot)
            progressed = False
            for slot in list(busy):
                done, outs, _ = busy[slot]
                if done.query():
                    del busy[slot]
                    self._finish(slot, outs)
                    free.append(slot)
                    progressed = True
            if busy and not progressed:
                time.sleep(2e-5)

    def close(self):
        """Serves every queued event, stops the worker and frees the slots;
        then raises a deferred device-side error of any slot, if there was one."""
        with self._cv:
            self._closing = True
            self._cv.notify()
        self._thread.join()
        err = None
        for sl in self._slots:
            try:
                sl.ctx.status(sl.stream)
            except Exception as e:
                err = err or e
            sl.ctx.close()
        self._slots = []
        if err is not None:
            raise err

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
