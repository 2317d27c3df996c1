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
HIP library on a device-resident event pool; tests also drive it with a CPU
backend and a virtual clock.
"""
from __future__ import annotations

import gc
import time
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

    def summary(self):
        lat = self.latencies()
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
                    max_inflight_bytes=int(self.max_inflight_bytes), failures=self.failures)


class Scheduler:
    """Admission by HBM budget and continuous batching over backend slots."""

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
            while queued and (self.event_budget is None or
                              inflight + self.footprint(recs[queued[0]].n_hits) <= self.event_budget):
                i = queued.pop(0)
                recs[i].t_admit = now
                inflight += self.footprint(recs[i].n_hits)
                admitted.append(i)
            stats.max_inflight_bytes = max(stats.max_inflight_bytes, inflight)
            # launch: one batch per free slot, a maximal run of consecutive events
            while free and admitted:
                run = [admitted[0]]
                hits = recs[admitted[0]].n_hits
                k = 1
                while (k < len(admitted) and admitted[k] == run[-1] + 1 and len(run) < self.max_batch_events
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
            if not progressed and not (free and admitted) and not (queued and self.event_budget is None):
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
