"""CPU backend for the serving scheduler: the oracle computes each batch and a
virtual clock models the GPU (service time per batch, optional slot failure)."""
import numpy as np

import oracle
from paper_2001_09761_amd.gen import concat_events


class FakeBackend:
    def __init__(self, events, params, *, slots=2, service_time=lambda hits: 1e-3 + hits * 1e-8,
                 fail_once_on_slot=None, slot_bytes=1 << 20):
        self.events = events
        self.params = params
        self.n_slots = slots
        self.service_time = service_time
        self.fail_once_on_slot = fail_once_on_slot
        self._slot_bytes = slot_bytes
        self.offsets = np.concatenate([[0], np.cumsum([e["x"].size for e in events])]).astype(np.int64)
        n = int(self.offsets[-1])
        self.cluster_id = np.full(n, -7, np.int32)
        self.is_seed = np.full(n, 7, np.uint8)
        self.t = 0.0
        self.inflight = {}
        self.launches = []

    def slot_bytes(self):
        return self._slot_bytes

    def start(self):
        self.t = 0.0
        return 0.0

    def now(self):
        return self.t

    def launch(self, slot, first, count):
        evs = self.events[first:first + count]
        hits = sum(e["x"].size for e in evs)
        fail = self.fail_once_on_slot is not None and slot == self.fail_once_on_slot
        if fail:
            self.fail_once_on_slot = None
        else:
            b = concat_events(evs)
            o = oracle.run(b["x"], b["y"], b["layer"], b["energy"], dc=self.params["dc"],
                           rho_c=self.params["rho_c"], delta_c=self.params["delta_c"],
                           delta_o=self.params["delta_o"], bounds=self.params.get("bounds"),
                           extent=self.params.get("extent"), n_layers=self.params["n_layers"],
                           event=b["event"], n_events=count, want=())
            a, z = int(self.offsets[first]), int(self.offsets[first + count])
            self.cluster_id[a:z] = o["cluster_id"]
            self.is_seed[a:z] = o["is_seed"]
        h = (self.t + self.service_time(hits), fail)
        self.inflight[slot] = h
        self.launches.append((slot, first, count, hits))
        return h

    def poll(self, slot, handle):
        t_done, fail = handle
        if self.t >= t_done:
            self.inflight.pop(slot, None)
            return "failed" if fail else "ok"
        return None

    def idle(self, next_arrival, busy):
        cands = [h[0] for h in self.inflight.values()]
        if next_arrival is not None:
            cands.append(next_arrival)
        if cands:
            self.t = max(self.t, min(cands))


class FakeStagedBackend(FakeBackend):
    """FakeBackend whose events must first be admitted into a staging ring of
    ``ring_hits`` hits (the host-resident serving variant's bookkeeping):
    admission fails while there is no contiguous room, a batch may only take
    events that sit back to back in the ring, and completed events free their
    range. Records the ring offset of every admission and the peak use."""

    def __init__(self, events, params, *, ring_hits, **kw):
        super().__init__(events, params, **kw)
        from paper_2001_09761_amd.serve import StagingRing
        self.ring = StagingRing(ring_hits)
        self.offs = {}
        self.peak_used = 0

    def admit(self, i, n_hits):
        off = self.ring.allocate(i, n_hits)
        if off is None:
            return False
        self.offs[i] = off
        self.peak_used = max(self.peak_used, self.ring.used_hits())
        return True

    def adjacent(self, i, j):
        return self.ring.adjacent(i, j)

    def release(self, run):
        for i in run:
            self.ring.release(i)
