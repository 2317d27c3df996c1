"""Serving scheduler on the CPU: oracle-backed fake backend, virtual clock.

Checks admission by HBM budget, continuous batching of consecutive pool
events, slot concurrency, failure re-queueing, and that every event's result
equals the result of clustering it alone."""
import numpy as np
import pytest

import oracle
from fake_backend import FakeBackend
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen
from paper_2001_09761_amd.serve import POOL_BYTES_PER_HIT, Scheduler

P = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)


def _events(n=12):
    return [adversarial_event(100 + i, n=60 + 13 * i, n_layers=3) for i in range(n)]


def _alone(ev):
    return oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=P["dc"], rho_c=P["rho_c"],
                      delta_c=P["delta_c"], delta_o=P["delta_o"], bounds=P["bounds"], n_layers=3, want=())


def _check_results(be, evs):
    for i, ev in enumerate(evs):
        a, z = int(be.offsets[i]), int(be.offsets[i + 1])
        ref = _alone(ev)
        assert np.array_equal(be.cluster_id[a:z], ref["cluster_id"]), i
        assert np.array_equal(be.is_seed[a:z], ref["is_seed"]), i


def _check_times(stats):
    for r in stats.records:
        assert r.t_arrival <= r.t_admit <= r.t_launch <= r.t_done


def test_all_events_served_and_equal_alone():
    evs = _events()
    be = FakeBackend(evs, P, slots=2)
    n_hits = [e["x"].size for e in evs]
    arrivals = gen.poisson_arrivals(2000.0, len(evs))
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=64).run(arrivals, n_hits)
    _check_results(be, evs)
    _check_times(st)
    assert sum(b[2] for b in st.batches) == len(evs)


def test_continuous_batching_forms_multi_event_batches():
    evs = _events(20)
    # slow service, fast arrivals: events queue up behind the busy slot
    be = FakeBackend(evs, P, slots=1, service_time=lambda h: 5e-3)
    arrivals = np.linspace(0, 2e-3, len(evs))
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=5).run(arrivals, [e["x"].size for e in evs])
    sizes = [b[2] for b in st.batches]
    assert sizes[0] == 1 and max(sizes) == 5 and sum(sizes) == 20
    # each batch is a run of consecutive pool events
    for slot, first, count, hits, *_ in st.batches:
        assert hits == sum(evs[i]["x"].size for i in range(first, first + count))
    _check_results(be, evs)


def test_batch_respects_hit_capacity():
    evs = _events(10)
    n_hits = [e["x"].size for e in evs]
    cap = max(n_hits) + 10
    be = FakeBackend(evs, P, slots=1, service_time=lambda h: 5e-3)
    st = Scheduler(be, max_batch_hits=cap, max_batch_events=64).run(np.zeros(len(evs)), n_hits)
    assert all(b[3] <= cap for b in st.batches)
    _check_results(be, evs)


def test_hbm_budget_limits_inflight_events():
    evs = _events(8)
    n_hits = [e["x"].size for e in evs]
    be = FakeBackend(evs, P, slots=3, slot_bytes=1000)
    budget = 3 * 1000 + max(n_hits) * POOL_BYTES_PER_HIT  # room for one event at a time
    st = Scheduler(be, hbm_budget_bytes=budget, max_batch_hits=10_000, max_batch_events=64).run(
        np.zeros(len(evs)), n_hits)
    assert st.max_inflight_bytes <= budget - 3 * 1000
    # at every moment the events of overlapping batches fit the budget
    for b in st.batches:
        live = [c for c in st.batches if c[4] <= b[4] < c[5]]
        assert sum(c[3] for c in live) * POOL_BYTES_PER_HIT <= budget - 3 * 1000
    _check_results(be, evs)
    # without a budget the same arrivals put more in flight at once
    be2 = FakeBackend(evs, P, slots=3, slot_bytes=1000)
    st2 = Scheduler(be2, max_batch_hits=10_000, max_batch_events=64).run(np.zeros(len(evs)), n_hits)
    assert st2.max_inflight_bytes > budget - 3 * 1000


def test_slots_overlap_when_budget_allows():
    evs = _events(6)
    be = FakeBackend(evs, P, slots=3, service_time=lambda h: 1e-2)
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=1).run(np.zeros(6), [e["x"].size for e in evs])
    starts = [b[4] for b in st.batches[:3]]
    assert len(set(b[0] for b in st.batches[:3])) == 3 and max(starts) - min(starts) < 1e-2


def test_failed_slot_requeues_and_results_still_equal_alone():
    evs = _events(10)
    be = FakeBackend(evs, P, slots=2, fail_once_on_slot=0, service_time=lambda h: 2e-3)
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=4).run(np.zeros(len(evs)),
                                                                         [e["x"].size for e in evs])
    assert st.failures == 1
    assert any(r.attempts == 2 for r in st.records)
    _check_results(be, evs)
    _check_times(st)


def test_event_larger_than_budget_or_slot_is_rejected():
    evs = _events(3)
    n_hits = [e["x"].size for e in evs]
    be = FakeBackend(evs, P, slots=1, slot_bytes=100)
    with pytest.raises(ValueError):
        Scheduler(be, hbm_budget_bytes=100 + 10, max_batch_hits=10_000, max_batch_events=8).run(np.zeros(3), n_hits)
    with pytest.raises(ValueError):
        Scheduler(be, max_batch_hits=10, max_batch_events=8).run(np.zeros(3), n_hits)
    with pytest.raises(ValueError):
        Scheduler(be, hbm_budget_bytes=50, max_batch_hits=10_000, max_batch_events=8)


def test_summary_fields():
    evs = _events(5)
    be = FakeBackend(evs, P, slots=2)
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=8).run(gen.poisson_arrivals(500.0, 5),
                                                                        [e["x"].size for e in evs])
    s = st.summary()
    assert s["events"] == 5 and s["p99_ms"] >= s["p50_ms"] > 0 and s["hits"] == sum(e["x"].size for e in evs)


def test_plan_batch_takes_the_longest_fitting_prefix():
    from paper_2001_09761_amd.serve import plan_batch
    assert plan_batch([], 100, 4) == 0
    assert plan_batch([10], 10, 1) == 1
    assert plan_batch([5, 5, 5], 12, 10) == 2          # hit capacity
    assert plan_batch([5, 5, 5], 100, 2) == 2          # event capacity
    assert plan_batch([3, 9, 1], 10, 10) == 1          # FIFO: no reordering past a large event
    rng = np.random.default_rng(3)
    for _ in range(200):
        sizes = list(rng.integers(1, 50, rng.integers(1, 20)))
        cap_h, cap_e = int(rng.integers(50, 200)), int(rng.integers(1, 10))
        k = plan_batch(sizes, cap_h, cap_e)
        assert 1 <= k <= min(cap_e, len(sizes)) and sum(sizes[:k]) <= cap_h
        assert k == min(cap_e, len(sizes)) or sum(sizes[:k + 1]) > cap_h


def test_staging_ring_ranges_never_overlap():
    """Random admissions and out-of-order releases: every live range lies in
    the region, no two overlap, a range is freed for reuse only after all
    older ones, and an empty ring always takes an event that fits."""
    from paper_2001_09761_amd.serve import StagingRing
    rng = np.random.default_rng(0)
    for trial in range(40):
        cap = int(rng.integers(50, 400))
        ring = StagingRing(cap)
        live = {}
        nxt = 0
        for _ in range(300):
            if live and rng.random() < 0.45:
                k = int(rng.choice(list(live)))
                ring.release(k)
                del live[k]
            else:
                n = int(rng.integers(1, cap // 2 + 1))
                off = ring.allocate(nxt, n)
                if not live:
                    assert off == 0
                if off is not None:
                    assert 0 <= off and off + n <= cap
                    live[nxt] = (off, n)
                nxt += 1
            held = sorted((e[1], e[1] + e[2]) for e in ring.live)
            for (a0, a1), (b0, b1) in zip(held, held[1:]):
                assert a1 <= b0, (trial, held)
            assert ring.used_hits() <= cap
    with pytest.raises(ValueError):
        StagingRing(10).allocate(0, 11)


def test_staged_admission_waits_for_room_and_batches_stay_contiguous():
    """A staging ring that holds about two events: admission waits (the
    budget binds), batches only take events adjacent in the ring, the ring
    is never over-committed, and every result equals the event alone."""
    evs = _events(12)
    n_hits = [e["x"].size for e in evs]
    from fake_backend import FakeStagedBackend
    ring = 2 * max(n_hits) + 5
    be = FakeStagedBackend(evs, P, ring_hits=ring, slots=2, service_time=lambda h: 3e-3)
    st = Scheduler(be, max_batch_hits=10_000, max_batch_events=8).run(np.zeros(len(evs)), n_hits)
    _check_results(be, evs)
    _check_times(st)
    s = st.summary()
    assert s["admit_wait_p99_ms"] > 0 and be.peak_used <= ring
    for slot, first, count, hits, *_ in st.batches:
        for i in range(first, first + count - 1):
            assert be.offs[i + 1] == be.offs[i] + n_hits[i]
    assert sum(b[2] for b in st.batches) == len(evs)
