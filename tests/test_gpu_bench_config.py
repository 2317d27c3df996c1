"""GPU parity at the benchmark's full sizes and launch configuration.

The timed workloads (32 distinct 1M-hit events in one batched run, and the
64-event batch of 100 layers x U[1000, 10000] hits) run with the shipped MI355X
tuning. Sampled events are compared with the oracle bit for bit; every event is
compared with a run at the default tuning (the tuning may change speed only)."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import to_dev
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
PARAMS = dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=100)


def _run(events, tuned):
    import torch
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd import autotune
    dev = torch.device("cuda", 0)
    b = gen.concat_events(events)
    t = to_dev(b, dev)
    n, ne = b["x"].size, len(events)
    with clue.Context(PARAMS["dc"], PARAMS["rho_c"], PARAMS["delta_c"], PARAMS["delta_o"], max_hits=n,
                      max_events=ne, extent=200.0, n_layers=100) as ctx:
        if tuned:
            key = autotune.cache_key(PARAMS, n, ne)
            tun = autotune.load_cached(key, autotune.SHIPPED_CACHE)
            assert tun is not None, f"no shipped tuning for {key}"
            tun = dict(tun)
            tun["block"] = tuple(tun["block"])
            autotune._apply(ctx, tun)
        cid, seed = ctx.run_batch(t["event"], ne, t["x"], t["y"], t["layer"], t["energy"])
        torch.cuda.synchronize()
        ctx.status()
        return b, cid.cpu().numpy(), seed.cpu().numpy()


def _check(events, sample):
    b, cid, seed = _run(events, tuned=True)
    _, cid0, seed0 = _run(events, tuned=False)
    assert np.array_equal(cid, cid0) and np.array_equal(seed, seed0), "shipped tuning changed the output"
    offs = np.concatenate([[0], np.cumsum([e["x"].size for e in events])])
    for e in sample:
        a, z = offs[e], offs[e + 1]
        ref = oracle.run_event(events[e], PARAMS, n_threads=NT, want=())
        assert np.array_equal(cid[a:z], ref["cluster_id"]), f"event {e}: cluster ids differ"
        assert np.array_equal(seed[a:z], ref["is_seed"]), f"event {e}: seed flags differ"
    # every event: ids are 0..k-1 with k = number of seeds, noise is -1
    for e in range(len(events)):
        c, s = cid[offs[e]:offs[e + 1]], seed[offs[e]:offs[e + 1]]
        k = int(s.sum())
        assert c.min() >= -1 and c.max() == k - 1
        assert np.array_equal(np.sort(c[s == 1]), np.arange(k))


def test_bench_headline_batch():
    events = [gen.config2(seed=1, event_index=e)[0] for e in range(32)]
    _check(events, sample=[0, 13, 31])


def test_bench_64_event_batch():
    events = [gen.config4_event(e) for e in range(64)]
    _check(events, sample=[0, 63])
