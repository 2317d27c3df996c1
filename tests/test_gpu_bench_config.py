"""GPU parity at the benchmark's full sizes and launch configuration.

The timed workloads (32 distinct 1M-hit events in one batched run, and the
64-event batch of 100 layers x U[1000, 10000] hits) run with the shipped MI355X
tuning, as the benchmark runs them. Every event's cluster ids and seed flags
are compared with the oracle bit for bit, and so is every hit's density from a
second run of the same launch configuration that keeps the intermediates."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import to_dev
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
PARAMS = dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=100)


def _run(b, ne, keep):
    import torch
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd import autotune
    dev = torch.device("cuda", 0)
    t = to_dev(b, dev)
    n = b["x"].size
    with clue.Context(PARAMS["dc"], PARAMS["rho_c"], PARAMS["delta_c"], PARAMS["delta_o"], max_hits=n,
                      max_events=ne, extent=200.0, n_layers=100,
                      flags=clue.KEEP_INTERMEDIATES if keep else 0) as ctx:
        key = autotune.cache_key(PARAMS, n, ne)
        tun = autotune.load_cached(key, autotune.SHIPPED_CACHE)
        assert tun is not None, f"no shipped tuning for {key}"
        tun = dict(tun)
        tun["block"] = tuple(tun["block"])
        autotune._apply(ctx, tun)
        cid, seed = ctx.run_batch(t["event"], ne, t["x"], t["y"], t["layer"], t["energy"])
        rho = ctx.intermediates()["rho"] if keep else None
        torch.cuda.synchronize()
        ctx.status()
        return cid.cpu().numpy(), seed.cpu().numpy(), None if rho is None else rho.cpu().numpy()


def _check(events):
    b = gen.concat_events(events)
    ne = len(events)
    print(f"full-size batch: {ne} events, {b['x'].size} hits", flush=True)
    cid, seed, _ = _run(b, ne, keep=False)
    cid_k, seed_k, rho = _run(b, ne, keep=True)
    assert np.array_equal(cid, cid_k) and np.array_equal(seed, seed_k), "keeping intermediates changed the output"
    ref = oracle.run(b["x"], b["y"], b["layer"], b["energy"], event=b["event"], n_events=ne, n_threads=NT,
                     want=("rho",), **{k: PARAMS[k] for k in ("dc", "rho_c", "delta_c", "delta_o", "extent",
                                                               "n_layers")})
    offs = np.concatenate([[0], np.cumsum([e["x"].size for e in events])])
    for e in range(ne):
        a, z = offs[e], offs[e + 1]
        assert np.array_equal(cid[a:z], ref["cluster_id"][a:z]), f"event {e}: cluster ids differ"
        assert np.array_equal(seed[a:z], ref["is_seed"][a:z]), f"event {e}: seed flags differ"
        assert np.array_equal(rho[a:z].view(np.uint32), ref["rho"][a:z].view(np.uint32)), f"event {e}: rho differs"


def test_bench_headline_batch():
    events = [gen.config2(seed=1, event_index=e)[0] for e in range(32)]
    _check(events)


def test_bench_64_event_batch():
    events = [gen.config4_event(e) for e in range(64)]
    _check(events)
