"""GPU: the served form and the autotuner.

Each event's result is the same alone and in the mix (continuous batching
over two slots on separate streams), bit for bit, and equal to the oracle;
clue_run_batch_range equals clue_run_batch; the autotuner's candidates all
reproduce the reference output."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import to_dev
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


def _params(n_layers):
    return dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=n_layers)


def _events(n, n_layers=8, seed=11):
    return [gen.config4_event(e, seed=seed, n_layers=n_layers) for e in range(n)]


def test_served_results_equal_alone_and_oracle():
    import torch
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd.serve import GpuPoolBackend, Scheduler, make_pool
    dev = torch.device("cuda", 0)
    evs = _events(40, n_layers=100)  # config-5 events: 100 layers x U[1000, 10000] hits
    p = _params(100)
    print(f"served parity: {len(evs)} events, {sum(e['x'].size for e in evs)} hits", flush=True)
    pool = make_pool(evs, dev)
    n_hits = [e["x"].size for e in evs]
    cap = 12 * max(n_hits)
    be = GpuPoolBackend(p, pool, slots=2, max_batch_hits=cap, max_batch_events=12)
    arrivals = gen.poisson_arrivals(20000.0, len(evs))  # fast enough that batches form
    st = Scheduler(be, hbm_budget_bytes=0, max_batch_hits=cap, max_batch_events=12).run(arrivals, n_hits)
    torch.cuda.synchronize()
    summ = st.summary()
    assert summ["events"] == len(evs) and summ["max_batch_events"] > 1, summ
    got_cid = pool["cluster_id"].cpu().numpy()
    got_seed = pool["is_seed"].cpu().numpy()
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=max(n_hits), extent=200.0,
                      n_layers=100) as ctx:
        for i, ev in enumerate(evs):
            a, z = int(pool["offsets"][i]), int(pool["offsets"][i + 1])
            t = to_dev(ev, dev)
            cid, seed = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
            assert np.array_equal(got_cid[a:z], cid.cpu().numpy()), f"event {i} differs in the mix"
            assert np.array_equal(got_seed[a:z], seed.cpu().numpy()), f"event {i} seeds differ in the mix"
            ref = oracle.run_event(ev, p, n_threads=NT, want=())
            assert np.array_equal(got_cid[a:z], ref["cluster_id"]), f"event {i} differs from the oracle"
            assert np.array_equal(got_seed[a:z], ref["is_seed"]), f"event {i} seeds differ from the oracle"
        ctx.status()
    be.close()


def test_run_batch_range_equals_run_batch():
    import torch
    import paper_2001_09761_amd as clue
    dev = torch.device("cuda", 0)
    evs = _events(6, seed=13)
    b = gen.concat_events(evs)
    t = to_dev(b, dev)
    n = b["x"].size
    p = _params(8)
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=n, max_events=6, extent=200.0,
                      n_layers=8) as ctx:
        cid, seed = ctx.run_batch(t["event"], 6, t["x"], t["y"], t["layer"], t["energy"])
        cid, seed = cid.clone(), seed.clone()
        # events 2..4 of a pool whose ids start at 100
        offs = np.concatenate([[0], np.cumsum([e["x"].size for e in evs])])
        a, z = int(offs[2]), int(offs[5])
        ev_ids = (t["event"][a:z] + 98).contiguous()
        c2 = torch.empty(z - a, dtype=torch.int32, device=dev)
        s2 = torch.empty(z - a, dtype=torch.uint8, device=dev)
        ctx.run_batch_range(100, 3, ev_ids, t["x"][a:z], t["y"][a:z], t["layer"][a:z], t["energy"][a:z], c2, s2)
        torch.cuda.synchronize()
        ctx.status()
        assert torch.equal(c2, cid[a:z]) and torch.equal(s2, seed[a:z])


def test_autotuner_keeps_outputs_identical(tmp_path):
    import torch
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd import autotune
    dev = torch.device("cuda", 0)
    evs = _events(4, seed=17)
    b = gen.concat_events(evs)
    t = to_dev(b, dev)
    p = _params(8)
    space = [("density_quads", [1, 2]), ("block", [(8, 8), (4, 4)]), ("tile_size", [5.0]),
             ("nh_first_radius", [0.0, 1.0]), ("threads_per_query", [1, 4]), ("lds_cap", [256])]
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=b["x"].size, max_events=4,
                      extent=200.0, n_layers=8) as ctx:
        best, table = autotune.autotune(ctx, t, 4, p, reps=1, space=space, log=None)
        assert len(table) >= 8 and best["ms"] > 0
        cid, _ = ctx.run_batch(t["event"], 4, t["x"], t["y"], t["layer"], t["energy"])
        ref = oracle.run_event(b, p, n_threads=NT, want=())
        assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"])
        # cache round trip
        key = autotune.cache_key(p, b["x"].size, 4)
        autotune.store_cached(key, best, str(tmp_path / "t.json"))
        assert autotune.load_cached(key, str(tmp_path / "t.json"))["tile_size"] == best["tile_size"]


def test_online_server_futures_equal_run():
    """Server.submit from host arrays and from device tensors: every future
    holds the event's result as Context.run gives it alone; batches form over
    two slots; an event above max_batch_hits fails its own future only."""
    import torch
    import paper_2001_09761_amd as clue
    dev = torch.device("cuda", 0)
    evs = _events(24, n_layers=6, seed=13)
    p = _params(6)
    cap = 4 * max(e["x"].size for e in evs)
    srv = clue.Server(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_batch_hits=cap, max_batch_events=8,
                      slots=2, extent=200.0, n_layers=6)
    futs = []
    with srv:
        for i, ev in enumerate(evs):
            if i % 2:
                t = to_dev(ev, dev)
                futs.append(srv.submit(t["x"], t["y"], t["layer"], t["energy"]))
            else:
                futs.append(srv.submit(ev["x"], ev["y"], ev["layer"], ev["energy"]))
        big = np.zeros(cap + 1, np.float32)
        f_big = srv.submit(big, big, np.zeros(cap + 1, np.int32), big)
        results = [f.result(timeout=60) for f in futs]
    with pytest.raises(ValueError):
        f_big.result(timeout=1)
    with pytest.raises(RuntimeError):
        srv.submit(evs[0]["x"], evs[0]["y"], evs[0]["layer"], evs[0]["energy"])
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=max(e["x"].size for e in evs),
                      extent=200.0, n_layers=6) as ctx:
        for i, (ev, (cid, seed)) in enumerate(zip(evs, results)):
            t = to_dev(ev, dev)
            rc, rs = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
            assert torch.equal(cid, rc) and torch.equal(seed, rs), f"event {i}"
            if i % 6 == 0:
                ref = oracle.run_event(ev, p, n_threads=NT, want=())
                assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"])
        ctx.status()


def test_plain_cap_tuner_keeps_outputs():
    """The plain-form LDS cap tuner: every cap gives the same output (it
    raises otherwise) and the chosen cap is applied."""
    import torch
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd.autotune import tune_plain_cap
    dev = torch.device("cuda", 0)
    ev = gen.config4_event(0, n_layers=5)
    p = _params(5)
    t = to_dev(ev, dev)
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=ev["x"].size, extent=200.0,
                      n_layers=5) as ctx:
        cap = tune_plain_cap(ctx, t, caps=(96, 256, 960), reps=3, log=None)
        assert cap in (96, 256, 960) and ctx.tuning()["plain_lds_cap"] == cap
        cid, _ = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
        ref = oracle.run_event(ev, p, n_threads=NT, want=())
        assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"])


def test_online_server_validate_fails_only_the_bad_batch():
    """With VALIDATE, an event holding a non-finite coordinate fails the
    futures of its batch with CLUE_ERR_INPUT; the server keeps serving and
    later events resolve normally."""
    import torch
    import paper_2001_09761_amd as clue
    dev = torch.device("cuda", 0)
    evs = _events(3, n_layers=4, seed=17)
    p = _params(4)
    bad = {k: v.copy() for k, v in evs[0].items() if isinstance(v, np.ndarray)}
    bad["x"][5] = np.nan
    cap = max(e["x"].size for e in evs)
    with clue.Server(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_batch_hits=cap, max_batch_events=1,
                     slots=1, extent=200.0, n_layers=4, flags=clue.VALIDATE) as srv:
        f_bad = srv.submit(bad["x"], bad["y"], bad["layer"], bad["energy"])
        with pytest.raises(clue.ClueError) as ei:
            f_bad.result(timeout=60)
        assert ei.value.code == -5
        goods = [srv.submit(e["x"], e["y"], e["layer"], e["energy"]) for e in evs[1:]]
        outs = [f.result(timeout=60) for f in goods]
    for e, (cid, _) in zip(evs[1:], outs):
        ref = oracle.run_event(e, p, n_threads=NT, want=())
        assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"])
