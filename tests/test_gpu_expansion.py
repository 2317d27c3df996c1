"""GPU parity of the k-way expansion (Algorithm 3: one thread per seed walks
its follower tree) against the oracle, bit for bit, beside the default
pointer jumping; and the delta_o sweep of Fig. 4 (noise rejection) on the GPU.
"""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_parity, gpu_run
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
DFS = dict(expansion=2)


def _ref(ev, p, **kw):
    return oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=p["dc"], rho_c=p["rho_c"],
                      delta_c=p["delta_c"], delta_o=p["delta_o"], extent=p.get("extent"),
                      bounds=p.get("bounds"), n_layers=p["n_layers"], event=ev.get("event"),
                      n_events=ev.get("n_events"), n_threads=NT, **kw)


@pytest.mark.parametrize("batched", [False, True])
def test_dfs_config2(batched):
    ev, p = gen.config2()
    assert_parity(gpu_run(ev, p, batched=batched, tuning=DFS), _ref(ev, p), where=f"cfg2 dfs batched={batched}")


def test_dfs_batch_of_events():
    evs = [gen.config4_event(e, n_layers=20) for e in range(6)]
    ev = gen.concat_events(evs)
    p = dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=20)
    got = gpu_run(ev, p, batched=True, n_events=ev["n_events"], tuning=DFS)
    assert_parity(got, _ref(ev, p), where="cfg4 sample dfs")


def test_dfs_paper_workload():
    ev, p = gen.paper_event(10000, n_layers=10)
    assert_parity(gpu_run(ev, p, batched=True, tuning=dict(DFS, tile_size=gen.PAPER_BIN)), _ref(ev, p),
                  where="paper dfs")


def test_dfs_long_chain():
    """Equally spaced unit-weight hits on a line: the interior ties in rho, so
    every interior hit follows its higher-index neighbour, and one cluster is
    a single chain about n deep (the worst case for a one-thread walk)."""
    n = 20000
    x = (np.arange(n, dtype=np.float64) * 0.5 + 1.0).astype(np.float32)
    ev = dict(x=x, y=np.full(n, 5.0, np.float32), layer=np.zeros(n, np.int32), energy=np.ones(n, np.float32))
    p = dict(dc=2.0, rho_c=3.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 10002, 10), n_layers=1)
    ref = _ref(ev, p)
    assert ref["is_seed"].sum() == 1 and (ref["cluster_id"] == 0).sum() > n - 10
    for batched in (False, True):
        assert_parity(gpu_run(ev, p, batched=batched, tuning=DFS), ref, where=f"chain batched={batched}")


def test_dfs_without_follower_output():
    """CLUE_NO_FOLLOWERS with the k-way expansion: the context grows its arena
    for the lists the walks need, still reports no lists, and switching back
    to pointer jumping gives the same ids."""
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    ev = adversarial_event(21, n=800, n_layers=3)
    p = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
    ref = _ref(ev, p)
    t = to_dev(ev, torch.device("cuda", 0))
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=800, bounds=p["bounds"],
                      n_layers=3, flags=clue.NO_FOLLOWERS) as ctx:
        for expansion in (2, 1, 2):
            ctx.set_tuning(expansion=expansion)
            assert ctx.tuning()["expansion"] == expansion
            for run in ("plain", "batched"):
                if run == "plain":
                    cid, seed = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
                else:
                    ev_ids = torch.zeros(800, dtype=torch.int32, device=t["x"].device)
                    cid, seed = ctx.run_batch(ev_ids, 1, t["x"], t["y"], t["layer"], t["energy"])
                ctx.status()
                assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"]), (expansion, run)
                assert np.array_equal(seed.cpu().numpy(), ref["is_seed"].astype(np.uint8)), (expansion, run)
        with pytest.raises(clue.ClueError):
            ctx.followers()
        with pytest.raises(clue.ClueError):
            ctx.set_tuning(expansion=3)


@pytest.mark.parametrize("expansion", [1, 2])
def test_delta_o_sweep_fig4(expansion):
    """Fig. 4 on the GPU: for each delta_o the outputs equal the oracle's bit
    for bit; across the sweep the seeds and every clustered hit's id stay
    fixed while the noise set shrinks strictly at 10, 20 and 60."""
    ev, p = gen.noise_sweep_event()
    prev = None
    noise = []
    for do in (5.0,) + gen.NOISE_SWEEP_DELTA_O + (100.0,):
        q = dict(p, delta_o=do)
        got = gpu_run(ev, q, tuning=dict(expansion=expansion))
        assert_parity(got, _ref(ev, q), where=f"delta_o={do}")
        cid = got["cluster_id"]
        if prev is not None:
            assert np.array_equal(got["is_seed"], prev["is_seed"])
            kept = prev["cluster_id"] >= 0
            assert np.array_equal(cid[kept], prev["cluster_id"][kept])
            assert np.all((cid < 0) <= (prev["cluster_id"] < 0))
        noise.append(int((cid < 0).sum()))
        prev = got
    assert noise[0] > noise[1] > noise[2] > noise[3] >= noise[4], noise


def test_dfs_paper_strict_and_batches():
    """The k-way walk under the paper's strict ties (equal densities never
    higher) and over a batch whose events share no numbering."""
    import paper_2001_09761_amd as clue
    ev = adversarial_event(12, n=900, n_layers=3, unit_weights=True)
    p = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
    for batched in (False, True):
        got = gpu_run(ev, p, batched=batched, tuning=DFS, flags=clue.KEEP_INTERMEDIATES | clue.TIE_PAPER_STRICT)
        assert_parity(got, _ref(ev, p, paper_strict=True), where=f"strict dfs batched={batched}")
    evs = [adversarial_event(40 + e, n=300 + 40 * e, n_layers=3) for e in range(5)]
    b = gen.concat_events(evs)
    got = gpu_run(b, p, batched=True, n_events=b["n_events"], tuning=DFS)
    assert_parity(got, _ref(b, p), where="adversarial batch dfs")
