"""The no-allocation entry point (clue_run_noalloc) through the C ABI: bit
for bit the same as clue_run, the plain one-event form it is a variant of,
on two calls in a row (the second smaller, over the first call's leftover
scratch), with no change in free device memory across a call; and its
refusals (too large, flags that need a context)."""
import numpy as np
import pytest

from paper_2001_09761_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(ev):
    return {k: torch.from_numpy(ev[k]).cuda() for k in ("x", "y", "layer", "energy")}


def _plain(ctx, t):
    cid, seed = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
    return cid, seed


def _outputs(n):
    return (torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            torch.full((n,), 7, dtype=torch.uint8, device="cuda"))


def _noalloc(p, t, tuning=None, flags=0, out=None):
    import paper_2001_09761_amd as clue
    n = t["x"].numel()
    cid, seed = _outputs(n) if out is None else out
    clue.run_noalloc(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], t["x"], t["y"], t["layer"], t["energy"],
                     cid, seed, extent=p["extent"], n_layers=p["n_layers"], flags=flags, tuning=tuning)
    return cid, seed


def test_noalloc_equals_clue_run_twice():
    import paper_2001_09761_amd as clue
    big, p = gen.config2(event_index=3)             # 1M hits, the largest workload event
    small, p_small = gen.config2(event_index=4, n_layers=37, hits_per_layer=7000)
    for ev, pp, name in ((big, p, "1M-hit event"), (small, p_small, "259k-hit event")):
        print(f"no-alloc parity: {name}, n = {ev['x'].size}", flush=True)
        t = _dev(ev)
        n = ev["x"].size
        with clue.Context(pp["dc"], pp["rho_c"], pp["delta_c"], pp["delta_o"], max_hits=n, extent=pp["extent"],
                          n_layers=pp["n_layers"]) as ctx:
            want_cid, want_seed = _plain(ctx, t)
            tuning = ctx.tuning()
            torch.cuda.synchronize()
            ctx.status()
        # default tuning: the same as a fresh context's
        cid, seed = _noalloc(pp, t)
        torch.cuda.synchronize()
        assert torch.equal(cid, want_cid) and torch.equal(seed, want_seed)
        # an explicit tuning, and no device allocation inside the call
        out = _outputs(n)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        cid2, seed2 = _noalloc(pp, t, tuning=dict(tuning, block_x=10, block_y=10, plain_lds_cap=768), out=out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert torch.equal(cid2, want_cid) and torch.equal(seed2, want_seed)


def test_noalloc_against_oracle_small():
    import oracle
    ev, p = gen.config1()
    ref = oracle.run_event(ev, p)
    cid, seed = _noalloc(p, _dev(ev))
    torch.cuda.synchronize()
    assert np.array_equal(cid.cpu().numpy(), ref["cluster_id"])
    assert np.array_equal(seed.cpu().numpy(), ref["is_seed"])


def test_noalloc_refusals():
    import paper_2001_09761_amd as clue
    from paper_2001_09761_amd._lib import ClueError
    ev, p = gen.config1()
    t = _dev(ev)
    for flags in (clue.VALIDATE, clue.KEEP_INTERMEDIATES):
        with pytest.raises(ClueError) as e:
            _noalloc(p, t, flags=flags)
        assert e.value.code == -1
    # a run whose arena exceeds the fixed scratch is refused before any launch
    n = 2_000_000
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    zi = torch.zeros(n, dtype=torch.int32, device="cuda")
    cid = torch.empty(n, dtype=torch.int32, device="cuda")
    seed = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(ClueError) as e:
        clue.run_noalloc(2.0, 5.0, 2.0, 4.0, z, z, zi, z, cid, seed, extent=200.0, n_layers=100)
    assert e.value.code == -2 and "scratch" in str(e.value)
