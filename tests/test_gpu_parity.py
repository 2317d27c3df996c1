"""GPU parity: the HIP path (through the C ABI) against the oracle, element
by element and bit for bit (rho, nh, delta^2, follower lists, cluster ids,
seed flags), plain and batched forms, across tunings and edge cases."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_parity, gpu_run
from golden_cases import load_cases
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
CASES = load_cases()


def _ref(ev, p, **kw):
    return oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=p["dc"], rho_c=p["rho_c"],
                      delta_c=p["delta_c"], delta_o=p["delta_o"], extent=p.get("extent"),
                      bounds=p.get("bounds"), n_layers=p["n_layers"], event=ev.get("event"),
                      n_events=ev.get("n_events"), kernel=p.get("kernel", "flat"),
                      kernel_scale=p.get("kernel_scale", 0.0), n_threads=NT, **kw)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
@pytest.mark.parametrize("batched", [False, True])
def test_hand_cases(case, batched):
    p = dict(case["params"])
    ev = case["event"]
    got = gpu_run(ev, p, batched=batched)
    assert np.array_equal(got["rho"].view(np.uint32), case["rho"].view(np.uint32)), (got["rho"], case["rho"])
    assert np.array_equal(got["nh"], case["nh"])
    assert np.array_equal(got["cluster_id"], case["cluster_id"])
    assert np.array_equal(got["is_seed"], case["is_seed"])
    assert np.array_equal(got["fstart"], case["fstart"]) and np.array_equal(got["flist"], case["flist"])


ADV_P = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("batched", [False, True])
def test_adversarial(seed, batched):
    ev = adversarial_event(seed, n=400 + 50 * seed, n_layers=3, unit_weights=seed % 2 == 1)
    assert_parity(gpu_run(ev, ADV_P, batched=batched), _ref(ev, ADV_P), where=f"adv{seed}")


TUNINGS = [
    dict(tile_size=2.5),                      # 3x3 density lists, halo 2
    dict(tile_size=2.1, block_x=4, block_y=4),
    dict(tile_size=8.0, block_x=2, block_y=2),  # 2x2 lists, few tiles
    dict(tile_size=25.0),                     # one tile covers the extent
    dict(threads_per_query=2),
    dict(threads_per_query=4, block_x=16, block_y=4),
    dict(threads_per_query=8),
    dict(lds_cap=64),                         # blocks overflow LDS: quarters, single tiles, then global
    dict(lds_cap=128),                        # quarter blocks fit where whole blocks do not
    dict(lds_cap=96, block_x=4, block_y=4),
    dict(lds_cap=64, tile_size=2.5, threads_per_query=4),
    dict(density_quads=3),                    # quad lists merged by one lane each
    dict(density_quads=3, tile_size=8.0, block_x=2, block_y=2, lds_cap=128),
    dict(density_quads=2),                    # per-query merges, no quad lists
    dict(nh_first_radius=0.0),                # single-phase nearest-higher search
    dict(nh_first_radius=0.5, threads_per_query=2),
    dict(nh_first_radius=3.99),
    dict(lds_cap=2048, block_x=16, block_y=16),
    dict(expansion=2),                        # k-way expansion: one thread per seed
    dict(plain_lds_cap=64),                   # plain form: fallbacks; batched form: default cap
    dict(lds_cap=64, plain_lds_cap=2048, block_x=16, block_y=16),
    dict(expansion=2, lds_cap=64, threads_per_query=4),
]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(t) for t in TUNINGS])
@pytest.mark.parametrize("batched", [False, True])
def test_tuning_invariance(tuning, batched):
    ev = adversarial_event(77, n=600, n_layers=3)
    assert_parity(gpu_run(ev, ADV_P, batched=batched, tuning=tuning), _ref(ev, ADV_P), where=str(tuning))


def test_config1():
    ev, p = gen.config1()
    ref = _ref(ev, p)
    assert_parity(gpu_run(ev, p), ref, where="cfg1 plain")
    assert_parity(gpu_run(ev, p, batched=True), ref, where="cfg1 batched")
    ev2, _ = gen.config1(shuffle=True)
    assert_parity(gpu_run(ev2, p), _ref(ev2, p), where="cfg1 shuffled")


@pytest.mark.parametrize("batched", [False, True])
def test_config2_full(batched):
    ev, p = gen.config2()
    assert_parity(gpu_run(ev, p, batched=batched), _ref(ev, p), where=f"cfg2 batched={batched}")


def test_config2_shuffled():
    ev, p = gen.config2(n_layers=20, shuffle=True)
    assert_parity(gpu_run(ev, p), _ref(ev, p), where="cfg2 shuffled")


@pytest.mark.parametrize("step", range(1, 11))
def test_config3_sweep(step):
    ev, p = gen.config3_sweep(step)
    assert_parity(gpu_run(ev, p, followers=False), _ref(ev, p, want=("rho", "nh", "delta2")),
                  where=f"cfg3 step {step}")


@pytest.mark.parametrize("dc", [1.0, 2.0, 3.0])
def test_config3_hard(dc):
    ev, p = gen.config3_hard(dc)
    assert_parity(gpu_run(ev, p), _ref(ev, p), where=f"cfg3 hard dc={dc}")


def test_batch_equals_events():
    """Batched run over several events == oracle per event, indices event-local."""
    evs = [adversarial_event(s, n=200 + 37 * s, n_layers=3) for s in range(7)]
    evs.insert(3, {k: v[:0] for k, v in evs[0].items()})  # an empty event in the middle
    batch = gen.concat_events(evs)
    ref = _ref(batch, ADV_P)
    got = gpu_run(batch, ADV_P, batched=True, n_events=batch["n_events"])
    assert_parity(got, ref, where="batch")


def test_config4_sample_events():
    """Four config-4 events (U[1k,10k] hits per layer) in one batch."""
    evs = [gen.config4_event(e) for e in range(4)]
    batch = gen.concat_events(evs)
    p = dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=100)
    assert_parity(gpu_run(batch, p, batched=True, n_events=4), _ref(batch, p), where="cfg4 sample")


def test_repeat_runs_bitwise_equal():
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    ev, p = gen.config2(n_layers=10)
    n = ev["x"].size
    t = to_dev(ev, torch.device("cuda", 0))
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=n, extent=p["extent"],
                      n_layers=p["n_layers"]) as ctx:
        first = [a.clone() for a in ctx.run(t["x"], t["y"], t["layer"], t["energy"])]
        for _ in range(20):
            cid, seed = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
            assert torch.equal(cid, first[0]) and torch.equal(seed, first[1])
        ev_ids = torch.zeros(n, dtype=torch.int32, device=t["x"].device)
        for _ in range(20):
            cid, seed = ctx.run_batch(ev_ids, 1, t["x"], t["y"], t["layer"], t["energy"])
            assert torch.equal(cid, first[0]) and torch.equal(seed, first[1])
        ctx.status()


def test_empty_and_single():
    z = {k: v[:0] for k, v in adversarial_event(1, n=10).items()}
    got = gpu_run(z, ADV_P, followers=False)
    assert got["cluster_id"].size == 0
    one = {k: v[:1] for k, v in adversarial_event(1, n=10).items()}
    assert_parity(gpu_run(one, ADV_P), _ref(one, ADV_P), where="single")


def test_dense_single_tile_and_outside_extent():
    """Every hit in one small spot (LDS overflow path) plus hits far outside
    the grid extent (clamped into edge tiles)."""
    rng = np.random.default_rng(5)
    n = 3000
    x = rng.normal(10, 0.7, n).astype(np.float32)
    y = rng.normal(10, 0.7, n).astype(np.float32)
    x[:50] = rng.uniform(-100, -50, 50)
    y[50:100] = rng.uniform(60, 90, 50)
    ev = dict(x=x, y=y, layer=np.zeros(n, np.int32), energy=rng.uniform(0, 1, n).astype(np.float32))
    p = dict(ADV_P, n_layers=1)
    assert_parity(gpu_run(ev, p), _ref(ev, p), where="dense")


def test_paper_strict_mode():
    import paper_2001_09761_amd as clue
    ev = adversarial_event(9, n=500, n_layers=2, unit_weights=True)
    p = dict(ADV_P, n_layers=2)
    got = gpu_run(ev, p, flags=clue.KEEP_INTERMEDIATES | clue.TIE_PAPER_STRICT)
    assert_parity(got, _ref(ev, p, paper_strict=True), where="strict")


def test_no_followers_flag():
    import paper_2001_09761_amd as clue
    ev = adversarial_event(10, n=500, n_layers=2)
    p = dict(ADV_P, n_layers=2)
    got = gpu_run(ev, p, flags=clue.KEEP_INTERMEDIATES | clue.NO_FOLLOWERS)
    assert_parity(got, _ref(ev, p), keys=("cluster_id", "is_seed", "rho", "nh", "delta2"), where="nofollow")


def test_validate_rejects_bad_input():
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    ev = adversarial_event(3, n=100, n_layers=1)
    ev["x"][7] = np.nan
    t = to_dev(ev, torch.device("cuda", 0))
    with clue.Context(2.0, 5.0, 2.0, 4.0, max_hits=100, bounds=(0, 0, 20, 20), n_layers=1,
                      flags=clue.VALIDATE) as ctx:
        with pytest.raises(clue.ClueError) as ei:
            ctx.run(t["x"], t["y"], t["layer"], t["energy"])
        assert ei.value.code == -5
        ev["x"][7] = 1.0
        ev["layer"][3] = 5
        t = to_dev(ev, torch.device("cuda", 0))
        with pytest.raises(clue.ClueError):
            ctx.run(t["x"], t["y"], t["layer"], t["energy"])


def test_capacity_and_argument_errors():
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    ev = adversarial_event(3, n=100, n_layers=1)
    t = to_dev(ev, torch.device("cuda", 0))
    with clue.Context(2.0, 5.0, 2.0, 4.0, max_hits=50, bounds=(0, 0, 20, 20), n_layers=1) as ctx:
        with pytest.raises(clue.ClueError) as ei:
            ctx.run(t["x"], t["y"], t["layer"], t["energy"])
        assert ei.value.code == -2
        ctx.reserve(100)
        ctx.run(t["x"], t["y"], t["layer"], t["energy"])
        ctx.status()
        with pytest.raises(clue.ClueError) as ei:
            ctx.set_tuning(tile_size=1.0)  # below dc: density window would span > 3 tiles
        assert ei.value.code == -1
    with pytest.raises(clue.ClueError):
        clue.Context(0.0, 5.0, 2.0, 4.0, max_hits=10, n_layers=1)


@pytest.mark.parametrize("hpl", [1000, 10000])
@pytest.mark.parametrize("tile", [0.0, 5.0])
def test_paper_workload(hpl, tile):
    """The paper's own study (Sec. 4.2): unit weights, sigma = 3 cm clusters,
    dc = 3, rho_c = 8, delta_c = delta_o = 5; at its 5 cm bin (windows span up
    to three tiles) and at the default tile."""
    ev, p = gen.paper_event(hpl)
    tuning = dict(tile_size=tile) if tile else None
    assert_parity(gpu_run(ev, p, tuning=tuning), _ref(ev, p), where=f"paper {hpl}/layer tile {tile}")


def test_paper_sweep_batched():
    """The paper's linear-scaling sweep (1k..10k hits per layer) as one batch."""
    evs = [gen.paper_event(1000 * s, event_index=s)[0] for s in range(1, 11)]
    batch = gen.concat_events(evs)
    p = dict(gen.PAPER_PARAMS, extent=200.0, n_layers=100)
    got = gpu_run(batch, p, batched=True, n_events=10, tuning=dict(tile_size=gen.PAPER_BIN))
    assert_parity(got, _ref(batch, p), where="paper sweep batched")


def test_events_at_and_beyond_packed_index_limit():
    """The nearest-higher search packs (event-local index, LDS position) into
    one word for events of up to 2**21 hits; larger events take the
    global-memory path. One batch holds an event of exactly 2**21 hits and one
    of 2.1M; the larger also runs alone in the plain form."""
    at, p_at = gen.config2(seed=12, event_index=6, n_layers=128, hits_per_layer=16384)
    beyond, p = gen.config2(seed=11, event_index=5, hits_per_layer=21000)
    assert at["x"].size == 2 ** 21 and beyond["x"].size > 2 ** 21
    p = dict(p, n_layers=128)
    batch = gen.concat_events([at, beyond])
    assert_parity(gpu_run(batch, p, batched=True, n_events=2), _ref(batch, p), where="2**21 and 2.1M batched")
    assert_parity(gpu_run(beyond, p), _ref(beyond, p), where="2.1M plain")


@pytest.mark.parametrize("n", [4095, 4096, 16383, 16384, 16385])
def test_scan_chunk_boundaries(n):
    """Seed numbering scans n + 1 elements in chunks of 256 threads x 16
    elements (plain launches) or x 64 (the batched form): hit counts whose
    n + 1 lands exactly on, or one past, a chunk edge of either form."""
    ev, p = gen.config2(seed=20 + n % 7, event_index=n, n_layers=1, hits_per_layer=n)
    ref = _ref(ev, p)
    assert_parity(gpu_run(ev, p), ref, where=f"n={n} plain")
    assert_parity(gpu_run(ev, p, batched=True), ref, where=f"n={n} batched")


def test_decreasing_event_ids_without_validation():
    """Event ids that decrease break the batched form's contract; without
    CLUE_VALIDATE the result is unspecified but the run must stay within its
    buffers. Here the first event's hits resume after the second's, so the
    second event's recorded first hit can lie past its own hits (the packed
    nearest-higher index would wrap; such regions take the global search).
    The run completes, reports no device error, and the context then clusters
    a valid batch bit-exactly."""
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    a = adversarial_event(21, n=3000, n_layers=2)
    b = adversarial_event(22, n=2000, n_layers=2)
    ev = {k: np.concatenate([a[k][:1500], b[k], a[k][1500:]]) for k in ("x", "y", "layer", "energy")}
    ev["event"] = np.r_[np.zeros(1500, np.int32), np.ones(2000, np.int32), np.zeros(1500, np.int32)]
    n = ev["x"].size
    p = dict(ADV_P, n_layers=2)
    dev = torch.device("cuda", 0)
    t = to_dev(ev, dev)
    with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=n, max_events=2,
                      bounds=p["bounds"], n_layers=2, flags=clue.KEEP_INTERMEDIATES) as ctx:
        for _ in range(3):
            cid, seed = ctx.run_batch(t["event"], 2, t["x"], t["y"], t["layer"], t["energy"])
            fs, fl = ctx.followers()
            torch.cuda.synchronize()
            ctx.status()
            assert set(np.unique(seed.cpu().numpy())) <= {0, 1}
            f = fs.cpu().numpy()
            assert f[0] == 0 and np.all(np.diff(f) >= 0) and f[-1] <= n
        good = gen.concat_events([a, b])
        got = gpu_run(good, p, batched=True, n_events=2, ctx=ctx)
    assert_parity(got, _ref(good, p), where="valid batch after decreasing ids")


@pytest.mark.parametrize("tuning", [None, dict(threads_per_query=1), dict(threads_per_query=8)])
def test_dense_cores_in_a_batch_go_through_the_spill_kernels(tuning):
    """Three events in one batched run (graph form): two hold a core of 1500
    hits in one tile next to sparse hits, so the density and nearest-higher
    stages queue those tiles' queries for the spill kernels (chunks of 256
    and of 256 / tpq queries, several per tile, from two events and several
    layers); the third event stays on the staged path. Every output equals
    the oracle's."""
    rng = np.random.default_rng(11)
    evs = []
    for e in range(3):
        x = rng.uniform(0, 20, 400).astype(np.float32)
        y = rng.uniform(0, 20, 400).astype(np.float32)
        layer = rng.integers(0, 3, 400).astype(np.int32)
        if e != 1:
            for L in (0, 2):
                x = np.concatenate([x, rng.normal(5.0 + 3 * e, 0.3, 1500).astype(np.float32)])
                y = np.concatenate([y, rng.normal(12.0, 0.3, 1500).astype(np.float32)])
                layer = np.concatenate([layer, np.full(1500, L, np.int32)])
        evs.append(dict(x=x, y=y, layer=layer, energy=rng.uniform(0.1, 1.0, x.size).astype(np.float32)))
    b = gen.concat_events(evs)
    print(f"dense cores in a batch: {b['x'].size} hits, tuning {tuning}", flush=True)
    assert_parity(gpu_run(b, ADV_P, batched=True, n_events=3, tuning=tuning), _ref(b, ADV_P), where="dense batch")


def test_dense_core_takes_the_global_merge_and_scales():
    """A core far denser than any LDS cap: m hits inside one tile, all within
    dc of one another, so every query has about m neighbours and exact
    densities need O(m^2) work in all. The tile's queries are queued for the
    spill kernels, which spread them over the GPU's workgroups; each query
    merges the window's index-sorted tile lists once. The run stays bit-exact,
    doubling m costs well under the 8x a rescan of the window per neighbour
    would, and 8000 hits in one tile take well under the 194 ms that one
    workgroup serving the whole tile took."""
    import torch
    import paper_2001_09761_amd as clue
    from gpu_helpers import to_dev
    times = {}
    for m in (4000, 8000):
        rng = np.random.default_rng(m)
        x = rng.normal(10.0, 0.3, m).astype(np.float32)
        y = rng.normal(10.0, 0.3, m).astype(np.float32)
        ev = dict(x=x, y=y, layer=np.zeros(m, np.int32), energy=rng.uniform(0.5, 1.5, m).astype(np.float32))
        p = dict(ADV_P, n_layers=1)
        print(f"dense core: m = {m}", flush=True)
        assert_parity(gpu_run(ev, p), _ref(ev, p), where=f"dense core m={m}")
        t = to_dev(ev, torch.device("cuda", 0))
        with clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=m, bounds=p["bounds"],
                          n_layers=1) as ctx:
            ctx.run(t["x"], t["y"], t["layer"], t["energy"])
            ms = []
            for _ in range(5):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                ctx.run(t["x"], t["y"], t["layer"], t["energy"])
                e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            ctx.status()
        times[m] = float(np.median(ms))
    print(f"dense core device ms: {times}", flush=True)
    assert times[8000] < 6.0 * times[4000], times
    assert times[8000] < 50.0, times


@pytest.mark.parametrize("tuning", [dict(lds_cap=2048, plain_lds_cap=2048, block_x=16, block_y=16),
                                    dict(lds_cap=1280, plain_lds_cap=1280)])
@pytest.mark.parametrize("batched", [False, True])
def test_staged_dense_tiles_long_lower_bound_searches(tuning, batched):
    """Tiles of 600, 250, 128 (a power of two) and 1 hits side by side, plus
    sparse hits, all in one staged region (an LDS cap above the region's
    total): the quad-list build's lower-bound searches then take ten
    power-of-two steps, with probes clamped at the ends of tiles of every
    size, including empty ones. Every output equals the oracle's."""
    rng = np.random.default_rng(21)

    def box(n, x0, x1, y0, y1):
        return rng.uniform(x0, x1, n).astype(np.float32), rng.uniform(y0, y1, n).astype(np.float32)

    parts = [box(600, 4.1, 7.9, 4.1, 7.9), box(250, 8.2, 11.9, 4.1, 7.9), box(128, 4.1, 7.9, 8.2, 11.9),
             (np.array([10.0], np.float32), np.array([10.0], np.float32)), box(100, 0.0, 20.0, 0.0, 20.0)]
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    layer = np.zeros(x.size, np.int32)
    xs, ys = box(300, 0.0, 20.0, 0.0, 20.0)  # a sparse second layer
    x, y = np.concatenate([x, xs]), np.concatenate([y, ys])
    layer = np.concatenate([layer, np.ones(300, np.int32)])
    order = rng.permutation(x.size)  # caller order unrelated to position
    ev = dict(x=x[order], y=y[order], layer=layer[order], energy=rng.uniform(0.1, 1.0, x.size).astype(np.float32))
    p = dict(ADV_P, n_layers=2)
    print(f"staged dense tiles: {x.size} hits, tuning {tuning}, batched {batched}", flush=True)
    assert_parity(gpu_run(ev, p, batched=batched, tuning=tuning), _ref(ev, p), where="staged dense tiles")


@pytest.mark.parametrize("tuning", [dict(density_quads=2, lds_cap=2048, plain_lds_cap=2048, block_x=16, block_y=16),
                                    dict(tile_size=2.5, lds_cap=2048, plain_lds_cap=2048, block_x=8, block_y=8)])
@pytest.mark.parametrize("batched", [False, True])
def test_staged_dense_tiles_per_query_merges(tuning, batched):
    """The same dense staged tiles through the per-query merges instead of
    quad lists: without quad lists at the default tile (12-byte records, the
    two-tile instance) and at a 2.5 cm tile, where a window spans three tiles
    (16-byte records, the three-tile instance). Tiles of more than 64 hits
    take the full merge. Every output equals the oracle's."""
    rng = np.random.default_rng(22)
    x = np.concatenate([rng.uniform(4.1, 7.9, 600), rng.uniform(8.2, 11.9, 250), rng.uniform(0.0, 20.0, 200)])
    y = np.concatenate([rng.uniform(4.1, 7.9, 600), rng.uniform(4.1, 7.9, 250), rng.uniform(0.0, 20.0, 200)])
    order = rng.permutation(x.size)
    ev = dict(x=x[order].astype(np.float32), y=y[order].astype(np.float32), layer=np.zeros(x.size, np.int32),
              energy=rng.uniform(0.1, 1.0, x.size).astype(np.float32))
    p = dict(ADV_P, n_layers=1)
    print(f"per-query merges on dense tiles: tuning {tuning}, batched {batched}", flush=True)
    assert_parity(gpu_run(ev, p, batched=batched, tuning=tuning), _ref(ev, p), where="per-query merges")



@pytest.mark.parametrize("tuning", [dict(tile_size=4.5, block_x=4, block_y=4, lds_cap=2048, plain_lds_cap=2048),
                                    dict(tile_size=4.5, block_x=8, block_y=8, lds_cap=64, plain_lds_cap=64),
                                    dict(tile_size=4.5, block_x=8, block_y=8, lds_cap=96, plain_lds_cap=96),
                                    dict(tile_size=4.5, block_x=4, block_y=4, density_quads=2, lds_cap=256,
                                         plain_lds_cap=256)])
@pytest.mark.parametrize("kernel", ["flat", "gaussian"])
@pytest.mark.parametrize("batched", [False, True])
def test_quad_lists_of_every_length_residue(tuning, kernel, batched):
    """Quad lists of every length modulo four, which the density queries read
    padded to a multiple of four entries with a record at infinite distance.
    On a 24 x 24 grid of 4.5 cm tiles, two layers hold 0..7 hits per tile, so
    the lists take every residue. The third layer is a checkerboard of single
    hits. With 8 x 8-tile blocks, an interior block stages 50 of them and its
    81 quads hold two each: 324 padded entries, which overflow the entry
    array at a 64-hit cap (the per-query merge runs instead) and fit at a
    96-hit cap; a corner block's 64 quads fill the 256 entries of the 64-hit
    cap exactly. Every output equals the oracle's, also with the Gaussian
    kernel, whose term is evaluated (and discarded) for the padding record."""
    rng = np.random.default_rng(23)
    t, nt = 4.5, 24
    xs, ys, ls = [], [], []
    for layer in range(3):
        for ty in range(nt):
            for tx in range(nt):
                k = (tx + nt * ty + 3 * layer) % 8 if layer < 2 else (tx + ty + 1) % 2
                xs.append(rng.uniform(tx * t + 0.01, (tx + 1) * t - 0.01, k))
                ys.append(rng.uniform(ty * t + 0.01, (ty + 1) * t - 0.01, k))
                ls.append(np.full(k, layer, np.int32))
    x, y, layer = np.concatenate(xs), np.concatenate(ys), np.concatenate(ls)
    order = rng.permutation(x.size)
    ev = dict(x=x[order].astype(np.float32), y=y[order].astype(np.float32), layer=layer[order],
              energy=rng.uniform(0.1, 1.0, x.size).astype(np.float32))
    p = dict(ADV_P, bounds=(0, 0, nt * t, nt * t), n_layers=3)
    if kernel != "flat":
        p.update(kernel=kernel, kernel_scale=1.0)
    print(f"quad lists of every residue: {x.size} hits, {kernel}, tuning {tuning}, batched {batched}", flush=True)
    assert_parity(gpu_run(ev, p, batched=batched, tuning=tuning), _ref(ev, p), where="quad list residues")


@pytest.mark.parametrize("tuning", [dict(tile_size=4.5, block_x=4, block_y=4, lds_cap=2048, plain_lds_cap=2048),
                                    dict(tile_size=4.5, block_x=3, block_y=5, lds_cap=256, plain_lds_cap=256,
                                         threads_per_query=8),
                                    dict(tile_size=4.5, block_x=5, block_y=3, lds_cap=2048, plain_lds_cap=2048,
                                         threads_per_query=1, nh_first_radius=0.0)])
@pytest.mark.parametrize("batched", [False, True])
def test_nh_core_positions_with_empty_rows(tuning, batched):
    """Nearest-higher reads each core query's staged position from an array
    filled per region row. Every third tile row is empty, the others hold
    0..6 hits per tile, so cores have empty rows, rows of one tile's hits and
    ragged rows, and interior blocks start their core past the region's first
    column; with phase 1 off every query goes through the phase-2 queue.
    Every output equals the oracle's."""
    rng = np.random.default_rng(24)
    t, nt = 4.5, 24
    xs, ys, ls = [], [], []
    for layer in range(2):
        for ty in range(nt):
            for tx in range(nt):
                k = 0 if (ty + layer) % 3 == 1 else (3 * tx + ty + layer) % 7
                xs.append(rng.uniform(tx * t + 0.01, (tx + 1) * t - 0.01, k))
                ys.append(rng.uniform(ty * t + 0.01, (ty + 1) * t - 0.01, k))
                ls.append(np.full(k, layer, np.int32))
    x, y, layer = np.concatenate(xs), np.concatenate(ys), np.concatenate(ls)
    order = rng.permutation(x.size)
    ev = dict(x=x[order].astype(np.float32), y=y[order].astype(np.float32), layer=layer[order],
              energy=rng.uniform(0.1, 1.0, x.size).astype(np.float32))
    p = dict(ADV_P, bounds=(0, 0, nt * t, nt * t), n_layers=2)
    print(f"nh core positions: {x.size} hits, tuning {tuning}, batched {batched}", flush=True)
    assert_parity(gpu_run(ev, p, batched=batched, tuning=tuning), _ref(ev, p), where="nh core positions")
