"""GPU: the host-resident batched form (clue_run_batch_host).

Host arrays are streamed through a context smaller than the batch, in chunks
of whole events with copies overlapping the kernels; the results equal the
device-resident batched form bit for bit, and the oracle."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import to_dev
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
P = dict(gen.DEFAULT_PARAMS, extent=200.0, n_layers=8)


def _events(n=7, seed=21):
    return [gen.config4_event(e, seed=seed, n_layers=8) for e in range(n)]


def _ctx(max_hits, max_events):
    import paper_2001_09761_amd as clue
    return clue.Context(P["dc"], P["rho_c"], P["delta_c"], P["delta_o"], max_hits=max_hits, max_events=max_events,
                        extent=200.0, n_layers=8)


def _device_reference(b, ne):
    import torch
    t = to_dev(b, torch.device("cuda", 0))
    with _ctx(b["x"].size, ne) as ctx:
        cid, seed = ctx.run_batch(t["event"], ne, t["x"], t["y"], t["layer"], t["energy"])
        torch.cuda.synchronize()
        ctx.status()
        return cid.cpu().numpy(), seed.cpu().numpy()


@pytest.mark.parametrize("pinned", [False, True])
def test_host_form_chunks_equal_device_form(pinned):
    import torch
    evs = _events()
    b = gen.concat_events(evs)
    ne = len(evs)
    sizes = [e["x"].size for e in evs]
    cap = int(max(sizes) * 2.5)  # about two events per chunk
    arrays = {k: b[k] for k in ("event", "x", "y", "layer", "energy")}
    if pinned:
        arrays = {k: torch.from_numpy(v).pin_memory() for k, v in arrays.items()}
    with _ctx(cap, ne) as ctx:
        cid, seed = ctx.run_batch_host(arrays["event"], ne, arrays["x"], arrays["y"], arrays["layer"],
                                       arrays["energy"])
        cid2, seed2 = ctx.run_batch_host(arrays["event"], ne, arrays["x"], arrays["y"], arrays["layer"],
                                         arrays["energy"])
    ref_cid, ref_seed = _device_reference(b, ne)
    assert np.array_equal(cid, ref_cid) and np.array_equal(seed, ref_seed)
    assert np.array_equal(cid2, ref_cid) and np.array_equal(seed2, ref_seed)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for e in (0, ne - 1):
        ref = oracle.run_event(evs[e], P, n_threads=NT, want=())
        assert np.array_equal(cid[offs[e]:offs[e + 1]], ref["cluster_id"])


def test_host_form_single_event_and_empty():
    ev = _events(1, seed=22)[0]
    with _ctx(ev["x"].size, 1) as ctx:
        cid, seed = ctx.run_batch_host(None, 1, ev["x"], ev["y"], ev["layer"], ev["energy"])
        ref = oracle.run_event(ev, P, n_threads=NT, want=())
        assert np.array_equal(cid, ref["cluster_id"]) and np.array_equal(seed, ref["is_seed"])
        z = np.zeros(0, np.float32)
        cid0, seed0 = ctx.run_batch_host(None, 1, z, z, np.zeros(0, np.int32), z)
        assert cid0.size == 0 and seed0.size == 0


def test_host_form_event_larger_than_capacity():
    import paper_2001_09761_amd as clue
    evs = _events(3, seed=23)
    b = gen.concat_events(evs)
    with _ctx(min(e["x"].size for e in evs) - 1, 3) as ctx:
        with pytest.raises(clue.ClueError) as ei:
            ctx.run_batch_host(b["event"], 3, b["x"], b["y"], b["layer"], b["energy"])
        assert ei.value.code == -2  # CLUE_ERR_CAPACITY
