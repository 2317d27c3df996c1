"""Pin P1: the fixed grid never changes a result (Eq. 1 is a superset of Eq. 2).

The oracle's grid form must equal its O(n^2) form bit for bit (rho, rho64,
nh, delta2, followers, labels) on tiny adversarial events, for every bin size
from a third of dc to larger than the whole extent."""
import numpy as np
import pytest

import oracle
from oracle_cases import adversarial_event

KEYS = ("rho", "rho64", "nh", "delta2", "cluster_id", "is_seed", "fstart", "flist")


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("unit", [False, True])
def test_grid_equals_bruteforce(seed, unit):
    dc = 2.0
    ev = adversarial_event(seed, n=300 + 20 * seed, n_layers=1 + seed % 3, unit_weights=unit, dc=dc)
    kw = dict(dc=dc, rho_c=3.0 if unit else 5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20),
              n_layers=3)
    ref = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], brute_force=True, **kw)
    for b in (dc / 3, dc, 4.0, 12.0, 50.0):
        o = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], bin_size=b, **kw)
        for k in KEYS:
            assert np.array_equal(o[k], ref[k]), (k, b)


def test_threads_do_not_change_results():
    ev = adversarial_event(42, n=400, n_layers=3)
    kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
    a = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], n_threads=1, **kw)
    b = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], n_threads=3, **kw)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_multi_event_equals_separate_events():
    """Events are independent and indices are event-local."""
    evs = [adversarial_event(s, n=150, n_layers=2) for s in (1, 2, 3)]
    kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=2)
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("x", "y", "layer", "energy")}
    event = np.concatenate([np.full(e["x"].size, i, np.int32) for i, e in enumerate(evs)])
    batch = oracle.run(cat["x"], cat["y"], cat["layer"], cat["energy"], event=event, n_events=3, **kw)
    off = 0
    for i, e in enumerate(evs):
        one = oracle.run(e["x"], e["y"], e["layer"], e["energy"], **kw)
        sl = slice(off, off + e["x"].size)
        for k in ("rho", "nh", "delta2", "cluster_id", "is_seed"):
            assert np.array_equal(batch[k][sl], one[k]), (i, k)
        assert batch["n_clusters"][i] == one["n_clusters"][0]
        off += e["x"].size


def _followers_from_links(o, event, params):
    """F_i of Eq. 5 rebuilt from the oracle's per-hit decision inputs: hit j is
    registered with i = nh_j exactly when it is neither a seed (rho > rho_c
    and delta > delta_c) nor an outlier (rho < rho_c and delta > delta_o) and
    has a nearest-higher; lists hold event-local indices in ascending order
    and the CSR offsets run over the whole batch in caller order."""
    rho, d2, nh = o["rho"], o["delta2"], o["nh"]
    n = rho.size
    f32 = np.float32
    seed = (rho > f32(params["rho_c"])) & (d2 > f32(params["delta_c"]) * f32(params["delta_c"]))
    outl = (rho < f32(params["rho_c"])) & (d2 > f32(params["delta_o"]) * f32(params["delta_o"]))
    follower = ~seed & ~outl & (nh >= 0)
    first = np.zeros(n, np.int64)
    starts = np.r_[0, np.nonzero(np.diff(event))[0] + 1]
    for s, e in zip(starts, np.r_[starts[1:], n]):
        first[s:e] = s
    lists = [[] for _ in range(n)]
    for j in range(n):  # ascending j: each list fills in ascending order
        if follower[j]:
            lists[first[j] + nh[j]].append(j - first[j])
    fstart = np.zeros(n + 1, np.int32)
    fstart[1:] = np.cumsum([len(v) for v in lists])
    flist = np.array([v for vs in lists for v in vs], np.int32)
    return seed, fstart, flist


@pytest.mark.parametrize("seed", range(3))
def test_follower_lists_multi_event(seed):
    """Pin of the follower lists (Eq. 5; Algorithm 3, first loop) over a
    multi-event batch with lists of several entries: membership, ascending
    event-local entries and batch-global CSR offsets, rebuilt in numpy from
    the per-hit nh, rho and delta^2."""
    evs = [adversarial_event(100 * seed + s, n=250, n_layers=2) for s in range(4)]
    kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=2)
    cat = {k: np.concatenate([e[k] for e in evs]) for k in ("x", "y", "layer", "energy")}
    event = np.concatenate([np.full(e["x"].size, i, np.int32) for i, e in enumerate(evs)])
    o = oracle.run(cat["x"], cat["y"], cat["layer"], cat["energy"], event=event, n_events=len(evs),
                   n_threads=2, **kw)
    is_seed, fstart, flist = _followers_from_links(o, event, kw)
    assert np.array_equal(o["is_seed"].astype(bool), is_seed)
    lens = np.diff(fstart)
    assert lens.max() >= 3 and (lens >= 2).sum() >= 10  # lists of several entries occur
    assert np.array_equal(o["fstart"], fstart)
    assert np.array_equal(o["flist"], flist)
    # each event's lists equal the same event run alone
    off = 0
    for e in evs:
        n1 = e["x"].size
        one = oracle.run(e["x"], e["y"], e["layer"], e["energy"], **kw)
        seg = o["flist"][o["fstart"][off]:o["fstart"][off + n1]]
        assert np.array_equal(seg, one["flist"])
        assert np.array_equal(o["fstart"][off:off + n1 + 1] - o["fstart"][off], one["fstart"])
        off += n1
