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
