"""Oracle pins: hand-built cases and closed forms (no GPU).

Expected values are derived by hand from the paper's definitions (Eq. 3-5,
Algorithms 1-3) and stored in tests/golden/hand_cases.txt; closed forms are
computed in the test from geometry, not from the oracle."""
import numpy as np
import pytest

import oracle
from golden_cases import load_cases

CASES = load_cases()


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
@pytest.mark.parametrize("brute", [False, True])
def test_hand_case(case, brute):
    p = case["params"]
    ev = case["event"]
    o = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=p["dc"], rho_c=p["rho_c"],
                   delta_c=p["delta_c"], delta_o=p["delta_o"], bounds=p["bounds"],
                   n_layers=p["n_layers"], brute_force=brute)
    assert np.array_equal(o["rho"].view(np.uint32), case["rho"].view(np.uint32)), (o["rho"], case["rho"])
    assert np.array_equal(o["nh"], case["nh"]), (o["nh"], case["nh"])
    assert np.array_equal(o["cluster_id"], case["cluster_id"]), (o["cluster_id"], case["cluster_id"])
    assert np.array_equal(o["is_seed"], case["is_seed"])
    # follower lists F_i (Eq. 5), written out by hand in the fixture
    assert np.array_equal(o["fstart"], case["fstart"]), (o["fstart"], case["fstart"])
    assert np.array_equal(o["flist"], case["flist"]), (o["flist"], case["flist"])


def test_hand_cases_as_one_batch():
    """The hand cases that share one parameter set, run as consecutive events
    of one batch: every output stays event-local (nh, follower entries, ids
    from 0 per event) and the follower CSR offsets run over the whole batch.
    The expected CSR is assembled here from the hand-written per-case lists."""
    p0 = CASES[0]["params"]
    group = [c for c in CASES if c["params"] == p0]
    assert len(group) >= 5 and any(len(c["flist"]) >= 4 for c in group)
    cat = {k: np.concatenate([c["event"][k] for c in group]) for k in ("x", "y", "layer", "energy")}
    event = np.concatenate([np.full(c["event"]["x"].size, i, np.int32) for i, c in enumerate(group)])
    o = oracle.run(cat["x"], cat["y"], cat["layer"], cat["energy"], event=event, n_events=len(group),
                   dc=p0["dc"], rho_c=p0["rho_c"], delta_c=p0["delta_c"], delta_o=p0["delta_o"],
                   bounds=p0["bounds"], n_layers=p0["n_layers"], n_threads=3)
    fstart = [0]
    for c in group:
        fstart.extend((fstart[-1] + c["fstart"][1:]).tolist())
    flist = np.concatenate([c["flist"] for c in group])
    assert np.array_equal(o["fstart"], np.array(fstart, np.int32))
    assert np.array_equal(o["flist"], flist)
    assert np.array_equal(o["nh"], np.concatenate([c["nh"] for c in group]))
    assert np.array_equal(o["cluster_id"], np.concatenate([c["cluster_id"] for c in group]))
    assert np.array_equal(o["n_clusters"], np.array([c["is_seed"].sum() for c in group], np.int32))


def _lattice(nx, ny, pitch=1.0):
    gx, gy = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    return (gx.ravel() * pitch + 1.0).astype(np.float32), (gy.ravel() * pitch + 1.0).astype(np.float32)


@pytest.mark.parametrize("dc,expect", [(1.2, (3, 4, 5)), (1.7, (4, 6, 9))])
def test_lattice_density_closed_form(dc, expect):
    """Square lattice, unit weights: dc in (a, sqrt2 a) counts the 4-neighbourhood
    (corner 3, edge 4, interior 5); dc in (sqrt2 a, 2a) the 8-neighbourhood
    (corner 4, edge 6, interior 9). Eq. 3 with chi = 1 and self included."""
    nx = ny = 7
    x, y = _lattice(nx, ny)
    n = x.size
    o = oracle.run(x, y, np.zeros(n, np.int32), np.ones(n, np.float32), dc=dc, rho_c=1.0, delta_c=dc,
                   delta_o=dc, bounds=(0, 0, 9, 9))
    ix = np.tile(np.arange(nx), ny)
    iy = np.repeat(np.arange(ny), nx)
    border = (ix == 0).astype(int) + (ix == nx - 1) + (iy == 0) + (iy == ny - 1)
    want = np.where(border == 2, expect[0], np.where(border == 1, expect[1], expect[2]))
    assert np.array_equal(o["rho"], want.astype(np.float32))


def test_coincident_hits_closed_form():
    """c coincident hits of weight E: rho = c*E exactly for small c (Eq. 3)."""
    for c in (1, 2, 5, 17):
        x = np.full(c, 3.0, np.float32)
        o = oracle.run(x, x, np.zeros(c, np.int32), np.full(c, 0.5, np.float32), dc=1.0, rho_c=0.1,
                       delta_c=1.0, delta_o=1.0, bounds=(0, 0, 10, 10))
        assert np.all(o["rho"] == np.float32(0.5 * c))
        # all tie in rho: the largest index is the single seed, every other hit
        # follows the next index (d2 = 0 ties break to the smallest higher index)
        assert o["is_seed"].sum() == 1 and o["is_seed"][-1] == 1
        assert np.array_equal(o["nh"][:-1], np.arange(1, c, dtype=np.int32))
        assert np.all(o["cluster_id"] == 0)


def test_chain_depth():
    """A chain of increasing energy at 1 cm spacing with dc = 0.5: every hit is
    its own density, its nearest-higher is the next hit, and the single seed at
    the top labels the whole chain through a depth-(n-1) follower tree."""
    n = 500
    x = np.arange(n, dtype=np.float32)
    y = np.zeros(n, np.float32)
    e = (1.0 + np.arange(n)).astype(np.float32)
    o = oracle.run(x, y, np.zeros(n, np.int32), e, dc=0.5, rho_c=0.5, delta_c=2.0, delta_o=2.0,
                   bounds=(0, 0, n, 1))
    assert np.array_equal(o["rho"], e)
    assert np.array_equal(o["nh"][:-1], np.arange(1, n, dtype=np.int32)) and o["nh"][-1] == -1
    assert np.all(o["delta2"][:-1] == 1.0) and np.isinf(o["delta2"][-1])
    assert np.array_equal(o["is_seed"], (np.arange(n) == n - 1).astype(np.uint8))
    assert np.all(o["cluster_id"] == 0)
    # follower lists: F_{i+1} = [i]
    assert np.array_equal(np.diff(o["fstart"]), np.r_[0, np.ones(n - 1, int)])
    assert np.array_equal(o["flist"], np.arange(n - 1, dtype=np.int32))


def test_layers_do_not_interact():
    """Identical hits on two layers give identical per-layer results (one grid
    per layer, Sec. 2.1)."""
    from oracle_cases import adversarial_event
    ev = adversarial_event(11, n=200, n_layers=1)
    n = ev["x"].size
    x = np.concatenate([ev["x"], ev["x"]])
    y = np.concatenate([ev["y"], ev["y"]])
    e = np.concatenate([ev["energy"], ev["energy"]])
    lay = np.r_[np.zeros(n, np.int32), np.ones(n, np.int32)]
    kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20))
    two = oracle.run(x, y, lay, e, n_layers=2, **kw)
    one = oracle.run(ev["x"], ev["y"], np.zeros(n, np.int32), ev["energy"], n_layers=1, **kw)
    assert np.array_equal(two["rho"][:n], one["rho"]) and np.array_equal(two["rho"][n:], one["rho"])
    assert np.array_equal(two["nh"][:n], one["nh"])
    assert np.array_equal(two["nh"][n:], np.where(one["nh"] >= 0, one["nh"] + n, -1))
    k = one["n_clusters"][0]
    assert np.array_equal(two["cluster_id"][:n], one["cluster_id"])
    # second copy's seeds come after the first copy's in index order
    assert np.array_equal(two["cluster_id"][n:], np.where(one["cluster_id"] >= 0, one["cluster_id"] + k, -1))


def test_paper_strict_ties_split_clusters():
    """With the literal strict rho_j > rho_i of Eq. 4, coincident equal hits
    have no nearest-higher and every one becomes a seed; the (rho, index)
    order keeps them in one cluster."""
    x = np.full(4, 2.0, np.float32)
    kw = dict(dc=1.0, rho_c=1.0, delta_c=1.0, delta_o=1.0, bounds=(0, 0, 5, 5))
    strict = oracle.run(x, x, np.zeros(4, np.int32), np.ones(4, np.float32), paper_strict=True, **kw)
    total = oracle.run(x, x, np.zeros(4, np.int32), np.ones(4, np.float32), **kw)
    assert np.all(strict["nh"] == -1) and strict["is_seed"].sum() == 4
    assert np.array_equal(strict["cluster_id"], np.arange(4, dtype=np.int32))
    assert total["is_seed"].sum() == 1 and np.all(total["cluster_id"] == 0)


def test_bad_inputs_rejected():
    x = np.array([1.0, np.nan], np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.run(x, x, np.zeros(2, np.int32), np.ones(2, np.float32), dc=1, rho_c=1, delta_c=1,
                   delta_o=1, extent=5)
    x = np.array([1.0, 2.0], np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.run(x, x, np.array([0, 3], np.int32), np.ones(2, np.float32), dc=1, rho_c=1, delta_c=1,
                   delta_o=1, extent=5, n_layers=2)
    with pytest.raises(oracle.OracleError):
        oracle.run(x, x, np.zeros(2, np.int32), np.ones(2, np.float32), dc=0.0, rho_c=1, delta_c=1,
                   delta_o=1, extent=5)
    with pytest.raises(oracle.OracleError):
        oracle.run(x, x, np.zeros(2, np.int32), np.ones(2, np.float32), dc=1, rho_c=1, delta_c=1,
                   delta_o=1, extent=5, event=np.array([1, 0], np.int32), n_events=2)


def test_empty_input():
    z = np.zeros(0, np.float32)
    o = oracle.run(z, z, np.zeros(0, np.int32), z, dc=1, rho_c=1, delta_c=1, delta_o=1, extent=5,
                   n_layers=1)
    assert o["cluster_id"].size == 0 and o["n_clusters"][0] == 0
