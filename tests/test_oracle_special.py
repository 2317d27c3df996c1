"""Oracle pins against library routines and an independent algorithm.

P3: with unit weights rho_i is the number of points within dc, which
    scipy's KD-tree counts independently (inputs keep every pair at least 1e-4
    away from dc so the open/closed ball and float32 rounding cannot differ).
P3: the follower forest (each non-seed, non-outlier hit linked to its
    nearest-higher) has exactly one root per connected component
    (scipy.sparse.csgraph), and a hit's label is its root's seed id or -1.
P4: labels equal an independent CFSFDP-style assignment that visits hits in
    decreasing (rho, index) order and copies the label of the nearest-higher
    (the assignment CLUE replaces, Sec. 2 intro and Sec. 2.2).
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

import oracle
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen


def _far_from_dc(x, y, layer, dc, tol=1e-4):
    keep = np.ones(x.size, bool)
    pts = np.stack([x, y], 1).astype(np.float64)
    for lay in np.unique(layer):
        idx = np.nonzero(layer == lay)[0]
        d = np.sqrt(((pts[idx, None, :] - pts[None, idx, :]) ** 2).sum(-1))
        bad = np.abs(d - dc) < tol
        np.fill_diagonal(bad, False)
        # drop one endpoint of every ambiguous pair
        for a, b in zip(*np.nonzero(np.triu(bad))):
            if keep[idx[a]] and keep[idx[b]]:
                keep[idx[b]] = False
    return keep


@pytest.mark.parametrize("seed", range(4))
def test_unit_weight_density_is_kdtree_count(seed):
    dc = 1.5 + 0.25 * seed
    ev = adversarial_event(100 + seed, n=400, n_layers=2, unit_weights=True, dc=dc)
    keep = _far_from_dc(ev["x"], ev["y"], ev["layer"], dc)
    ev = {k: v[keep] for k, v in ev.items()}
    o = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=dc, rho_c=3, delta_c=2, delta_o=4,
                   bounds=(0, 0, 20, 20), n_layers=2)
    pts = np.stack([ev["x"], ev["y"]], 1).astype(np.float64)
    for lay in (0, 1):
        idx = np.nonzero(ev["layer"] == lay)[0]
        tree = cKDTree(pts[idx])
        cnt = tree.query_ball_point(pts[idx], r=dc, return_length=True)
        assert np.array_equal(o["rho"][idx], cnt.astype(np.float32))


def _forest_checks(o, rho_c, delta_c, delta_o):
    n = o["rho"].size
    seed = o["is_seed"].astype(bool)
    outlier = (o["rho"] < np.float32(rho_c)) & (o["delta2"] > np.float32(delta_o) * np.float32(delta_o))
    follower = ~seed & ~outlier & (o["nh"] >= 0)
    src = np.nonzero(follower)[0]
    g = coo_matrix((np.ones(src.size), (src, o["nh"][src])), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    roots = np.nonzero(~follower)[0]
    # one root per component
    assert np.array_equal(np.bincount(comp[roots], minlength=ncomp), np.ones(ncomp, int))
    root_of_comp = np.empty(ncomp, int)
    root_of_comp[comp[roots]] = roots
    root = root_of_comp[comp]
    seed_id = np.cumsum(seed) - 1
    want = np.where(seed[root], seed_id[root], -1)
    assert np.array_equal(o["cluster_id"], want.astype(np.int32))


@pytest.mark.parametrize("seed", range(3))
def test_labels_follow_forest_components(seed):
    ev = adversarial_event(200 + seed, n=500, n_layers=3)
    kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0)
    o = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], bounds=(0, 0, 20, 20), n_layers=3, **kw)
    _forest_checks(o, kw["rho_c"], kw["delta_c"], kw["delta_o"])


def test_labels_follow_forest_components_config1():
    ev, p = gen.config1()
    o = oracle.run_event(ev, p)
    _forest_checks(o, p["rho_c"], p["delta_c"], p["delta_o"])


def _cfsfdp_assign(rho, nh, is_seed, is_outlier):
    """Visit hits in decreasing (rho, index) order; a seed opens the next
    cluster in seed-index order, an outlier or a hit without nearest-higher is
    noise, anything else copies its nearest-higher's label (already set,
    because the nearest-higher comes earlier in this order)."""
    n = rho.size
    order = sorted(range(n), key=lambda i: (-float(rho[i]), -i))
    seed_id = np.cumsum(is_seed) - 1
    lab = np.full(n, -2, np.int64)
    for i in order:
        if is_seed[i]:
            lab[i] = seed_id[i]
        elif is_outlier[i] or nh[i] < 0:
            lab[i] = -1
        else:
            assert lab[nh[i]] != -2, "nearest-higher visited later"
            lab[i] = lab[nh[i]]
    return lab


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("wide", [False, True])
def test_labels_equal_density_order_assignment(seed, wide):
    ev = adversarial_event(300 + seed, n=300, n_layers=1)
    if wide:  # P4: no window limit (d_m >= extent diagonal), no outliers possible
        kw = dict(dc=2.0, rho_c=-1.0, delta_c=40.0, delta_o=40.0)
    else:
        kw = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0)
    o = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], bounds=(0, 0, 20, 20), n_layers=1, **kw)
    outl = (o["rho"] < np.float32(kw["rho_c"])) & (o["delta2"] > np.float32(kw["delta_o"]) ** 2)
    lab = _cfsfdp_assign(o["rho"], o["nh"], o["is_seed"].astype(bool), outl)
    assert np.array_equal(o["cluster_id"], lab.astype(np.int32))
    if wide:
        # with an unlimited window every layer has exactly one hit without a
        # nearest-higher: its density maximum, the only seed (rho_c < 0)
        assert o["is_seed"].sum() == 1 and (o["nh"] < 0).sum() == 1
        assert np.all(o["cluster_id"] == 0)
        top = max(range(o["rho"].size), key=lambda i: (float(o["rho"][i]), i))
        assert o["is_seed"][top] == 1
