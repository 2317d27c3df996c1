"""Oracle pins for the Gaussian and exponential kernels of Eq. 3.

The kernels use the oracle's own binary32 exponential (Cody-Waite range
reduction plus a degree-7 Taylor polynomial). It is pinned against float64
exp; the kernel densities are pinned against a direct float64 evaluation, a
huge kernel scale must reproduce the flat kernel bit for bit, and the grid
must not change results (brute force)."""
import numpy as np
import pytest

import oracle
from oracle_cases import adversarial_event

P = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
U = 2.0 ** -24


def test_exp32_accuracy_and_shape():
    x = -np.linspace(0.0, 86.0, 1_000_001).astype(np.float32)
    e = oracle.exp32(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(e - ref) / ulp) <= 1.5
    assert oracle.exp32(np.array([0.0], np.float32))[0] == 1.0
    assert np.all(np.diff(e[::-1]) >= 0)  # non-decreasing in x
    assert np.all(oracle.exp32(np.array([-87.5, -100.0, -1e30], np.float32)) == 0.0)


def _direct(ev, kernel, s, dc):
    """rho by a float64 sum over the float32-decided neighbour set."""
    x, y, e, l = ev["x"], ev["y"], ev["energy"], ev["layer"]
    s = float(np.float32(s))  # the scale as the float32 parameter holds it
    rho = np.zeros(x.size)
    m = np.zeros(x.size, int)
    dc2 = np.float32(dc) * np.float32(dc)
    for i in range(x.size):
        dx = (x[i] - x).astype(np.float32)
        dy = (y[i] - y).astype(np.float32)
        d2 = (dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)
        nb = (l == l[i]) & (d2 < dc2)
        d2n = d2[nb].astype(np.float64)
        w = np.exp(-d2n / (2 * s * s)) if kernel == "gaussian" else np.exp(-np.sqrt(d2n) / s)
        rho[i] = np.sum(w * e[nb])
        m[i] = nb.sum()
    return rho, m


@pytest.mark.parametrize("kernel,s", [("gaussian", 1.0), ("gaussian", 0.4), ("exponential", 1.5),
                                      ("exponential", 0.3)])
def test_kernel_density_matches_float64(kernel, s):
    ev = adversarial_event(5, n=300, n_layers=3)
    r = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **P, kernel=kernel, kernel_scale=s,
                   want=("rho", "rho64"))
    ref, m = _direct(ev, kernel, s, P["dc"])
    # rho64 sums float64 weights in another order: agrees to rounding
    assert np.allclose(r["rho64"], ref, rtol=1e-12, atol=1e-300)
    # float32 rho: each term carries at most 1.5 ulp (exp) + 1 ulp (sqrt, scale,
    # product), and m - 1 additions of non-negative terms
    bound = (m - 1 + 4) * U / (1 - (m + 3) * U)
    rel = np.abs(r["rho"] - ref) / np.maximum(ref, 1e-30)
    assert np.all(rel <= bound), float(np.max(rel - bound))


@pytest.mark.parametrize("kernel,s", [("gaussian", 1e6), ("exponential", 1e12)])
def test_huge_scale_equals_flat(kernel, s):
    ev = adversarial_event(8, n=400, n_layers=3)
    flat = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **P)
    wide = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **P, kernel=kernel, kernel_scale=s)
    for k in ("rho", "nh", "cluster_id", "is_seed"):
        assert np.array_equal(flat[k].view(np.uint32) if flat[k].dtype == np.float32 else flat[k],
                              wide[k].view(np.uint32) if wide[k].dtype == np.float32 else wide[k]), k


@pytest.mark.parametrize("kernel,s", [("gaussian", 0.8), ("exponential", 0.7)])
@pytest.mark.parametrize("bin_size", [0.5, 2.0, 7.0])
def test_kernel_grid_equals_brute_force(kernel, s, bin_size):
    ev = adversarial_event(11, n=350, n_layers=3)
    kw = dict(P, kernel=kernel, kernel_scale=s)
    brute = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **kw, brute_force=True)
    grid = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **kw, bin_size=bin_size)
    for k in ("rho", "rho64", "nh", "delta2", "cluster_id", "is_seed", "fstart", "flist"):
        a, b = brute[k], grid[k]
        if a.dtype in (np.float32, np.float64):
            a, b = a.view(np.uint32 if a.dtype == np.float32 else np.uint64), b.view(
                np.uint32 if b.dtype == np.float32 else np.uint64)
        assert np.array_equal(a, b), k


def test_kernel_arguments_checked():
    ev = adversarial_event(3, n=50, n_layers=3)
    with pytest.raises(oracle.OracleError):
        oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], **P, kernel="gaussian", kernel_scale=0.0)
