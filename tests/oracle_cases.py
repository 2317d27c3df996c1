"""Seeded tiny adversarial events shared by the oracle pins and the GPU
parity tests (inputs only: no clustering arithmetic lives here)."""
import numpy as np


def adversarial_event(seed, n=300, n_layers=3, extent=20.0, unit_weights=False, dc=2.0):
    """Random tiny event with the corner cases the grid must survive:
    duplicates, hits exactly on bin edges, hits outside the extent, and pairs
    one float32 ulp either side of distance dc along an axis."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, extent, n)
    y = rng.uniform(0, extent, n)
    k = n // 10
    # clusters of points so that densities and ties are non-trivial
    cx = rng.uniform(0, extent, 5)
    cy = rng.uniform(0, extent, 5)
    idx = rng.integers(0, 5, k * 3)
    x[: 3 * k] = cx[idx] + rng.normal(0, 1.0, 3 * k)
    y[: 3 * k] = cy[idx] + rng.normal(0, 1.0, 3 * k)
    # exact duplicates
    x[3 * k: 4 * k] = x[: k]
    y[3 * k: 4 * k] = y[: k]
    # on bin/tile edges (integers and multiples of dc/2)
    x[4 * k: 5 * k] = np.round(x[4 * k: 5 * k])
    y[4 * k: 5 * k] = np.round(y[4 * k: 5 * k] / (dc / 2)) * (dc / 2)
    # outside the extent
    x[5 * k: 5 * k + k // 2] = rng.uniform(-5, 0, k // 2)
    y[5 * k + k // 2: 6 * k] = rng.uniform(extent, extent + 5, k - k // 2)
    x = x.astype(np.float32)
    y = y.astype(np.float32)
    # pairs at dc +- 1 ulp along x
    for t in range(k // 2):
        i = 6 * k + 2 * t
        base = np.float32(rng.uniform(2, extent - 4))
        x[i] = base
        y[i + 1] = y[i]
        target = np.float32(base + np.float32(dc))
        if t % 3 == 0:
            target = np.nextafter(target, np.float32(np.inf))
        elif t % 3 == 1:
            target = np.nextafter(target, np.float32(-np.inf))
        x[i + 1] = target
    layer = rng.integers(0, n_layers, n).astype(np.int32)
    if unit_weights:
        e = np.ones(n, np.float32)
    else:
        e = rng.uniform(0, 3, n).astype(np.float32)
        e[: 3 * k] *= 4
    return dict(x=x, y=y, layer=layer, energy=e)
