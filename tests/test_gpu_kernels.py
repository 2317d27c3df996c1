"""GPU parity for the Gaussian and exponential kernels chi of Eq. 3.

Both sides evaluate the same fixed binary32 exponential, so rho, nh, delta2,
labels and follower lists are compared bit for bit with the oracle, on every
density path (quad lists, per-query merges, three-tile windows, global
fallback), plain and batched."""
import numpy as np
import pytest

from gpu_helpers import assert_parity, gpu_run
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen
from test_gpu_parity import _ref

pytestmark = pytest.mark.gpu
ADV = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
KERNELS = [("gaussian", 0.8), ("exponential", 0.7), ("gaussian", 1e6)]
TUNINGS = [None, dict(density_quads=2), dict(density_quads=3), dict(tile_size=2.5), dict(lds_cap=64),
           dict(tile_size=8.0, block_x=2, block_y=2)]


@pytest.mark.parametrize("kernel,s", KERNELS)
@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(t) for t in TUNINGS])
@pytest.mark.parametrize("batched", [False, True])
def test_kernels_adversarial(kernel, s, tuning, batched):
    p = dict(ADV, kernel=kernel, kernel_scale=s)
    ev = adversarial_event(31, n=500, n_layers=3)
    assert_parity(gpu_run(ev, p, batched=batched, tuning=tuning), _ref(ev, p),
                  where=f"{kernel} {s} {tuning} batched={batched}")


@pytest.mark.parametrize("kernel,s", [("gaussian", 1.0), ("exponential", 1.0)])
def test_kernels_config2(kernel, s):
    ev, p = gen.config2(n_layers=30)
    p = dict(p, kernel=kernel, kernel_scale=s)
    assert_parity(gpu_run(ev, p, batched=True), _ref(ev, p), where=f"cfg2 {kernel}")


def test_kernel_paper_workload_bin5():
    ev, p = gen.paper_event(10000, n_layers=20)
    p = dict(p, kernel="gaussian", kernel_scale=1.5)
    assert_parity(gpu_run(ev, p, tuning=dict(tile_size=gen.PAPER_BIN)), _ref(ev, p), where="paper gaussian")


def test_kernel_argument_errors():
    import paper_2001_09761_amd as clue
    with pytest.raises(clue.ClueError):
        clue.Context(2.0, 5.0, 2.0, 4.0, max_hits=10, extent=20.0, n_layers=1, kernel="gaussian", kernel_scale=0.0)
