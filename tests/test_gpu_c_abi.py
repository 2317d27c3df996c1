"""GPU: the C ABI from a plain C program (no Python binding, no torch).

tests/c_abi/clue_c_consumer (built by __graft_entry__.build) clusters one
event with clue_run and clue_run_batch, checks that they agree and that
argument errors come back as codes, and writes its outputs; here they are
compared with the oracle bit for bit."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle_cases import adversarial_event
from paper_2001_09761_amd import gen

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "clue_c_consumer")


def _run(tmp_path, ev, p):
    n = ev["x"].size
    b = p.get("bounds") or (0.0, 0.0, p["extent"], p["extent"])
    src, out = tmp_path / "event.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.array([p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], *b], np.float32).tobytes())
        f.write(np.int32(p["n_layers"]).tobytes())
        for k, dt in (("x", np.float32), ("y", np.float32), ("layer", np.int32), ("energy", np.float32)):
            f.write(np.ascontiguousarray(ev[k], dtype=dt).tobytes())
    print(f"c consumer: {n} hits", flush=True)
    r = subprocess.run([EXE, str(src), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    raw = np.fromfile(out, dtype=np.uint8)
    return raw[: 4 * n].view(np.int32), raw[4 * n:]


@pytest.mark.skipif(not os.path.exists(EXE), reason="C consumer not built (__graft_entry__.build)")
@pytest.mark.parametrize("case", ["cfg1", "adversarial"])
def test_c_consumer_equals_oracle(tmp_path, case):
    if case == "cfg1":
        ev, p = gen.config1()
    else:
        ev = adversarial_event(31, n=700, n_layers=3)
        p = dict(dc=2.0, rho_c=5.0, delta_c=2.0, delta_o=4.0, bounds=(0, 0, 20, 20), n_layers=3)
    cid, seed = _run(tmp_path, ev, p)
    ref = oracle.run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=p["dc"], rho_c=p["rho_c"],
                     delta_c=p["delta_c"], delta_o=p["delta_o"], extent=p.get("extent"), bounds=p.get("bounds"),
                     n_layers=p["n_layers"])
    assert np.array_equal(cid, ref["cluster_id"])
    assert np.array_equal(seed, ref["is_seed"].astype(np.uint8))
