"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle element by element."""
import numpy as np

import oracle


def to_dev(ev, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in ev.items() if isinstance(v, np.ndarray)}


def gpu_run(ev, p, *, batched=False, n_events=1, flags=None, tuning=None, ctx=None, followers=True):
    """Runs the GPU path with intermediates kept; returns numpy outputs."""
    import torch
    import paper_2001_09761_amd as clue
    dev = torch.device("cuda", 0)
    f = clue.KEEP_INTERMEDIATES if flags is None else flags
    t = to_dev(ev, dev)
    n = ev["x"].size
    own = ctx is None
    if own:
        ctx = clue.Context(p["dc"], p["rho_c"], p["delta_c"], p["delta_o"], max_hits=max(n, 1),
                           max_events=max(n_events, 1), extent=p.get("extent"), bounds=p.get("bounds"),
                           n_layers=p["n_layers"], flags=f, kernel=p.get("kernel", "flat"),
                           kernel_scale=p.get("kernel_scale", 0.0))
    try:
        if tuning:
            ctx.set_tuning(**tuning)
        if batched:
            ev_ids = t.get("event")
            if ev_ids is None:
                ev_ids = torch.zeros(n, dtype=torch.int32, device=dev)
            cid, seed = ctx.run_batch(ev_ids, n_events, t["x"], t["y"], t["layer"], t["energy"])
        else:
            cid, seed = ctx.run(t["x"], t["y"], t["layer"], t["energy"])
        out = dict(cluster_id=cid, is_seed=seed)
        if f & clue.KEEP_INTERMEDIATES:
            out.update(ctx.intermediates())
        if followers and not (f & clue.NO_FOLLOWERS):
            fs, fl = ctx.followers()
            out["fstart"], out["flist"] = fs, fl
        torch.cuda.synchronize()
        ctx.status()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        if own:
            ctx.close()


def assert_parity(got, ref, keys=("cluster_id", "is_seed", "rho", "nh", "delta2", "fstart", "flist"), where=""):
    for k in keys:
        if k not in got or k not in ref:
            continue
        a, b = got[k], ref[k]
        if a.dtype == np.float32:
            a, b = a.view(np.uint32), b.view(np.uint32)
        if a.dtype == np.uint8:
            b = b.astype(np.uint8)
        assert a.shape == b.shape, (where, k, a.shape, b.shape)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{where}: {k} differs at {bad.size} positions, first {bad[:8]}: got {got[k][bad[:8]]} want {ref[k][bad[:8]]}"
