"""CLUE per-layer clustering on AMD Instinct MI355X (gfx950).

``Context`` wraps one libclue context: ``run`` clusters one event with
per-stage launches (plain form), ``run_batch`` clusters many events with
persistent kernels replayed from a HIP graph (batched form). Inputs and
outputs are torch tensors on the GPU; work is enqueued on the current torch
stream. ``Server`` (from ``paper_2001_09761_amd.serve``) is the online served
form: events are submitted as they come and come back as futures.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (ClueError, KEEP_INTERMEDIATES, NO_FOLLOWERS, TIE_PAPER_STRICT, VALIDATE,  # noqa: F401
                   make_params)

__all__ = ["Context", "Server", "ClueError", "VALIDATE", "KEEP_INTERMEDIATES", "TIE_PAPER_STRICT", "NO_FOLLOWERS",
           "footprint_bytes", "run_noalloc"]


def _torch():
    import torch
    return torch


def _bounds(extent=None, bounds=None):
    if bounds is not None:
        return tuple(float(b) for b in bounds)
    s = 200.0 if extent is None else float(extent)
    return (0.0, 0.0, s, s)


def footprint_bytes(dc, rho_c, delta_c, delta_o, max_hits, max_events=1, *, extent=None, bounds=None,
                    n_layers=100, tile_size=0.0, flags=0, kernel="flat", kernel_scale=0.0) -> int:
    p = make_params(dc, rho_c, delta_c, delta_o, _bounds(extent, bounds), n_layers, tile_size, 0, flags, kernel,
                    kernel_scale)
    out = ctypes.c_uint64(0)
    _lib.check(_lib.load().clue_footprint_bytes(ctypes.byref(p), int(max_hits), int(max_events),
                                                ctypes.byref(out)))
    return int(out.value)


def run_noalloc(dc, rho_c, delta_c, delta_o, x, y, layer, energy, cluster_id, is_seed, *, extent=None,
                bounds=None, n_layers=100, tile_size=0.0, threads_per_query=0, flags=0, kernel="flat",
                kernel_scale=0.0, tuning=None, stream=None):
    """One event through ``clue_run_noalloc``: the plain form over the
    library's fixed per-device scratch, for callers that cannot allocate.
    The caller passes the outputs (``cluster_id`` int32, ``is_seed`` uint8);
    ``tuning`` is a dict as returned by ``Context.tuning()`` or None."""
    torch = _torch()
    L = _lib.load()
    p = make_params(dc, rho_c, delta_c, delta_o, _bounds(extent, bounds), n_layers, tile_size, threads_per_query,
                    flags, kernel, kernel_scale)
    t = None
    if tuning is not None:
        t = _lib.ClueTuning(float(tuning.get("tile_size", 0.0)), int(tuning.get("threads_per_query", 0)),
                            int(tuning.get("block_x", 0)), int(tuning.get("block_y", 0)),
                            int(tuning.get("lds_cap", 0)), float(tuning.get("nh_first_radius", -1.0)),
                            int(tuning.get("density_quads", 0)), int(tuning.get("plain_lds_cap", 0)),
                            int(tuning.get("expansion", 0)))
    n = int(x.numel())
    dev = Context._dev
    s = torch.cuda.current_stream() if stream is None else stream
    rc = L.clue_run_noalloc(ctypes.byref(p), ctypes.byref(t) if t is not None else None, n,
                            dev(None, x, torch.float32, "x", n), dev(None, y, torch.float32, "y", n),
                            dev(None, layer, torch.int32, "layer", n), dev(None, energy, torch.float32, "energy", n),
                            dev(None, cluster_id, torch.int32, "cluster_id", n),
                            dev(None, is_seed, torch.uint8, "is_seed", n), ctypes.c_void_p(s.cuda_stream))
    _lib.check(rc, None)
    return cluster_id, is_seed


class Context:
    """One libclue context (scratch arena, captured graph) on one device."""

    def __init__(self, dc, rho_c, delta_c, delta_o, *, max_hits, max_events=1, extent=None, bounds=None,
                 n_layers=100, tile_size=0.0, threads_per_query=0, flags=0, device=None, hbm_budget=0,
                 kernel="flat", kernel_scale=0.0):
        torch = _torch()
        self._L = _lib.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.params = make_params(dc, rho_c, delta_c, delta_o, _bounds(extent, bounds), n_layers, tile_size,
                                  threads_per_query, flags, kernel, kernel_scale)
        self.flags = int(flags)
        self._ctx = ctypes.c_void_p(None)
        rc = self._L.clue_create(ctypes.byref(self._ctx), ctypes.byref(self.params), self.device, int(max_hits),
                                 int(max_events), int(hbm_budget))
        if rc != 0:
            raise ClueError(rc, self._L.clue_last_error(None).decode(errors="replace"))
        self.max_hits = int(max_hits)
        self.max_events = int(max_events)
        self._last_n = 0

    # -- helpers ---------------------------------------------------------
    def _check(self, rc):
        _lib.check(rc, self._ctx)

    @staticmethod
    def _stream(stream):
        torch = _torch()
        s = torch.cuda.current_stream() if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def _dev(self, t, dtype, name, n):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be contiguous with at least {n} elements")
        return ctypes.c_void_p(t.data_ptr() if n > 0 else 0)

    def _outputs(self, n, cluster_id, is_seed, device):
        torch = _torch()
        if cluster_id is None:
            cluster_id = torch.empty(n, dtype=torch.int32, device=device)
        if is_seed is None:
            is_seed = torch.empty(n, dtype=torch.uint8, device=device)
        return cluster_id, is_seed

    # -- runs ------------------------------------------------------------
    def run(self, x, y, layer, energy, cluster_id=None, is_seed=None, stream=None):
        """Cluster one event (plain form). Returns (cluster_id, is_seed)."""
        torch = _torch()
        n = int(x.numel())
        cluster_id, is_seed = self._outputs(n, cluster_id, is_seed, x.device)
        self._check(self._L.clue_run(self._ctx, n, self._dev(x, torch.float32, "x", n),
                                     self._dev(y, torch.float32, "y", n),
                                     self._dev(layer, torch.int32, "layer", n),
                                     self._dev(energy, torch.float32, "energy", n),
                                     self._dev(cluster_id, torch.int32, "cluster_id", n),
                                     self._dev(is_seed, torch.uint8, "is_seed", n), self._stream(stream)))
        self._last_n = n
        return cluster_id, is_seed

    def run_batch(self, event, n_events, x, y, layer, energy, cluster_id=None, is_seed=None, stream=None):
        """Cluster a batch of events (batched form). ``event`` holds
        non-decreasing event ids in [0, n_events)."""
        torch = _torch()
        n = int(x.numel())
        cluster_id, is_seed = self._outputs(n, cluster_id, is_seed, x.device)
        self._check(self._L.clue_run_batch(self._ctx, n, int(n_events), self._dev(event, torch.int32, "event", n),
                                           self._dev(x, torch.float32, "x", n),
                                           self._dev(y, torch.float32, "y", n),
                                           self._dev(layer, torch.int32, "layer", n),
                                           self._dev(energy, torch.float32, "energy", n),
                                           self._dev(cluster_id, torch.int32, "cluster_id", n),
                                           self._dev(is_seed, torch.uint8, "is_seed", n), self._stream(stream)))
        self._last_n = n
        return cluster_id, is_seed

    @staticmethod
    def _host(t, np_dtype, name, n):
        """Pointer to a contiguous host array (numpy array or CPU tensor)."""
        torch = _torch()
        if isinstance(t, torch.Tensor):
            if t.device.type != "cpu":
                raise TypeError(f"{name} must be in host memory")
            t = t.numpy()
        if not isinstance(t, np.ndarray) or t.dtype != np_dtype or not t.flags.c_contiguous or t.size < n:
            raise TypeError(f"{name} must be a contiguous {np.dtype(np_dtype).name} host array of >= {n} elements")
        return ctypes.c_void_p(t.ctypes.data if n > 0 else 0)

    def run_batch_host(self, event, n_events, x, y, layer, energy, cluster_id=None, is_seed=None):
        """Batched form over HOST arrays (numpy arrays or CPU tensors; pinned
        tensors let copies overlap the kernels). The batch may exceed the
        context capacity: it is streamed through in chunks of whole events.
        Synchronous. Returns (cluster_id, is_seed) as host arrays."""
        n = int(np.asarray(x).size) if not hasattr(x, "numel") else int(x.numel())
        if cluster_id is None:
            cluster_id = np.empty(n, dtype=np.int32)
        if is_seed is None:
            is_seed = np.empty(n, dtype=np.uint8)
        ev = ctypes.c_void_p(0) if event is None else self._host(event, np.int32, "event", n)
        self._check(self._L.clue_run_batch_host(self._ctx, n, int(n_events), ev, self._host(x, np.float32, "x", n),
                                                self._host(y, np.float32, "y", n),
                                                self._host(layer, np.int32, "layer", n),
                                                self._host(energy, np.float32, "energy", n),
                                                self._host(cluster_id, np.int32, "cluster_id", n),
                                                self._host(is_seed, np.uint8, "is_seed", n)))
        return cluster_id, is_seed

    def run_batch_range(self, first_event, n_events, event, x, y, layer, energy, cluster_id, is_seed,
                        stream=None):
        """Batched form over a contiguous run of pool events with ids in
        [first_event, first_event + n_events); tensors may be views into a pool."""
        torch = _torch()
        n = int(x.numel())
        self._check(self._L.clue_run_batch_range(
            self._ctx, n, int(first_event), int(n_events), self._dev(event, torch.int32, "event", n),
            self._dev(x, torch.float32, "x", n), self._dev(y, torch.float32, "y", n),
            self._dev(layer, torch.int32, "layer", n), self._dev(energy, torch.float32, "energy", n),
            self._dev(cluster_id, torch.int32, "cluster_id", n), self._dev(is_seed, torch.uint8, "is_seed", n),
            self._stream(stream)))
        self._last_n = n
        return cluster_id, is_seed

    def intermediates(self, stream=None):
        """rho, nh (event-local) and delta^2 of the last run (needs KEEP_INTERMEDIATES)."""
        torch = _torch()
        n = self._last_n
        dev = torch.device("cuda", self.device)
        rho = torch.empty(n, dtype=torch.float32, device=dev)
        nh = torch.empty(n, dtype=torch.int32, device=dev)
        d2 = torch.empty(n, dtype=torch.float32, device=dev)
        self._check(self._L.clue_get_intermediates(self._ctx, ctypes.c_void_p(rho.data_ptr() if n else 0),
                                                   ctypes.c_void_p(nh.data_ptr() if n else 0),
                                                   ctypes.c_void_p(d2.data_ptr() if n else 0),
                                                   self._stream(stream)))
        return dict(rho=rho, nh=nh, delta2=d2)

    def followers(self, stream=None):
        """Follower lists F_i of the last run as (fstart[n+1], flist[n_followers])."""
        torch = _torch()
        n = self._last_n
        dev = torch.device("cuda", self.device)
        fstart = torch.empty(n + 1, dtype=torch.int32, device=dev)
        flist = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        tot = ctypes.c_int64(0)
        self._check(self._L.clue_get_followers(self._ctx, ctypes.c_void_p(fstart.data_ptr()),
                                               ctypes.c_void_p(flist.data_ptr()), ctypes.byref(tot),
                                               self._stream(stream)))
        return fstart, flist[: int(tot.value)]

    def status(self, stream=None):
        self._check(self._L.clue_status(self._ctx, self._stream(stream)))

    def reserve(self, max_hits, max_events=None):
        me = self.max_events if max_events is None else int(max_events)
        self._check(self._L.clue_reserve(self._ctx, int(max_hits), me))
        self.max_hits = max(self.max_hits, int(max_hits))
        self.max_events = max(self.max_events, me)

    def set_tuning(self, tile_size=0.0, threads_per_query=0, block_x=0, block_y=0, lds_cap=0,
                   nh_first_radius=-1.0, density_quads=0, expansion=0, plain_lds_cap=0):
        """Change the kernel tuning (results are identical for every tuning)."""
        t = _lib.ClueTuning(float(tile_size), int(threads_per_query), int(block_x), int(block_y), int(lds_cap),
                            float(nh_first_radius), int(density_quads), int(plain_lds_cap), int(expansion))
        self._check(self._L.clue_set_tuning(self._ctx, ctypes.byref(t)))

    def tuning(self):
        t = _lib.ClueTuning()
        h = ctypes.c_int32()
        self._check(self._L.clue_get_tuning(self._ctx, ctypes.byref(t), ctypes.byref(h)))
        return dict(tile_size=t.tile_size, threads_per_query=t.threads_per_query, block_x=t.block_x,
                    block_y=t.block_y, lds_cap=t.lds_cap, nh_first_radius=t.nh_first_radius,
                    density_quads=t.density_quads, plain_lds_cap=t.plain_lds_cap, expansion=t.expansion,
                    halo=h.value)

    def enable_stage_timing(self, on=True):
        self._check(self._L.clue_enable_stage_timing(self._ctx, 1 if on else 0))

    def stage_times(self):
        ms = (ctypes.c_float * 16)()
        names = (ctypes.c_char_p * 16)()
        k = self._L.clue_stage_times(self._ctx, ms, names, 16)
        if k < 0:
            self._check(k)
        return {names[i].decode(): float(ms[i]) for i in range(k)}

    def close(self):
        if self._ctx:
            self._L.clue_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


from .serve import Server  # noqa: E402  (the served form builds on Context)
