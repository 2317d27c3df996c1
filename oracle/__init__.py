"""CLUE oracle: TEST INFRASTRUCTURE ONLY.

A plain CPU implementation of the paper's Algorithms 1-3 (see
``clue_oracle.h``). Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it. The GPU library does not and
must never route through it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("dc", ctypes.c_float), ("rho_c", ctypes.c_float),
        ("delta_c", ctypes.c_float), ("delta_o", ctypes.c_float),
        ("x_min", ctypes.c_float), ("y_min", ctypes.c_float),
        ("x_max", ctypes.c_float), ("y_max", ctypes.c_float),
        ("n_layers", ctypes.c_int32), ("bin_size", ctypes.c_float),
        ("paper_strict", ctypes.c_int32), ("brute_force", ctypes.c_int32),
        ("kernel", ctypes.c_int32), ("kernel_scale", ctypes.c_float),
    ]

KERNELS = {"flat": 0, "gaussian": 1, "exponential": 2}


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_run.argtypes = [ctypes.POINTER(OracleParams), ctypes.c_int64, ctypes.c_int32, P,
                                 P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_exp32.argtypes = [P, P, ctypes.c_int64]
        L.oracle_exp32.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def run(x, y, layer, energy, *, dc, rho_c, delta_c, delta_o, extent=None, bounds=None,
        n_layers=None, event=None, n_events=None, bin_size=0.0, paper_strict=False,
        brute_force=False, kernel="flat", kernel_scale=0.0, n_threads=1,
        want=("rho", "rho64", "nh", "delta2", "followers")):
    """Run the oracle on host arrays. Returns a dict of numpy arrays.

    ``bounds=(x_min, y_min, x_max, y_max)`` or ``extent=s`` for [0, s]^2."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    energy = np.ascontiguousarray(energy, dtype=np.float32)
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    n = x.shape[0]
    if bounds is None:
        s = 200.0 if extent is None else float(extent)
        bounds = (0.0, 0.0, s, s)
    if n_layers is None:
        n_layers = int(layer.max()) + 1 if n else 1
    ev = None
    if event is not None:
        ev = np.ascontiguousarray(event, dtype=np.int32)
        if n_events is None:
            n_events = int(ev.max()) + 1 if n else 1
    if n_events is None:
        n_events = 1
    p = OracleParams(dc, rho_c, delta_c, delta_o, bounds[0], bounds[1], bounds[2], bounds[3],
                     int(n_layers), float(bin_size), int(bool(paper_strict)), int(bool(brute_force)),
                     KERNELS[kernel], float(kernel_scale))
    out = dict(cluster_id=np.empty(n, np.int32), is_seed=np.empty(n, np.uint8))
    if "rho" in want:
        out["rho"] = np.empty(n, np.float32)
    if "rho64" in want:
        out["rho64"] = np.empty(n, np.float64)
    if "nh" in want:
        out["nh"] = np.empty(n, np.int32)
    if "delta2" in want:
        out["delta2"] = np.empty(n, np.float32)
    if "followers" in want:
        out["fstart"] = np.empty(n + 1, np.int32)
        out["flist"] = np.empty(max(n, 1), np.int32)
    out["n_clusters"] = np.empty(n_events, np.int32)
    rc = lib().oracle_run(ctypes.byref(p), n, n_events, _ptr(ev), _ptr(x), _ptr(y), _ptr(layer),
                          _ptr(energy), _ptr(out["cluster_id"]), _ptr(out["is_seed"]),
                          _ptr(out.get("rho")), _ptr(out.get("rho64")), _ptr(out.get("nh")),
                          _ptr(out.get("delta2")), _ptr(out.get("fstart")), _ptr(out.get("flist")),
                          _ptr(out["n_clusters"]), int(n_threads))
    if rc != 0:
        raise OracleError(rc, lib().oracle_last_error().decode())
    if "followers" in want:
        out["flist"] = out["flist"][: out["fstart"][n]]
    return out


def exp32(x):
    """The oracle's binary32 exponential (x <= 0) on an array."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    lib().oracle_exp32(_ptr(x), _ptr(out), x.size)
    return out


def run_event(ev, params, **kw):
    """Convenience wrapper: ``ev`` from the input generators, ``params`` dict
    with dc, rho_c, delta_c, delta_o, extent and n_layers."""
    return run(ev["x"], ev["y"], ev["layer"], ev["energy"], dc=params["dc"], rho_c=params["rho_c"],
               delta_c=params["delta_c"], delta_o=params["delta_o"],
               extent=params.get("extent"), bounds=params.get("bounds"),
               n_layers=params.get("n_layers"), event=ev.get("event"),
               n_events=ev.get("n_events"), kernel=params.get("kernel", "flat"),
               kernel_scale=params.get("kernel_scale", 0.0), **kw)
