"""ctypes binding of libclue (include/clue.h): argument marshalling only.

PyTorch supplies device memory and streams; every step of the clustering
runs in the library's HIP kernels. Importing this module never builds
anything: if libclue.so is missing the loader raises, loudly.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclue.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "clue.h")

CLUE_OK = 0
ERRORS = {-1: "CLUE_ERR_ARG", -2: "CLUE_ERR_CAPACITY", -3: "CLUE_ERR_NOMEM", -4: "CLUE_ERR_HIP",
          -5: "CLUE_ERR_INPUT", -6: "CLUE_ERR_BUDGET", -7: "CLUE_ERR_STATE", -8: "CLUE_ERR_DEVICE"}
VALIDATE, KEEP_INTERMEDIATES, TIE_PAPER_STRICT, NO_FOLLOWERS = 1, 2, 4, 8
NOALLOC_SCRATCH_BYTES = 64 << 20  # CLUE_NOALLOC_SCRATCH_BYTES


class ClueParams(ctypes.Structure):
    _fields_ = [
        ("dc", ctypes.c_float), ("rho_c", ctypes.c_float),
        ("delta_c", ctypes.c_float), ("delta_o", ctypes.c_float),
        ("x_min", ctypes.c_float), ("y_min", ctypes.c_float),
        ("x_max", ctypes.c_float), ("y_max", ctypes.c_float),
        ("n_layers", ctypes.c_int32), ("tile_size", ctypes.c_float),
        ("threads_per_query", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("kernel", ctypes.c_int32), ("kernel_scale", ctypes.c_float),
    ]


KERNELS = {"flat": 0, "gaussian": 1, "exponential": 2}


class ClueTuning(ctypes.Structure):
    _fields_ = [
        ("tile_size", ctypes.c_float), ("threads_per_query", ctypes.c_int32),
        ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
        ("lds_cap", ctypes.c_int32), ("nh_first_radius", ctypes.c_float),
        ("density_quads", ctypes.c_int32), ("plain_lds_cap", ctypes.c_int32), ("expansion", ctypes.c_int32),
    ]


class ClueError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/clue.h."""
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(clue_[a-z_0-9]+)\s*\(", src)))


def load(path: str = LIB_PATH):
    """Loads libclue.so (PyTorch's HIP runtime must be loaded first so both
    share one runtime; importing torch does that)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libclue.so not found at {path}: build it with "
                          f"`python -c 'import __graft_entry__ as g; g.build()'`")
    import torch  # noqa: F401  (loads the HIP runtime that libclue binds to)
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    sig = {
        "clue_create": ([ctypes.POINTER(P), ctypes.POINTER(ClueParams), ctypes.c_int, i64, i32, u64], ctypes.c_int),
        "clue_reserve": ([P, i64, i32], ctypes.c_int),
        "clue_footprint_bytes": ([ctypes.POINTER(ClueParams), i64, i32, ctypes.POINTER(u64)], ctypes.c_int),
        "clue_run": ([P, i64, P, P, P, P, P, P, P], ctypes.c_int),
        "clue_run_batch": ([P, i64, i32, P, P, P, P, P, P, P, P], ctypes.c_int),
        "clue_run_batch_range": ([P, i64, i32, i32, P, P, P, P, P, P, P, P], ctypes.c_int),
        "clue_run_batch_host": ([P, i64, i32, P, P, P, P, P, P, P], ctypes.c_int),
        "clue_get_intermediates": ([P, P, P, P, P], ctypes.c_int),
        "clue_get_followers": ([P, P, P, ctypes.POINTER(i64), P], ctypes.c_int),
        "clue_status": ([P, P], ctypes.c_int),
        "clue_set_tuning": ([P, ctypes.POINTER(ClueTuning)], ctypes.c_int),
        "clue_get_tuning": ([P, ctypes.POINTER(ClueTuning), ctypes.POINTER(i32)], ctypes.c_int),
        "clue_enable_stage_timing": ([P, ctypes.c_int], ctypes.c_int),
        "clue_stage_times": ([P, ctypes.POINTER(f32), ctypes.POINTER(ctypes.c_char_p), ctypes.c_int], ctypes.c_int),
        "clue_run_noalloc": ([ctypes.POINTER(ClueParams), ctypes.POINTER(ClueTuning), i64, P, P, P, P, P, P, P],
                             ctypes.c_int),
        "clue_last_error": ([P], ctypes.c_char_p),
        "clue_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def make_params(dc, rho_c, delta_c, delta_o, bounds, n_layers, tile_size=0.0, threads_per_query=0, flags=0,
                kernel="flat", kernel_scale=0.0):
    return ClueParams(float(dc), float(rho_c), float(delta_c), float(delta_o), float(bounds[0]),
                      float(bounds[1]), float(bounds[2]), float(bounds[3]), int(n_layers), float(tile_size),
                      int(threads_per_query), int(flags), KERNELS[kernel], float(kernel_scale))


def check(rc: int, ctx=None):
    if rc != CLUE_OK:
        msg = load().clue_last_error(ctx).decode(errors="replace")
        raise ClueError(rc, msg)
