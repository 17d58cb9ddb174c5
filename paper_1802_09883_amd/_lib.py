"""ctypes loader for librepro.so (the HIP library); marshalling only.

The library must have been built (``__graft_entry__.build()``); there is no
fallback: a missing or unloadable library raises at first use.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librepro.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "repro.h")

REPRO_OK, REPRO_EINVAL, REPRO_EHIP = 0, -1, -2
ERR_KEY, ERR_NONFINITE, ERR_RANGE = 1, 2, 4
F32, F64 = 0, 1
I32, I64 = 0, 1

_lib = None


class BatchJob(ctypes.Structure):
    """repro_batch_job of include/repro.h."""
    _fields_ = [("keys", ctypes.c_void_p), ("values", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("num_groups", ctypes.c_int64), ("L", ctypes.c_int), ("accumulate", ctypes.c_int),
                ("states", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    """repro_batch_config of include/repro.h."""
    _fields_ = [("chunk_rows", ctypes.c_int64), ("max_slice_groups", ctypes.c_int), ("order", ctypes.c_int),
                ("merge", ctypes.c_int), ("split", ctypes.c_int)]


MAX_COLS, MAX_AGGS = 8, 4
NOALLOC_SCRATCH_BYTES = 64 << 20  # REPRO_NOALLOC_SCRATCH_BYTES


class Query(ctypes.Structure):
    """repro_query of include/repro.h."""
    _fields_ = [("keys", ctypes.c_void_p), ("cols", ctypes.c_void_p * MAX_COLS), ("n", ctypes.c_int64),
                ("num_groups", ctypes.c_int64), ("L", ctypes.c_int), ("naggs", ctypes.c_int),
                ("agg_a", ctypes.c_int * MAX_AGGS), ("agg_b", ctypes.c_int * MAX_AGGS),
                ("out", ctypes.c_void_p * MAX_AGGS), ("status", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    """repro_server_config of include/repro.h."""
    _fields_ = [("slots", ctypes.c_int), ("chunk_rows", ctypes.c_int64), ("no_batch_path", ctypes.c_int),
                ("query_workgroups", ctypes.c_int), ("max_bypass", ctypes.c_int)]


class BatchPlan(ctypes.Structure):
    """repro_batch_plan of include/repro.h."""
    _fields_ = [("workspace", ctypes.c_void_p), ("items", ctypes.c_int64), ("grid", ctypes.c_int),
                ("lds_bytes", ctypes.c_int), ("kt", ctypes.c_int), ("vt", ctypes.c_int), ("T", ctypes.c_int),
                ("reserved", ctypes.c_int * 4)]


def header_functions():
    """Names of the functions declared in include/repro.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(repro_[a-z_0-9]+)\s*\(", text, re.M)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    lib.repro_state_bytes.restype = sz
    lib.repro_state_bytes.argtypes = [i64, i32, i32]
    lib.repro_workspace_bytes.restype = sz
    lib.repro_workspace_bytes.argtypes = [i64, i64, i32, i32, i32, i32]
    lib.repro_state_init.argtypes = [vp, i64, i32, i32, vp]
    lib.repro_groupby_sum.argtypes = [vp, i32, vp, i32, i64, i64, i32, i32, vp, vp, sz, vp, vp]
    lib.repro_merge.argtypes = [vp, vp, i64, i32, i32, vp]
    lib.repro_finalize.argtypes = [vp, i64, i32, i32, vp, vp]
    lib.repro_plain_groupby_sum.argtypes = [vp, i32, vp, i32, i64, i64, vp, vp, sz, vp, vp]
    lib.repro_plain_workspace_bytes.restype = sz
    lib.repro_plain_workspace_bytes.argtypes = [i64, i64, i32, i32]
    lib.repro_profile_arm.argtypes = [i32]
    lib.repro_profile_arm.restype = ctypes.c_int
    lib.repro_profile_read.argtypes = [vp, i32, vp]
    lib.repro_profile_read.restype = ctypes.c_int
    bj, bc, bp = ctypes.POINTER(BatchJob), ctypes.POINTER(BatchConfig), ctypes.POINTER(BatchPlan)
    lib.repro_batch_workspace_bytes.restype = sz
    lib.repro_batch_workspace_bytes.argtypes = [bj, i32, i32, i32, i32, bc]
    lib.repro_batch_prepare.restype = ctypes.c_int
    lib.repro_batch_prepare.argtypes = [bj, i32, i32, i32, i32, bc, vp, sz, bp, vp]
    lib.repro_batch_launch.restype = ctypes.c_int
    lib.repro_batch_launch.argtypes = [bp, vp, vp]
    lib.repro_batch_tune.restype = ctypes.c_int
    lib.repro_batch_tune.argtypes = [bj, i32, i32, i32, i32, vp, sz, bc, ctypes.POINTER(ctypes.c_float), vp]
    lib.repro_sum_workspace_bytes.restype = sz
    lib.repro_sum_workspace_bytes.argtypes = [i64, i32]
    lib.repro_sum.restype = ctypes.c_int
    lib.repro_sum.argtypes = [vp, i32, i64, i32, i32, vp, vp, sz, vp, vp]
    lib.repro_groupby_count.restype = ctypes.c_int
    lib.repro_groupby_count.argtypes = [vp, i32, i64, i64, vp, vp, vp]
    lib.repro_derive_stats.restype = ctypes.c_int
    lib.repro_derive_stats.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    lib.repro_mul.restype = ctypes.c_int
    lib.repro_mul.argtypes = [vp, i32, vp, i32, i64, vp, vp]
    qp, scp = ctypes.POINTER(Query), ctypes.POINTER(ServerConfig)
    lib.repro_query_bytes.restype = sz
    lib.repro_query_bytes.argtypes = [qp, scp]
    lib.repro_server_create.restype = ctypes.c_int
    lib.repro_server_create.argtypes = [vp, sz, scp, ctypes.POINTER(vp)]
    lib.repro_server_submit.restype = ctypes.c_int
    lib.repro_server_submit.argtypes = [vp, qp, ctypes.POINTER(i64)]
    lib.repro_server_poll.restype = ctypes.c_int
    lib.repro_server_poll.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double), i32,
                                      ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(i64)]
    lib.repro_server_clock.restype = ctypes.c_double
    lib.repro_server_clock.argtypes = []
    lib.repro_server_destroy.restype = ctypes.c_int
    lib.repro_server_destroy.argtypes = [vp]
    lib.repro_workspace_bytes_cols.restype = sz
    lib.repro_workspace_bytes_cols.argtypes = [i64, i64, i32, i32, vp, i32, i32]
    lib.repro_groupby_sum_cols.restype = ctypes.c_int
    lib.repro_groupby_sum_cols.argtypes = [vp, i32, i32, vp, vp, i64, i64, i32, i32, vp, vp, sz, vp, vp]
    lib.repro_plain_groupby_sum_cols.restype = ctypes.c_int
    lib.repro_plain_groupby_sum_cols.argtypes = [vp, i32, i32, vp, vp, i64, i64, vp, vp, vp]
    lib.repro_groupby_sum_noalloc.restype = ctypes.c_int
    lib.repro_groupby_sum_noalloc.argtypes = [vp, i32, vp, i32, i64, i64, i32, i32, vp, vp, vp]
    lib.repro_read_probe.restype = ctypes.c_int
    lib.repro_read_probe.argtypes = [vp, sz, i32, i32, vp, vp]
    lib.repro_atomic_probe.restype = ctypes.c_int
    lib.repro_atomic_probe.argtypes = [vp, i64, vp, i64, i32, vp]
    lib.repro_version.restype = ctypes.c_char_p
    lib.repro_version.argtypes = []
    for name in ("repro_state_init", "repro_groupby_sum", "repro_merge", "repro_finalize",
                 "repro_plain_groupby_sum"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int, what: str):
    if rc == REPRO_EINVAL:
        raise ValueError(f"{what}: invalid argument")
    if rc != REPRO_OK:
        raise RuntimeError(f"{what}: HIP error (code {rc})")
