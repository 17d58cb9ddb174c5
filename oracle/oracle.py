"""CPU oracle for reproducible GroupBy-SUM into repro<T,L> (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  Nothing here is shared with the HIP
library; the state layout is restated from the interface documentation.

All arithmetic lives in ``repro_oracle.c``; this module only marshals numpy
arrays.  See that file for the paper passages each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "repro_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ERR_KEY, ERR_NONFINITE, ERR_RANGE = 1, 2, 4

# format tuples (m, W, B, jmax, emin, emax), restated from the paper:
# W = 18 (float) / 40 (double), m = fraction bits, B = emin.
FMT_DOUBLE = (52, 40, -1022, 51, -1022, 1023)
FMT_FLOAT = (23, 18, -126, 14, -126, 127)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-fno-strict-aliasing", "-Wall", "-o", tmp, _SRC,
               "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.orc_state_bytes.restype = ctypes.c_size_t
    lib.orc_state_bytes.argtypes = [i64, i32, i32]
    lib.orc_state_init.argtypes = [vp, i64, i32, i32]
    lib.orc_groupby_sum.argtypes = [vp, i32, vp, i32, i64, i64, i32, i32, vp, vp]
    lib.orc_groupby_sum_threads.argtypes = [vp, i32, vp, i32, i64, i64, i32, i32, vp, vp, i32]
    lib.orc_merge.argtypes = [vp, vp, i64, i32, i32]
    lib.orc_finalize.argtypes = [vp, i64, i32, i32, vp]
    lib.orc_sum_fmt.argtypes = [vp, i64, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.orc_jreq.argtypes = [ctypes.c_double, i32, i32, i32]
    lib.orc_extract.argtypes = [ctypes.c_double, i32, i32, i32, i32, i32, vp]
    lib.orc_extract.restype = None
    lib.orc_round.argtypes = [i64, ctypes.c_uint64, i32, i32, i32, i32]
    lib.orc_round.restype = ctypes.c_double
    lib.orc_encode.argtypes = [i64, ctypes.c_uint64, i32, i32, vp, vp]
    lib.orc_derive_stats.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def state_bytes(G: int, T64: bool, L: int) -> int:
    return int(_load().orc_state_bytes(G, int(T64), L))


def state_init(G: int, T64: bool = True, L: int = 2) -> np.ndarray:
    st = np.zeros(state_bytes(G, T64, L), dtype=np.uint8)
    _check(_load().orc_state_init(_ptr(st), G, int(T64), L), "state_init")
    return st


def _cols(keys, values):
    keys = np.ascontiguousarray(keys)
    values = np.ascontiguousarray(values)
    if keys.dtype not in (np.int32, np.int64):
        raise TypeError("keys must be int32 or int64")
    if values.dtype not in (np.float32, np.float64):
        raise TypeError("values must be float32 or float64")
    if keys.shape != values.shape or keys.ndim != 1:
        raise ValueError("keys and values must be 1-D of equal length")
    return keys, values


def groupby_sum(keys, values, G: int, L: int = 2, T64: bool = True, states=None, threads: int = 1):
    """Accumulate (key, value) rows into canonical states; returns (states, status)."""
    keys, values = _cols(keys, values)
    lib = _load()
    st = state_init(G, T64, L) if states is None else np.array(states, dtype=np.uint8, copy=True)
    status = np.zeros(1, dtype=np.uint32)
    args = (_ptr(keys), int(keys.dtype == np.int64), _ptr(values), int(values.dtype == np.float64),
            keys.shape[0], G, int(T64), L, _ptr(st), _ptr(status))
    if threads > 1:
        rc = lib.orc_groupby_sum_threads(*args, threads)
    else:
        rc = lib.orc_groupby_sum(*args)
    _check(rc, "groupby_sum")
    return st, int(status[0])


def merge(dst, src, G: int, L: int = 2, T64: bool = True) -> np.ndarray:
    d = np.array(dst, dtype=np.uint8, copy=True)
    s = np.ascontiguousarray(src, dtype=np.uint8)
    _check(_load().orc_merge(_ptr(d), _ptr(s), G, int(T64), L), "merge")
    return d


def finalize(states, G: int, L: int = 2, T64: bool = True) -> np.ndarray:
    s = np.ascontiguousarray(states, dtype=np.uint8)
    out = np.zeros(G, dtype=np.float64 if T64 else np.float32)
    _check(_load().orc_finalize(_ptr(s), G, int(T64), L, _ptr(out)), "finalize")
    return out


def split_states(states, G: int, L: int, T64: bool = True):
    """Views (S[L,G], C[L,G]) of a state buffer in the documented layout."""
    st = np.ascontiguousarray(states, dtype=np.uint8)
    sb = G * L * (8 if T64 else 4)
    sb = (sb + 7) & ~7
    S = st[: G * L * (8 if T64 else 4)].view(np.float64 if T64 else np.float32).reshape(L, G)
    C = st[sb: sb + G * L * 8].view(np.int64).reshape(L, G)
    return S, C


def sum_fmt(values, fmt, L: int):
    """Reproducible sum of one stream in format fmt=(m,W,B,jmax,emin,emax).

    Returns (top_index, [K_1..K_L] as Python ints, finalised value)."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    top = ctypes.c_int(0)
    khi = np.zeros(8, dtype=np.int64)
    klo = np.zeros(8, dtype=np.uint64)
    res = ctypes.c_double(0.0)
    m, W, B, jmax, emin, emax = fmt
    rc = _load().orc_sum_fmt(_ptr(v), v.shape[0], m, W, B, jmax, emin, emax, L, ctypes.byref(top),
                             _ptr(khi), _ptr(klo), ctypes.byref(res))
    _check(rc, "sum_fmt")
    K = [(int(khi[i]) << 64) | int(klo[i]) for i in range(L)]
    return top.value, K, res.value


def jreq(b: float, m: int, W: int, B: int) -> int:
    return int(_load().orc_jreq(float(b), m, W, B))


def extract(b: float, top: int, L: int, m: int, W: int, B: int):
    k = np.zeros(8, dtype=np.int64)
    _load().orc_extract(float(b), top, L, m, W, B, _ptr(k))
    return [int(x) for x in k[:L]]


def round_exact(K: int, s: int, m: int, emin: int, emax: int) -> float:
    """Nearest number of the format to K * 2^s (ties to even), as a float."""
    hi = K >> 64
    lo = K & ((1 << 64) - 1)
    return float(_load().orc_round(hi, lo, s, m, emin, emax))


def encode(K: int, E: int, m: int):
    """Canonical (S, C) of one level whose exact sum is K units of 2^(E-m)."""
    S = ctypes.c_double(0.0)
    C = ctypes.c_int64(0)
    rc = _load().orc_encode(K >> 64, K & ((1 << 64) - 1), E, m, ctypes.byref(S), ctypes.byref(C))
    _check(rc, "encode")
    return S.value, C.value


def derive_stats(sums, sumsq, counts):
    """AVG, sample VAR and sample STDDEV per group from finalised SUM(x),
    SUM(x*x) (float64) and exact COUNT (int64); returns three float64 arrays."""
    s = np.ascontiguousarray(sums, dtype=np.float64)
    q = np.ascontiguousarray(sumsq, dtype=np.float64)
    c = np.ascontiguousarray(counts, dtype=np.int64)
    G = s.shape[0]
    if q.shape != (G,) or c.shape != (G,):
        raise ValueError("sums, sumsq and counts must have one entry per group")
    avg, var, sd = (np.empty(G, dtype=np.float64) for _ in range(3))
    _check(_load().orc_derive_stats(_ptr(s), _ptr(q), _ptr(c), G, _ptr(avg), _ptr(var), _ptr(sd)), "derive_stats")
    return avg, var, sd
