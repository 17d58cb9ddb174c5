"""The allocation-free GroupBy-SUM entry point (repro_groupby_sum_noalloc,
called through the C interface) gives the bits of repro_groupby_sum with a
caller workspace, and of the oracle, on consecutive calls that share the
library's static scratch array: the second and later calls are smaller and
must not see what an earlier call left in it (spill words, partials)."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1802_09883_amd import _lib, api
else:  # collected on CPU-only hosts, never run there
    _lib = api = None


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rising(n, G, seed):
    """Magnitudes grow along the rows and a few huge values come late, so a
    workgroup's tops keep rising and rows go through the spill array."""
    rng = np.random.default_rng(seed)
    e = (-900 + (np.arange(n) * 1800) // n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), e + rng.integers(-3, 4, n))
    late = rng.choice(n, 100, replace=False)
    vals[late] = np.ldexp(rng.standard_normal(100), rng.integers(950, 1000, 100))
    keys = rng.integers(0, G, n).astype(np.int32)
    return keys, vals


def noalloc_call(keys_t, vals_t, G, L, T64):
    """One call of the C entry point on the current stream."""
    lib = _lib.load()
    T = _lib.F64 if T64 else _lib.F32
    states = api.state_init(G, L, torch.float64 if T64 else torch.float32)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    kt = _lib.I32 if keys_t.dtype == torch.int32 else _lib.I64
    vt = _lib.F64 if vals_t.dtype == torch.float64 else _lib.F32
    rc = lib.repro_groupby_sum_noalloc(ctypes.c_void_p(keys_t.data_ptr()), kt, ctypes.c_void_p(vals_t.data_ptr()),
                                       vt, keys_t.numel(), G, T, L, ctypes.c_void_p(states.data_ptr()),
                                       ctypes.c_void_p(status.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.REPRO_OK, rc
    torch.cuda.synchronize()
    return states, int(status.item())


def check(keys, vals, G, L, T64, what):
    say(f"case {what}: n={len(keys)} G={G} L={L} T64={T64}")
    kt, vt = dev(keys), dev(vals)
    st_na, status_na = noalloc_call(kt, vt, G, L, T64)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    st_ws = api.groupby_sum(kt, vt, G, L, torch.float64 if T64 else torch.float32, status=status)
    torch.cuda.synchronize()
    assert status_na == int(status.item()), what
    assert torch.equal(st_na, st_ws), f"{what}: noalloc states differ from the workspace entry point"
    orc, ost = O.groupby_sum(keys, vals, G, L, T64, threads=8)
    assert status_na == ost, what
    assert np.array_equal(st_na.cpu().numpy(), orc), f"{what}: noalloc states differ from the oracle"


def test_noalloc_matches_workspace_entry_on_consecutive_calls():
    # 1: spill array in use (several tiles per workgroup, rising tops)
    keys, vals = rising(3_000_000, 64, 1)
    check(keys, vals, 64, 2, True, "noalloc 1: rising tops, spill path")
    # 2: smaller, same shape: nothing of call 1 may leak in
    keys, vals = rising(500_000, 64, 2)
    check(keys, vals, 64, 2, True, "noalloc 2: smaller rising-tops input")
    # 3: smaller still, more groups and levels, error rows
    rng = np.random.default_rng(3)
    n, G = 100_003, 1000
    keys = rng.integers(-3, G + 3, n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-500, 500, n))
    vals[rng.random(n) < 0.001] = np.inf
    check(keys, vals, G, 3, True, "noalloc 3: error rows, int64 keys")
    # 4: a small high-cardinality call (partitioned path) inside the array
    n, G = 200_000, 50_000
    keys = rng.integers(0, G, n).astype(np.int32)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-60, 60, n)).astype(np.float32)
    check(keys, vals, G, 2, False, "noalloc 4: partitioned, float accumulators")


def test_noalloc_rejects_calls_beyond_the_array():
    lib = _lib.load()
    n, G = 10_000_000, 1 << 22  # partitioned: about 180 MiB of scratch
    assert lib.repro_workspace_bytes(n, G, _lib.I64, _lib.F64, _lib.F64, 2) > _lib.NOALLOC_SCRATCH_BYTES
    p = ctypes.c_void_p(0x1000)  # never dereferenced: the size check fails first
    rc = lib.repro_groupby_sum_noalloc(p, _lib.I64, p, _lib.F64, n, G, _lib.F64, 2, p, None, None)
    assert rc == _lib.REPRO_EINVAL
