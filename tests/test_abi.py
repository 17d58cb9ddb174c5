"""The C interface library loads and exports what include/repro.h declares;
host-side argument checks behave as documented (no GPU work is issued)."""
import ctypes
import os

import pytest

from paper_1802_09883_amd import _lib


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1802_09883_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_function(lib):
    names = _lib.header_functions()
    assert set(names) >= {"repro_state_bytes", "repro_workspace_bytes", "repro_state_init", "repro_groupby_sum",
                          "repro_merge", "repro_finalize", "repro_plain_groupby_sum", "repro_version"}
    for name in names:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.repro_version()


def test_state_bytes_layout(lib):
    # S block (padded to 8 bytes) + int64 C block
    assert lib.repro_state_bytes(16, _lib.F64, 2) == 16 * 2 * 8 + 16 * 2 * 8
    assert lib.repro_state_bytes(3, _lib.F32, 1) == 16 + 3 * 8
    assert lib.repro_state_bytes(0, _lib.F64, 2) == 0
    assert lib.repro_state_bytes(4, _lib.F64, 5) == 0


def test_workspace_depends_on_sizes_only(lib):
    a = lib.repro_workspace_bytes(10 ** 6, 16, _lib.I32, _lib.F64, _lib.F64, 2)
    b = lib.repro_workspace_bytes(10 ** 6, 16, _lib.I64, _lib.F32, _lib.F64, 2)
    assert a == b > 0
    assert lib.repro_workspace_bytes(10 ** 6, 16, _lib.I32, _lib.F64, _lib.F64, 0) == 0


def test_invalid_arguments_return_einval_without_gpu(lib):
    p = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    null = ctypes.c_void_p(0)
    # float64 values into float accumulators
    assert lib.repro_groupby_sum(p, 0, p, _lib.F64, 10, 4, _lib.F32, 2, p, p, 1 << 30, null, null) == _lib.REPRO_EINVAL
    # L out of range, no groups, negative n, missing states
    assert lib.repro_groupby_sum(p, 0, p, 1, 10, 4, 1, 5, p, p, 1 << 30, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_groupby_sum(p, 0, p, 1, 10, 0, 1, 2, p, p, 1 << 30, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_groupby_sum(p, 0, p, 1, -1, 4, 1, 2, p, p, 1 << 30, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_groupby_sum(p, 0, p, 1, 10, 4, 1, 2, null, p, 1 << 30, null, null) == _lib.REPRO_EINVAL
    # workspace too small
    assert lib.repro_groupby_sum(p, 0, p, 1, 10 ** 6, 16, 1, 2, p, p, 16, null, null) == _lib.REPRO_EINVAL
    # n = 0 is a no-op
    assert lib.repro_groupby_sum(null, 0, null, 1, 0, 4, 1, 2, p, null, 0, null, null) == _lib.REPRO_OK
    assert lib.repro_merge(p, p, 4, 1, 2, null) == _lib.REPRO_EINVAL
    assert lib.repro_finalize(p, 4, 1, 2, null, null) == _lib.REPRO_EINVAL
    # products: negative n, unknown type, missing output; n = 0 is a no-op
    assert lib.repro_mul(p, _lib.F64, p, _lib.F64, -1, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_mul(p, 7, p, _lib.F64, 10, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_mul(p, _lib.F32, p, _lib.F64, 10, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_mul(null, _lib.F32, null, _lib.F64, 0, null, null) == _lib.REPRO_OK
    # a server poll without a server, or with a negative capacity
    n = ctypes.c_int(5)
    assert lib.repro_server_poll(null, None, None, 4, ctypes.byref(n), None, None, None) == _lib.REPRO_EINVAL


def test_noalloc_entry_rejects_without_gpu(lib):
    p = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    null = ctypes.c_void_p(0)
    # the arguments repro_groupby_sum rejects
    assert lib.repro_groupby_sum_noalloc(p, 0, p, _lib.F64, 10, 4, _lib.F32, 2, p, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_groupby_sum_noalloc(p, 0, p, 1, 10, 4, 1, 5, p, null, null) == _lib.REPRO_EINVAL
    assert lib.repro_groupby_sum_noalloc(p, 0, p, 1, 10, 4, 1, 2, null, null, null) == _lib.REPRO_EINVAL
    # more scratch than the static array holds
    n, G = 10_000_000, 1 << 22
    assert lib.repro_workspace_bytes(n, G, _lib.I64, _lib.F64, _lib.F64, 2) > _lib.NOALLOC_SCRATCH_BYTES
    assert lib.repro_groupby_sum_noalloc(p, 1, p, 1, n, G, 1, 2, p, null, null) == _lib.REPRO_EINVAL
    # every LDS-path call up to 2^31 rows fits
    for L, G in ((1, 7679), (2, 5484), (3, 4265), (4, 3489)):
        assert 0 < lib.repro_workspace_bytes(1 << 31, G, _lib.I32, _lib.F64, _lib.F64, L) <= _lib.NOALLOC_SCRATCH_BYTES
    # n = 0 is a no-op
    assert lib.repro_groupby_sum_noalloc(null, 0, null, 1, 0, 4, 1, 2, p, null, null) == _lib.REPRO_OK


def test_every_group_count_has_a_plan(lib):
    # one LDS workgroup, one partitioning level, two levels, up to 2^31 - 1 groups
    for L in (1, 2, 3, 4):
        for G in (16, 10 ** 5, (1 << 23) + 1, (1 << 24) + 1, 10 ** 9, (1 << 31) - 1):
            assert lib.repro_workspace_bytes(10 ** 6, G, _lib.I64, _lib.F64, _lib.F64, L) > 0, (L, G)
    assert lib.repro_workspace_bytes(10 ** 6, 1 << 31, _lib.I64, _lib.F64, _lib.F64, 2) == 0


def test_plain_baseline_workspace_and_probe_checks(lib):
    # groups that fit LDS need no workspace; beyond, the partitioned baseline does
    assert lib.repro_plain_workspace_bytes(10 ** 6, 1024, _lib.I32, _lib.F64) == 0
    big = lib.repro_plain_workspace_bytes(10 ** 6, 1 << 22, _lib.I64, _lib.F64)
    assert big >= 10 ** 6 * 10  # the partitioned (local key, value) columns
    assert lib.repro_plain_workspace_bytes(10 ** 6, 0, _lib.I32, _lib.F64) == 0
    p = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    assert lib.repro_plain_groupby_sum(p, 0, p, 1, 10, 4, p, ctypes.c_void_p(0x1001), 1 << 20, null, null) == \
        _lib.REPRO_EINVAL  # misaligned workspace
    # the read probe rejects bad shapes before launching anything
    assert lib.repro_read_probe(p, 1024, 0, 256, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_read_probe(p, 1024, 4, 100, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_read_probe(p, 1000, 4, 256, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_read_probe(null, 1024, 4, 256, p, null) == _lib.REPRO_EINVAL
    assert lib.repro_atomic_probe(p, 10, p, 0, 4, null) == _lib.REPRO_EINVAL
    assert lib.repro_atomic_probe(p, 10, p, 16, 0, null) == _lib.REPRO_EINVAL
    assert lib.repro_atomic_probe(null, 10, p, 16, 4, null) == _lib.REPRO_EINVAL
    assert lib.repro_atomic_probe(p, -1, p, 16, 4, null) == _lib.REPRO_EINVAL
    assert lib.repro_atomic_probe(null, 0, null, 16, 4, null) == _lib.REPRO_OK  # nothing to do


def _jobs(specs):
    """Host job records with fake device addresses (the planner never
    dereferences them)."""
    arr = (_lib.BatchJob * len(specs))()
    for i, (n, G, L) in enumerate(specs):
        arr[i] = _lib.BatchJob(0x10000 * (i + 1), 0x20000000 + 0x10000 * i, n, G, L, 0, 0x40000000 + 0x1000 * i, None)
    return arr


def test_batch_workspace_and_validation_without_gpu(lib):
    ok = [(1000, 16, 2), (0, 5, 3), (2_000_000, 70_000, 3), (300_000, 4000, 1)]
    jobs = _jobs(ok)
    need = lib.repro_batch_workspace_bytes(jobs, len(ok), _lib.I32, _lib.F64, _lib.F64, None)
    assert need > 0 and need % 256 == 0
    # the partial sums of split jobs grow with the number of chunks
    small = _lib.BatchConfig(1 << 20, 0, 0, 0)
    assert lib.repro_batch_workspace_bytes(jobs, len(ok), _lib.I32, _lib.F64, _lib.F64, ctypes.byref(small)) < need
    for bad in ([(10, 0, 2)], [(10, 4, 0)], [(10, 4, 5)], [(-1, 4, 2)]):
        assert lib.repro_batch_workspace_bytes(_jobs(bad), 1, _lib.I32, _lib.F64, _lib.F64, None) == 0
    assert lib.repro_batch_workspace_bytes(jobs, len(ok), _lib.I32, _lib.F64, _lib.F32, None) == 0  # narrowing
    nostate = _jobs([(10, 4, 2)])
    nostate[0].states = None
    assert lib.repro_batch_workspace_bytes(nostate, 1, _lib.I32, _lib.F64, _lib.F64, None) == 0
    plan = _lib.BatchPlan()
    # invalid arguments are rejected before anything touches the GPU
    assert lib.repro_batch_prepare(_jobs([(10, 4, 5)]), 1, _lib.I32, _lib.F64, _lib.F64, None, ctypes.c_void_p(256),
                                   1 << 20, ctypes.byref(plan), None) == _lib.REPRO_EINVAL
    assert lib.repro_batch_prepare(jobs, len(ok), _lib.I32, _lib.F64, _lib.F64, None, ctypes.c_void_p(256), need - 1,
                                   ctypes.byref(plan), None) == _lib.REPRO_EINVAL
    assert lib.repro_batch_prepare(jobs, len(ok), _lib.I32, _lib.F64, _lib.F64, None, ctypes.c_void_p(257), need,
                                   ctypes.byref(plan), None) == _lib.REPRO_EINVAL


def test_batch_split_modes_without_gpu(lib):
    """Jobs beyond one workgroup's LDS: sorting their chunks (split 0, the
    default) needs a scratch copy of the rows in the workspace, re-reading
    them per slice (split 1) does not; past 64 slices a job falls back to
    re-reading, so the two modes then need the same workspace."""
    def need(specs, split, cap=0):
        cfg = _lib.BatchConfig(1 << 19, cap, 0, 0, split)
        return lib.repro_batch_workspace_bytes(_jobs(specs), len(specs), _lib.I32, _lib.F64, _lib.F64,
                                               ctypes.byref(cfg))
    big = [(5_000_000, 60_000, 2)]
    sorted_ws, reread_ws = need(big, 0), need(big, 1)
    assert sorted_ws > 0 and reread_ws > 0
    assert sorted_ws - reread_ws >= 5_000_000 * (2 + 8)  # 16-bit local keys and the values
    small = [(5_000_000, 4000, 2)]  # fits one workgroup's LDS: no slices, no copy
    assert need(small, 0) == need(small, 1)
    many = [(5_000_000, 60_000, 2)]  # slices of at most 256 groups: more than 64 of them
    assert need(many, 0, cap=256) == need(many, 1, cap=256)
    bad = _lib.BatchConfig(1 << 19, 0, 0, 0, 2)
    assert lib.repro_batch_workspace_bytes(_jobs(big), 1, _lib.I32, _lib.F64, _lib.F64, ctypes.byref(bad)) == 0


def test_query_bytes_without_gpu(lib):
    q = _lib.Query()
    q.keys = 0x1000
    for i in range(6):
        q.cols[i] = 0x100000 * (i + 1)
    q.n, q.num_groups, q.L, q.naggs = 1_000_000, 1000, 2, 4
    for i, (a, b) in enumerate(((0, -1), (1, -1), (2, 3), (4, 5))):
        q.agg_a[i], q.agg_b[i], q.out[i] = a, b, 0x9000000 + 0x10000 * i
    cfg = _lib.ServerConfig(4, 1 << 20, 0, 0, 0)
    need = lib.repro_query_bytes(ctypes.byref(q), ctypes.byref(cfg))
    # four states, two product columns (8 B per row each), one chunk's workspace
    assert need >= 4 * lib.repro_state_bytes(1000, _lib.F64, 2) + 2 * 8 * 1_000_000
    q.naggs = 5
    assert lib.repro_query_bytes(ctypes.byref(q), ctypes.byref(cfg)) == 0
    q.naggs = 4
    q.cols[5] = None  # a product aggregate without its column
    assert lib.repro_query_bytes(ctypes.byref(q), ctypes.byref(cfg)) == 0
    srv = ctypes.c_void_p()
    bad = _lib.ServerConfig(4, 1 << 20, 0, 0, -1)  # negative bypass bound
    assert lib.repro_server_create(ctypes.c_void_p(256), 1 << 20, ctypes.byref(bad), ctypes.byref(srv)) == \
        _lib.REPRO_EINVAL
    assert lib.repro_server_create(ctypes.c_void_p(257), 1 << 20, ctypes.byref(cfg), ctypes.byref(srv)) == \
        _lib.REPRO_EINVAL  # misaligned arena, rejected before any GPU call


def test_server_poll_error_path_keeps_completions():
    """The binding's poll on the library's error return: the completions the
    call reported are kept in Server.completed and leave the live set, the
    dropped query's ticket leaves it too, and the error names that ticket.
    A stand-in library writes the outputs the C poll writes on that path."""
    from paper_1802_09883_amd import api

    class FakeLib:
        def repro_server_poll(self, h, tk, tm, cap, nd, nq, nr, dr):
            tk[0], tm[0], tk[1], tm[1] = 3, 1.5, 5, 2.5
            nd._obj.value, nq._obj.value, nr._obj.value = 2, 1, 0
            dr._obj.value = 7
            return _lib.REPRO_EHIP

    srv = object.__new__(api.Server)
    srv.lib, srv.h = FakeLib(), None
    srv.live = {3: "a", 5: "b", 7: "c", 9: "d"}
    srv.completed = []
    with pytest.raises(RuntimeError, match="dropped query 7"):
        srv.poll(cap=4)
    assert srv.completed == [(3, 1.5), (5, 2.5)]
    assert set(srv.live) == {9}
