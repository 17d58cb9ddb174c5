"""Python front end of librepro: reproducible GroupBy-SUM into repro<T,L>.

Thin wrappers over the C interface in include/repro.h: PyTorch tensors carry
device memory and streams; every step of the computation runs in the HIP
kernels of librepro.so.  Paper: Mueller, Arteaga, Hoefler, Alonso,
"Reproducible Floating-Point Aggregation in RDBMSs" (arXiv 1802.09883);
RSum(expression, L) of Sec. V-D is ``groupby_sum`` + ``finalize``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

_SCALAR = {torch.float32: _lib.F32, torch.float64: _lib.F64}
_KEY = {torch.int32: _lib.I32, torch.int64: _lib.I64}


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _T(T):
    if T not in _SCALAR:
        raise TypeError("T must be torch.float32 or torch.float64")
    return _SCALAR[T]


def state_bytes(num_groups: int, L: int = 2, T=torch.float64) -> int:
    return int(_lib.load().repro_state_bytes(num_groups, _T(T), L))


def workspace_bytes(n: int, num_groups: int, key_dtype=torch.int32, value_dtype=torch.float64,
                    L: int = 2, T=torch.float64) -> int:
    return int(_lib.load().repro_workspace_bytes(n, num_groups, _KEY[key_dtype], _SCALAR[value_dtype], _T(T), L))


def split_states(states: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64):
    """Views (S[L, G] of dtype T, C[L, G] int64) of a state buffer."""
    es = 8 if T == torch.float64 else 4
    sb = (num_groups * L * es + 7) // 8 * 8
    S = states[: num_groups * L * es].view(T).view(L, num_groups)
    C = states[sb: sb + num_groups * L * 8].view(torch.int64).view(L, num_groups)
    return S, C


def _new(shape, dtype, device, stream, zero=False):
    """A tensor allocated on the stream its kernels run on (the caching
    allocator then hands its memory to no other stream while they may run)."""
    s = stream if stream is not None else torch.cuda.current_stream(device)
    with torch.cuda.stream(s):
        return (torch.zeros if zero else torch.empty)(shape, dtype=dtype, device=device)


def state_init(num_groups: int, L: int = 2, T=torch.float64, device="cuda", stream=None) -> torch.Tensor:
    lib = _lib.load()
    st = _new(state_bytes(num_groups, L, T), torch.uint8, torch.device(device), stream)
    _lib.check(lib.repro_state_init(_vp(st), num_groups, _T(T), L, _stream(st.device, stream)), "state_init")
    return st


_WS = {}


def _workspace(nbytes: int, device, stream=None) -> torch.Tensor:
    """A cached workspace per (device, stream): calls on one stream are
    ordered, so they may share it; calls on different streams get their own.
    It is allocated on that stream, so the caching allocator does not hand its
    memory to another stream while a kernel may still use it."""
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (torch.device(device), s.cuda_stream)
    ws = _WS.get(key)
    if ws is None or ws.numel() < nbytes:
        with torch.cuda.stream(s):
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS[key] = ws
    return ws


def groupby_sum(keys: torch.Tensor, values: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64,
                states: torch.Tensor | None = None, status: torch.Tensor | None = None,
                workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Accumulate rows (keys[i], values[i]) into repro<T,L> states per group.

    Returns ``states`` (a fresh state buffer if none is given).  ``status`` is
    an optional device uint32 tensor OR-ed with REPRO_ERR_* bits."""
    lib = _lib.load()
    if keys.dtype not in _KEY or values.dtype not in _SCALAR:
        raise TypeError("keys int32/int64, values float32/float64")
    if keys.shape != values.shape or keys.dim() != 1:
        raise ValueError("keys and values must be 1-D of equal length")
    if not (keys.is_cuda and values.is_cuda) or keys.device != values.device:
        raise ValueError("keys and values must be on the same GPU")
    keys, values = keys.contiguous(), values.contiguous()
    dev = keys.device
    if states is None:
        states = state_init(num_groups, L, T, dev, stream)
    n = keys.numel()
    need = workspace_bytes(n, num_groups, keys.dtype, values.dtype, L, T)
    ws = workspace if workspace is not None else (_workspace(need, dev, stream) if need else None)
    rc = lib.repro_groupby_sum(_vp(keys), _KEY[keys.dtype], _vp(values), _SCALAR[values.dtype], n, num_groups,
                               _T(T), L, _vp(states), _vp(ws), ws.numel() if ws is not None else 0, _vp(status),
                               _stream(dev, stream))
    _lib.check(rc, "groupby_sum")
    return states


def groupby_sum_noalloc(keys: torch.Tensor, values: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64,
                       states: torch.Tensor | None = None, status: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """``groupby_sum`` through the entry point that allocates nothing: its
    scratch memory is the library's static device array, shared by every call
    on the GPU (calls that may overlap on one GPU race).  ``states`` must be
    given where the caller cannot allocate (a fresh state buffer is made
    otherwise)."""
    lib = _lib.load()
    if keys.dtype not in _KEY or values.dtype not in _SCALAR:
        raise TypeError("keys int32/int64, values float32/float64")
    if keys.shape != values.shape or keys.dim() != 1:
        raise ValueError("keys and values must be 1-D of equal length")
    if not (keys.is_cuda and values.is_cuda) or keys.device != values.device:
        raise ValueError("keys and values must be on the same GPU")
    if not (keys.is_contiguous() and values.is_contiguous()):
        raise ValueError("keys and values must be contiguous")
    dev = keys.device
    if states is None:
        states = state_init(num_groups, L, T, dev, stream)
    with torch.cuda.device(dev):
        rc = lib.repro_groupby_sum_noalloc(_vp(keys), _KEY[keys.dtype], _vp(values), _SCALAR[values.dtype],
                                           keys.numel(), num_groups, _T(T), L, _vp(states), _vp(status),
                                           _stream(dev, stream))
    _lib.check(rc, "groupby_sum_noalloc")
    return states


def workspace_bytes_cols(n: int, num_groups: int, key_dtype, value_dtypes, L: int = 2, T=torch.float64) -> int:
    vts = (ctypes.c_int * len(value_dtypes))(*[_SCALAR[d] for d in value_dtypes])
    return int(_lib.load().repro_workspace_bytes_cols(n, num_groups, _KEY[key_dtype], len(value_dtypes), vts,
                                                      _T(T), L))


def _check_cols(keys, columns):
    if keys.dtype not in _KEY or keys.dim() != 1 or not keys.is_cuda:
        raise TypeError("keys must be a 1-D int32/int64 GPU tensor")
    if not 1 <= len(columns) <= _lib.MAX_COLS:
        raise ValueError(f"1..{_lib.MAX_COLS} value columns")
    for v in columns:
        if v.dtype not in _SCALAR or v.shape != keys.shape or v.device != keys.device:
            raise ValueError("value columns must be float32/float64 of the keys' shape, on the keys' GPU")


def groupby_sum_cols(keys: torch.Tensor, columns, num_groups: int, L: int = 2, T=torch.float64, states=None,
                     status: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None):
    """Several SUM aggregates over one GROUP BY: states[c] += the GroupBy-SUM
    of columns[c] (one key pass for up to four columns).  Returns the list of
    states (fresh ones where none are given); each has the bits
    ``groupby_sum`` gives for its column alone."""
    lib = _lib.load()
    _check_cols(keys, columns)
    keys = keys.contiguous()
    columns = [v.contiguous() for v in columns]
    dev = keys.device
    if states is None:
        states = [state_init(num_groups, L, T, dev, stream) for _ in columns]
    if len(states) != len(columns):
        raise ValueError("one state per column")
    n = keys.numel()
    need = workspace_bytes_cols(n, num_groups, keys.dtype, [v.dtype for v in columns], L, T)
    ws = workspace if workspace is not None else (_workspace(need, dev, stream) if need else None)
    nc = len(columns)
    vals = (ctypes.c_void_p * nc)(*[v.data_ptr() for v in columns])
    vts = (ctypes.c_int * nc)(*[_SCALAR[v.dtype] for v in columns])
    sts = (ctypes.c_void_p * nc)(*[s.data_ptr() for s in states])
    rc = lib.repro_groupby_sum_cols(_vp(keys), _KEY[keys.dtype], nc, vals, vts, n, num_groups, _T(T), L, sts,
                                    _vp(ws), ws.numel() if ws is not None else 0, _vp(status), _stream(dev, stream))
    _lib.check(rc, "groupby_sum_cols")
    return states


def plain_groupby_sum_cols(keys: torch.Tensor, columns, num_groups: int, outs=None, status=None, stream=None):
    """Non-reproducible baseline over several columns (plain double atomics,
    one key pass for up to four columns); outs are accumulated into."""
    lib = _lib.load()
    _check_cols(keys, columns)
    keys = keys.contiguous()
    columns = [v.contiguous() for v in columns]
    if outs is None:
        outs = [_new(num_groups, torch.float64, keys.device, stream, zero=True) for _ in columns]
    nc = len(columns)
    vals = (ctypes.c_void_p * nc)(*[v.data_ptr() for v in columns])
    vts = (ctypes.c_int * nc)(*[_SCALAR[v.dtype] for v in columns])
    ops = (ctypes.c_void_p * nc)(*[o.data_ptr() for o in outs])
    rc = lib.repro_plain_groupby_sum_cols(_vp(keys), _KEY[keys.dtype], nc, vals, vts, keys.numel(), num_groups, ops,
                                          _vp(status), _stream(keys.device, stream))
    _lib.check(rc, "plain_groupby_sum_cols")
    return outs


def sum(values: torch.Tensor, L: int = 2, T=torch.float64, state: torch.Tensor | None = None,
        status: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Ungrouped reproducible sum of a column into a one-group state
    (returned; a fresh one if none is given)."""
    lib = _lib.load()
    if values.dtype not in _SCALAR or values.dim() != 1 or not values.is_cuda:
        raise TypeError("values: 1-D float32/float64 device tensor")
    values = values.contiguous()
    if state is None:
        state = state_init(1, L, T, values.device, stream)
    need = int(lib.repro_sum_workspace_bytes(values.numel(), L))
    ws = _workspace(need, values.device, stream) if need else None
    _lib.check(lib.repro_sum(_vp(values), _SCALAR[values.dtype], values.numel(), _T(T), L, _vp(state), _vp(ws),
                             need, _vp(status), _stream(values.device, stream)), "sum")
    return state


def groupby_count(keys: torch.Tensor, num_groups: int, counts=None, status=None, stream=None) -> torch.Tensor:
    """Exact int64 row counts per group (accumulated into ``counts``)."""
    lib = _lib.load()
    keys = keys.contiguous()
    if counts is None:
        counts = _new(num_groups, torch.int64, keys.device, stream, zero=True)
    _lib.check(lib.repro_groupby_count(_vp(keys), _KEY[keys.dtype], keys.numel(), num_groups, _vp(counts),
                                       _vp(status), _stream(keys.device, stream)), "groupby_count")
    return counts


def mul(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """out[i] = a[i] * b[i] in float64, one IEEE rounding (float inputs widen
    exactly): the expression column of an aggregate such as SUM(a * b)."""
    for t in (a, b):
        if t.dtype not in _SCALAR or t.dim() != 1 or not t.is_cuda:
            raise TypeError("mul: 1-D float32/float64 device tensors")
    if a.shape != b.shape or a.device != b.device:
        raise ValueError("mul: columns of equal length on one GPU")
    a, b = a.contiguous(), b.contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(a.device)
    if out is None:
        out = _new(a.numel(), torch.float64, a.device, s)
    _lib.check(_lib.load().repro_mul(_vp(a), _SCALAR[a.dtype], _vp(b), _SCALAR[b.dtype], a.numel(), _vp(out),
                                     ctypes.c_void_p(s.cuda_stream)), "mul")
    return out


def groupby_stats(keys: torch.Tensor, values: torch.Tensor, num_groups: int, L: int = 2, status=None, stream=None):
    """Reproducible AVG, sample VAR and sample STDDEV per group, derived from
    the reproducible SUM(x), SUM(x*x) (x*x rounded once per row, in a HIP
    kernel) and the exact COUNT.  Every step runs on ``stream`` (default: the
    current one); ``status`` is OR-ed with the REPRO_ERR_* bits of the rows.
    Returns a dict of device tensors."""
    lib = _lib.load()
    if keys.dtype not in _KEY or values.dtype not in _SCALAR or keys.shape != values.shape or keys.dim() != 1:
        raise TypeError("keys int32/int64 and values float32/float64, 1-D of equal length")
    dev = keys.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    sq = mul(values, values, stream=s)
    c = _new(num_groups, torch.int64, dev, s, zero=True)
    avg, var, sd = (_new(num_groups, torch.float64, dev, s) for _ in range(3))
    sum_x = finalize(groupby_sum(keys, values, num_groups, L, status=status, stream=s), num_groups, L, stream=s)
    sum_q = finalize(groupby_sum(keys, sq, num_groups, L, status=status, stream=s), num_groups, L, stream=s)
    groupby_count(keys, num_groups, counts=c, status=status, stream=s)
    _lib.check(lib.repro_derive_stats(_vp(sum_x), _vp(sum_q), _vp(c), num_groups, _vp(avg), _vp(var), _vp(sd),
                                      ctypes.c_void_p(s.cuda_stream)), "derive_stats")
    return {"sum": sum_x, "sumsq": sum_q, "count": c, "avg": avg, "var_samp": var, "stddev_samp": sd}


def merge(dst: torch.Tensor, src: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64, stream=None):
    """dst += src group by group (operator+=(repro)); returns dst."""
    lib = _lib.load()
    _lib.check(lib.repro_merge(_vp(dst), _vp(src), num_groups, _T(T), L, _stream(dst.device, stream)), "merge")
    return dst


def finalize(states: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64, out=None, stream=None):
    """Finalised sums (type T) of every group."""
    lib = _lib.load()
    if out is None:
        out = _new(num_groups, T, states.device, stream)
    _lib.check(lib.repro_finalize(_vp(states), num_groups, _T(T), L, _vp(out), _stream(states.device, stream)),
               "finalize")
    return out


def plain_groupby_sum(keys: torch.Tensor, values: torch.Tensor, num_groups: int, out=None, status=None,
                      stream=None) -> torch.Tensor:
    """Non-reproducible baseline: double-precision GroupBy-SUM (LDS atomics;
    partitioned first when the groups do not fit LDS, as the reproducible
    path is)."""
    lib = _lib.load()
    keys, values = keys.contiguous(), values.contiguous()
    if out is None:
        out = _new(num_groups, torch.float64, keys.device, stream, zero=True)
    need = int(lib.repro_plain_workspace_bytes(keys.numel(), num_groups, _KEY[keys.dtype], _SCALAR[values.dtype]))
    ws = _workspace(need, keys.device, stream) if need else None
    rc = lib.repro_plain_groupby_sum(_vp(keys), _KEY[keys.dtype], _vp(values), _SCALAR[values.dtype], keys.numel(),
                                     num_groups, _vp(out), _vp(ws), need, _vp(status), _stream(keys.device, stream))
    _lib.check(rc, "plain_groupby_sum")
    return out


def rsum(keys, values, num_groups: int, L: int = 2, T=torch.float64, stream=None):
    """RSum(expression, L): GroupBy-SUM and finalisation in one call."""
    st = groupby_sum(keys, values, num_groups, L, T, stream=stream)
    return finalize(st, num_groups, L, T, stream=stream)


def profile_arm(max_launches: int = 1):
    """Time the aggregation kernels of this thread's next groupby_sum calls."""
    _lib.check(_lib.load().repro_profile_arm(max_launches), "profile_arm")


def profile_read(cap: int = 4096):
    """Milliseconds of each armed aggregation kernel, in call order."""
    ms = (ctypes.c_float * cap)()
    cnt = ctypes.c_int(0)
    _lib.check(_lib.load().repro_profile_read(ms, cap, ctypes.byref(cnt)), "profile_read")
    return [float(ms[i]) for i in range(cnt.value)]


def state_reset(states: torch.Tensor, num_groups: int, L: int = 2, T=torch.float64, stream=None):
    """Re-initialise an existing state buffer in place (empty groups)."""
    _lib.check(_lib.load().repro_state_init(_vp(states), num_groups, _T(T), L, _stream(states.device, stream)),
               "state_init")
    return states


# ----------------------------------------------------------------- batches

class Job:
    """One GroupBy-SUM of a batch: its key and value columns (device tensors),
    group count, levels and state buffer; ``out`` (optional) receives the
    finalised sums; ``accumulate`` adds into the states instead of
    overwriting them."""

    def __init__(self, keys, values, num_groups, L, states, out=None, accumulate=False):
        self.keys, self.values, self.num_groups, self.L = keys, values, int(num_groups), int(L)
        self.states, self.out, self.accumulate = states, out, bool(accumulate)


def _batch_jobs(jobs):
    arr = (_lib.BatchJob * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        if j.keys.dtype != jobs[0].keys.dtype or j.values.dtype != jobs[0].values.dtype:
            raise TypeError("all jobs of a batch share the key and value dtypes")
        arr[i] = _lib.BatchJob(_vp(j.keys).value, _vp(j.values).value, j.keys.numel(), j.num_groups, j.L,
                               int(j.accumulate), _vp(j.states).value, _vp(j.out).value if j.out is not None else None)
    return arr


def _batch_config(config):
    if config is None:
        return None
    return ctypes.byref(_lib.BatchConfig(int(config.get("chunk_rows", 0)), int(config.get("max_slice_groups", 0)),
                                         int(config.get("order", 0)), int(config.get("merge", 0)),
                                         int(config.get("split", 0))))


class BatchRun:
    """A prepared batch: the plan, its workspace and references to the jobs'
    tensors (kept alive while the plan may be launched)."""

    def __init__(self, plan, workspace, jobs):
        self.plan, self.workspace, self.jobs = plan, workspace, jobs


def batch_prepare(jobs, T=torch.float64, config=None, stream=None) -> BatchRun:
    """Plans the batch and uploads the plan into a fresh workspace."""
    lib = _lib.load()
    if not jobs:
        raise ValueError("empty batch")
    for j in jobs:
        if j.keys.shape != j.values.shape or j.keys.dim() != 1 or not j.keys.is_contiguous() \
                or not j.values.is_contiguous():
            raise ValueError("job columns must be contiguous 1-D tensors of equal length")
    dev = jobs[0].keys.device
    arr = _batch_jobs(jobs)
    kt, vt = _KEY[jobs[0].keys.dtype], _SCALAR[jobs[0].values.dtype]
    cfg = _batch_config(config)
    need = lib.repro_batch_workspace_bytes(arr, len(jobs), kt, vt, _T(T), cfg)
    if need == 0:
        raise ValueError("batch_prepare: invalid jobs or configuration")
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.stream(s):
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    plan = _lib.BatchPlan()
    _lib.check(lib.repro_batch_prepare(arr, len(jobs), kt, vt, _T(T), cfg, _vp(ws), need, ctypes.byref(plan),
                                       ctypes.c_void_p(s.cuda_stream)), "batch_prepare")
    return BatchRun(plan, ws, list(jobs))


def batch_launch(run: BatchRun, status=None, stream=None):
    """Runs a prepared batch (kernels only; may be captured into a graph)."""
    s = stream if stream is not None else torch.cuda.current_stream(run.workspace.device)
    _lib.check(_lib.load().repro_batch_launch(ctypes.byref(run.plan), _vp(status), ctypes.c_void_p(s.cuda_stream)),
               "batch_launch")


def batch_groupby_sum(jobs, T=torch.float64, config=None, status=None, stream=None) -> BatchRun:
    """Prepare and launch a batch; returns the prepared run for re-launches."""
    run = batch_prepare(jobs, T, config, stream)
    batch_launch(run, status, stream)
    return run


def batch_tune(jobs, T=torch.float64, stream=None):
    """The autotuner: returns (best config dict, its milliseconds).  The jobs'
    states and outputs hold unspecified values afterwards."""
    lib = _lib.load()
    dev = jobs[0].keys.device
    arr = _batch_jobs(jobs)
    kt, vt = _KEY[jobs[0].keys.dtype], _SCALAR[jobs[0].values.dtype]
    # the largest workspace over the candidates the tuner times
    need = max(lib.repro_batch_workspace_bytes(arr, len(jobs), kt, vt, _T(T), _batch_config(
        {"chunk_rows": c, "max_slice_groups": cap, "merge": m, "split": sp}))
               for c in (65536, 131072, 262144, 524288, 1048576, 2097152) for cap in (0, 1024) for m in (0, 1)
               for sp in (0, 1))
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.stream(s):
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    best = _lib.BatchConfig()
    ms = ctypes.c_float(0)
    _lib.check(lib.repro_batch_tune(arr, len(jobs), kt, vt, _T(T), _vp(ws), need, ctypes.byref(best),
                                    ctypes.byref(ms), ctypes.c_void_p(s.cuda_stream)), "batch_tune")
    return {"chunk_rows": best.chunk_rows, "max_slice_groups": best.max_slice_groups, "order": best.order,
            "merge": best.merge, "split": best.split}, ms.value


# ----------------------------------------------------------------- serving

class QuerySpec:
    """A GroupBy query with up to four SUM aggregates: each aggregate is
    SUM(cols[a]) or SUM(cols[a] * cols[b]).  ``keys`` int32 and ``cols``
    float64 device tensors of equal length; ``out`` receives one float64
    tensor of num_groups finalised sums per aggregate."""

    def __init__(self, keys, cols, num_groups, aggs, L=2, status=None):
        self.keys, self.cols, self.num_groups, self.aggs, self.L = keys, list(cols), int(num_groups), list(aggs), L
        self.status = status
        self.out = [torch.empty(self.num_groups, dtype=torch.float64, device=keys.device) for _ in self.aggs]

    def record(self):
        q = _lib.Query()
        q.keys = _vp(self.keys).value
        for i, c in enumerate(self.cols[:_lib.MAX_COLS]):
            q.cols[i] = _vp(c).value
        q.n = self.keys.numel()
        q.num_groups = self.num_groups
        q.L = self.L
        q.naggs = len(self.aggs)  # more than MAX_AGGS is rejected by the library
        for i, (a, b) in enumerate(self.aggs[:_lib.MAX_AGGS]):
            q.agg_a[i], q.agg_b[i] = a, (-1 if b is None else b)
            q.out[i] = _vp(self.out[i]).value
        q.status = _vp(self.status).value if self.status is not None else None
        return q


class Server:
    """Request loop over a device arena (see include/repro.h): submit()
    queues a query, poll() retires finished queries and admits queued ones
    without blocking."""

    def __init__(self, arena_bytes, slots=4, chunk_rows=0, batch_path=True, query_workgroups=0, max_bypass=0,
                 device="cuda"):
        self.lib = _lib.load()
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        self.cfg = _lib.ServerConfig(slots, chunk_rows, 0 if batch_path else 1, query_workgroups, max_bypass)
        h = ctypes.c_void_p()
        _lib.check(self.lib.repro_server_create(_vp(self.arena), arena_bytes, ctypes.byref(self.cfg),
                                                ctypes.byref(h)), "server_create")
        self.h = h
        self.live = {}  # ticket -> query (keeps its tensors alive)
        self.completed = []  # completions reported by a poll that raised

    def query_bytes(self, spec):
        return int(self.lib.repro_query_bytes(ctypes.byref(spec.record()), ctypes.byref(self.cfg)))

    def submit(self, spec):
        t = ctypes.c_int64()
        _lib.check(self.lib.repro_server_submit(self.h, ctypes.byref(spec.record()), ctypes.byref(t)), "submit")
        self.live[t.value] = spec
        return t.value

    def poll(self, cap=256):
        """Returns ([(ticket, completion time)], queued, running).  If a
        query's work could not be enqueued, the completions of this call are
        kept in ``completed``, the dropped query is forgotten and
        RuntimeError is raised naming its ticket."""
        tk = (ctypes.c_int64 * cap)()
        tm = (ctypes.c_double * cap)()
        nd, nq, nr, dr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(-1)
        rc = self.lib.repro_server_poll(self.h, tk, tm, cap, ctypes.byref(nd), ctypes.byref(nq), ctypes.byref(nr),
                                        ctypes.byref(dr))
        done = [(tk[i], tm[i]) for i in range(min(nd.value, cap))]
        for t, _ in done:
            self.live.pop(t, None)
        if dr.value >= 0:
            self.live.pop(dr.value, None)
        if rc != _lib.REPRO_OK:
            self.completed.extend(done)
            raise RuntimeError(f"poll: HIP error (code {rc}); dropped query {dr.value}; "
                               f"{len(done)} completions kept in Server.completed")
        return done, nq.value, nr.value

    def clock(self):
        return self.lib.repro_server_clock()

    def close(self):
        if self.h:
            _lib.check(self.lib.repro_server_destroy(self.h), "server_destroy")
            self.h = None
