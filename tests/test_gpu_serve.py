"""Serving: queries admitted by memory into a fixed set of slots, their
states resident and fed chunk by chunk; every result must be bit-identical
alone and in the mix, and equal to the oracle (needs a GPU)."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1802_09883_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1802_09883_amd import api
else:  # collected on CPU-only hosts, never run there
    api = None


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_queries(count, max_rows, max_groups, salt):
    rows, groups, gaps = WL.served_queries(count, min_rows=10_000, max_rows=max_rows, max_groups=max_groups, salt=salt)
    pool = WL.decimal_columns(int(rows.max()), 6, salt=salt)
    pool_t = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in pool]
    host, specs = [], []
    rng = np.random.default_rng(salt)
    for q, (n, G) in enumerate(zip(rows, groups)):
        off = int(rng.integers(0, int(rows.max()) - int(n) + 1))
        keys = WL.served_keys(int(n), int(G), q, salt)
        host.append((keys, off, int(n), int(G)))
        specs.append(api.QuerySpec(torch.from_numpy(keys).cuda(), [c[off:off + n] for c in pool_t], int(G),
                                   WL.SERVED_AGGS, L=2))
    return pool, host, specs, gaps


def oracle_sums(pool, keys, off, n, G, L=2):
    cols = [c[off:off + n] for c in pool]
    outs = []
    for a, b in WL.SERVED_AGGS:
        v = cols[a] if b is None else cols[a] * cols[b]  # one IEEE rounding, as on the device
        st, status = O.groupby_sum(keys, v, G, L, True, threads=8)
        assert status == 0
        outs.append(O.finalize(st, G, L))
    return outs


def run_server(specs, arrival_gaps=None, slots=4, arena_bytes=4 << 30, chunk_rows=300_000, timeout=120.0,
               batch_path=True):
    srv = api.Server(arena_bytes, slots=slots, chunk_rows=chunk_rows, batch_path=batch_path)
    try:
        t0 = srv.clock()
        arr = t0 + (np.cumsum(arrival_gaps) if arrival_gaps is not None else np.zeros(len(specs)))
        done, i, peak = {}, 0, 0
        while len(done) < len(specs):
            now = srv.clock()
            while i < len(specs) and arr[i] <= now:
                assert srv.submit(specs[i]) == i
                i += 1
            comp, nq, nr = srv.poll()
            peak = max(peak, nr)
            for t, tm in comp:
                done[t] = tm
            assert srv.clock() - t0 < timeout, "server did not finish"
        torch.cuda.synchronize()
        return [done[k] - arr[k] for k in range(len(specs))], peak
    finally:
        srv.close()


@pytest.mark.parametrize("batch_path", [True, False])
def test_each_result_same_alone_and_in_the_mix(batch_path):
    """Alone uses the other execution path for queries that fit LDS (one
    batch launch vs chunked repro_groupby_sum), so the paths are compared too."""
    pool, host, specs, gaps = make_queries(14, max_rows=1_500_000, max_groups=1 << 20, salt=1)
    say(f"case serve mix: {len(specs)} queries, rows {[h[2] for h in host]}, groups {[h[3] for h in host]}")
    alone = []
    for s in specs:
        run_server([s], slots=1, batch_path=not batch_path)
        alone.append([o.clone() for o in s.out])
    for s in specs:
        for o in s.out:
            o.fill_(float("nan"))
    # in the mix: arrivals 50 us apart on average, 4 slots, chunked states
    lat, peak = run_server(specs, arrival_gaps=gaps * 50e-6, slots=4, batch_path=batch_path)
    say(f"mix: peak running {peak}, latencies ms {np.round(np.array(lat) * 1e3, 2)}")
    assert peak >= 2, "queries should have overlapped"
    for q, (s, a, (keys, off, n, G)) in enumerate(zip(specs, alone, host)):
        ref = oracle_sums(pool, keys, off, n, G)
        for k, (o, b, r) in enumerate(zip(s.out, a, ref)):
            got = o.cpu().numpy()
            assert np.array_equal(got.view(np.uint8), b.cpu().numpy().view(np.uint8)), \
                f"query {q} aggregate {k}: differs between alone and in the mix"
            assert np.array_equal(got.view(np.uint8), r.view(np.uint8)), f"query {q} aggregate {k}: differs from oracle"


def test_admission_waits_for_memory():
    """Six queries of one size, all submitted at once, into an arena that
    holds two of them: never more than two run, and all finish correctly."""
    n, G = 300_000, 3000
    pool = WL.decimal_columns(n, 6, salt=2)
    pool_t = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in pool]
    host, specs = [], []
    for q in range(6):
        keys = WL.served_keys(n, G, q, salt=2)
        host.append(keys)
        specs.append(api.QuerySpec(torch.from_numpy(keys).cuda(), pool_t, G, WL.SERVED_AGGS, L=2))
    probe = api.Server(1 << 30, slots=8, chunk_rows=300_000)
    need = probe.query_bytes(specs[0])
    probe.close()
    arena = (need // 256 + 1) * 256 * 2 + need // 2  # two fit, three do not
    lat, peak = run_server(specs, slots=8, arena_bytes=arena)
    assert peak == 2, f"memory admits exactly two queries at a time, saw {peak}"
    for s, keys in zip(specs, host):
        for o, r in zip(s.out, oracle_sums(pool, keys, 0, n, G)):
            assert np.array_equal(o.cpu().numpy(), r)


def test_invalid_and_oversized_queries_are_rejected():
    keys = torch.zeros(100, dtype=torch.int32, device="cuda")
    col = torch.ones(100, dtype=torch.float64, device="cuda")
    srv = api.Server(1 << 20, slots=2)
    try:
        with pytest.raises(ValueError):
            srv.submit(api.QuerySpec(keys, [col], 4, [(0, None)] * 5))  # too many aggregates
        with pytest.raises(ValueError):
            srv.submit(api.QuerySpec(keys, [col], 4, [(3, None)]))  # missing column
        with pytest.raises(ValueError):
            srv.submit(api.QuerySpec(keys, [col], 1 << 20, [(0, None)]))  # states larger than the arena
        spec = api.QuerySpec(keys, [col], 4, [(0, None), (0, 0)])
        assert srv.submit(spec) == 0
        while True:
            done, nq, nr = srv.poll()
            if done:
                break
            time.sleep(0.001)
        torch.cuda.synchronize()
        assert spec.out[0].cpu().tolist() == [100.0, 0.0, 0.0, 0.0]
        assert spec.out[1].cpu().tolist() == [100.0, 0.0, 0.0, 0.0]
    finally:
        srv.close()


def test_status_bits_and_empty_query():
    rng = np.random.default_rng(12)
    n, G = 50_000, 300
    keys = rng.integers(0, G, n).astype(np.int32)
    keys[::1000] = G + 5  # bad keys
    cols = WL.decimal_columns(n, 2, salt=12)
    cols[0][17] = np.nan
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    spec = api.QuerySpec(torch.from_numpy(keys).cuda(), [torch.from_numpy(c).cuda() for c in cols], G,
                         [(0, None), (0, 1)], L=3, status=status)
    empty = api.QuerySpec(torch.zeros(0, dtype=torch.int32, device="cuda"),
                          [torch.zeros(0, dtype=torch.float64, device="cuda")] * 2, 7, [(0, None), (0, 1)], L=2)
    run_server([spec, empty], slots=2)
    assert int(status.item()) == 1 | 2
    for o, v in zip(spec.out, (cols[0], cols[0] * cols[1])):
        st, s = O.groupby_sum(keys, v, G, 3)
        assert s == 3
        assert np.array_equal(o.cpu().numpy(), O.finalize(st, G, 3))
    for o in empty.out:
        assert o.cpu().numpy().tolist() == [0.0] * 7


def test_poll_reports_every_completion_within_cap():
    """Completions beyond the caller's `cap` stay in their slots and are
    reported by later polls: no ticket is lost, the counts are always
    written, and no poll reports more than `cap`."""
    n, G = 20_000, 64
    keys = torch.from_numpy(WL.served_keys(n, G, 0, salt=5)).cuda()
    cols = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in WL.decimal_columns(n, 2, salt=5)]
    specs = [api.QuerySpec(keys, cols, G, [(0, None), (0, 1)], L=2) for _ in range(6)]
    srv = api.Server(1 << 28, slots=6)
    try:
        for s in specs:
            srv.submit(s)
        _, nq, nr = srv.poll(cap=6)  # admits all six
        assert nq == 0 and nr == 6
        torch.cuda.synchronize()
        time.sleep(0.01)
        seen = []
        for _ in range(50):
            done, nq, nr = srv.poll(cap=2)
            assert len(done) <= 2
            seen += [t for t, _ in done]
            if len(seen) == 6:
                break
        assert sorted(seen) == list(range(6)) and nr == 0 and nq == 0
        assert not srv.live
    finally:
        srv.close()
    want = O.finalize(O.groupby_sum(keys.cpu().numpy(), cols[0].cpu().numpy(), G, 2)[0], G, 2)
    for s in specs:
        assert np.array_equal(s.out[0].cpu().numpy(), want)



@pytest.mark.parametrize("max_bypass", [0, 1, 4])
def test_admission_bypass_with_aging(max_bypass):
    """A queued query whose memory does not fit yet is passed by later
    queries that fit at most max_bypass times (0: strict arrival order);
    every result still equals the oracle."""
    G = 3000
    sizes = [2_000_000, 4_000_000, 20_000, 20_000]  # A runs; B does not fit beside it; C and D do
    pool = WL.decimal_columns(max(sizes), 6, salt=7)
    pool_t = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in pool]
    host, specs = [], []
    for q, n in enumerate(sizes):
        keys = WL.served_keys(n, G, q, salt=7)
        host.append(keys)
        specs.append(api.QuerySpec(torch.from_numpy(keys).cuda(), [c[:n] for c in pool_t], G, WL.SERVED_AGGS, L=2))
    probe = api.Server(1 << 32, slots=4, chunk_rows=300_000)
    need = [probe.query_bytes(s) for s in specs]
    probe.close()
    # B alone fits the arena, and so do A, C and D together, but not A and B
    arena = max(need[1], sum(need[i] // 256 * 256 + 512 for i in (0, 2, 3))) // 256 * 256 + 512
    assert need[1] <= arena < need[0] + need[1]
    srv = api.Server(arena, slots=4, chunk_rows=300_000, max_bypass=max_bypass)
    try:
        for s in specs:
            srv.submit(s)
        _, nq, nr = srv.poll()
        # strict: A only; one bypass: A and C (B aged, D waits); more: A, C and D
        want_running = {0: 1, 1: 2, 4: 3}[max_bypass]
        assert (nr, nq) == (want_running, 4 - want_running), (nr, nq)
        seen = 0
        t0 = time.time()
        while seen < 4:
            done, nq, nr = srv.poll()
            seen += len(done)
            assert time.time() - t0 < 120, "server did not finish"
        torch.cuda.synchronize()
    finally:
        srv.close()
    for s, keys, n in zip(specs, host, sizes):
        for o, r in zip(s.out, oracle_sums(pool, keys, 0, n, G)):
            assert np.array_equal(o.cpu().numpy(), r)


def test_full_served_workload_sampled_against_oracle():
    """The full served workload (128 queries, rows log-uniform 1e4..5e7,
    groups 4..2^20, 4 aggregates over 6 decimal-like columns) in the launch
    configuration the serving benchmark times (4 slots, bypass bound 8,
    64M-row chunks, a 24 GiB arena, every query submitted at once).  The
    oracle checks a seeded sample of the queries, the largest always among
    them, bit for bit."""
    import os
    Q = 128
    rows, groups, _ = WL.served_queries(Q)
    n_max = int(rows.max())
    pool = WL.decimal_columns(n_max, 6)
    pool_t = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in pool]
    rng = np.random.default_rng(7)
    offs = [int(rng.integers(0, n_max - int(n) + 1)) for n in rows]
    say(f"case full served workload: {Q} queries, {int(rows.sum())} rows, largest {n_max}")
    specs = []
    for q, (n, G) in enumerate(zip(rows, groups)):
        keys = torch.from_numpy(WL.served_keys(int(n), int(G), q)).cuda()
        specs.append(api.QuerySpec(keys, [c[offs[q]:offs[q] + int(n)] for c in pool_t], int(G), WL.SERVED_AGGS, L=2))
    srv = api.Server(24 << 30, slots=4, max_bypass=8, chunk_rows=64 << 20)
    try:
        for s in specs:
            srv.submit(s)
        done = set()
        t0 = time.monotonic()
        while len(done) < Q:
            comp, _, _ = srv.poll()
            done.update(t for t, _ in comp)
            assert time.monotonic() - t0 < 60.0, "server did not finish"
        torch.cuda.synchronize()
    finally:
        srv.close()
    sample = sorted({int(np.argmax(rows))} | set(np.random.default_rng(11).choice(Q, 7, replace=False).tolist()))
    threads = max(1, min(16, os.cpu_count() or 1))
    for q in sample:
        n, G = int(rows[q]), int(groups[q])
        say(f"oracle: query {q}, {n} rows, {G} groups")
        keys = WL.served_keys(n, G, q)
        cols = [c[offs[q]:offs[q] + n] for c in pool]
        for k, (a, b) in enumerate(WL.SERVED_AGGS):
            v = cols[a] if b is None else cols[a] * cols[b]  # one IEEE rounding, as on the device
            st, status = O.groupby_sum(keys, v, G, 2, True, threads=threads)
            assert status == 0
            ref = O.finalize(st, G, 2)
            got = specs[q].out[k].cpu().numpy()
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), f"query {q} aggregate {k} differs"
