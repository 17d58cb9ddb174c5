"""Batched GroupBy-SUM (many independent jobs in one persistent launch):
bit-exact parity of every job with the CPU oracle, independence of the
configuration and schedule, graph capture and the autotuner (needs a GPU)."""
import sys

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed_jobs(seed, count, max_rows=400_000, max_groups=70_000, errors=True):
    """Jobs of uneven sizes: rows log-uniform (some empty), groups log-uniform
    (several beyond one workgroup's LDS, so cut into group slices), L 1..4."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = 0 if j % 11 == 3 else int(np.exp(rng.uniform(np.log(50), np.log(max_rows))))
        G = int(np.exp(rng.uniform(0, np.log(max_groups))))
        L = int(rng.integers(1, 5))
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = np.ldexp(rng.standard_normal(n), rng.integers(-30, 31, n))
        if errors and j % 7 == 5 and n > 10:
            keys[::97] = G + 3
            vals[5] = np.nan
        out.append((keys, vals, G, L))
    return out


def oracle_job(keys, vals, G, L, prior=None):
    st, status = O.groupby_sum(keys, vals, G, L, True, threads=8)
    if prior is not None:
        st = O.merge(prior, st, G, L, True)
    return st, status


def make_batch(specs, accumulate=None, with_out=True):
    jobs, priors = [], []
    for i, (keys, vals, G, L) in enumerate(specs):
        acc = bool(accumulate and accumulate(i))
        prior = None
        if acc:
            # earlier rows of this group set, already in the states
            rng = np.random.default_rng(1000 + i)
            pk = rng.integers(0, G, 3000).astype(np.int32)
            pv = np.ldexp(rng.standard_normal(3000), rng.integers(-60, 61, 3000))
            st = api.groupby_sum(dev(pk), dev(pv), G, L)
            prior = O.groupby_sum(pk, pv, G, L)[0]
        else:
            st = torch.full((api.state_bytes(G, L),), 0xAB, dtype=torch.uint8, device="cuda")  # overwritten
        out = torch.full((G,), float("nan"), dtype=torch.float64, device="cuda") if with_out else None
        jobs.append(api.Job(dev(keys), dev(vals), G, L, st, out, accumulate=acc))
        priors.append(prior)
    return jobs, priors


def check_jobs(jobs, specs, priors, status, what):
    want_status = 0
    for i, (job, (keys, vals, G, L), prior) in enumerate(zip(jobs, specs, priors)):
        ref, st = oracle_job(keys, vals, G, L, prior)
        want_status |= st
        got = job.states.cpu().numpy()
        Sg, Cg = O.split_states(got, G, L, True)
        So, Co = O.split_states(ref, G, L, True)
        assert np.array_equal(Sg.view(np.uint8), So.view(np.uint8)) and np.array_equal(Cg, Co), \
            f"{what}: job {i} (n={len(keys)}, G={G}, L={L}) states differ from the oracle"
        if job.out is not None:
            assert np.array_equal(job.out.cpu().numpy().view(np.uint8), O.finalize(ref, G, L).view(np.uint8)), \
                f"{what}: job {i} finalised sums differ"
    assert status == want_status, f"{what}: status {status} vs oracle {want_status}"


@pytest.mark.parametrize("config", [None, {"merge": 1, "chunk_rows": 65536}])
def test_batch_matches_oracle_per_job(config):
    specs = mixed_jobs(1, 40)
    say(f"case batch of {len(specs)} mixed jobs, {sum(len(s[0]) for s in specs)} rows, config {config}")
    jobs, priors = make_batch(specs, accumulate=lambda i: i % 3 == 1)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    api.batch_groupby_sum(jobs, config=config, status=status)
    torch.cuda.synchronize()
    check_jobs(jobs, specs, priors, int(status.item()), "mixed batch")


@pytest.mark.parametrize("config", [
    {"chunk_rows": 8192}, {"chunk_rows": 1 << 20}, {"max_slice_groups": 300}, {"order": 1},
    {"chunk_rows": 16384, "max_slice_groups": 1000, "order": 1}, {"merge": 1}, {"chunk_rows": 8192, "merge": 1},
    {"chunk_rows": 16384, "max_slice_groups": 300, "order": 1, "merge": 1},
    {"split": 1}, {"split": 1, "chunk_rows": 8192, "merge": 1}, {"split": 1, "max_slice_groups": 300, "order": 1}])
def test_batch_configuration_does_not_change_bits(config):
    specs = mixed_jobs(2, 24, max_rows=200_000, errors=False)
    say(f"case batch config {config}")
    jobs, priors = make_batch(specs)
    run = api.batch_groupby_sum(jobs, config=config)
    torch.cuda.synchronize()
    check_jobs(jobs, specs, priors, 0, f"config {config}")
    # launching the same plan again (overwrite mode) gives the same bits
    before = [j.states.clone() for j in jobs]
    api.batch_launch(run)
    torch.cuda.synchronize()
    for a, j in zip(before, jobs):
        assert torch.equal(a, j.states)


@pytest.mark.parametrize("split,merge", [(0, 0), (0, 1), (1, 0)])
def test_batch_sorted_slices_status_and_edges(split, merge):
    """Jobs beyond one workgroup's LDS, run with their chunks sorted by group
    slice (split 0) or read once per slice (split 1): status bits when the
    only NaN, Inf and out-of-domain values sit on rows with invalid keys,
    and separately on rows with valid keys; a job whose rows all fall in
    one slice; the last slice shorter than the others; several chunks.
    States, sums and status equal the oracle's."""
    rng = np.random.default_rng([11, split, merge])
    specs = []
    G = 20_000
    # only the bad-key rows hold unusable values: KEY | NONFINITE | RANGE
    n = 70_000
    keys = rng.integers(0, G, n).astype(np.int32)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-30, 31, n))
    keys[[7, 900, 50_000]] = [G, -1, G + 99]
    vals[[7, 900, 50_000]] = [np.nan, np.inf, 1.7e308]
    specs.append((keys, vals, G, 2))
    # valid keys with NaN / -Inf values: NONFINITE only
    keys2 = rng.integers(0, 9_000, 40_000).astype(np.int32)
    vals2 = rng.standard_normal(40_000)
    vals2[[3, 30_001]] = [np.nan, -np.inf]
    specs.append((keys2, vals2, 9_000, 3))
    # every row in the last slice, which is shorter than the others
    G3 = 3 * 4096 + 5
    keys3 = rng.integers(3 * 4096, G3, 30_000).astype(np.int32)
    specs.append((keys3, np.ldexp(rng.standard_normal(30_000), rng.integers(-60, 61, 30_000)), G3, 1))
    # many slices, many chunks, cancelling pairs
    G4 = 60_000
    half = rng.standard_normal(100_000) * 2.0 ** 40
    keys4 = np.concatenate([rng.integers(0, G4, 100_000)] * 2).astype(np.int32)
    specs.append((keys4, np.concatenate([half, -half]), G4, 4))
    # no rows at all
    specs.append((np.zeros(0, np.int32), np.zeros(0), 30_000, 2))
    jobs, priors = make_batch(specs, accumulate=lambda i: i == 1)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    config = {"split": split, "merge": merge, "chunk_rows": 16384}
    say(f"case sorted slices {config}")
    api.batch_groupby_sum(jobs, config=config, status=status)
    torch.cuda.synchronize()
    check_jobs(jobs, specs, priors, int(status.item()), f"sorted slices {config}")
    assert int(status.item()) == 7  # KEY | NONFINITE | RANGE
    # the status word of the first job alone, against the oracle's
    status.zero_()
    only, _ = make_batch(specs[:1])
    api.batch_groupby_sum(only, config=config, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == O.groupby_sum(*specs[0])[1] == 7


def test_batch_accumulating_launches_add_the_batch_each_time():
    specs = mixed_jobs(3, 10, max_rows=50_000, errors=False)
    jobs, _ = make_batch(specs, with_out=False)
    for j in jobs:
        j.states = api.state_init(j.num_groups, j.L)
        j.accumulate = True
    run = api.batch_prepare(jobs)
    api.batch_launch(run)
    api.batch_launch(run)
    torch.cuda.synchronize()
    for j, (keys, vals, G, L) in zip(jobs, specs):
        ref, _ = O.groupby_sum(np.concatenate([keys, keys]), np.concatenate([vals, vals]), G, L)
        assert np.array_equal(j.states.cpu().numpy(), ref)


def test_batch_graph_capture_and_replay():
    specs = mixed_jobs(4, 16, max_rows=100_000, errors=False)
    jobs, priors = make_batch(specs)
    run = api.batch_prepare(jobs)
    api.batch_launch(run)
    torch.cuda.synchronize()
    eager = [j.states.clone() for j in jobs]
    outs = [j.out.clone() for j in jobs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        api.batch_launch(run, stream=s)
    for rep in range(3):
        for j in jobs:  # eager work between replays: scribble over the results
            j.states.fill_(0x5A)
            j.out.fill_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, j in enumerate(jobs):
            assert torch.equal(j.states, eager[i]), f"replay {rep}: job {i} states differ from the eager launch"
            assert torch.equal(j.out, outs[i]), f"replay {rep}: job {i} sums differ"
    check_jobs(jobs, specs, priors, 0, "graph replay")


def test_batch_autotuner_result_is_bit_neutral():
    specs = mixed_jobs(5, 20, max_rows=300_000, errors=False)
    jobs, priors = make_batch(specs)
    best, ms = api.batch_tune(jobs)
    say(f"tuned config {best}, {ms:.3f} ms")
    assert ms > 0 and best["chunk_rows"] > 0 and best["order"] in (0, 1)
    for j in jobs:
        j.states.fill_(0)
    api.batch_groupby_sum(jobs, config=best)
    torch.cuda.synchronize()
    check_jobs(jobs, specs, priors, 0, "tuned config")


def test_batch_invalid_jobs_are_rejected():
    k = dev(np.zeros(10, np.int32))
    v = dev(np.zeros(10))
    st = api.state_init(4, 2)
    for bad in (dict(L=0), dict(L=5), dict(num_groups=0)):
        args = dict(keys=k, values=v, num_groups=4, L=2, states=st)
        args.update(bad)
        with pytest.raises(ValueError):
            api.batch_prepare([api.Job(**args)])
    with pytest.raises(ValueError):
        api.batch_prepare([api.Job(k, dev(np.zeros(10)), 4, 2, st)], T=torch.float32)  # f64 -> float narrows


def test_batch_full_size_512_jobs():
    """The batched workload at its full size (512 jobs, rows log-uniform
    1e3..1e7, groups log-uniform 1..2^16, L in {2, 3}): every job's states
    and finalised sums against the oracle, tolerance 0."""
    rows, groups, Ls = WL.batched_jobs()
    say(f"case full batch: {len(rows)} jobs, {int(rows.sum())} rows")
    specs = [(*WL.batched_job(int(r), int(g), j), int(g), int(l)) for j, (r, g, l) in enumerate(zip(rows, groups, Ls))]
    jobs, priors = make_batch(specs, with_out=True)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    api.batch_groupby_sum(jobs, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    want_status = 0
    for i, (job, (keys, vals, G, L)) in enumerate(zip(jobs, specs)):
        ref, st = O.groupby_sum(keys, vals, G, L, True, threads=16)
        want_status |= st
        Sg, Cg = O.split_states(job.states.cpu().numpy(), G, L, True)
        So, Co = O.split_states(ref, G, L, True)
        assert np.array_equal(Sg.view(np.uint8), So.view(np.uint8)) and np.array_equal(Cg, Co), \
            f"full batch: job {i} (n={len(keys)}, G={G}, L={L}) states differ from the oracle"
        assert np.array_equal(job.out.cpu().numpy().view(np.uint8), O.finalize(ref, G, L).view(np.uint8)), \
            f"full batch: job {i} finalised sums differ"
        if i % 64 == 63:
            say(f"  checked {i + 1} jobs")
    assert want_status == 0


def _headroom_values(n, L, sign):
    """Values whose units sit just below 2^(W-1) = 2^39 at every level they
    reach, all of one sign, in one group at top index 26 (E = 18, grid of the
    first level 2^-34): b = 32 - 2^-35 - 2^-48 has units 2^39 - 1 and
    2^39 - 2^26; b * 2^-40 has units 0, 2^39 - 1 and 2^39 - 2^26."""
    b = 32.0 - 2.0 ** -35 - 2.0 ** -48
    if L <= 2:
        v = np.full(n, b)
    else:
        v = np.empty(n)
        v[0::2], v[1::2] = b, b * 2.0 ** -40
    return sign * v


@pytest.mark.parametrize("L,sign", [(2, 1.0), (2, -1.0), (3, 1.0), (4, -1.0)])
def test_carry_headroom_one_item_of_2_23_rows(L, sign):
    """The tiling bound of Sec. III-D taken as at most 2^23 rows into one
    workgroup's int64 level words: one batch item of exactly 2^23 rows of one
    group whose units are all just below 2^39 and of one sign, so a level
    word reaches about 2^62.  States and sums match the oracle bit for bit."""
    n = 1 << 23
    vals = _headroom_values(n, L, sign)
    keys = np.zeros(n, np.int32)
    units = O.extract(float(abs(vals[0])), 26, L, 52, 40, -1022)
    assert units[0] == 2 ** 39 - 1 and units[1] == 2 ** 39 - 2 ** 26
    say(f"case headroom: {n} rows, one group, L={L}, sign {sign:+.0f}, one item")
    st = torch.empty(api.state_bytes(1, L), dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    run = api.batch_groupby_sum([api.Job(dev(keys), dev(vals), 1, L, st, out)], config={"chunk_rows": n},
                                status=status)
    torch.cuda.synchronize()
    assert run.plan.items == 1, "the job must run as one item of 2^23 rows"
    ref, rst = O.groupby_sum(keys, vals, 1, L, True, threads=8)
    assert int(status.item()) == rst == 0
    Sg, Cg = O.split_states(st.cpu().numpy(), 1, L, True)
    So, Co = O.split_states(ref, 1, L, True)
    assert np.array_equal(Sg.view(np.uint8), So.view(np.uint8)) and np.array_equal(Cg, Co)
    # the level sums did reach about 2^62 (C counts 2^50 units each)
    assert int(np.abs(Co).max()) >= (2 ** 61) >> 50
    assert out.cpu().numpy().view(np.uint64)[0] == O.finalize(ref, 1, L).view(np.uint64)[0]


@pytest.mark.parametrize("T64", [True, False])
def test_batch_int64_keys_float_values_and_unaligned_columns(T64):
    rng = np.random.default_rng([6, T64])
    specs, jobs = [], []
    for j in range(12):
        n = int(rng.integers(1, 150_000))
        G = int(np.exp(rng.uniform(0, np.log(20_000))))
        L = int(rng.integers(1, 5))
        keys = rng.integers(-2, G + 2, n + 1).astype(np.int64)  # a few bad keys
        vals = np.ldexp(rng.standard_normal(n + 1), rng.integers(-40, 40, n + 1)).astype(np.float32)
        kt, vt = dev(keys), dev(vals)
        if j % 2:  # start one row in: columns not 16-byte aligned, scalar loads
            kt, vt, keys, vals = kt[1:], vt[1:], keys[1:], vals[1:]
        else:
            kt, vt, keys, vals = kt[:n], vt[:n], keys[:n], vals[:n]
        T = torch.float64 if T64 else torch.float32
        st = torch.zeros(api.state_bytes(G, L, T), dtype=torch.uint8, device="cuda")
        jobs.append(api.Job(kt, vt, G, L, st, torch.empty(G, dtype=T, device="cuda")))
        specs.append((keys, vals, G, L))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    api.batch_groupby_sum(jobs, T=torch.float64 if T64 else torch.float32, status=status)
    torch.cuda.synchronize()
    want = 0
    for i, (job, (keys, vals, G, L)) in enumerate(zip(jobs, specs)):
        ref, st = O.groupby_sum(keys, vals, G, L, T64)
        want |= st
        Sg, Cg = O.split_states(job.states.cpu().numpy(), G, L, T64)
        So, Co = O.split_states(ref, G, L, T64)
        assert np.array_equal(Sg.view(np.uint8), So.view(np.uint8)) and np.array_equal(Cg, Co), f"job {i}"
        assert np.array_equal(job.out.cpu().numpy().view(np.uint8), O.finalize(ref, G, L, T64).view(np.uint8))
    assert int(status.item()) == want and want & 1
