"""Bit-exact parity of the HIP library with the CPU oracle (needs a GPU).

Every comparison is on whole state buffers (canonical S and C bits) and on
finalised sums, element by element, with tolerance 0: the method is exact,
so any difference is a bug.  Inputs are seeded and synthetic (see
paper_1802_09883_amd.workloads).
"""
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


def TT(T64):
    return torch.float64 if T64 else torch.float32


def gpu_groupby(keys, vals, G, L, T64=True, states=None, keys_t=None, vals_t=None):
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = api.groupby_sum(dev(keys) if keys_t is None else keys_t, dev(vals) if vals_t is None else vals_t, G, L,
                         TT(T64), states=states, status=status)
    torch.cuda.synchronize()
    return st, int(status.item())


def assert_same_states(gpu_st, orc_st, G, L, T64, what=""):
    a = gpu_st.cpu().numpy()
    Sg, Cg = O.split_states(a, G, L, T64)
    So, Co = O.split_states(orc_st, G, L, T64)
    if np.array_equal(Sg.view(np.uint8), So.view(np.uint8)) and np.array_equal(Cg, Co):
        return
    bad = np.nonzero(np.any((Sg != So) | (Cg != Co), axis=0))[0]
    g = int(bad[0])
    raise AssertionError(f"{what}: {len(bad)} groups differ, first g={g}: gpu S={Sg[:, g]!r} C={Cg[:, g]!r} "
                         f"oracle S={So[:, g]!r} C={Co[:, g]!r}")


def check_case(keys, vals, G, L, T64=True, what=""):
    say(f"case {what}: n={len(keys)} G={G} L={L} T64={T64} kt={keys.dtype} vt={vals.dtype}")
    orc, ost = O.groupby_sum(keys, vals, G, L, T64, threads=8)
    st, status = gpu_groupby(keys, vals, G, L, T64)
    assert status == ost, f"{what}: status {status} vs oracle {ost}"
    assert_same_states(st, orc, G, L, T64, what)
    out = api.finalize(st, G, L, TT(T64))
    torch.cuda.synchronize()
    ref = O.finalize(orc, G, L, T64)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), ref.view(np.uint8)), f"{what}: finalize differs"
    return st


# ------------------------------------------------------------ configs

def test_plain_config_full():
    keys, vals = WL.plain()
    check_case(keys, vals, 16, 2, True, "plain 1M x 16 groups, repro<double,2>")


def test_lowcard_config_reduced():
    keys, v64, v32 = WL.lowcard(n=3_000_001)
    check_case(keys, v64, 1024, 3, True, "lowcard f64, repro<double,3>")
    check_case(keys, v32, 1024, 3, True, "lowcard f32 -> repro<double,3>")


def test_lowcard_config_full():
    keys, v64, v32 = WL.lowcard()
    kt = dev(keys)
    for name, vals in (("f64", v64), ("f32", v32)):
        say(f"case lowcard full {name}")
        orc, ost = O.groupby_sum(keys, vals, 1024, 3, True, threads=16)
        st, status = gpu_groupby(keys, vals, 1024, 3, True, keys_t=kt)
        assert status == ost == 0
        assert_same_states(st, orc, 1024, 3, True, f"lowcard full {name}")
        out = api.finalize(st, 1024, 3).cpu().numpy()
        assert np.array_equal(out, O.finalize(orc, 1024, 3))


def test_float_config_full():
    """The float-accumulator workload at its full size: 200M f32 values
    (exponents 2^U(-60,60), exact cancellation pairs) over 1024 groups into
    repro<float,2>, in the launch the benchmark times."""
    keys, _, v32 = WL.lowcard()
    say("case float full: 2e8 rows, 1024 groups, repro<float,2>")
    orc, ost = O.groupby_sum(keys, v32, 1024, 2, False, threads=16)
    st, status = gpu_groupby(keys, v32, 1024, 2, False)
    assert status == ost == 0
    assert_same_states(st, orc, 1024, 2, False, "float full")
    out = api.finalize(st, 1024, 2, TT(False)).cpu().numpy()
    ref = O.finalize(orc, 1024, 2, False)
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))


# ------------------------------------------------------- shapes, types

@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("kdt", [np.int32, np.int64])
@pytest.mark.parametrize("n", [1, 5, 2047, 2048, 2049, 100_003])
def test_shapes_and_levels(L, kdt, n):
    rng = np.random.default_rng([L, n, np.dtype(kdt).itemsize])
    G = int(rng.choice([1, 7, 16, 100, 1024]))
    keys = rng.integers(0, G, n).astype(kdt)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-200, 200, n))
    check_case(keys, vals, G, L, True, "shapes f64")
    check_case(keys, vals.astype(np.float32), G, L, False, "shapes f32 acc")


# largest group count whose bins fit one workgroup's LDS: (G + 1) * (8L + 12)
# bytes within 150 KiB; one more group takes the partitioned path
LDS_MAX_G = {1: 7679, 2: 5484, 3: 4265, 4: 3489}


@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("extra", [0, 1])
def test_largest_lds_group_count(L, extra):
    G = LDS_MAX_G[L] + extra
    rng = np.random.default_rng([L, extra])
    n = 300_000
    keys = rng.integers(0, G, n).astype(np.int32)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-40, 40, n))
    check_case(keys, vals, G, L, True, "largest LDS G" if extra == 0 else "one group beyond LDS")


@pytest.mark.parametrize("G,tiles", [(4096, 256), (4097, 256), (1024, 65), (1025, 8), (16, 256)])
def test_merge_launch_limits(G, tiles):
    """Few partials (partials x groups <= 2^20: one workgroup per tile here)
    are merged by one launch, more by two; around that limit, and resumed
    from a state whose tops are above the new rows'."""
    rng = np.random.default_rng([G, tiles])
    n = tiles * 8192
    keys = rng.integers(0, G, n).astype(np.int32)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-100, 100, n))
    check_case(keys, vals, G, 2, True, f"merge launch limits G={G} tiles={tiles}")
    big = np.ldexp(rng.standard_normal(G), rng.integers(300, 400, G))
    orc, _ = O.groupby_sum(np.concatenate([np.arange(G, dtype=np.int32), keys]), np.concatenate([big, vals]), G, 2)
    st, _ = gpu_groupby(np.arange(G, dtype=np.int32), big, G, 2)
    st, status = gpu_groupby(keys, vals, G, 2, states=st)
    assert status == 0
    assert_same_states(st, orc, G, 2, True, "resumed from higher tops")


def test_misaligned_columns_take_scalar_loads():
    keys, vals = WL.plain(n=50_001, salt=3)
    kt, vt = dev(keys), dev(vals)
    st, status = gpu_groupby(None, None, 16, 2, keys_t=kt[1:], vals_t=vt[1:])
    orc, _ = O.groupby_sum(keys[1:], vals[1:], 16, 2)
    assert status == 0
    assert_same_states(st, orc, 16, 2, True, "misaligned")


def test_extreme_values():
    rng = np.random.default_rng(77)
    n = 200_000
    parts = [
        np.ldexp(rng.standard_normal(n // 5), rng.integers(-1074, -1000, n // 5)),  # subnormal / tiny
        np.ldexp(rng.standard_normal(n // 5), rng.integers(900, 1004, n // 5)),     # near the domain edge
        np.ldexp(np.ones(n // 5), rng.integers(-1074, 1004, n // 5)),               # powers of two
        np.zeros(n // 10), -np.zeros(n // 10),
        np.ldexp(rng.integers(-(2 ** 39), 2 ** 39, n // 5).astype(np.float64) + 0.5, -10),  # halves: ties
    ]
    vals = np.concatenate(parts)
    keys = rng.integers(0, 9, len(vals)).astype(np.int32)
    for L in (1, 2, 3, 4):
        check_case(keys, vals, 9, L, True, "extreme f64")
    v32 = np.concatenate([np.ldexp(rng.standard_normal(n), rng.integers(-149, 119, n)).astype(np.float32),
                          np.zeros(1000, np.float32)])
    k32 = rng.integers(0, 5, len(v32)).astype(np.int32)
    for L in (1, 2, 3, 4):
        check_case(k32, v32, 5, L, False, "extreme f32 acc")
        check_case(k32, v32, 5, L, True, "extreme f32 -> double")


def test_single_group_many_rows_carry():
    """Carry stress: one group, large units at every level, many workgroups."""
    rng = np.random.default_rng(5)
    n = 6_000_000
    vals = np.ldexp(1.0 + rng.random(n), 40)  # all near one binade: units near 2^39
    keys = np.zeros(n, np.int32)
    check_case(keys, vals, 1, 3, True, "carry stress")
    check_case(keys, -vals, 1, 2, True, "carry stress negative")


def test_error_rows_status_and_skip():
    keys = np.array([0, 1, 5, -1, 1, 0, 2, 3] * 1000, np.int32)
    vals = np.array([1.5, 2.0, 3.0, 4.0, np.nan, np.inf, 2.0 ** 1005, -np.inf] * 1000)
    st = check_case(keys, vals, 4, 2, True, "error rows")
    v32 = np.array([1.0, 2.0 ** 121, np.nan, 3.0] * 100, np.float32)
    k32 = np.array([0, 0, 1, 7] * 100, np.int32)
    check_case(k32, v32, 2, 2, False, "error rows f32")


@pytest.mark.parametrize("G", [4, 1000, 5484, 5485, 300_000])
@pytest.mark.parametrize("T64", [True, False])
def test_bad_key_rows_carry_their_value_status(G, T64):
    """The only non-finite and out-of-domain values sit on rows whose keys are
    out of range: the status word still holds KEY | NONFINITE | RANGE, as the
    oracle classifies every row's value whatever its key, on the LDS path
    (G up to 5484 at L = 2) and on the partitioned path (above)."""
    rng = np.random.default_rng([61, G, T64])
    n = 200_003
    keys = rng.integers(0, G, n).astype(np.int64)
    big = 2.0 ** 1006 if T64 else 2.0 ** 121
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-60, 60, n))
    bad = rng.choice(n, 60, replace=False)
    keys[bad[:20]] = G + 7
    keys[bad[20:40]] = -3
    keys[bad[40:]] = G
    vals[bad[:10]] = np.nan
    vals[bad[10:20]] = np.inf
    vals[bad[20:30]] = -big
    vals[bad[30:40]] = big
    vals = vals if T64 else vals.astype(np.float32)
    st = check_case(keys, vals, G, 2, T64, f"bad-key rows only (G={G})")
    orc_status = O.groupby_sum(keys, vals, G, 2, T64)[1]
    assert orc_status == 7, orc_status  # KEY | NONFINITE | RANGE
    # only a bad key: KEY alone
    k2 = keys.copy()
    v2 = np.where(np.isfinite(vals) & (np.abs(vals) < big), vals, 1.0).astype(vals.dtype)
    check_case(k2, v2, G, 2, T64, f"bad keys, finite values (G={G})")
    del st


def test_bad_key_rows_status_other_paths():
    """The same rows through the multi-column call, a batch and the
    ungrouped sum (whose rows have no key: value bits only)."""
    rng = np.random.default_rng(62)
    n, G = 100_000, 1024
    keys = rng.integers(0, G, n).astype(np.int32)
    v = np.ldexp(rng.standard_normal(n), rng.integers(-30, 30, n))
    keys[[5, 6, 7]] = G + 1
    v[5], v[6], v[7] = np.nan, 2.0 ** 1006, -np.inf
    want = O.groupby_sum(keys, v, G, 3)[1]
    assert want == 7
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    api.groupby_sum_cols(dev(keys), [dev(v), dev(v.astype(np.float32))], G, 3, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 7 | O.groupby_sum(keys, v.astype(np.float32), G, 3)[1]
    status.zero_()
    st = torch.empty(api.state_bytes(G, 3), dtype=torch.uint8, device="cuda")
    api.batch_groupby_sum([api.Job(dev(keys), dev(v), G, 3, st)], status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == want
    status.zero_()
    api.sum(dev(v), 3, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == O.groupby_sum(np.zeros(n, np.int32), v, 1, 3)[1] == 6


# ------------------------------------------- schedule / resume / merge

def test_chunked_calls_and_host_roundtrip_resume():
    keys, v64, _ = WL.lowcard(n=1_000_000, salt=9, with_f32=False)
    orc, _ = O.groupby_sum(keys, v64, 1024, 3)
    st = api.state_init(1024, 3)
    cuts = [0, 1, 999, 2048 * 7 + 3, 400_000, 1_000_000]
    kt, vt = dev(keys), dev(v64)
    for i, (b, e) in enumerate(zip(cuts[:-1], cuts[1:])):
        st = api.groupby_sum(kt[b:e], vt[b:e], 1024, 3, states=st)
        if i == 2:  # checkpoint to host and restore
            torch.cuda.synchronize()
            st = torch.from_numpy(st.cpu().numpy().copy()).cuda()
    torch.cuda.synchronize()
    assert_same_states(st, orc, 1024, 3, True, "chunked resume")


def test_permutation_invariance_on_gpu():
    keys, v64, _ = WL.lowcard(n=500_000, salt=4, with_f32=False)
    a, _ = gpu_groupby(keys, v64, 1024, 3)
    p = np.random.default_rng(1).permutation(len(keys))
    b, _ = gpu_groupby(keys[p], v64[p], 1024, 3)
    assert torch.equal(a, b)


@pytest.mark.parametrize("T64", [True, False])
def test_merge_and_finalize_match_oracle(T64):
    rng = np.random.default_rng([3, T64])
    G = 333
    for L in (1, 2, 3, 4):
        ka = rng.integers(0, G, 50_000).astype(np.int64)
        kb = rng.integers(0, G, 70_000).astype(np.int64)
        span = (-1000, 1000) if T64 else (-140, 110)
        va = np.ldexp(rng.standard_normal(50_000), rng.integers(*span, 50_000))
        vb = np.ldexp(rng.standard_normal(70_000), rng.integers(*span, 70_000))
        if not T64:
            va, vb = va.astype(np.float32), vb.astype(np.float32)
        oa, _ = O.groupby_sum(ka, va, G, L, T64)
        ob, _ = O.groupby_sum(kb, vb, G, L, T64)
        ga, gb = dev(oa), dev(ob)
        api.merge(ga, gb, G, L, TT(T64))
        torch.cuda.synchronize()
        assert_same_states(ga, O.merge(oa, ob, G, L, T64), G, L, T64, "merge")
        out = api.finalize(dev(oa), G, L, TT(T64)).cpu().numpy()
        assert np.array_equal(out.view(np.uint8), O.finalize(oa, G, L, T64).view(np.uint8))


def test_state_init_and_empty_input():
    for T64 in (True, False):
        for L in (1, 2, 3, 4):
            st = api.state_init(37, L, TT(T64))
            torch.cuda.synchronize()
            assert np.array_equal(st.cpu().numpy(), O.state_init(37, T64, L))
            before = st.clone()
            api.groupby_sum(torch.zeros(0, dtype=torch.int32, device="cuda"),
                            torch.zeros(0, dtype=TT(T64), device="cuda"), 37, L, TT(T64), states=st)
            torch.cuda.synchronize()
            assert torch.equal(st, before)
            out = api.finalize(st, 37, L, TT(T64)).cpu().numpy()
            assert np.all(out == 0) and not np.any(np.signbit(out))


def test_invalid_arguments_are_rejected():
    k = torch.zeros(4, dtype=torch.int32, device="cuda")
    v = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        api.groupby_sum(k, v, 4, 2, torch.float32)  # f64 values into float states
    with pytest.raises(ValueError):
        api.groupby_sum(k, v, 4, 5)  # L out of range
    with pytest.raises(ValueError):
        api.groupby_sum(k, v, 0, 2)  # no groups


def test_plain_baseline_close_to_exact():
    keys, vals = WL.plain(n=200_000, salt=2)
    out = api.plain_groupby_sum(dev(keys), dev(vals), 16).cpu().numpy()
    orc, _ = O.groupby_sum(keys, vals, 16, 3)
    ref = O.finalize(orc, 16, 3)
    scale = np.array([np.abs(vals[keys == g]).sum() for g in range(16)])
    assert np.all(np.abs(out - ref) <= 1e-12 * scale)


@pytest.mark.parametrize("G,kdt", [(100_003, np.int32), (1 << 22, np.int64)])
def test_partitioned_plain_baseline_close_to_exact(G, kdt):
    """The baseline for groups beyond LDS partitions first (the same
    algorithm on doubles); its sums are within rounding of the exact ones,
    bad keys and NaN rows are skipped and reported."""
    rng = np.random.default_rng([G, 7])
    n = 1_500_000
    keys = rng.integers(-2, G + 2, n).astype(kdt)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-30, 30, n))
    vals[rng.random(n) < 1e-4] = np.nan
    need = api._lib.load().repro_plain_workspace_bytes(n, G, 0 if kdt == np.int32 else 1, 1)
    assert need > 0  # the partitioned baseline, not global atomics
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = api.plain_groupby_sum(dev(keys), dev(vals), G, status=status).cpu().numpy()
    torch.cuda.synchronize()
    orc, ost = O.groupby_sum(keys, vals, G, 3)
    assert int(status.item()) == ost == (1 | 2)
    ref = O.finalize(orc, G, 3)
    ok = (keys >= 0) & (keys < G) & np.isfinite(vals)
    scale = np.bincount(keys[ok].astype(np.int64), weights=np.abs(vals[ok]), minlength=G)
    assert np.all(np.abs(out - ref) <= 1e-12 * scale)


@pytest.mark.parametrize("G,L", [(16, 2), (1024, 3), (300, 4)])
def test_tops_rising_late_use_spill_path(G, L):
    """Magnitudes grow along the rows (tops keep rising inside every
    workgroup's chunk) and a few huge values arrive late: rows above their
    group's frozen top go through the spill array; bits must not change."""
    rng = np.random.default_rng([G, L])
    n = 3_000_000
    e = (-900 + (np.arange(n) * 1800) // n).astype(np.int64)  # rising exponents
    vals = np.ldexp(rng.standard_normal(n), e + rng.integers(-3, 4, n))
    late = rng.choice(n, 200, replace=False)
    vals[late] = np.ldexp(rng.standard_normal(200), rng.integers(950, 1000, 200))
    keys = rng.integers(0, G, n).astype(np.int32)
    check_case(keys, vals, G, L, True, "rising tops f64")
    with np.errstate(over="ignore"):  # values beyond float's range become +-Inf: skipped rows
        v_narrow = vals.astype(np.float32)
    check_case(keys, v_narrow, G, L, True, "rising tops f32 -> double")
    v32 = np.ldexp(rng.standard_normal(n), (-140 + (np.arange(n) * 250) // n)).astype(np.float32)
    check_case(keys, v32, G, L, False, "rising tops float acc")


# ------------------------------------------------ high cardinality (partitioned)

def test_highcard_config_reduced():
    keys, vals = WL.highcard(n=2_000_000, salt=1)
    check_case(keys, vals, 1 << 22, 2, True, "highcard reduced: Zipf int64 keys, 2^22 groups")


def test_highcard_config_full():
    keys, vals = WL.highcard()
    say("case highcard full: 1e8 rows, 2^22 groups, repro<double,2>")
    orc, ost = O.groupby_sum(keys, vals, 1 << 22, 2, True, threads=16)
    st, status = gpu_groupby(keys, vals, 1 << 22, 2, True)
    assert status == ost == 0
    assert_same_states(st, orc, 1 << 22, 2, True, "highcard full")
    out = api.finalize(st, 1 << 22, 2).cpu().numpy()
    assert np.array_equal(out, O.finalize(orc, 1 << 22, 2))


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_partitioned_uniform_keys_all_levels(L):
    rng = np.random.default_rng([21, L])
    G, n = 100_003, 1_500_000
    keys = rng.integers(0, G, n).astype(np.int32)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-300, 300, n))
    check_case(keys, vals, G, L, True, "partitioned f64")
    v32 = np.ldexp(rng.standard_normal(n), rng.integers(-60, 60, n)).astype(np.float32)
    check_case(keys, v32, G, L, False, "partitioned float acc")
    # f32 values widened into double accumulators: two atomics per row
    w32 = np.ldexp(rng.standard_normal(n), rng.integers(-149, 128, n)).astype(np.float32)
    w32[~np.isfinite(w32)] = 1.5
    check_case(keys, w32, G, L, True, "partitioned f32 -> double")


def test_partitioned_error_rows_and_resume():
    rng = np.random.default_rng(33)
    G, n = 300_000, 400_000
    keys = rng.integers(-5, G + 5, n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-1000, 1010, n))
    vals[rng.random(n) < 0.001] = np.nan
    check_case(keys, vals, G, 3, True, "partitioned error rows")
    # resume: two calls with a host round trip equal one call
    orc, _ = O.groupby_sum(keys, vals, G, 3)
    kt, vt = dev(keys), dev(vals)
    st = api.groupby_sum(kt[:123_457], vt[:123_457], G, 3)
    torch.cuda.synchronize()
    st = torch.from_numpy(st.cpu().numpy().copy()).cuda()
    st = api.groupby_sum(kt[123_457:], vt[123_457:], G, 3, states=st)
    torch.cuda.synchronize()
    assert_same_states(st, orc, G, 3, True, "partitioned resume")


def test_mid_cardinality_lds_path_large_lds():
    """Groups between the 64 KiB and 150 KiB LDS budgets stay on the LDS path."""
    rng = np.random.default_rng(44)
    for G, L in ((3000, 3), (5000, 2), (6000, 1)):
        n = 1_000_000
        keys = rng.integers(0, G, n).astype(np.int32)
        vals = np.ldexp(rng.standard_normal(n), rng.integers(-80, 80, n))
        check_case(keys, vals, G, L, True, "mid cardinality")


@pytest.mark.parametrize("L,G", [(2, (1 << 24) + 1000), (4, (1 << 23) + 5), (1, (1 << 26) + 3)])
def test_two_partitioning_levels(L, G):
    """More groups than one partitioning level holds: a first scatter into
    super-partitions, then the one-level path per super-partition; bad keys
    and non-finite values on the way, and a resumed second call."""
    rng = np.random.default_rng([L, G % 1000])
    n = 2_000_000
    keys = rng.integers(-3, G + 3, n).astype(np.int64)
    keys[: n // 4] = rng.integers(G - 2000, G, n // 4)  # the last, small super-partition gets rows too
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-200, 200, n))
    vals[rng.random(n) < 1e-4] = np.nan
    check_case(keys, vals, G, L, True, f"two partitioning levels G={G} L={L}")
    orc, _ = O.groupby_sum(keys, vals, G, L)
    st = api.groupby_sum(dev(keys[:700_001]), dev(vals[:700_001]), G, L)
    st = api.groupby_sum(dev(keys[700_001:]), dev(vals[700_001:]), G, L, states=st)
    torch.cuda.synchronize()
    assert_same_states(st, orc, G, L, True, "two levels, resumed")


def test_partitioned_multi_tile_slabs_over_several_rounds():
    """About 2000 partitions: the partition passes take slabs of two tiles,
    and with 10M rows the scatter workgroups go through several rounds, so
    rows land by (round, XCD-major workgroup order) with multi-tile runs.
    Bad keys and NaN rows on the way."""
    rng = np.random.default_rng(57)
    G, n = 8_000_000, 10_000_000
    keys = rng.integers(-2, G + 2, n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-100, 100, n))
    vals[rng.random(n) < 1e-5] = np.nan
    say(f"case multi-tile slabs: n={n}, G={G}, L=2")
    check_case(keys, vals, G, 2, True, "multi-tile slabs, several rounds")


def test_partitioned_many_partitions_small_tiles():
    """Thousands of partitions (the scatter falls back to 4096-row tiles)."""
    rng = np.random.default_rng(55)
    G, n = 7_000_000, 1_000_000
    keys = rng.integers(0, G, n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-100, 100, n))
    check_case(keys, vals, G, 4, True, "7M groups, L=4")
