"""Several SUM aggregates over one GROUP BY in one call (needs a GPU).

repro_groupby_sum_cols must give, for every column, the bits the CPU oracle
gives for that column alone (tolerance 0), on the fused one-pass kernel and
on every shape that runs column by column (T = float, groups beyond one
workgroup's LDS, unaligned columns).  Inputs are seeded and synthetic.
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


def same_bits(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def check_cols(keys, cols, G, L, T64=True, what="", keys_t=None, cols_t=None, threads=8):
    say(f"case {what}: n={len(keys)} G={G} L={L} T64={T64} kt={keys.dtype} "
        f"cols={[str(c.dtype) for c in cols]}")
    T = torch.float64 if T64 else torch.float32
    kt = dev(keys) if keys_t is None else keys_t
    ct = [dev(c) for c in cols] if cols_t is None else cols_t
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    states = api.groupby_sum_cols(kt, ct, G, L, T, status=status)
    outs = [api.finalize(st, G, L, T) for st in states]
    torch.cuda.synchronize()
    ost_all = 0
    for c, (col, st, out) in enumerate(zip(cols, states, outs)):
        orc, ost = O.groupby_sum(keys, col, G, L, T64, threads=threads)
        ost_all |= ost
        assert same_bits(st.cpu().numpy(), orc), f"{what}: column {c} states differ from the oracle"
        assert same_bits(out.cpu().numpy(), O.finalize(orc, G, L, T64)), f"{what}: column {c} sums differ"
    assert int(status.item()) == ost_all, f"{what}: status {int(status.item())} vs oracle {ost_all}"
    return states


def mixed_cols(n, ncols, seed, spread=60):
    rng = np.random.default_rng(seed)
    cols = []
    for c in range(ncols):
        v = np.ldexp(rng.standard_normal(n), rng.integers(-spread, spread + 1, n))
        cols.append(v.astype(np.float32) if c % 2 else v)
    return cols


def test_lowcard_two_columns_reduced():
    keys, v64, v32 = WL.lowcard(n=3_000_001, salt=4)
    check_cols(keys, [v64, v32], 1024, 3, True, "lowcard f64+f32 fused")


def test_lowcard_two_columns_full():
    keys, v64, v32 = WL.lowcard()
    check_cols(keys, [v64, v32], 1024, 3, True, "lowcard full f64+f32 fused", threads=16)


@pytest.mark.parametrize("ncols", [2, 3, 4])
@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("kdt", [np.int32, np.int64])
def test_fused_widths_levels_keys(ncols, L, kdt):
    n = 250_003  # several tiles per workgroup and a ragged tail
    rng = np.random.default_rng([ncols, L, np.dtype(kdt).itemsize])
    G = int(rng.choice([1, 16, 300]))
    keys = rng.integers(0, G, n).astype(kdt)
    check_cols(keys, mixed_cols(n, ncols, [ncols, L, 7]), G, L, True, f"{ncols} cols fused")


@pytest.mark.parametrize("mask", [0, 1, 2, 3])
def test_two_column_type_combinations(mask):
    """Every float/double combination of two fused columns (bit c of mask:
    column c is float32), with subnormal, non-finite and out-of-domain values
    and enough rows for the sampled seed tops and epoch mode."""
    n = 2_000_003
    rng = np.random.default_rng([mask, 5])
    G = 500
    keys = rng.integers(0, G, n).astype(np.int32)
    cols = []
    for c in range(2):
        if (mask >> c) & 1:
            v = np.ldexp(rng.standard_normal(n), rng.integers(-149, 120, n)).astype(np.float32)
            v[rng.random(n) < 1e-4] = np.inf
        else:
            v = np.ldexp(rng.standard_normal(n), rng.integers(-1074, 1010, n))
            v[rng.random(n) < 1e-4] = np.nan
        cols.append(v)
    check_cols(keys, cols, G, 3, True, f"two columns, float mask {mask}")


@pytest.mark.parametrize("n", [1, 7, 4095, 4096, 4097, 8193])
def test_fused_small_and_ragged(n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 100, n).astype(np.int32)
    check_cols(keys, mixed_cols(n, 2, [n]), 100, 2, True, "small fused")
    check_cols(keys, mixed_cols(n, 3, [n, 3]), 100, 3, True, "small fused x3")


def test_more_columns_than_one_pass():
    n = 120_001
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 64, n).astype(np.int32)
    check_cols(keys, mixed_cols(n, 7, [7]), 64, 2, True, "7 columns (4 + 3)")
    check_cols(keys, mixed_cols(n, 5, [5]), 64, 3, True, "5 columns (4 + 1)")


def test_groups_beyond_fused_lds_run_per_column():
    n = 200_000
    rng = np.random.default_rng(12)
    # two columns of 3000 groups at L = 3 do not fit one workgroup's LDS
    # together (each alone does); 9000 groups take the partitioned path
    for G in (3000, 9000):
        keys = rng.integers(0, G, n).astype(np.int32)
        check_cols(keys, mixed_cols(n, 2, [G]), G, 3, True, f"G={G} per column")


def test_float_accumulators_run_per_column():
    n = 100_001
    rng = np.random.default_rng(13)
    keys = rng.integers(0, 50, n).astype(np.int32)
    cols = [np.ldexp(rng.standard_normal(n), rng.integers(-20, 21, n)).astype(np.float32) for _ in range(3)]
    check_cols(keys, cols, 50, 2, False, "T=float per column")


def test_unaligned_columns_run_per_column():
    n = 60_001
    rng = np.random.default_rng(14)
    keys = rng.integers(0, 16, n + 1).astype(np.int32)
    cols = mixed_cols(n + 1, 2, [14])
    kt, ct = dev(keys), [dev(c) for c in cols]
    check_cols(keys[1:], [c[1:] for c in cols], 16, 2, True, "unaligned", keys_t=kt[1:], cols_t=[c[1:] for c in ct])


def test_error_rows_per_column():
    base_k = np.array([0, 1, 5, -1, 1, 0, 2, 3], np.int32)
    a = np.array([1.5, 2.0, 3.0, 4.0, np.nan, np.inf, 2.0 ** 1005, -np.inf])
    b = np.array([2.5, -2.0, 1.0, 4.0, 7.0, 1.0, 3.0, 9.0], np.float32)
    keys, ca, cb = np.tile(base_k, 1000), np.tile(a, 1000), np.tile(b, 1000)
    check_cols(keys, [ca, cb], 4, 2, True, "error rows, fused")


def test_resume_and_equal_to_single_column_calls():
    keys, v64, v32 = WL.lowcard(n=1_000_000, salt=15)
    G, L = 1024, 3
    kt, a, b = dev(keys), dev(v64), dev(v32)
    h = 400_000
    states = api.groupby_sum_cols(kt[:h], [a[:h], b[:h]], G, L)
    states = api.groupby_sum_cols(kt[h:], [a[h:], b[h:]], G, L, states=states)
    single = [api.groupby_sum(kt, a, G, L), api.groupby_sum(kt, b, G, L)]
    torch.cuda.synchronize()
    for c, (x, y) in enumerate(zip(states, single)):
        assert same_bits(x.cpu().numpy(), y.cpu().numpy()), f"column {c}: resumed fused != single-column call"


def test_empty_input_and_invalid_arguments():
    G, L = 8, 2
    kt = torch.zeros(0, dtype=torch.int32, device="cuda")
    cols = [torch.zeros(0, dtype=torch.float64, device="cuda") for _ in range(2)]
    states = api.groupby_sum_cols(kt, cols, G, L)
    torch.cuda.synchronize()
    empty = O.state_init(G, True, L)
    assert all(same_bits(s.cpu().numpy(), empty) for s in states)
    k1 = torch.zeros(10, dtype=torch.int32, device="cuda")
    c1 = torch.ones(10, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):  # f64 column into float accumulators
        api.groupby_sum_cols(k1, [c1, c1.float()], G, L, torch.float32)
    st = api.state_init(G, L)
    with pytest.raises(ValueError):  # one state for two aggregates
        api.groupby_sum_cols(k1, [c1, c1], G, L, states=[st, st])
    with pytest.raises(ValueError):
        api.groupby_sum_cols(k1, [c1] * 9, G, L)


def test_plain_columns_close_to_exact():
    keys, vals = WL.plain(n=500_000, salt=16)
    cols = [vals, (vals * 3.0).astype(np.float32)]
    outs = api.plain_groupby_sum_cols(dev(keys), [dev(c) for c in cols], 16)
    torch.cuda.synchronize()
    for c, o in zip(cols, outs):
        ref = np.zeros(16)
        np.add.at(ref, keys, c.astype(np.float64))
        assert np.allclose(o.cpu().numpy(), ref, rtol=1e-9, atol=1e-6)
