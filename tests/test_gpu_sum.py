"""Ungrouped reproducible sum: bit-exact parity with the oracle (one group,
every key 0), and the accuracy of the level sums against the error bound of
the method on the distributions of the paper's accuracy study (needs a GPU)."""
import sys
from fractions import Fraction

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


def gpu_sum(vals, L, T64=True, state=None, vt=None):
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = torch.from_numpy(np.ascontiguousarray(vals)).cuda() if vt is None else vt
    st = api.sum(v, L, torch.float64 if T64 else torch.float32, state=state, status=status)
    torch.cuda.synchronize()
    return st, int(status.item())


def oracle_sum(vals, L, T64=True):
    return O.groupby_sum(np.zeros(len(vals), np.int32), vals, 1, L, T64, threads=8)


@pytest.mark.parametrize("L", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 7, 2047, 2048, 2049, 100_003, 3_000_001])
def test_sum_matches_oracle(L, n):
    rng = np.random.default_rng([n, L])
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-200, 200, n))
    st, status = gpu_sum(vals, L)
    ref, rs = oracle_sum(vals, L)
    assert status == rs == 0
    assert np.array_equal(st.cpu().numpy(), ref)
    v32 = np.ldexp(rng.standard_normal(n), rng.integers(-60, 60, n)).astype(np.float32)
    for T64 in (True, False):
        st, _ = gpu_sum(v32, L, T64)
        ref, _ = oracle_sum(v32, L, T64)
        assert np.array_equal(st.cpu().numpy(), ref), f"float values, T64={T64}"


def test_sum_error_rows_resume_and_unaligned():
    rng = np.random.default_rng(5)
    n = 1_000_003
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-1000, 1010, n))
    vals[::1001] = np.nan
    vals[7] = np.inf
    ref, rs = oracle_sum(vals, 3)
    st, status = gpu_sum(vals, 3)
    assert status == rs and rs & 2 and rs & 4
    assert np.array_equal(st.cpu().numpy(), ref)
    # two calls into one state equal one call; an unaligned start uses scalar loads
    vt = torch.from_numpy(vals).cuda()
    st = api.sum(vt[:1], 3)
    st = api.sum(vt[1:], 3, state=st)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), ref)


def test_sum_full_size_column():
    keys, v64, v32 = WL.lowcard()
    say("case sum of 2e8 float64 values, repro<double,3>")
    st, status = gpu_sum(v64, 3)
    ref, rs = O.groupby_sum(np.zeros(len(v64), np.int32), v64, 1, 3, True, threads=16)
    assert status == rs == 0
    assert np.array_equal(st.cpu().numpy(), ref)


def exact_level_value(state, L):
    """Sum over levels of K_l * g_l, exactly, from a canonical double state."""
    S, C = O.split_states(state, 1, L, True)
    total = Fraction(0)
    for l in range(L):
        s = float(S[l, 0])
        bits = int(np.array([s]).view(np.uint64)[0])
        E = ((bits >> 52) & 0x7FF) - 1023
        lo = bits & ((1 << 50) - 1)
        K = int(C[l, 0]) * (1 << 50) + lo
        total += Fraction(K) * Fraction(2) ** (E - 52)
    return total


def exact_sum(vals):
    m, e = np.frexp(vals)
    mi = (m * 2.0 ** 53).astype(np.int64)
    sh = (e - 53 + 1074).astype(np.int64)
    tot = 0
    for a, b in zip(mi.tolist(), sh.tolist()):
        tot += a << b
    return Fraction(tot, 1 << 1074)


@pytest.mark.parametrize("dist", ["uniform12", "exp1"])
@pytest.mark.parametrize("n", [1000, 1_000_000])
def test_accuracy_within_bound(dist, n):
    """The accuracy study: |sum_l K_l g_l - sum b| <= n * 2^((1-L)W) * max|b|
    (the method's bound) for L = 1, 2, 3, and the finalised double is that
    value rounded a few times; the measured errors are printed."""
    rng = np.random.default_rng([n, 17])
    vals = rng.uniform(1.0, 2.0, n) if dist == "uniform12" else rng.exponential(1.0, n)
    ex = exact_sum(vals)
    mx = Fraction(float(np.max(np.abs(vals))))
    rows = []
    for L in (1, 2, 3):
        st, _ = gpu_sum(vals, L)
        err = abs(exact_level_value(st.cpu().numpy(), L) - ex)
        bound = n * Fraction(2) ** ((1 - L) * 40) * mx
        assert err <= bound, f"L={L}: error {float(err):.3e} above the bound {float(bound):.3e}"
        fin = float(api.finalize(st, 1, L).cpu().numpy()[0])
        rows.append((L, float(err), float(bound), abs(fin - float(ex))))
    say(f"accuracy {dist} n={n}: " + "; ".join(f"L={L} level error {e:.3e} (bound {b:.3e}), final {f:.3e}"
                                              for L, e, b, f in rows))


def test_counts_and_derived_statistics():
    """COUNT is exact; AVG / VAR / STDDEV derived from reproducible sums are
    bit-identical to the oracle's derivation (the same fixed IEEE sequence,
    square root included) from the oracle's sums, and do not change with the
    row order.  Tolerance 0."""
    rng = np.random.default_rng(9)
    n, G = 2_000_003, 5000
    keys = rng.integers(0, G, n).astype(np.int32)
    keys[:10] = G - 1  # group G-1 has rows; make one group empty and one with a single row
    keys[keys == 7] = 8
    keys[11] = 7
    keys[keys == 12] = 13  # group 12 empty
    vals = np.round(np.exp(rng.uniform(0, np.log(1e6), n)) * 100) / 100
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = api.groupby_stats(torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda(), G, L=2, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    cnt = np.bincount(keys, minlength=G)
    assert np.array_equal(out["count"].cpu().numpy(), cnt)
    s_ref = O.finalize(O.groupby_sum(keys, vals, G, 2, threads=8)[0], G, 2)
    q_ref = O.finalize(O.groupby_sum(keys, vals * vals, G, 2, threads=8)[0], G, 2)
    assert np.array_equal(out["sum"].cpu().numpy(), s_ref) and np.array_equal(out["sumsq"].cpu().numpy(), q_ref)
    m, v, sd = O.derive_stats(s_ref, q_ref, cnt)
    for name, want in (("avg", m), ("var_samp", v), ("stddev_samp", sd)):
        got = out[name].cpu().numpy()
        assert np.array_equal(np.isnan(got), np.isnan(want)), name
        fin = ~np.isnan(want)
        assert np.array_equal(got[fin].view(np.uint64), want[fin].view(np.uint64)), f"{name} differs from the oracle"
    got_m, got_v = out["avg"].cpu().numpy(), out["var_samp"].cpu().numpy()
    assert np.isnan(got_v[7]) and not np.isnan(got_m[7])  # one row: AVG defined, VAR not
    assert np.isnan(got_m[12])  # no row: AVG undefined
    # another order of the same rows: the same bits
    perm = rng.permutation(n)
    out2 = api.groupby_stats(torch.from_numpy(keys[perm]).cuda(), torch.from_numpy(vals[perm]).cuda(), G, L=2)
    for k in ("avg", "var_samp", "stddev_samp"):
        assert np.array_equal(out2[k].cpu().numpy().view(np.uint64), out[k].cpu().numpy().view(np.uint64))


def test_derived_statistics_float_values_side_stream_and_status():
    """float32 values (widened exactly; their squares are exact in double),
    a non-default stream, and error rows reported through the status word."""
    rng = np.random.default_rng(10)
    n, G = 300_001, 700
    keys = rng.integers(0, G, n).astype(np.int64)
    vals = np.ldexp(rng.standard_normal(n), rng.integers(-20, 20, n)).astype(np.float32)
    keys[3], vals[4] = G + 1, np.nan
    side = torch.cuda.Stream()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    kt, vt = torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda()
    side.wait_stream(torch.cuda.current_stream())
    out = api.groupby_stats(kt, vt, G, L=3, status=status, stream=side)
    side.synchronize()
    ok = (keys >= 0) & (keys < G)
    s_ref, st1 = O.groupby_sum(keys, vals, G, 3)
    q_ref, _ = O.groupby_sum(keys, vals.astype(np.float64) ** 2, G, 3)
    s_ref, q_ref = O.finalize(s_ref, G, 3), O.finalize(q_ref, G, 3)
    cnt = np.bincount(keys[ok], minlength=G)
    assert int(status.item()) == st1 == (1 | 2)
    assert np.array_equal(out["count"].cpu().numpy(), cnt)
    for name, want in zip(("avg", "var_samp", "stddev_samp"), O.derive_stats(s_ref, q_ref, cnt)):
        got = out[name].cpu().numpy()
        assert np.array_equal(np.isnan(got), np.isnan(want)), name
        fin = ~np.isnan(want)
        assert np.array_equal(got[fin].view(np.uint64), want[fin].view(np.uint64)), name
