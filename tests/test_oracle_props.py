"""Invariance properties of the CPU oracle (bit-reproducibility, Sec. II-A).

The aggregate of each group must have the same bits for any execution: any
physical order of the rows, any split into chunks accumulated one after the
other (resumable state, Alg. 2), any merge tree of partial states
(operator+=(repro), Sec. IV; merge phase of Alg. 4) and any thread count.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import oracle as O


def make_rows(seed, n, G, spread, T64, zipf=False):
    rng = np.random.default_rng(seed)
    if zipf:
        keys = np.minimum(rng.zipf(1.5, n) - 1, G - 1)
    else:
        keys = rng.integers(0, G, n)
    keys = keys.astype(np.int32 if seed % 2 else np.int64)
    v = np.ldexp(rng.standard_normal(n), rng.integers(-spread, spread + 1, n))
    if n >= 4:  # exact cancellation pairs inside groups
        h = n // 4
        v[h:2 * h] = -v[:h]
        keys[h:2 * h] = keys[:h]
    return keys, (v if T64 else v.astype(np.float32))


settings.register_profile("oracle", max_examples=40, deadline=None)
settings.load_profile("oracle")

common = dict(
    seed=st.integers(0, 2 ** 31),
    n=st.integers(0, 3000),
    G=st.integers(1, 40),
    L=st.integers(1, 4),
    T64=st.booleans(),
)


@given(**common)
def test_permutation_invariance(seed, n, G, L, T64):
    spread = 300 if T64 else 60
    keys, v = make_rows(seed, n, G, spread, T64)
    a, sa = O.groupby_sum(keys, v, G, L, T64)
    p = np.random.default_rng(seed + 1).permutation(n)
    b, sb = O.groupby_sum(keys[p], v[p], G, L, T64)
    assert sa == sb == 0
    assert np.array_equal(a, b)


@given(**common, cuts=st.lists(st.integers(0, 3000), max_size=6))
def test_chunked_resume_invariance(seed, n, G, L, T64, cuts):
    keys, v = make_rows(seed, n, G, 300 if T64 else 60, T64, zipf=True)
    whole, _ = O.groupby_sum(keys, v, G, L, T64)
    bounds = sorted({0, n, *[c for c in cuts if c <= n]})
    states = O.state_init(G, T64, L)
    for b, e in zip(bounds[:-1], bounds[1:]):
        states, _ = O.groupby_sum(keys[b:e], v[b:e], G, L, T64, states=states)
    assert np.array_equal(whole, states)


@given(**common, parts=st.integers(1, 7), order_seed=st.integers(0, 1000))
def test_merge_tree_invariance(seed, n, G, L, T64, parts, order_seed):
    keys, v = make_rows(seed, n, G, 300 if T64 else 60, T64)
    whole, _ = O.groupby_sum(keys, v, G, L, T64)
    rng = np.random.default_rng(order_seed)
    assign = rng.integers(0, parts, n)
    partial = [O.groupby_sum(keys[assign == p], v[assign == p], G, L, T64)[0] for p in range(parts)]
    # random binary merge tree
    while len(partial) > 1:
        i, j = sorted(rng.choice(len(partial), 2, replace=False))
        merged = O.merge(partial[i], partial[j], G, L, T64)
        partial = [x for k, x in enumerate(partial) if k not in (i, j)] + [merged]
    assert np.array_equal(whole, partial[0])


@given(seed=st.integers(0, 2 ** 31), n=st.integers(0, 20000), threads=st.integers(2, 9))
def test_thread_count_invariance(seed, n, threads):
    keys, v = make_rows(seed, n, 17, 500, True)
    a, _ = O.groupby_sum(keys, v, 17, 3)
    b, _ = O.groupby_sum(keys, v, 17, 3, threads=threads)
    assert np.array_equal(a, b)


def test_f32_values_widen_exactly_into_double_states():
    """A float32 column summed into repro<double,L> equals the same values
    given as float64 (widening is exact)."""
    keys, v = make_rows(5, 5000, 9, 60, False)
    a, _ = O.groupby_sum(keys, v, 9, 3, True)
    b, _ = O.groupby_sum(keys, v.astype(np.float64), 9, 3, True)
    assert np.array_equal(a, b)
