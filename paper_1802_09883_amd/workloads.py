"""Seeded synthetic GroupBy-SUM inputs (numpy only).

These generators hold none of the method's arithmetic: they only draw
(key, value) columns.  The same arrays feed the HIP library and the CPU
oracle.  They stand in for the paper's uniform-key workload (Sec. VI-A:
n pairs, keys uniform in [0, n_groups), identity-hashed; value
distributions U[1,2) and Exp(1) in Sec. VI-B) with the shapes of the
benchmark configurations:

  plain       n rows, int32 keys U[0,16), float64 N(0,1) * 2^k, k ~ U{-20..20}
  lowcard     n rows, int32 keys U[0,1024), float64 and float32 columns
              s * |z| * 2^k, k ~ U{-60..60}, s = +-1, and half of every
              group's rows are exact negations of its other rows, in random
              positions (sign-mixed cancellation)
  highcard    n rows, int64 keys Zipf(s=1) over 2^22 groups (rank r drawn
              with P ~ 1/r by inverse CDF, key = seeded permutation of r),
              float64 s * lognormal(0, 4)
Seeds: SeedSequence([0x5EED, config_id, column_id]).
"""
from __future__ import annotations

import numpy as np

SEED = 0x5EED


def rng_for(config_id: int, column_id: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED, config_id, column_id, salt]))


def plain(n: int = 10 ** 6, groups: int = 16, salt: int = 0):
    """Plain GroupBy-SUM: int32 keys U[0,groups), N(0,1) * 2^U{-20..20}."""
    rk, rv, re = rng_for(1, 0, salt), rng_for(1, 1, salt), rng_for(1, 2, salt)
    keys = rk.integers(0, groups, n, dtype=np.int32)
    vals = np.ldexp(rv.standard_normal(n), re.integers(-20, 21, n))
    return keys, vals


def lowcard(n: int = 2 * 10 ** 8, groups: int = 1024, salt: int = 0, with_f32: bool = True):
    """Low-cardinality scan with exact cancellation pairs (see module doc).
    Returns keys (int32), values float64, values float32 (or None)."""
    half = n // 2
    rk, rv, re, rs, rp = (rng_for(2, c, salt) for c in range(5))
    bkeys = rk.integers(0, groups, half, dtype=np.int32)
    mag = np.abs(rv.standard_normal(half))
    mag[mag == 0] = 1.0
    base = np.ldexp(mag, re.integers(-60, 61, half))
    base[rs.random(half) < 0.5] *= -1.0
    extra = n - 2 * half  # odd n: one unpaired row
    ekeys = rk.integers(0, groups, extra, dtype=np.int32)
    evals = np.ldexp(np.abs(rv.standard_normal(extra)) + 1.0, re.integers(-60, 61, extra))
    perm = rp.permutation(n)
    keys = np.concatenate([bkeys, bkeys, ekeys])[perm]
    v64 = np.concatenate([base, -base, evals])[perm]
    v32 = None
    if with_f32:
        b32 = base.astype(np.float32)
        v32 = np.concatenate([b32, -b32, evals.astype(np.float32)])[perm]
    return keys, v64, v32


def zipf_ranks(rng: np.random.Generator, n: int, N: int, s: float = 1.0) -> np.ndarray:
    """n ranks in [1, N] with P(r) proportional to r^-s (inverse CDF)."""
    w = 1.0 / np.arange(1, N + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, N)


def highcard(n: int = 10 ** 8, groups: int = 1 << 22, salt: int = 0):
    """High-cardinality skewed: int64 Zipf(1) keys, +-lognormal(0, 4) values."""
    rr, rperm, rv, rs = (rng_for(3, c, salt) for c in range(4))
    ranks = zipf_ranks(rr, n, groups)
    perm = rperm.permutation(groups).astype(np.int64)
    keys = perm[ranks - 1]
    vals = rv.lognormal(0.0, 4.0, n)
    vals[rs.random(n) < 0.5] *= -1.0
    return keys, vals


def batched_jobs(count: int = 512, salt: int = 0):
    """Sizes of independent GroupBy jobs: rows log-uniform in [1e3, 1e7],
    groups log-uniform in [1, 2^16], L in {2, 3}."""
    r = rng_for(4, 0, salt)
    rows = np.exp(r.uniform(np.log(1e3), np.log(1e7), count)).astype(np.int64)
    groups = np.exp(r.uniform(0.0, np.log(2.0 ** 16), count)).astype(np.int64)
    Ls = r.choice([2, 3], count)
    return rows, np.maximum(groups, 1), Ls


def batched_job(rows: int, groups: int, job: int, salt: int = 0):
    """One batched job's columns: int32 keys U[0,groups), N(0,1) * 2^U{-30..30}."""
    rk, rv, re = (rng_for(4, 1 + c, salt * 100003 + job) for c in range(3))
    keys = rk.integers(0, groups, rows, dtype=np.int32)
    vals = np.ldexp(rv.standard_normal(rows), re.integers(-30, 31, rows))
    return keys, vals


def decimal_columns(n: int, ncols: int = 6, salt: int = 0):
    """Decimal-like float64 columns: x log-uniform in [1, 1e6], rounded to
    two decimals (round(x * 100) / 100)."""
    rng = rng_for(5, 0, salt)
    x = np.exp(rng.uniform(0.0, np.log(1e6), (ncols, n)))
    return np.round(x * 100.0) / 100.0


def served_queries(count: int = 128, min_rows: int = 10_000, max_rows: int = 50_000_000, min_groups: int = 4,
                   max_groups: int = 1 << 20, salt: int = 0):
    """Sizes of a stream of GroupBy queries: rows log-uniform in
    [min_rows, max_rows], groups log-uniform in [min_groups, max_groups],
    and unit-rate exponential inter-arrival gaps (scale them by 1/rate for
    a Poisson process of that rate)."""
    r = rng_for(5, 1, salt)
    rows = np.exp(r.uniform(np.log(min_rows), np.log(max_rows), count)).astype(np.int64)
    groups = np.exp(r.uniform(np.log(min_groups), np.log(max_groups), count)).astype(np.int64)
    gaps = r.exponential(1.0, count)
    return rows, groups, gaps


def served_keys(n: int, groups: int, query: int, salt: int = 0):
    """int32 keys U[0, groups) of one served query."""
    return rng_for(5, 2, salt * 1000003 + query).integers(0, groups, n, dtype=np.int32)


# The four aggregates of a served query: SUM(c0), SUM(c1), SUM(c2*c3), SUM(c4*c5).
SERVED_AGGS = ((0, None), (1, None), (2, 3), (4, 5))
