"""Independent exact model of the paper's one-pass RSum (Alg. 2), in rationals.

Test-side only.  It follows the structure of Alg. 2 (Sec. III-C) step by step:
running sums S^(l) and carry counts C^(l) per level, the level-shift loop when
|b| >= 2^h * ulp(S^(1)), per-level extraction, and carry-bit propagation after
every value; finalisation by the equation of Sec. III-C from the last level
up.  Merging two states follows the lane merge of Alg. 3 (Sec. III-D) after
aligning the lower state with the same level-shift step.

It shares no code with the C oracle, which uses the two-pass "maximum
exponent first" form with integer level sums; agreement between the two is
therefore a real check (one-pass == two-pass, order independence).

Everything is exact (``fractions.Fraction``); the only rounding is the
explicit ``round_fmt`` into the target binary format.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Sequence


def ufp_exp(x: Fraction) -> int:
    """e with |x| in [2^e, 2^(e+1)), x != 0 (exact)."""
    x = abs(Fraction(x))
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    return e


def pow2(e: int) -> Fraction:
    return Fraction(2) ** e


def round_fmt(x: Fraction, m: int, emin: int, emax: int, mode: str = "even"):
    """Round x to a binary format with m fraction bits and exponent range
    [emin, emax] (gradual underflow).  mode 'even': nearest, ties to even;
    'trunc': toward zero.  Returns a Fraction, or +-inf as a float."""
    x = Fraction(x)
    if x == 0:
        return Fraction(0)
    sgn = -1 if x < 0 else 1
    a = abs(x)
    e = max(ufp_exp(a), emin)
    ulp = pow2(e - m)
    q, rem = divmod(a, ulp)
    if mode == "even":
        half = ulp / 2
        if rem > half or (rem == half and q % 2 == 1):
            q += 1
    elif mode != "trunc":
        raise ValueError(mode)
    r = q * ulp
    if r >= pow2(emax + 1):
        return math.inf * sgn
    return sgn * r


def rne_int(x: Fraction) -> int:
    """Nearest integer to x, ties to the even integer."""
    x = Fraction(x)
    fl = math.floor(x)
    d = x - fl
    if d > Fraction(1, 2) or (d == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


class OnePassRSum:
    """State of Alg. 2 for one group, in exact arithmetic.

    m: fraction bits; W: level spacing; f0: exponent of the first extractor
    of a fresh state (the paper's f); h: level-shift threshold exponent
    (the text's h = W-1); tie: 'state-free' rounds r / ulp(S) half-even,
    'literal' computes (r (+) S) (-) S with one rounding to the format, the
    literal form of Alg. 2 whose ties depend on S."""

    def __init__(self, m: int, W: int, f0: int, L: int, h: int | None = None, tie: str = "state-free"):
        self.m, self.W, self.L = m, W, L
        self.h = W - 1 if h is None else h
        self.tie = tie
        # exponents E^(l) of the extractors; S^(l) = 1.5 * 2^E^(l) initially
        self.E = [f0 - l * W for l in range(L)]
        self.S = [Fraction(3, 2) * pow2(E) for E in self.E]
        self.C = [0] * L

    def ulp(self, l: int) -> Fraction:
        return pow2(self.E[l] - self.m)

    def _shift_up(self):
        # drop the last level, demote the others, new first level 2^W higher
        top = self.E[0]
        for l in range(self.L - 1, 0, -1):
            self.S[l], self.C[l], self.E[l] = self.S[l - 1], self.C[l - 1], self.E[l - 1]
        self.E[0] = top + self.W
        self.S[0] = Fraction(3, 2) * pow2(self.E[0])
        self.C[0] = 0

    def _carry(self, l: int):
        u = pow2(self.E[l])
        lo = self.S[l] - Fraction(3, 2) * u
        d = math.floor(lo / (u / 4))
        self.S[l] -= d * (u / 4)
        self.C[l] += d
        assert Fraction(3, 2) * u <= self.S[l] < Fraction(7, 4) * u

    def add(self, b):
        b = Fraction(b)
        if b == 0:
            return
        while abs(b) >= pow2(self.h) * self.ulp(0):
            self._shift_up()
        r = b
        for l in range(self.L):
            if self.tie == "state-free":
                q = rne_int(r / self.ulp(l)) * self.ulp(l)
            else:
                s = round_fmt(r + self.S[l], self.m, -10**6, 10**6)
                q = s - self.S[l]
            self.S[l] += q
            r -= q
        for l in range(self.L):
            self._carry(l)

    def merge(self, other: "OnePassRSum"):
        """operator+=(repro): align tops by level shifts, then the lane merge
        S := 1.5 ufp + sum (S_v - 1.5 ufp(S_v)), C := sum C_v, then carries."""
        o = OnePassRSum(self.m, self.W, 0, self.L, self.h, self.tie)
        o.E, o.S, o.C = list(other.E), list(other.S), list(other.C)
        while self.E[0] < o.E[0]:
            self._shift_up()
        while o.E[0] < self.E[0]:
            o._shift_up()
        for l in range(self.L):
            u = pow2(self.E[l])
            self.S[l] = Fraction(3, 2) * u + (self.S[l] - Fraction(3, 2) * u) + (o.S[l] - Fraction(3, 2) * u)
            self.C[l] += o.C[l]
            self._carry(l)

    def level_values(self) -> List[Fraction]:
        """Exact value of each level: (S - 1.5 ufp(S)) + 0.25 ufp(S) * C."""
        out = []
        for l in range(self.L):
            u = pow2(self.E[l])
            out.append((self.S[l] - Fraction(3, 2) * u) + (u / 4) * self.C[l])
        return out

    def exact_value(self) -> Fraction:
        return sum(self.level_values(), Fraction(0))

    def finalize(self, emin: int, emax: int, m_out: int | None = None):
        """Equation of Sec. III-C: round each level once, add from the last
        level to the first, rounding every addition to the format."""
        m = self.m if m_out is None else m_out
        vals = [round_fmt(v, m, emin, emax) for v in self.level_values()]
        acc = vals[-1]
        for v in reversed(vals[:-1]):
            if isinstance(acc, float) or isinstance(v, float):
                acc = float(acc) + float(v)
            else:
                acc = round_fmt(acc + v, m, emin, emax)
        return acc


def onepass_sum(values: Sequence, m: int, W: int, f0: int, L: int, emin: int, emax: int, **kw):
    st = OnePassRSum(m, W, f0, L, **kw)
    for v in values:
        st.add(v)
    return st.finalize(emin, emax)


def conventional_sum(values: Sequence, m: int, emin: int, emax: int, mode: str = "even"):
    """Left-to-right sum rounding after each addition (the non-reproducible
    built-in sum)."""
    acc = Fraction(0)
    for v in values:
        acc = round_fmt(acc + Fraction(v), m, emin, emax, mode)
    return acc
