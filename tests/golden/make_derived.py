"""Writes tests/golden/derived_by_oracle.txt: the values of the worked
examples that the paper does not print, computed by the CPU oracle alone.

The paper prints the Fig. 2 result for one reading of its toy format (14)
and the Fig. 3 adjusting number (d = 1).  Under the same readings this
script records what the oracle gives for the other cases the pins use:

* Fig. 2 (Sec. III-C) with m = 4 fraction bits instead of 3;
* Fig. 3 (Sec. III-C): the canonical (S, C) of the level after the carry.

The pins then check these values against the independent one-pass exact
model in tests/exact_ref.py.  Run from the repository root:

    python tests/golden/make_derived.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402


def load(name):
    out = {}
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = (s.strip() for s in line.split("=", 1))
                out[k] = v
    return out


def main():
    f2 = load("fig2_rsum_example.txt")
    vals = [float(x) for x in f2["values"].split()]
    W, f, L = int(f2["W"]), int(f2["f"]), int(f2["L"])
    B = f - (L - 1) * W  # lattice through the first extractor of a fresh state
    _, _, m4 = O.sum_fmt(vals, (4, W, B, 30, -20, 20), L)

    f3 = load("fig3_carry.txt")
    m, E = int(f3["m"]), int(f3["E"])
    # level sum after the value: (S - 1.5 ufp) / ulp + the value's units
    ulp = 2.0 ** (E - m)
    K = int((int(f3["S.before"]) - 1.5 * 2.0**E) / ulp) + round(float(f3["value"]) / ulp)
    S, C = O.encode(K, E, m)

    lines = [
        "# Written by tests/golden/make_derived.py from the CPU oracle alone; do not edit.",
        "# Fig. 2 (Sec. III-C) in the format with m = 4 fraction bits:",
        f"fig2.result.m4 = {m4:g}",
        "# Fig. 3 (Sec. III-C): canonical level state after the carry:",
        f"fig3.S.after = {S:g}",
        f"fig3.C.after = {C}",
    ]
    with open(os.path.join(HERE, "derived_by_oracle.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
