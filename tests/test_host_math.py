"""Host-side checks of the integer identities the kernels rely on."""


def test_jreq_multiply_shift_matches_division():
    """The kernels compute floor(x / W) as (x * ceil(2^16 / W)) >> 16 for the
    whole range of x that finite values produce (x = e + m - B + 1 with
    e = floor(log2|b|)): double lattice W = 40, x in [1, 2098]; float
    lattice W = 18, x in [1, 277]; float values on the double lattice lie
    inside the first range."""
    for W, hi in ((40, 2098), (18, 277)):
        mul = (65536 + W - 1) // W
        for x in range(1, hi + 1):
            assert (x * mul) >> 16 == x // W


def test_spill_word_carry_rule():
    """Spill words hold H * 2^64 + w with w unsigned; adding a signed unit k
    changes H by the carry out: +1 if k >= 0 and w wrapped, -1 if k < 0 and
    w borrowed.  Checked against exact integers on random sequences."""
    import random

    rnd = random.Random(5)
    M = 1 << 64
    for _ in range(200):
        w, H, exact = rnd.randrange(M), rnd.randrange(-5, 5), 0
        exact = H * M + w
        for _ in range(200):
            k = rnd.randrange(-(1 << 39), 1 << 39) if rnd.random() < 0.9 else rnd.randrange(-(1 << 63), 1 << 63)
            old = w
            w = (w + k) % M
            c = (1 if w < old else 0) if k >= 0 else (-1 if w > old else 0)
            H += c
            exact += k
            assert H * M + w == exact
