"""The integer products' multiply-add forms, checked on the host with exact
integers.

The kernels compute Shoup's product (x w mod p in [0, 2p) from the
precomputed quotient wq = floor(w 2^k / p)) with 32x32->64-bit
multiply-adds only.  These tests model each multiply-add as (a b + c) mod
2^64 plus its carry-out bit and check the identities the device code rests
on:

* the high word floor(x wq / 2^64) from t = x0 y1 + hi(x0 y0) and
  u = x1 y0 + t, whose 65th bit (the carry) becomes the high word of the
  last multiply-add's addend;
* the remainder x w - q p (mod 2^64) as x w + q (2^64 - p), with the four
  cross products accumulated in one 64-bit word, shifted up by 32 and used
  as the addend of x0 w0;
* for p < 2^31, the remainder as the low word of x w + q (2^32 - p);
* a thread's sum as two 64-bit sums of the values' 32-bit halves, folded to
  96 bits;
* a 96-bit segment sum hi 2^64 + lo folded to one 64-bit word congruent to
  it (the partial coefficients): lo + hi R with R = 2^64 mod p, and on a
  carry out of 64 bits R added in place of the carry, which never carries
  again for p < 2^63.

A dropped carry, a wrong cross product or a missing shift fails here.
"""
import random

import pytest

M64 = 1 << 64
M32 = 1 << 32


def mad(a, b, c):
    """v_mad_u64_u32: (a b + c) mod 2^64 and the carry-out bit."""
    v = a * b + c
    return v % M64, v >> 64


def mulhi64(x, y, use_carry=True):
    x0, x1, y0, y1 = x % M32, x >> 32, y % M32, y >> 32
    t, _ = mad(x0, y1, (x0 * y0) >> 32)
    u, c = mad(x1, y0, t)
    s = (u >> 32) | ((c if use_carry else 0) << 32)
    q, _ = mad(x1, y1, s)
    return q


def shoup64(x, w, wq, p):
    n = (M64 - p) % M64
    x0, x1, w0, w1 = x % M32, x >> 32, w % M32, w >> 32
    q = mulhi64(x, wq)
    q0, q1, n0, n1 = q % M32, q >> 32, n % M32, n >> 32
    h, _ = mad(x1, w0, 0)
    h, _ = mad(x0, w1, h)
    h, _ = mad(q1, n0, h)
    h, _ = mad(q0, n1, h)
    h = (h << 32) % M64
    r, _ = mad(x0, w0, h)
    r, _ = mad(q0, n0, r)
    return r


def shoup32(x, w, wq, p):
    q = (x * wq) >> 32
    t, _ = mad(x, w, 0)
    r, _ = mad(q, (M32 - p) % M32, t)
    return r % M32


def half_sums(vals):
    lo = hi = 0
    for v in vals:
        lo, _ = mad(v % M32, 1, lo)
        hi, _ = mad(v >> 32, 1, hi)
    t = (lo >> 32) + hi % M32
    w0, w1, w2 = lo % M32, t % M32, ((hi >> 32) + (t >> 32)) % M32
    return w0 + (w1 << 32) + (w2 << 64)


def _edge_words(rng, bits):
    top = (1 << bits) - 1
    return [0, 1, 2, top, top - 1, 1 << (bits - 1), (1 << (bits - 1)) - 1] + [rng.randrange(1 << bits)
                                                                              for _ in range(60)]


def test_high_word_exact_and_carry_needed():
    rng = random.Random(1)
    words = _edge_words(rng, 64)
    carries = 0
    for x in words:
        for y in words:
            assert mulhi64(x, y) == (x * y) >> 64, (x, y)
            x0, x1, y0, y1 = x % M32, x >> 32, y % M32, y >> 32
            t = x0 * y1 + ((x0 * y0) >> 32)
            carries += (x1 * y0 + t) >= M64
    assert carries > 0
    # dropping the carry is caught
    assert any(mulhi64(x, y, use_carry=False) != (x * y) >> 64 for x in words for y in words)


@pytest.mark.parametrize("p", [3, 5, (1 << 31) + 11, (1 << 50) - 27, (1 << 62) - 57, (1 << 63) - 25, (1 << 63) - 1])
def test_shoup64_remainder(p):
    rng = random.Random(p)
    for _ in range(4000):
        w = rng.randrange(p)
        wq = (w << 64) // p
        x = rng.choice([rng.randrange(2 * p), 2 * p - 1, 0, rng.randrange(M64), M64 - 1])
        r = shoup64(x, w, wq, p)
        assert r < 2 * p and (r - x * w) % p == 0, (x, w)


@pytest.mark.parametrize("p", [3, 97, 65537, (1 << 31) - 1, (1 << 31) - 4095, (1 << 30) + 3])
def test_shoup32_remainder(p):
    rng = random.Random(p)
    for _ in range(4000):
        w = rng.randrange(p)
        wq = (w << 32) // p
        x = rng.choice([rng.randrange(2 * p), 2 * p - 1, 0, rng.randrange(M32), M32 - 1])
        r = shoup32(x, w, wq, p)
        assert r < 2 * p and (r - x * w) % p == 0, (x, w)


def test_half_sums_fold_to_96_bits():
    rng = random.Random(7)
    cases = [[M64 - 1] * 16, [0] * 16, [M32 - 1] * 16, [M64 - M32] * 16]
    cases += [[rng.randrange(M64) for _ in range(rng.randrange(1, 17))] for _ in range(2000)]
    for vals in cases:
        assert half_sums(vals) == sum(vals)


def fold96(lo, hi, p):
    """The partial coefficients' fold: y = hi R lazily, lo + y, a carry
    replaced by R (R = 2^64 mod p)."""
    R = M64 % p
    y = shoup64(hi, R, (R << 64) // p, p)
    s = lo + y
    if s >= M64:
        s = s - M64 + R
        assert s < M64, "second carry"
    return s


@pytest.mark.parametrize("p", [3, 5, (1 << 31) + 11, (1 << 50) - 27, (1 << 62) - 57, (1 << 62) + 135,
                               (1 << 63) - 25, (1 << 63) - 1])
def test_fold96_congruent_and_below_2_64(p):
    rng = random.Random(p ^ 0x5EED)
    R = M64 % p
    # extremes: the largest lo with the largest lazy y (hi chosen so that
    # hi R mod p is p - 1, when p - 1 is a multiple of gcd(R, p) = 1)
    hi_max = ((p - 1) * pow(R, -1, p)) % p % M32 if R else 0
    cases = [(M64 - 1, M32 - 1), (M64 - 1, hi_max), (0, 0), (M64 - 1, 0), (p - 1, 1)]
    cases += [(rng.randrange(M64), rng.randrange(M32)) for _ in range(5000)]
    carried = 0
    for lo, hi in cases:
        v = fold96(lo, hi, p)
        assert v < M64 and (v - (hi * M64 + lo)) % p == 0, (lo, hi)
        carried += lo + shoup64(hi, R, (R << 64) // p, p) >= M64
    assert carried > 0 or p < (1 << 32)
