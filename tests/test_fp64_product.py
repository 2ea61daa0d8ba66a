"""The FP64 product's range argument (Section 3.1, Alg. 2 and 3), checked on
the host with exact arithmetic.

The FP64 policy keeps running values signed: the left operand x of Alg. 2
lies in (-p, p), the right one y (a power of a monomial value) in [0, p),
and the quotient estimate c is rounded to nearest instead of down.  The
claim is that g = x y - c p is exact and lies within 7p/8 of zero, so with
no correction step it is congruent to x y and lies in (-p, p) again; and
that a sum of at most 8
such values (|s| < 2^53) is folded by s - rint(s u) p into (-p, p) with no
correction, as is the sum of two folded values in the walks between
threads, and that one conditional addition makes a folded value canonical.

Each IEEE operation is modelled with Python floats (round to nearest, ties
to even, as the device runs) and each FMA as the exact rational result
rounded once (int / int true division is correctly rounded).  These are
properties of the mathematics the kernels rely on, not a copy of a kernel;
a wrong bound (a quotient rounded down with no correction, a p beyond
2^50) fails here.
"""
import math
import random
from fractions import Fraction

import pytest


def fma(a: float, b: float, c: float) -> float:
    exact = Fraction(a) * Fraction(b) + Fraction(c)
    return exact.numerator / exact.denominator


def alg2_signed(x: float, y: float, p: float, u: float, quotient=round):
    """Returns (g, c): the remainder and the quotient estimate.  round:
    Python's round on a float, to nearest with ties to even (v_rndne_f64)."""
    h = x * y
    l = fma(x, y, -h)
    b = h * u
    c = float(quotient(b))
    d = fma(-c, p, h)
    return d + l, c


def fold(s: float, p: float, u: float) -> float:
    c = float(round(s * u))  # Python's round: to nearest, ties to even, as v_rndne_f64
    return fma(-c, p, s)


def canonical(r: float, p: float) -> float:
    return r + p if r < 0.0 else r


# The last modulus is a 50-bit odd one whose double reciprocal lies well
# below 1/p (relative error -1.1e-16): there a quotient rounded down can
# fall short by one (for p = 2^50 - 27 it never does on random operands,
# since fl(1/p) is accurate to about 2^-100).
P_LOW_RECIP = 1123934916484611
MODULI = [2**31 + 11, 2**40 - 87, 2**49 + 9, 2**50 - 27, 2**50 - 1, P_LOW_RECIP]


def _operands(p: int, rng: random.Random):
    edge_x = [-(p - 1), -(p - 2), -(p // 2), -1, 0, 1, p // 2, p - 2, p - 1]
    edge_y = [0, 1, 2, p // 2, p // 2 + 1, p - 2, p - 1]
    for x in edge_x:
        for y in edge_y:
            yield x, y
    for _ in range(3000):
        yield rng.randrange(-(p - 1), p), rng.randrange(0, p)
    # operands near the top of the range, where the quotient estimate is tightest
    for _ in range(1000):
        yield rng.choice((-1, 1)) * (p - 1 - rng.randrange(1 << 20)), p - 1 - rng.randrange(1 << 20)


@pytest.mark.parametrize("p", MODULI)
def test_signed_product_exact_and_in_range(p):
    rng = random.Random(p)
    pf, u = float(p), 1.0 / float(p)
    for x, y in _operands(p, rng):
        g, c = alg2_signed(float(x), float(y), pf, u)
        assert g == x * y - int(c) * p, (x, y)            # remainder exact
        assert abs(g) <= 7 * p / 8, (x, y)                # a valid left operand again, no correction


@pytest.mark.parametrize("p", MODULI)
def test_chain_of_signed_products(p):
    """A running value kept signed over a long chain stays congruent to the
    exact power product and never leaves (-p, p)."""
    rng = random.Random(p + 1)
    pf, u = float(p), 1.0 / float(p)
    for _ in range(20):
        lam = rng.randrange(0, p)
        gamma = rng.randrange(0, p)
        x, want = float(lam), lam
        for _ in range(200):
            x = alg2_signed(x, float(gamma), pf, u)[0]
            want = want * gamma % p
            assert -p < x < p and (int(x) - want) % p == 0


@pytest.mark.parametrize("p", MODULI)
def test_sum_of_eight_folded(p):
    rng = random.Random(p + 2)
    pf, u = float(p), 1.0 / float(p)
    cases = [[-(p - 1)] * 8, [p - 1] * 8, [0] * 8, [-(p - 1), p - 1] * 4, [p - 1] * 7 + [-1]]
    cases += [[rng.randrange(-(p - 1), p) for _ in range(rng.randrange(1, 9))] for _ in range(3000)]
    for vals in cases:
        s = 0.0
        for v in vals:
            s += float(v)
        assert s == sum(vals)                             # the thread's sum is exact
        r = fold(s, pf, u)
        assert r == int(r) and -p < r < p and (int(r) - sum(vals)) % p == 0, vals
        assert abs(r) <= p / 2 + p * 2.0**-30              # rounded quotient: within p/2 of zero
        c = canonical(r, pf)
        assert 0 <= c < p and c == sum(vals) % p


@pytest.mark.parametrize("p", MODULI)
def test_walk_of_folded_values(p):
    """The walks between threads add two folded values and fold again: a
    long walk stays in (-p, p) and congruent to the exact sum."""
    rng = random.Random(p + 3)
    pf, u = float(p), 1.0 / float(p)
    for _ in range(40):
        acc, want = 0.0, 0
        for _ in range(200):
            v = fold(float(rng.randrange(-(8 * (p - 1)), 8 * p)), pf, u)
            want += int(v)
            acc = fold(acc + v, pf, u)
            assert -p < acc < p and (int(acc) - want) % p == 0
        assert canonical(acc, pf) == want % p


def test_quotient_rounded_down_needs_a_correction():
    """An operand pair for which a quotient rounded down (as Alg. 2 is
    printed) falls short and leaves g in [p, 2p): the rounded-to-nearest
    estimate the kernels use lands within 7p/8 of zero there too."""
    p = P_LOW_RECIP
    x, y = 726220303110107, 618400639462378
    pf, u = float(p), 1.0 / float(p)
    g_floor, c = alg2_signed(float(x), float(y), pf, u, quotient=math.floor)
    assert g_floor >= p and g_floor == x * y - int(c) * p
    g, c = alg2_signed(float(x), float(y), pf, u)
    assert abs(g) <= 7 * p / 8 and g == x * y - int(c) * p


def test_checks_catch_planted_mistakes():
    """The checks above are sharp enough to see a broken argument: near
    p = 2^53 (outside the policy's p < 2^50) the remainder stops being
    exact."""
    rng = random.Random(7)
    p = 2**53 - 111
    pf, u = float(p), 1.0 / float(p)
    inexact = 0
    for _ in range(500):
        x, y = -(p - 1 - rng.randrange(1 << 20)), p - 1 - rng.randrange(1 << 20)
        g, c = alg2_signed(float(x), float(y), pf, u)
        inexact += g != x * y - int(c) * p
    assert inexact > 0
