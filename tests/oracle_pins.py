"""Pins for the CPU oracle: checks that do not reuse the oracle's own formula.

Each function takes an ``oracle.Oracle`` and raises AssertionError on a
mismatch.  They are run as ordinary tests (test_oracle_pins.py) and against
deliberately broken copies of the oracle (test_oracle_mutations.py), which
must each fail at least one of them.

What pins what (paper sections in brackets):

* ``pin_full_point_bigint``: the images b_t(x1, x2) are checked by evaluating
  f at full points (x1, x2, beta^t) over the integers, with no modular
  reduction until the very end [Section 2.1, definition of b_t].  This never
  groups terms and never forms coefficients, so it is a different
  computation from the oracle's.
* ``pin_small_prime_exhaustive``: for p <= 13 and x1, x2 degrees < p, equality
  of b_t as a function on all of F_p^2 fixes every coefficient; all base
  points in F_p^{n-2} (zero included) are tried, and Fermat periodicity
  b_{t+p-1} = b_t is checked when no beta_k is zero.
* ``pin_closed_forms``: single term a*x1^d*x2^e*M(x) gives a*M(beta)^t at
  (d, e) [Section 2.3: M_i(beta^t) = m_i^t]; beta = (1,..,1) gives the grouped
  coefficient sums for every t; beta_k = 0 kills exactly the terms using x_k.
* ``pin_linearity``: images are linear in the coefficient vector; duplicate
  exponent rows add up.
* ``pin_power_consistency``: row j*k of the images at beta equals row j of the
  images at beta^k [Section 2.3: powers of beta].
* ``pin_group_order``: columns are the distinct (d, e) in descending
  lexicographic order [Section 2.3: lex order x1 > x2 > ... makes like
  monomials adjacent].
* ``pin_gcd_example``: the worked example of Section 2.1 (golden fixture).

Arbitrary points (the random points of Zippel's method, Section 2.1):

* ``pin_points_full_point_bigint``: as above, at full points (x1, x2, x_t)
  with x_t arbitrary (zeros and unreduced values included).
* ``pin_points_character_sums``: for small p, summing the images over every
  point of (F_p^*)^m weighted by prod_k x_k^{-j_k} gives (p-1)^m times the
  sum of a_i over the terms whose tail exponents are congruent to j modulo
  p-1 (orthogonality of the characters x -> x^j of F_p^*), and the plain sum
  over all of F_p^m gives sum_i a_i prod_k S(g_ik) with S(0) = 0 and
  S(g) = -1 if (p-1) | g > 0, else 0.  Both identities are number theory,
  not the oracle's formula.
* ``pin_points_match_powers``: the points beta^1 .. beta^T give the images
  of the power mode (each side pinned on its own above).
* ``pin_points_zero_and_linearity``: at x = 0 only terms without tail
  variables survive; images are linear in the coefficients.

Interpolation (coefficients back from the images, Section 2.1):

* ``pin_interp_round_trip``: images from the (separately pinned) evaluation
  give back the coefficients, for several primes and shapes.
* ``pin_interp_exhaustive``: for p = 7 and a group of three terms, every one
  of the 7^3 coefficient vectors comes back (the map is a bijection).
* ``pin_interp_closed_forms``: a one-term group gives c_1 / m; extra image
  rows beyond the group size do not matter; a group with two equal monomial
  values is reported singular.
"""
from __future__ import annotations

import itertools
import os
import random

import numpy as np

from paper_2004_11571_amd import workloads as W

PRIMES_SMALL = [2, 3, 5, 7, 11, 13]
PRIMES_WORD = [3, 5, 7, 13, W.P31, W.P50, W.P63]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def image_at(out_row, gd, ge, x1, x2, p):
    """Evaluate a dense bivariate image at (x1, x2) in F_p."""
    acc = 0
    for c, d, e in zip(out_row, gd, ge):
        acc += int(c) * pow(x1, int(d), p) * pow(x2, int(e), p)
    return acc % p


def full_value(exps, coeffs, p, x1, x2, beta, t):
    """f(x1, x2, beta^t) over the integers, reduced only at the end."""
    total = 0
    bt = [int(b) ** t for b in beta]
    for row, a in zip(exps.tolist(), coeffs.tolist()):
        term = int(a) * x1 ** row[0] * x2 ** row[1]
        for k in range(2, len(row)):
            term *= bt[k - 2] ** row[k]
        total += term
    return total % p


def pin_full_point_bigint(orc, seed=1, cases=24):
    rng = np.random.default_rng(seed)
    pyr = random.Random(seed)
    for case in range(cases):
        p = PRIMES_WORD[case % len(PRIMES_WORD)]
        n = 2 + case % 4
        s = [1, 3, 7, 20][case % 4]
        T = 1 + case % 6
        poly = W.random_small(rng, p, n, s, T, dmax=5, allow_dup=(case % 3 == 0))
        if case % 5 == 0 and p > 3:
            poly.beta[:] = np.asarray([pyr.randrange(0, p) for _ in range(n - 2)], np.uint64)
        out = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, T)
        gd, ge = orc.groups(poly.exps)
        for t in range(1, T + 1):
            for _ in range(3):
                x1, x2 = pyr.randrange(0, p), pyr.randrange(0, p)
                want = full_value(poly.exps, poly.coeffs, p, x1, x2, poly.beta, t)
                got = image_at(out[t - 1], gd, ge, x1, x2, p)
                assert got == want, (case, p, n, s, t)


def pin_small_prime_exhaustive(orc, seed=2, primes=PRIMES_SMALL):
    rng = np.random.default_rng(seed)
    for p in primes:
        for n in ([3, 4] if p <= 7 else [3]):
            s = 6 if p <= 3 else 12
            exps = np.concatenate([
                rng.integers(0, p, size=(s, 2)),            # x1, x2 degree < p
                rng.integers(0, 2 * p + 1, size=(s, n - 2)),
            ], axis=1).astype(np.uint32)
            coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
            gd, ge = orc.groups(exps)
            T = 2 * p
            for beta in itertools.product(range(p), repeat=n - 2):
                beta = np.asarray(beta, np.uint64)
                out = orc.evaluate(p, exps, coeffs, beta, T)
                for t in range(1, T + 1):
                    for x1 in range(p):
                        for x2 in range(p):
                            want = full_value(exps, coeffs, p, x1, x2, beta, t)
                            assert image_at(out[t - 1], gd, ge, x1, x2, p) == want, (p, n, tuple(beta), t)
                if all(int(b) != 0 for b in beta):
                    for t in range(1, T - (p - 1) + 1):
                        assert np.array_equal(out[t - 1], out[t - 1 + p - 1]), (p, tuple(beta), t)


def _group_sums(exps, coeffs, p):
    sums = {}
    for row, a in zip(exps.tolist(), coeffs.tolist()):
        key = (row[0], row[1])
        sums[key] = (sums.get(key, 0) + int(a)) % p
    return sums


def pin_closed_forms(orc, seed=3):
    rng = np.random.default_rng(seed)
    pyr = random.Random(seed)
    for p in PRIMES_WORD:
        # single term: a * x1^d x2^e * prod x_k^{g_k}  ->  a * (prod beta_k^{g_k})^t
        for n in (2, 3, 6):
            row = [pyr.randrange(0, 9) for _ in range(n)]
            a = pyr.randrange(0, p)
            beta = [pyr.randrange(1, p) if p > 2 else 1 for _ in range(n - 2)]
            m = 1
            for k in range(2, n):
                m = m * pow(beta[k - 2], row[k], p) % p
            T = 7
            out = orc.evaluate(p, np.asarray([row], np.uint32), np.asarray([a], np.uint64),
                               np.asarray(beta, np.uint64), T)
            assert out.shape == (T, 1)
            for t in range(1, T + 1):
                assert int(out[t - 1, 0]) == a * pow(m, t, p) % p, (p, n, t)
        # beta = (1, ..., 1): every row is the grouped coefficient sum
        poly = W.random_small(rng, p, 5, 25, 4, dmax=3, allow_dup=True)
        ones = np.ones(3, np.uint64)
        out = orc.evaluate(p, poly.exps, poly.coeffs, ones, 4)
        gd, ge = orc.groups(poly.exps)
        sums = _group_sums(poly.exps, poly.coeffs, p)
        for g, key in enumerate(zip(gd.tolist(), ge.tolist())):
            for t in range(4):
                assert int(out[t, g]) == sums[key], (p, key, t)
        # beta_k = 0: only terms with exponent 0 in x_k survive (0^0 = 1)
        if p > 2:
            beta = np.asarray([pyr.randrange(1, p), 0, pyr.randrange(1, p)], np.uint64)
            out0 = orc.evaluate(p, poly.exps, poly.coeffs, beta, 3)
            keep = poly.exps[:, 3] == 0
            out1 = orc.evaluate(p, poly.exps[keep], poly.coeffs[keep], beta, 3)
            gd1, ge1 = orc.groups(poly.exps[keep])
            col = {k: j for j, k in enumerate(zip(gd.tolist(), ge.tolist()))}
            for j, key in enumerate(zip(gd1.tolist(), ge1.tolist())):
                assert np.array_equal(out0[:, col[key]], out1[:, j])
            absent = set(col) - set(zip(gd1.tolist(), ge1.tolist()))
            for key in absent:
                assert not out0[:, col[key]].any()


def pin_linearity(orc, seed=4):
    rng = np.random.default_rng(seed)
    for p in (W.P31, W.P50, W.P63, 7):
        poly = W.random_small(rng, p, 5, 40, 5, dmax=4)
        a2 = rng.integers(0, p, size=poly.s, dtype=np.uint64)
        c = int(rng.integers(1, p))
        r1 = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 5)
        r2 = orc.evaluate(p, poly.exps, a2, poly.beta, 5)
        summed = np.asarray([(int(x) + int(y)) % p for x, y in zip(poly.coeffs, a2)], np.uint64)
        r12 = orc.evaluate(p, poly.exps, summed, poly.beta, 5)
        for x, y, z in zip(r1.ravel(), r2.ravel(), r12.ravel()):
            assert (int(x) + int(y)) % p == int(z)
        scaled = np.asarray([int(x) * c % p for x in poly.coeffs], np.uint64)
        rc = orc.evaluate(p, poly.exps, scaled, poly.beta, 5)
        for x, z in zip(r1.ravel(), rc.ravel()):
            assert int(x) * c % p == int(z)
        # duplicate rows add: terms (row, a) and (row, b) == (row, a + b)
        exps2 = np.concatenate([poly.exps, poly.exps[:5]], axis=0)
        co2 = np.concatenate([poly.coeffs, a2[:5]])
        merged = poly.coeffs.copy()
        merged[:5] = [(int(x) + int(y)) % p for x, y in zip(poly.coeffs[:5], a2[:5])]
        assert np.array_equal(orc.evaluate(p, exps2, co2, poly.beta, 5),
                              orc.evaluate(p, poly.exps, merged, poly.beta, 5))


def pin_power_consistency(orc, seed=5):
    rng = np.random.default_rng(seed)
    for p in (W.P31, W.P63, 11):
        poly = W.random_small(rng, p, 6, 30, 12, dmax=4)
        full = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 12)
        for k in (2, 3, 4):
            bk = np.asarray([pow(int(b), k, p) for b in poly.beta], np.uint64)
            rows = orc.evaluate(p, poly.exps, poly.coeffs, bk, 12 // k)
            for j in range(1, 12 // k + 1):
                assert np.array_equal(rows[j - 1], full[j * k - 1]), (p, k, j)
        # t0 offset: rows t0.. of a longer run
        part = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 5, t0=6)
        assert np.array_equal(part, full[5:10])


def pin_group_order(orc, seed=6):
    rng = np.random.default_rng(seed)
    poly = W.random_small(rng, W.P31, 4, 60, 1, dmax=3, allow_dup=True)
    gd, ge = orc.groups(poly.exps)
    want = sorted({(r[0], r[1]) for r in poly.exps.tolist()}, reverse=True)
    assert list(zip(gd.tolist(), ge.tolist())) == want
    # a zero coefficient keeps its group
    co = poly.coeffs.copy()
    co[:] = 0
    out = orc.evaluate(W.P31, poly.exps, co, poly.beta, 2)
    assert out.shape == (2, len(want)) and not out.any()


def load_golden_gcd():
    """Parse tests/golden/gcd_example.txt into {name: (terms, beta, expected)}."""
    polys = {}
    cur = None
    with open(os.path.join(GOLDEN, "gcd_example.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "poly":
                cur = polys.setdefault(tok[1], {"terms": [], "beta": None, "expect": {}})
            elif tok[0] == "term":
                cur["terms"].append((int(tok[1]), [int(x) for x in tok[2:]]))
            elif tok[0] == "beta":
                cur["beta"] = [int(x) for x in tok[1:]]
            elif tok[0] == "expect":
                cur["expect"][(int(tok[1]), int(tok[2]))] = int(tok[3])
    return polys


def _poly_mul(f, g, p):
    h = {}
    for ef, cf in f.items():
        for eg, cg in g.items():
            e = tuple(x + y for x, y in zip(ef, eg))
            h[e] = (h.get(e, 0) + cf * cg) % p
    return h


def pin_gcd_example(orc, p=W.P63, T=5, seed=7):
    """Section 2.1: with c = x1 x2 + x3 x4 and d = x3 - x4, d vanishes at
    beta = (1, 1) and c becomes x1 x2 + 1, so every image of gc and gc + gd at
    (1, 1)^t coincides (the point is unlucky); at a random beta they differ."""
    gold = load_golden_gcd()
    for name, spec in gold.items():
        exps = np.asarray([e for _, e in spec["terms"]], np.uint32)
        coeffs = np.asarray([a % p for a, _ in spec["terms"]], np.uint64)
        out = orc.evaluate(p, exps, coeffs, np.asarray(spec["beta"], np.uint64), T)
        gd, ge = orc.groups(exps)
        got = {(int(d), int(e)): out[:, j] for j, (d, e) in enumerate(zip(gd, ge))}
        for key, val in spec["expect"].items():
            assert key in got, (name, key)
            assert all(int(v) == val % p for v in got[key]), (name, key)
        assert set(got) == set(spec["expect"]), name
    rng = random.Random(seed)
    g = {}
    for _ in range(6):
        g[tuple(rng.randrange(0, 3) for _ in range(4))] = rng.randrange(1, p)
    c = {(1, 1, 0, 0): 1, (0, 0, 1, 1): 1}
    d = {(0, 0, 1, 0): 1, (0, 0, 0, 1): p - 1}
    f = _poly_mul(g, c, p)
    h = dict(f)
    for e, v in _poly_mul(g, d, p).items():
        h[e] = (h.get(e, 0) + v) % p

    def run(poly, beta):
        ex = np.asarray(list(poly.keys()), np.uint32)
        co = np.asarray(list(poly.values()), np.uint64)
        out = orc.evaluate(p, ex, co, np.asarray(beta, np.uint64), T)
        gd, ge = orc.groups(ex)
        return {(int(a), int(b)): out[:, j] for j, (a, b) in enumerate(zip(gd, ge))}

    def same(u, v):
        keys = set(u) | set(v)
        zero = np.zeros(T, np.uint64)
        return all(np.array_equal(u.get(k, zero), v.get(k, zero)) for k in keys)

    assert same(run(f, [1, 1]), run(h, [1, 1]))
    beta = [rng.randrange(2, p), rng.randrange(2, p)]
    assert not same(run(f, beta), run(h, beta))
    # image of f at (1,1)^t is g(x1, x2, 1, 1) * (x1 x2 + 1)
    gb = {}
    for e, v in g.items():
        gb[(e[0], e[1])] = (gb.get((e[0], e[1]), 0) + v) % p
    want = {}
    for (a, b), v in gb.items():
        for (da, db) in ((1, 1), (0, 0)):
            k = (a + da, b + db)
            want[k] = (want.get(k, 0) + v) % p
    got = run(f, [1, 1])
    for k in set(want) | set(got):
        vals = got.get(k, np.zeros(T, np.uint64))
        assert all(int(x) == want.get(k, 0) for x in vals), k




# ---------------------------------------------------------------------------
# Arbitrary points
# ---------------------------------------------------------------------------

def full_value_at(exps, coeffs, p, x1, x2, x):
    """f(x1, x2, x) over the integers, reduced only at the end."""
    total = 0
    for row, a in zip(exps.tolist(), coeffs.tolist()):
        term = int(a) * x1 ** row[0] * x2 ** row[1]
        for k in range(2, len(row)):
            term *= int(x[k - 2]) ** row[k]
        total += term
    return total % p


def pin_points_full_point_bigint(orc, seed=21, cases=20):
    rng = np.random.default_rng(seed)
    pyr = random.Random(seed)
    for case in range(cases):
        p = PRIMES_WORD[case % len(PRIMES_WORD)]
        n = 2 + case % 5
        s = [1, 4, 9, 25][case % 4]
        T = 1 + case % 5
        poly = W.random_small(rng, p, n, s, T, dmax=4, allow_dup=(case % 3 == 1))
        pts = [[pyr.choice([0, 1, p - 1, pyr.randrange(0, p), p + pyr.randrange(0, 1000)])
                for _ in range(n - 2)] for _ in range(T)]
        points = np.asarray(pts, np.uint64).reshape(T, n - 2)
        out = orc.evaluate_points(p, poly.exps, poly.coeffs, points)
        gd, ge = orc.groups(poly.exps)
        for t in range(T):
            for _ in range(3):
                x1, x2 = pyr.randrange(0, p), pyr.randrange(0, p)
                want = full_value_at(poly.exps, poly.coeffs, p, x1, x2, pts[t])
                assert image_at(out[t], gd, ge, x1, x2, p) == want, (case, p, n, s, t)


def pin_points_character_sums(orc, seed=22):
    rng = np.random.default_rng(seed)
    for p, m in ((5, 2), (7, 1), (7, 2), (3, 3)):
        s = 16
        exps = np.concatenate([rng.integers(0, 3, size=(s, 2)),
                               rng.integers(0, 3 * (p - 1) + 1, size=(s, m))], axis=1).astype(np.uint32)
        # a few terms whose tail exponents are all positive multiples of p-1
        exps[:3, 2:] = (p - 1) * rng.integers(1, 3, size=(3, m))
        coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
        gd, ge = orc.groups(exps)
        G = len(gd)
        col = {(int(d), int(e)): j for j, (d, e) in enumerate(zip(gd, ge))}
        # every point of F_p^m
        allpts = np.asarray(list(itertools.product(range(p), repeat=m)), np.uint64)
        out = orc.evaluate_points(p, exps, coeffs, allpts)
        S = lambda g: (p - 1) if (g > 0 and g % (p - 1) == 0) else 0     # -1 mod p, else 0
        want = [0] * G
        for row, a in zip(exps.tolist(), coeffs.tolist()):
            v = int(a)
            for g in row[2:]:
                v *= S(g)
            want[col[(row[0], row[1])]] += v
        got = [int(x) for x in (out.astype(object).sum(axis=0) % p)]
        assert got == [w % p for w in want], (p, m)
        # weighted sums over (F_p^*)^m pick out exponent classes mod p-1
        units = np.asarray(list(itertools.product(range(1, p), repeat=m)), np.uint64)
        outu = orc.evaluate_points(p, exps, coeffs, units)
        for j in itertools.product(range(p - 1), repeat=m):
            w = [1] * len(units)
            for r, x in enumerate(units.tolist()):
                for k in range(m):
                    w[r] = w[r] * pow(int(x[k]), (p - 1 - j[k]) % (p - 1), p) % p
            lhs = [sum(w[r] * int(outu[r, g]) for r in range(len(units))) % p for g in range(G)]
            rhs = [0] * G
            for row, a in zip(exps.tolist(), coeffs.tolist()):
                if all(row[2 + k] % (p - 1) == j[k] for k in range(m)):
                    rhs[col[(row[0], row[1])]] += int(a)
            scale = pow(p - 1, m, p)
            assert lhs == [scale * r % p for r in rhs], (p, m, j)


def pin_points_match_powers(orc, seed=23):
    rng = np.random.default_rng(seed)
    for p, n, s, T in ((W.P63, 6, 40, 7), (W.P31, 4, 30, 5), (101, 3, 10, 9), (W.P50, 8, 25, 3)):
        poly = W.random_small(rng, p, n, s, T, dmax=5)
        pts = np.asarray([[pow(int(b), t, p) for b in poly.beta] for t in range(1, T + 1)],
                         np.uint64).reshape(T, n - 2)
        a = orc.evaluate_points(p, poly.exps, poly.coeffs, pts)
        b = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, T)
        assert np.array_equal(a, b), (p, n)


def pin_points_zero_and_linearity(orc, seed=24):
    rng = np.random.default_rng(seed)
    p, n, s, T = W.P63, 5, 60, 4
    poly = W.random_small(rng, p, n, s, T, dmax=3)
    poly.exps[:10, 2:] = 0                       # some terms without tail variables
    zero = np.zeros((1, n - 2), np.uint64)
    out = orc.evaluate_points(p, poly.exps, poly.coeffs, zero)
    gd, ge = orc.groups(poly.exps)
    want = {}
    for row, a in zip(poly.exps.tolist(), poly.coeffs.tolist()):
        if not any(row[2:]):
            want[(row[0], row[1])] = (want.get((row[0], row[1]), 0) + int(a)) % p
    for j, (d, e) in enumerate(zip(gd, ge)):
        assert int(out[0, j]) == want.get((int(d), int(e)), 0)
    pts = rng.integers(0, p, size=(T, n - 2), dtype=np.uint64)
    c2 = rng.integers(0, p, size=s, dtype=np.uint64)
    k = 987654321
    mix = np.asarray([(int(a) * k + int(b)) % p for a, b in zip(poly.coeffs, c2)], np.uint64)
    o1 = orc.evaluate_points(p, poly.exps, poly.coeffs, pts).astype(object)
    o2 = orc.evaluate_points(p, poly.exps, c2, pts).astype(object)
    om = orc.evaluate_points(p, poly.exps, mix, pts).astype(object)
    assert np.array_equal(om, (o1 * k + o2) % p)


# ---------------------------------------------------------------------------
# Interpolation
# ---------------------------------------------------------------------------

def _distinct_support(rng, p, n, s, dmax, d12=3):
    exps = W.draw_exponents(rng, s, n, d12, dmax, per_var=True)
    return exps


def pin_interp_round_trip(orc, seed=31):
    rng = np.random.default_rng(seed)
    for p, n, s in ((W.P63, 5, 300), (W.P50, 6, 200), (W.P31, 4, 150), (1000003, 3, 60), (101, 4, 12)):
        exps = _distinct_support(rng, p, n, s, 6 if n > 3 else 40)
        coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
        T = s  # more rows than any group needs
        for attempt in range(20):
            beta = rng.integers(1, p, size=n - 2, dtype=np.uint64)
            images = orc.evaluate(p, exps, coeffs, beta, T)
            try:
                got = orc.interpolate(p, exps, beta, images)
            except Exception:        # an unlucky beta (equal monomial values) for tiny p
                if p > 10**6:
                    raise
                continue
            assert np.array_equal(got, coeffs % np.uint64(p)), (p, n, s)
            break
        else:
            raise AssertionError(f"no usable beta for p={p}")


def pin_interp_exhaustive(orc, p=7):
    exps = np.asarray([[1, 0, 1, 0], [1, 0, 0, 1], [1, 0, 2, 2]], np.uint32)
    beta = np.asarray([2, 3], np.uint64)       # monomial values 2, 3, 36 = 1 mod 7: distinct
    seen = set()
    for a in itertools.product(range(p), repeat=3):
        coeffs = np.asarray(a, np.uint64)
        images = orc.evaluate(p, exps, coeffs, beta, 3)
        got = tuple(int(x) for x in orc.interpolate(p, exps, beta, images))
        assert got == a, (a, got)
        seen.add(tuple(int(x) for x in images[:, 0]))
    assert len(seen) == p ** 3                 # distinct coefficient vectors give distinct images


def pin_interp_closed_forms(orc, seed=32):
    import oracle as O
    rng = np.random.default_rng(seed)
    p = W.P63
    exps = np.asarray([[2, 1, 3, 1], [0, 0, 2, 5]], np.uint32)     # two one-term groups
    beta = rng.integers(2, p, size=2, dtype=np.uint64)
    images = rng.integers(0, p, size=(4, 2), dtype=np.uint64)       # any values are consistent
    gd, ge = orc.groups(exps)
    got = orc.interpolate(p, exps, beta, images)
    for i, row in enumerate(exps.tolist()):
        g = [j for j in range(len(gd)) if (int(gd[j]), int(ge[j])) == (row[0], row[1])][0]
        m = pow(int(beta[0]), row[2], p) * pow(int(beta[1]), row[3], p) % p
        assert int(got[i]) == int(images[0, g]) * pow(m, p - 2, p) % p
    # rows past the largest group are not used
    exps = _distinct_support(rng, p, 5, 120, 5)
    coeffs = rng.integers(0, p, size=120, dtype=np.uint64)
    beta = rng.integers(1, p, size=3, dtype=np.uint64)
    images = orc.evaluate(p, exps, coeffs, beta, 200)
    sizes = {}
    for row in exps.tolist():
        sizes[(row[0], row[1])] = sizes.get((row[0], row[1]), 0) + 1
    mx = max(sizes.values())
    noisy = images.copy()
    noisy[mx:] = rng.integers(0, p, size=noisy[mx:].shape, dtype=np.uint64)
    assert np.array_equal(orc.interpolate(p, exps, beta, noisy), coeffs)
    # beta_3 = 1 makes terms that differ only in x3 share a monomial value
    exps = np.asarray([[1, 1, 0, 2], [1, 1, 3, 2]], np.uint32)
    try:
        orc.interpolate(p, exps, np.asarray([1, 5], np.uint64), np.ones((2, 1), np.uint64))
    except O.SingularError:
        pass
    else:
        raise AssertionError("singular system not reported")


ALL_PINS = [pin_full_point_bigint, pin_small_prime_exhaustive, pin_closed_forms,
            pin_linearity, pin_power_consistency, pin_group_order, pin_gcd_example,
            pin_points_full_point_bigint, pin_points_character_sums, pin_points_match_powers,
            pin_points_zero_and_linearity, pin_interp_round_trip, pin_interp_exhaustive,
            pin_interp_closed_forms]
