"""Seeded generators: shapes, bounds, distinctness, reproducibility."""
import math

import numpy as np

from paper_2004_11571_amd import workloads as W


def _distinct(exps):
    return np.unique(exps, axis=0).shape[0] == exps.shape[0]


def test_n4_s1e3_shape_and_bounds():
    p = W.n4_s1e3_p31_T64()
    assert (p.n, p.s, p.T, p.p) == (4, 1000, 64, W.P31)
    assert p.exps.dtype == np.uint32 and p.exps.max() <= 10
    assert _distinct(p.exps)
    assert p.coeffs.max() < p.p and p.beta.min() >= 1 and p.beta.max() < p.p


def test_reproducible():
    a, b = W.n4_s1e3_p31_T64(), W.n4_s1e3_p31_T64()
    assert np.array_equal(a.exps, b.exps) and np.array_equal(a.coeffs, b.coeffs)
    assert np.array_equal(a.beta, b.beta)
    c = W.n4_s1e3_p31_T64(instance=1)
    assert not np.array_equal(a.coeffs, c.coeffs)


def test_total_degree_tail():
    rng = np.random.default_rng(0)
    e = W.draw_exponents(rng, 5000, 6, 40, 20)
    assert e[:, :2].max() <= 40 and e[:, 2:].sum(axis=1).max() <= 20
    assert _distinct(e)
    # every tail total degree 0..20 occurs (uniform over the simplex favours high totals)
    assert set(e[:, 2:].sum(axis=1).tolist()) >= set(range(5, 21))


def test_raise_dr_makes_room():
    dr = W.raise_dr(1_000_000, 4, 40, 20)
    assert 41 ** 2 * math.comb(dr + 2, 2) >= 2_000_000
    assert 41 ** 2 * math.comb(dr + 1, 2) < 2_000_000
    assert W.raise_dr(1000, 8, 40, 20) == 20


def test_uneven_batch_small():
    polys = W.uneven_batch(count=6, s_max=3e3)
    assert len(polys) == 6
    for q in polys:
        assert 4 <= q.n <= 8 and 1000 <= q.s <= 3000 and 32 <= q.T <= 2048
        assert q.p in (W.P31, W.P63) and _distinct(q.exps)


def test_serve_stream_poisson():
    pool = W.serve_pool(3, s_max=2e3)
    reqs = W.serve_stream(2000.0, 0.5, pool)
    assert 800 < len(reqs) < 1200
    times = [r.arrival_s for r in reqs]
    assert times == sorted(times) and times[-1] < 0.5
    for r in reqs:
        assert 64 <= r.T <= 2048 and r.beta.shape == (pool[r.poly_index].n - 2,)
