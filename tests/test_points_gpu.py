"""Point mode (images at T arbitrary points) vs the CPU oracle, bit-exact."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu

P_SMALL_W8 = (1 << 31) + 11
P_COMPOSITE = 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23 * 29 * 31 * 37 * 41 * 43 * 47


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _say(*a):
    print(*a, flush=True)


def random_points(rng, p, T, m, special=True):
    pts = rng.integers(0, p, size=(T, m), dtype=np.uint64)
    if special and T and m:
        # zeros, ones, p-1 and unreduced values (reduced on the device)
        mask = rng.random((T, m))
        pts[mask < 0.05] = 0
        pts[(mask >= 0.05) & (mask < 0.08)] = 1
        pts[(mask >= 0.08) & (mask < 0.11)] = p - 1
        big = (mask >= 0.11) & (mask < 0.15)
        pts[big] = pts[big] + np.uint64(p) * rng.integers(1, 3, size=int(big.sum()), dtype=np.uint64)
    return pts


def check_points(orc, p, exps, coeffs, points, K=0, C=0):
    exps = np.ascontiguousarray(exps, np.uint32)
    coeffs = np.ascontiguousarray(coeffs, np.uint64)
    points = np.ascontiguousarray(points, np.uint64)
    _say(f"points case p={p} s={exps.shape[0]} n={exps.shape[1]} T={points.shape[0]} K={K} C={C}")
    with PV.Poly(p, exps, coeffs) as poly:
        if K or C:
            poly.set_tuning(K, 0, C)
        tk, tp, tc = poly.points_tuning(points.shape[0])  # the tiles the run below takes
        assert tk <= 16 and tp == 8 and 1 <= tc <= max(points.shape[0], 1)
        if K:
            assert tk == min(K, 16)
        if C:
            assert tc == min(C, max(points.shape[0], 1))
        got = poly.run_points(points)
    want = orc.evaluate_points(p, exps, coeffs, points, threads=8).astype(got.dtype)
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"
    return got


@pytest.mark.parametrize("p", [3, 97, W.P31, P_SMALL_W8, W.P50, P_COMPOSITE, W.P63])
@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_random_polys_points(orc, p, n):
    rng = np.random.default_rng(p % 997 + 7 * n)
    poly = W.random_small(rng, p, n, 600, 1, dmax={2: 30, 3: 9}.get(n, 5))
    pts = random_points(rng, p, 29, n - 2)
    check_points(orc, p, poly.exps, poly.coeffs, pts)


@pytest.mark.parametrize("p", [W.P31, W.P63])
@pytest.mark.parametrize("K", [1, 2, 4, 8, 16])
def test_points_tuning(orc, p, K):
    rng = np.random.default_rng(K + 5)
    big = W.random_small(rng, p, 5, 3000, 1, dmax=12)
    big.exps[:1500, :2] = [3, 1]
    big.exps[1500:2200, :2] = [2, 2]
    big.exps = np.unique(big.exps, axis=0)
    big.coeffs = rng.integers(0, p, size=big.exps.shape[0], dtype=np.uint64)
    pts = random_points(rng, p, 21, 3)
    for C in (1, 3, 7):
        check_points(orc, p, big.exps, big.coeffs, pts, K=K, C=C)


@pytest.mark.parametrize("p", [W.P31, W.P63])
@pytest.mark.parametrize("tail", [[30], [20] * 4, [100] * 3, [30] * 6, [300], [65535, 3], [0, 5, 0]])
def test_factor_shapes(orc, p, tail):
    """Tail degree bounds that give one to four factor tables, digit splits,
    and variables that never occur."""
    rng = np.random.default_rng(len(tail) * 1000 + tail[0])
    s, m = 400, len(tail)
    exps = np.zeros((s, 2 + m), np.uint32)
    exps[:, :2] = rng.integers(0, 4, size=(s, 2))
    for k, D in enumerate(tail):
        exps[:, 2 + k] = rng.integers(0, D + 1, size=s)
        if D:
            exps[0, 2 + k] = D                     # the bound is reached
    coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
    w = 4 if p < 2**31 else 8
    nf, E = PV.points_factors(w, [int(exps[:, 2 + k].max()) for k in range(m)])
    _say(f"factors {nf} entries {E}")
    check_points(orc, p, exps, coeffs, random_points(rng, p, 17, m))


def test_points_match_power_mode(orc):
    """The points beta^1..beta^T give exactly the power mode's images."""
    rng = np.random.default_rng(77)
    for p in (W.P31, W.P63):
        poly = W.random_small(rng, p, 6, 2000, 50, dmax=8)
        pts = np.asarray([[pow(int(b), t, p) for b in poly.beta] for t in range(1, 51)], np.uint64)
        with PV.Poly(p, poly.exps, poly.coeffs) as h:
            a = h.run_points(pts)
            b = h.run(poly.beta, 50)
        assert np.array_equal(a, b)


def test_points_edges(orc):
    rng = np.random.default_rng(5)
    p = W.P63
    # one term, one point
    check_points(orc, p, np.asarray([[1, 2, 3, 4]], np.uint32), np.asarray([5], np.uint64),
                 np.asarray([[7, 0]], np.uint64))
    # every group a single term, T = 1
    poly = W.random_small(rng, p, 4, 300, 1, dmax=20)
    check_points(orc, p, poly.exps, poly.coeffs, random_points(rng, p, 1, 2))
    # duplicate rows and coefficient p-1
    poly = W.random_small(rng, p, 5, 500, 1, dmax=3, allow_dup=True)
    poly.coeffs[:50] = p - 1
    check_points(orc, p, poly.exps, poly.coeffs, random_points(rng, p, 33, 3))
    # T = 0 and s = 0 are no-ops
    with PV.Poly(p, poly.exps, poly.coeffs) as h:
        assert h.run_points(np.zeros((0, 3), np.uint64)).shape == (0, h.G)


def test_points_table_chunks(orc):
    """More points than one launch's table budget holds (the points are
    processed in several chunks of tables)."""
    rng = np.random.default_rng(9)
    p = W.P63
    s, m = 64, 6
    exps = np.zeros((s, 2 + m), np.uint32)
    exps[:, :2] = rng.integers(0, 3, size=(s, 2))
    exps[:, 2:] = rng.integers(0, 31, size=(s, m))
    exps[0, 2:] = 30
    coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
    nf, E = PV.points_factors(8, [30] * m)
    T = (256 << 20) // (E * 16) + 1000             # one chunk plus a ragged second one
    check_points(orc, p, exps, coeffs, random_points(rng, p, T, m, special=False))


def test_points_async_streams(orc):
    import torch
    rng = np.random.default_rng(12)
    p = W.P31
    poly = W.random_small(rng, p, 6, 5000, 1, dmax=6)
    T = 40
    pts = random_points(rng, p, T, 4)
    want = orc.evaluate_points(p, poly.exps, poly.coeffs, pts, threads=8).astype(np.uint32)
    st = torch.cuda.Stream()
    with PV.Poly(p, poly.exps, poly.coeffs) as h:
        dpts = torch.from_numpy(pts.view(np.int64)).to("cuda")
        out = torch.empty((T, h.G), dtype=torch.int32, device="cuda")
        with torch.cuda.stream(st):
            h.run_points_async(dpts, T, out, stream=st)
        st.synchronize()
        got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)


def test_points_unsupported():
    p = W.P63
    n = 32
    exps = np.full((2, n), 10, np.uint32)
    exps[1, 2:] = 9
    with PV.Poly(p, exps, np.asarray([1, 2], np.uint64)) as h:
        with pytest.raises(PV.PevalError) as ei:
            h.run_points(np.ones((3, n - 2), np.uint64))
        assert ei.value.code == PV.EUNSUPPORTED


def test_points_full_size_sampled(orc):
    """The 1e6-term workload at 1024 random points: sampled rows against the oracle."""
    w = W.n6_s1e6_p63_T1024()
    rng = np.random.default_rng(2004)
    pts = rng.integers(1, w.p, size=(w.T, w.n - 2), dtype=np.uint64)
    with PV.Poly(w.p, w.exps, w.coeffs) as h:
        got = h.run_points(pts)
    rows = [0, 1, 511, 1023]
    want = orc.evaluate_points(w.p, w.exps, w.coeffs, pts[rows], threads=16)
    assert np.array_equal(got[rows], want)


# 50-bit odd modulus whose double reciprocal lies well below 1/p (the FP64
# product's quotient estimate is least accurate there)
P_LOW_RECIP = 1123934916484611


@pytest.mark.parametrize("p", [P_SMALL_W8, W.P50, P_LOW_RECIP])
@pytest.mark.parametrize("K", [1, 2, 4, 8, 16])
def test_points_fp64_product(orc, p, K):
    """2^31 <= p < 2^50 takes the FP64 product by default (K capped at 8);
    the integer product on the same handle agrees, with runs alternating so
    that each product's slot arrays are prepared once and kept apart."""
    rng = np.random.default_rng(p % 1009 + K)
    poly = W.random_small(rng, p, 6, 3000, 1, dmax=7)
    poly.exps[:900, :2] = [3, 2]  # one group over several waves
    poly.exps = np.unique(poly.exps, axis=0)
    poly.coeffs = rng.integers(0, p, size=poly.exps.shape[0], dtype=np.uint64)
    exps = np.ascontiguousarray(poly.exps, np.uint32)
    pts = random_points(rng, p, 37, 4)
    want = orc.evaluate_points(p, exps, poly.coeffs, pts, threads=8)
    with PV.Poly(p, exps, poly.coeffs) as h:
        assert h.arith() == "fp64"
        h.set_tuning(K, 0, 3)
        for mode in ("auto", "int", "fp64", "int"):
            h.set_arith(mode)
            assert h.points_tuning(pts.shape[0])[0] == (min(K, 8) if mode != "int" else K)
            got = h.run_points(pts)
            assert np.array_equal(got.astype(np.uint64), want), (mode, K)


@pytest.mark.parametrize("tail", [[30], [20] * 4, [300], [65535, 3]])
def test_points_fp64_factor_shapes(orc, tail):
    """FP64 product with one to four factor tables and digit-split variables."""
    p = W.P50
    rng = np.random.default_rng(len(tail) * 31 + tail[0])
    s, m = 700, len(tail)
    exps = np.zeros((s, m + 2), np.uint32)
    exps[:, :2] = rng.integers(0, 12, size=(s, 2))
    for v, d in enumerate(tail):
        exps[:, 2 + v] = rng.integers(0, d + 1, size=s)
    exps[0, 2:] = tail
    exps = np.unique(exps, axis=0)
    coeffs = rng.integers(0, p, size=exps.shape[0], dtype=np.uint64)
    check_points(orc, p, exps, coeffs, random_points(rng, p, 23, m))


def test_points_table2_shape_sampled(orc):
    """The paper's Table 2 shape (5e5 terms, p = 2^50 - 27) at 1e4 random
    points with the FP64 product: sampled rows against the oracle."""
    w = W.paper_table2()
    pts = W.random_points(w)
    with PV.Poly(w.p, w.exps, w.coeffs) as h:
        assert h.arith() == "fp64"
        got = h.run_points(pts)
    rows = [0, 1, 4999, w.T - 1]
    want = orc.evaluate_points(w.p, w.exps, w.coeffs, pts[rows], threads=16)
    assert np.array_equal(got[rows].astype(np.uint64), want)
