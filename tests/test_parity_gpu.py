"""HIP path vs the CPU oracle, element by element (bit-exact: the images are
canonical residues, so there is exactly one correct answer)."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu

P_SMALL_W8 = (1 << 31) + 11        # smallest odd modulus size on the 64-bit path
P_COMPOSITE = 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23 * 29 * 31 * 37 * 41 * 43 * 47   # odd, not prime


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _say(*a):
    print(*a, flush=True)


def _run(poly, beta, T, t0):
    if t0 == 1:
        return poly.run(beta, T)
    import torch
    buf = torch.empty((T, max(poly.G, 1)), dtype=torch.int64 if poly.elem_bytes == 8 else torch.int32,
                      device="cuda")
    poly.run_async(beta, T, buf, t0=t0)
    torch.cuda.synchronize()
    return buf.cpu().numpy().view(poly.dtype)[:, :poly.G]


def check(orc, p, exps, coeffs, beta, T, tuning=None, t0=1, single=None):
    """Images of the HIP path against the oracle.  Without an explicit tuning
    the default path runs (single-launch where the run fits it) and then the
    multi-kernel path with its heuristic K and C; both must match.  single:
    whether the default path must be the single-launch one (None: either)."""
    exps = np.ascontiguousarray(exps, np.uint32)
    coeffs = np.ascontiguousarray(coeffs, np.uint64)
    beta = np.ascontiguousarray(beta, np.uint64)
    _say(f"case p={p} s={exps.shape[0]} n={exps.shape[1]} T={T} tuning={tuning} t0={t0}")
    runs = {}
    with PV.Poly(p, exps, coeffs) as poly:
        gd, ge = poly.groups()
        od, oe = orc.groups(exps)
        assert np.array_equal(gd, od) and np.array_equal(ge, oe)
        if tuning:
            poly.set_tuning(*tuning)
            runs["tuned"] = _run(poly, beta, T, t0)
        else:
            is_single = poly.get_tuning(T) == (0, 0, 0)
            if single is not None:
                assert is_single == single, poly.get_tuning(T)
            runs["single" if is_single else "default"] = _run(poly, beta, T, t0)
            if is_single:
                poly.set_tuning(0, 16, 0)  # the multi-kernel path, heuristic K and C
                assert poly.get_tuning(T)[0] != 0
                runs["multi"] = _run(poly, beta, T, t0)
    want = orc.evaluate(p, exps, coeffs, beta, T, t0=t0, threads=8)
    for name, got in runs.items():
        assert got.shape == want.shape, name
        bad = np.argwhere(got != want.astype(got.dtype))
        assert bad.size == 0, f"{name}: {len(bad)} mismatches, first at {bad[:3].tolist()}"
    return got


def test_n4_s1e3_full(orc):
    w = W.n4_s1e3_p31_T64()
    check(orc, w.p, w.exps, w.coeffs, w.beta, w.T)


@pytest.mark.parametrize("p", [3, 5, 97, P_COMPOSITE % (1 << 31) | 1, W.P31, P_SMALL_W8, W.P50,
                               P_COMPOSITE, W.P63])
@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_random_polys(orc, p, n):
    rng = np.random.default_rng(p % 1000 + n)
    poly = W.random_small(rng, p, n, 700, 37, dmax={2: 30, 3: 9}.get(n, 5))
    check(orc, p, poly.exps, poly.coeffs, poly.beta, poly.T)


@pytest.mark.parametrize("p,K,P", [(p, K, P) for p in (W.P31, W.P63) for K in (1, 2, 4, 8, 16) for P in (8, 16, 32)] +
                         [(W.P31, 32, 8), (W.P31, 32, 16)])   # 32 terms per thread: 32-bit residues, P <= 16
def test_tuning_grid(orc, p, K, P):
    rng = np.random.default_rng(K * 31 + P)
    # a few big groups (span several waves), many small ones, a ragged tail
    big = W.random_small(rng, p, 5, 3000, 1, dmax=12)
    big.exps[:1500, :2] = [3, 1]
    big.exps[1500:2200, :2] = [2, 2]
    big.exps = np.unique(big.exps, axis=0)
    big.coeffs = rng.integers(0, p, size=big.exps.shape[0], dtype=np.uint64)
    for C in (1, 3, 7):
        check(orc, p, big.exps, big.coeffs, big.beta, 45, tuning=(K, P, C))


def test_edge_single_term(orc):
    check(orc, W.P63, [[2, 3, 4, 0, 7]], [12345], [5, 6, 7], 9)
    check(orc, W.P31, [[0, 0, 1]], [W.P31 - 1], [W.P31 - 1], 1)


def test_edge_one_group(orc):
    rng = np.random.default_rng(3)
    e = W.draw_exponents(rng, 5000, 6, 0, 20)
    for p in (W.P31, W.P63):
        co = rng.integers(0, p, size=e.shape[0], dtype=np.uint64)
        check(orc, p, e, co, rng.integers(1, p, 4, dtype=np.uint64), 33)


def test_edge_all_groups_distinct(orc):
    rng = np.random.default_rng(4)
    e = np.stack([np.arange(2000) // 50, np.arange(2000) % 50, rng.integers(0, 9, 2000),
                  rng.integers(0, 9, 2000)], axis=1).astype(np.uint32)
    for p in (W.P31, W.P63):
        check(orc, p, e, rng.integers(0, p, 2000, dtype=np.uint64), [3, 5], 20)


def test_edge_T_values(orc):
    w = W.n4_s1e3_p31_T64()
    for T in (1, 2, 15, 16, 17, 97):
        check(orc, w.p, w.exps, w.coeffs, w.beta, T)


def test_edge_special_points(orc):
    rng = np.random.default_rng(5)
    for p in (W.P31, W.P63, 7):
        poly = W.random_small(rng, p, 6, 400, 12, dmax=4)
        check(orc, p, poly.exps, poly.coeffs, np.ones(4, np.uint64), 12)
        check(orc, p, poly.exps, poly.coeffs, np.asarray([0, 3, 0, 1], np.uint64), 12)
        check(orc, p, poly.exps, np.full(poly.s, p - 1, np.uint64), poly.beta, 12)
        check(orc, p, poly.exps, np.zeros(poly.s, np.uint64), poly.beta, 3)


def test_edge_unreduced_inputs_and_duplicates(orc):
    rng = np.random.default_rng(6)
    p = W.P63
    poly = W.random_small(rng, p, 5, 600, 10, dmax=3, allow_dup=True)
    co = rng.integers(0, 2**64 - 1, size=poly.s, dtype=np.uint64)
    beta = np.asarray([2**64 - 1, p, p + 5], np.uint64)
    check(orc, p, poly.exps, co, beta, 10)


def test_edge_large_exponents(orc):
    rng = np.random.default_rng(7)
    e = np.asarray([[2**32 - 1, 0, 65535, 1], [0, 2**32 - 1, 1, 65535], [5, 5, 65535, 65535],
                    [5, 5, 0, 0], [2**31, 7, 40000, 3]], np.uint32)
    for p in (W.P31, W.P63):
        check(orc, p, e, rng.integers(0, p, 5, dtype=np.uint64), rng.integers(1, p, 2, dtype=np.uint64), 6)


def test_edge_empty(orc):
    with PV.Poly(W.P63, np.zeros((0, 4), np.uint32), np.zeros(0, np.uint64)) as poly:
        assert poly.G == 0
        out = poly.run([2, 3], 5)
        assert out.shape == (5, 0)
    with PV.Poly(W.P63, [[1, 2, 3, 4]], [9]) as poly:
        assert poly.run([2, 3], 0).shape == (0, 1)


def test_run_async_offset(orc):
    w = W.n4_s1e3_p31_T64()
    check(orc, w.p, w.exps, w.coeffs, w.beta, 20, t0=40)
    rng = np.random.default_rng(8)
    poly = W.random_small(rng, W.P63, 6, 900, 1, dmax=4)
    check(orc, W.P63, poly.exps, poly.coeffs, poly.beta, 50, t0=1000, tuning=(4, 16, 5))


def _with_group(rng, p, size, others, n=6, dmax=10):
    """A polynomial whose largest (x1, x2) group has exactly `size` terms."""
    tails = W.draw_exponents(rng, size + others, n - 2, dmax, dmax, per_var=True)
    e = np.zeros((size + others, n), np.uint32)
    e[:, 2:] = tails
    e[:size, :2] = [7, 3]
    e[size:, 0] = rng.integers(0, 7, others)          # x1 degree below 7: never the big group
    e[size:, 1] = rng.integers(0, 20, others)
    e = np.unique(e, axis=0)
    assert np.max(np.unique(e[:, :2], axis=0, return_counts=True)[1]) == size
    return e, rng.integers(0, p, e.shape[0], dtype=np.uint64), rng.integers(1, p, n - 2, dtype=np.uint64)


@pytest.mark.parametrize("p", [W.P31, W.P63])
def test_single_launch_shapes(orc, p):
    """The single-launch path at the edges of where it is used: several
    evaluations per block, ragged last block, largest term count, largest
    group, s*T at the limit, no tail variables, and just beyond each limit
    (multi-kernel path)."""
    rng = np.random.default_rng(11 if p == W.P31 else 12)
    q = W.random_small(rng, p, 5, 50, 1, dmax=6)
    check(orc, p, q.exps, q.coeffs, q.beta, 4000, single=True)          # 16 evaluations per block
    check(orc, p, q.exps, q.coeffs, q.beta, 4001, single=True)          # ragged last block
    s_max = 8192 if p == W.P31 else 4096                                 # 32 KiB of term values per evaluation
    q = W.random_small(rng, p, 6, s_max, 1, dmax=10)
    check(orc, p, q.exps, q.coeffs, q.beta, 128, single=True)
    q = W.random_small(rng, p, 6, s_max + 1, 1, dmax=10)
    check(orc, p, q.exps, q.coeffs, q.beta, 16, single=False)
    q = W.random_small(rng, p, 6, 4096, 1, dmax=10)
    check(orc, p, q.exps, q.coeffs, q.beta, 256, single=True)           # s T = 2^20
    check(orc, p, q.exps, q.coeffs, q.beta, 257, single=False)
    e, co, beta = _with_group(rng, p, 256, 300)
    check(orc, p, e, co, beta, 40, single=True)
    e, co, beta = _with_group(rng, p, 257, 300)
    check(orc, p, e, co, beta, 40, single=False)
    q = W.random_small(rng, p, 2, 300, 1, dmax=40)                       # n = 2: no tables
    check(orc, p, q.exps, q.coeffs, np.zeros(0, np.uint64), 70, single=True)
    q = W.random_small(rng, p, 4, 900, 1, dmax=10)
    check(orc, p, q.exps, q.coeffs, q.beta, 33, t0=10**12 + 7, single=True)   # chain starts by exponentiation
    check(orc, p, q.exps, q.coeffs, q.beta, 600, t0=2**40 + 3, single=True)


def test_single_launch_selection():
    """Which runs take the single-launch path, and how it is switched off."""
    w = W.n4_s1e3_p31_T64()
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        assert poly.get_tuning(w.T) == (0, 0, 0)
        poly.set_tuning(0, 16, 0)
        assert poly.get_tuning(w.T)[0] in (1, 2, 4, 8, 16)
        poly.set_tuning(0, 0, 0)
        assert poly.get_tuning(w.T) == (0, 0, 0)
        poly.set_arith("int")
        assert poly.get_tuning(w.T) != (0, 0, 0)
        poly.set_arith("auto")
        assert poly.get_tuning(w.T) == (0, 0, 0)
        assert poly.get_tuning((1 << 20) // w.s + 1) != (0, 0, 0)
    big = W.random_small(np.random.default_rng(13), W.P31, 4, 9000, 1, dmax=30)
    with PV.Poly(big.p, big.exps, big.coeffs) as poly:
        assert poly.get_tuning(8) != (0, 0, 0)                            # s above 8192


def test_deterministic_repeat():
    w = W.n4_s1e3_p31_T64()
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        a = poly.run(w.beta, 64)
        for _ in range(3):
            assert np.array_equal(poly.run(w.beta, 64), a)


def test_streams_and_handles_are_independent():
    import torch
    rng = np.random.default_rng(9)
    polys = [W.random_small(rng, p, 6, 5000, 1, dmax=5) for p in (W.P31, W.P63, W.P63)]
    hs = [PV.Poly(q.p, q.exps, q.coeffs) for q in polys]
    try:
        ref = [h.run(q.beta, 64) for h, q in zip(hs, polys)]
        streams = [torch.cuda.Stream() for _ in hs]
        bufs = []
        for h, q, st in zip(hs, polys, streams):
            dt = torch.int32 if h.elem_bytes == 4 else torch.int64
            b = torch.empty((64, h.G), dtype=dt, device="cuda")
            h.run_async(q.beta, 64, b, stream=st)
            bufs.append(b)
        torch.cuda.synchronize()
        for h, b, r in zip(hs, bufs, ref):
            assert np.array_equal(b.cpu().numpy().view(h.dtype), r)
    finally:
        for h in hs:
            h.destroy()


def _sampled_rows(orc, w, rows, got):
    for t in rows:
        want = orc.evaluate(w.p, w.exps, w.coeffs, w.beta, 1, t0=t, threads=1)[0]
        assert np.array_equal(got[t - 1].astype(np.uint64), want), f"row t={t}"


def test_n6_s1e6_full_size_sampled(orc):
    """n=6, 1e6 terms, p = 2^63-25, T = 1024, automatic tuning (the benchmark
    configuration); full oracle rows at a few t."""
    import concurrent.futures as cf
    w = W.n6_s1e6_p63_T1024()
    _say("n6_s1e6_p63_T1024: generated")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        got = poly.run(w.beta, w.T)
        _say("n6_s1e6_p63_T1024: tuning", poly.get_tuning(w.T), "G", poly.G)
        gd, ge = poly.groups()
    rows = [1, 2, 5, 6, 513, w.T - 1, w.T]
    with cf.ThreadPoolExecutor(len(rows)) as ex:
        futs = {t: ex.submit(orc.evaluate, w.p, w.exps, w.coeffs, w.beta, 1, t, 1) for t in rows}
        for t, f in futs.items():
            want = f.result()[0]
            assert np.array_equal(got[t - 1], want), f"row t={t}"
    _say("n6_s1e6_p63_T1024: rows ok")


def test_single_hip_runtime():
    """libpeval and PyTorch must share one HIP runtime (pointers and streams
    cross between them)."""
    import re
    PV.lib()
    import torch
    torch.cuda.init()
    maps = open("/proc/self/maps").read()
    runtimes = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(runtimes) == 1, runtimes


P40 = (1 << 40) - 87   # prime below 2^40


# 50-bit odd modulus whose double reciprocal lies well below 1/p: the
# quotient estimate of Alg. 2 falls short by one now and then, so the
# product's correction is taken on the device (about 2e-5 of products).
P_LOW_RECIP = 1123934916484611


@pytest.mark.parametrize("p", [P_SMALL_W8, P40, W.P50, (1 << 50) - 1 - 2 * 12345, P_LOW_RECIP])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
@pytest.mark.parametrize("P", [8, 16, 32])
def test_fp64_product_path(orc, p, K, P):
    """The paper's FP64-FMA product (Alg. 2) on the evaluation kernel."""
    rng = np.random.default_rng(K * 7 + P + p % 97)
    poly = W.random_small(rng, p, 6, 1500, 1, dmax=6)
    poly.exps[:600, :2] = [4, 4]  # one group spanning several waves
    poly.exps = np.unique(poly.exps, axis=0)
    poly.coeffs = rng.integers(0, p, size=poly.exps.shape[0], dtype=np.uint64)
    poly.coeffs[:7] = p - 1
    for C in (1, 5):
        exps = np.ascontiguousarray(poly.exps, np.uint32)
        with PV.Poly(p, exps, poly.coeffs) as q:
            q.set_arith("fp64")
            q.set_tuning(K, P, C)
            got = q.run(poly.beta, 41)
        want = orc.evaluate(p, exps, poly.coeffs, poly.beta, 41, threads=8)
        assert np.array_equal(got, want), (p, K, P, C)


def test_fp64_offsets_and_edges(orc):
    p = W.P50
    rng = np.random.default_rng(77)
    poly = W.random_small(rng, p, 5, 400, 1, dmax=4)
    with PV.Poly(p, poly.exps, poly.coeffs) as q:
        q.set_arith("fp64")
        for beta in (poly.beta, np.ones(3, np.uint64), np.asarray([0, p - 1, 2], np.uint64)):
            assert np.array_equal(q.run(beta, 9), orc.evaluate(p, poly.exps, poly.coeffs, beta, 9))
    check(orc, p, poly.exps, poly.coeffs, poly.beta, 30, t0=500)


@pytest.mark.parametrize("p", [W.P50, P_LOW_RECIP])
def test_fp64_many_products(orc, p):
    """2e4 terms x 400 rows (8e6 products) under the FP64 product at its
    widest K, every image against the oracle."""
    rng = np.random.default_rng(p % 1013)
    poly = W.random_small(rng, p, 7, 20000, 1, dmax=8)
    want = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 400, threads=8)
    with PV.Poly(p, poly.exps, poly.coeffs) as q:
        q.set_arith("fp64")
        for tun in ((8, 16, 0), (8, 32, 3)):
            q.set_tuning(*tun)
            assert np.array_equal(q.run(poly.beta, 400), want), tun


def test_fp64_mode_limits():
    with PV.Poly(W.P31, [[1, 2, 3]], [5]) as q:
        with pytest.raises(PV.PevalError):
            q.set_arith("fp64")
    with PV.Poly(W.P63, [[1, 2, 3]], [5]) as q:
        with pytest.raises(PV.PevalError):
            q.set_arith("fp64")
        q.set_arith("int")


@pytest.mark.parametrize("p", [P_SMALL_W8, P40, W.P50])
def test_integer_product_below_2_50(orc, p):
    """2^31 <= p < 2^50 defaults to the FP64 product; the integer one must agree."""
    rng = np.random.default_rng(p % 1009)
    poly = W.random_small(rng, p, 6, 2500, 1, dmax=6)
    want = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 50, threads=8)
    with PV.Poly(p, poly.exps, poly.coeffs) as q:
        for mode in ("int", "fp64", "auto"):
            q.set_arith(mode)
            for tun in ((16, 16, 3), (8, 32, 1), (1, 8, 7)):
                q.set_tuning(*tun)
                assert np.array_equal(q.run(poly.beta, 50), want), (mode, tun)


# --- pseudo-Mersenne product (p = 2^63 - c or 2^31 - c, small c) -----------

PM_MODULI = [W.P63, (1 << 63) - 1, (1 << 63) - ((1 << 20) - 1), W.P31, (1 << 31) - 4095, (1 << 31) - 3]


def check_pm(orc, p, exps, coeffs, beta, T, K=0, C=0):
    exps = np.ascontiguousarray(exps, np.uint32)
    _say(f"pm case p={p} s={exps.shape[0]} n={exps.shape[1]} T={T} K={K} C={C}")
    with PV.Poly(p, exps, coeffs) as poly:
        poly.set_arith("pm")
        assert poly.arith() == "pm"
        if K or C:
            poly.set_tuning(K, 0, C)
        got = poly.run(beta, T)
    want = orc.evaluate(p, exps, coeffs, beta, T, threads=8).astype(got.dtype)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"


@pytest.mark.parametrize("p", PM_MODULI)
def test_pseudo_mersenne_random(orc, p):
    rng = np.random.default_rng(p % 4099)
    poly = W.random_small(rng, p, 5, 2500, 41, dmax=6)
    for K, C in ((0, 0), (1, 3), (4, 1), (16, 7)):
        check_pm(orc, p, poly.exps, poly.coeffs, poly.beta, poly.T, K=K, C=C)


@pytest.mark.parametrize("p", PM_MODULI)
def test_pseudo_mersenne_extremes(orc, p):
    """Coefficients and base point at p - 1 keep every running value and
    product at the top of its range."""
    rng = np.random.default_rng(7)
    poly = W.random_small(rng, p, 4, 800, 33, dmax=9)
    poly.coeffs[:] = p - 1
    beta = np.full(2, p - 1, np.uint64)
    check_pm(orc, p, poly.exps, poly.coeffs, beta, 33)
    beta = np.asarray([p - 2, 2], np.uint64)
    check_pm(orc, p, poly.exps, poly.coeffs, beta, 33)


def test_pseudo_mersenne_refused():
    for p in (W.P50, 1000003, (1 << 63) - (1 << 21) - 1):
        with PV.Poly(p, np.asarray([[1, 1, 1]], np.uint32), np.asarray([1], np.uint64)) as h:
            with pytest.raises(PV.PevalError) as ei:
                h.set_arith("pm")
            assert ei.value.code == PV.EUNSUPPORTED


def test_n8_s1e7_full_size_sampled(orc):
    """n=8, 1e7 terms, p = 2^63-25, T = 4096 (the large workload), automatic
    tuning: whole oracle rows at the first, a middle and the last t, and
    single coefficients spread over the table."""
    import concurrent.futures as cf
    w = W.n8_s1e7_p63_T4096()
    _say("n8_s1e7_p63_T4096: generated")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        got = poly.run(w.beta, w.T)
        _say("n8_s1e7_p63_T4096: tuning", poly.get_tuning(w.T), "G", poly.G)
        gd, ge = poly.groups()
    rows = [1, 2049, w.T]
    with cf.ThreadPoolExecutor(len(rows)) as ex:
        futs = {t: ex.submit(orc.evaluate, w.p, w.exps, w.coeffs, w.beta, 1, t, 1) for t in rows}
        for t, f in futs.items():
            assert np.array_equal(got[t - 1], f.result()[0]), t
    rng = np.random.default_rng(44)
    for _ in range(6):
        t, g = int(rng.integers(1, w.T + 1)), int(rng.integers(0, len(gd)))
        want = orc.entry(w.p, w.exps, w.coeffs, w.beta, t, int(gd[g]), int(ge[g]))
        assert int(got[t - 1, g]) == want, (t, g)


def test_table2_full_size_sampled(orc):
    """The paper's Table 2 shape (n = 6, 5e5 terms, p = 2^50-27, T = 1e4)
    under automatic tuning, which takes the FP64 product: whole oracle rows
    at the first, a middle and the last t."""
    import concurrent.futures as cf
    w = W.paper_table2()
    _say("paper_table2: generated")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        got = poly.run(w.beta, w.T)
        _say("paper_table2: tuning", poly.get_tuning(w.T), "arith", poly.arith(), "G", poly.G)
        assert poly.arith() == "fp64"
    rows = [1, 2, 5001, w.T]
    with cf.ThreadPoolExecutor(len(rows)) as ex:
        futs = {t: ex.submit(orc.evaluate, w.p, w.exps, w.coeffs, w.beta, 1, t, 1) for t in rows}
        for t, f in futs.items():
            assert np.array_equal(got[t - 1], f.result()[0]), t
    _say("paper_table2: rows ok")


def test_batch_full_size_sampled(orc):
    """The 256-member uneven batch of the benchmark (terms up to 1e6, T up to
    2048, both primes) as one graph replay: members' first and last images
    against the oracle for a spread of members."""
    import torch
    ws = W.uneven_batch(count=256)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    try:
        with PV.Batch(polys, Ts) as b:
            outs = [torch.empty((T, q.G), dtype=torch.int32 if q.elem_bytes == 4 else torch.int64, device="cuda")
                    for q, T in zip(polys, Ts)]
            b.run([w.beta for w in ws], outs)
            torch.cuda.synchronize()
            # the largest members and a few small ones
            order = sorted(range(len(ws)), key=lambda j: -ws[j].s * ws[j].T)
            for j in order[:3] + order[-3:] + [100, 200]:
                w, q = ws[j], polys[j]
                got = outs[j].cpu().numpy().view(q.dtype)
                for t in (1, w.T):
                    want = orc.evaluate(w.p, w.exps, w.coeffs, w.beta, 1, t, 8)[0]
                    assert np.array_equal(got[t - 1].astype(np.uint64), want), (j, t)
    finally:
        for q in polys:
            q.destroy()


# (the FP64 product, taken for the 50-bit modulus, holds at most 8 terms per thread)
@pytest.mark.parametrize("p,K", [(p, K) for p in (W.P31, W.P63, W.P50, P_SMALL_W8) for K in (1, 2, 4, 8, 16)
                                 if not (p == W.P50 and K > 8)])
def test_direct_layout(orc, p, K):
    """Every group within one thread's K terms: the evaluation kernel writes
    the images itself (no segmented sums, partial sums or combine).  Group
    sizes 1..K, several chains, a ragged T, a start past t = 1."""
    rng = np.random.default_rng(K * 13 + p % 101)
    G = 700
    sizes = rng.integers(1, K + 1, size=G)
    sizes[0] = K
    rows = []
    for g, m in enumerate(sizes):
        d, e = divmod(g, 40)
        for i in range(m):
            rows.append([d, e, i, (7 * i + g) % 5, i % 3])
    exps = np.asarray(rows, np.uint32)
    coeffs = rng.integers(0, p, size=exps.shape[0], dtype=np.uint64)
    coeffs[:5] = p - 1
    beta = rng.integers(1, p, size=3, dtype=np.uint64)
    for C, T, t0 in ((1, 37, 1), (5, 61, 1), (3, 29, 1000003)):
        with PV.Poly(p, exps, coeffs) as poly:
            if p == W.P50:
                poly.set_arith("fp64")
            poly.set_tuning(K, 16, C)
            got = _run(poly, beta, T, t0)
        want = orc.evaluate(p, exps, coeffs, beta, T, t0=t0, threads=8)
        assert np.array_equal(got.astype(np.uint64), want), (p, K, C, T, t0)
