"""Served requests: each result is identical alone and in the mix (tolerance
0: canonical residues), under continuous batching, slicing and a tight
memory budget."""
import threading
import time

import numpy as np
import pytest

from oracle import Oracle
from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pool(seed, count, s_max, moduli=(W.P63, W.P31)):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.integers(4, 9))
        s = int(round(10 ** rng.uniform(3, np.log10(s_max))))
        p = moduli[j % len(moduli)]
        out.append(W.make_poly(int(rng.integers(0, 2**62)), p, n, s, 1, 40, W.raise_dr(s, n, 40, 20)))
    return out


def _alone(pool, reqs):
    """Every request evaluated alone with a plain run on its own handle."""
    hs = [PV.Poly(w.p, w.exps, w.coeffs) for w in pool]
    try:
        return [hs[j].run(beta, T) for j, beta, T in reqs]
    finally:
        for h in hs:
            h.destroy()


def _requests(pool, count, seed, t_max=600):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        j = int(rng.integers(0, len(pool)))
        T = int(rng.integers(1, t_max))
        beta = rng.integers(1, pool[j].p, size=pool[j].n - 2, dtype=np.uint64)
        reqs.append((j, beta, T))
    return reqs


@pytest.mark.parametrize("slice_work", [2e9, 2e5])
def test_served_equals_alone(slice_work):
    pool = _pool(1, 6, 5e4)
    reqs = _requests(pool, 40, 2)
    want = _alone(pool, reqs)
    with PV.Server(8 << 30) as srv:
        srv.configure(slice_work=slice_work)
        pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]
        rids = []
        for k, (j, beta, T) in enumerate(reqs):
            rids.append(srv.submit(pids[j], beta, T))
            if k == 20:
                time.sleep(0.002)  # later arrivals join passes already in flight
        got = [srv.wait(r, 60000) for r in rids]
        st = srv.stats()
        print("stats", st, flush=True)
    for k, (g, w_) in enumerate(zip(got, want)):
        assert np.array_equal(g, w_), f"request {k}"
    assert st["completed"] == len(reqs) and st["rejected"] == 0


def test_served_tight_budget_and_oracle():
    pool = _pool(3, 4, 2e4)
    reqs = _requests(pool, 16, 4, t_max=300)
    orc = Oracle()
    with PV.Server(96 << 20) as srv:
        srv.configure(slice_work=1e6)
        pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]
        rids = [srv.submit(pids[j], beta, T) for j, beta, T in reqs]
        got = [srv.wait(r, 60000) for r in rids]
        st = srv.stats()
        print("stats", st, flush=True)
        assert st["hbm_peak"] <= 96 << 20
    for (j, beta, T), g in zip(reqs[:6], got[:6]):
        w = pool[j]
        assert np.array_equal(g.astype(np.uint64), orc.evaluate(w.p, w.exps, w.coeffs, beta, T, threads=8))
    want = _alone(pool, reqs)
    for g, w_ in zip(got, want):
        assert np.array_equal(g, w_)


def test_served_fp64_members():
    """Polynomials with 2^31 <= p < 2^50 are served with the FP64 product
    (their own queue in each pass) beside 32- and 64-bit integer ones."""
    pool = _pool(5, 6, 3e4, moduli=(W.P31, W.P50, W.P63))
    reqs = _requests(pool, 30, 6, t_max=400)
    orc = Oracle()
    with PV.Server(4 << 30) as srv:
        srv.configure(slice_work=5e6)
        pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]
        rids = [srv.submit(pids[j], beta, T) for j, beta, T in reqs]
        got = [srv.wait(r, 60000) for r in rids]
    want = _alone(pool, reqs)
    for k, (g, w_) in enumerate(zip(got, want)):
        assert np.array_equal(g, w_), f"request {k}"
    checked = 0
    for (j, beta, T), g in zip(reqs, got):
        w = pool[j]
        if w.p == W.P50 and checked < 5:
            assert np.array_equal(g.astype(np.uint64), orc.evaluate(w.p, w.exps, w.coeffs, beta, T, threads=8))
            checked += 1
    assert checked == 5


def test_concurrent_submitters():
    pool = _pool(5, 3, 1e4)
    reqs = _requests(pool, 30, 6, t_max=200)
    want = _alone(pool, reqs)
    got = [None] * len(reqs)
    with PV.Server(4 << 30) as srv:
        pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]

        def worker(k0):
            for k in range(k0, len(reqs), 3):
                j, beta, T = reqs[k]
                got[k] = srv.wait(srv.submit(pids[j], beta, T), 60000)

        ths = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    for g, w_ in zip(got, want):
        assert np.array_equal(g, w_)


def test_served_at_stream_sizes():
    """The served stream's sizes: terms up to 5e6, T up to 2048, 31- and
    63-bit primes, and a tenth of the requests for polynomials the server has
    not seen (registered just before, uploaded at admission, removed after).
    Every result equals the request run alone (stops at the first
    mismatch); a few small ones are checked by the oracle."""
    sizes = [5_000_000, 1_200_000, 300_000, 40_000, 3_000]
    rng = np.random.default_rng(11)
    pool = []
    for j, s in enumerate(sizes):
        n = int(rng.integers(4, 9))
        p = (W.P63, W.P31)[j % 2]
        pool.append(W.make_poly(int(rng.integers(0, 2**62)), p, n, s, 1, 40, W.raise_dr(s, n, 40, 20)))
    reqs = []
    for k in range(60):
        j = int(rng.integers(0, len(pool)))
        T = int(round(2 ** rng.uniform(6, 11)))
        beta = rng.integers(1, pool[j].p, size=pool[j].n - 2, dtype=np.uint64)
        fresh = rng.integers(0, pool[j].p, size=pool[j].s, dtype=np.uint64) if k % 10 == 3 else None
        reqs.append((j, beta, T, fresh))
    print("case served stream sizes:", [(w.s, w.n) for w in pool], flush=True)
    with PV.Server(64 << 30) as srv:
        pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]
        rids, new_ids = [], []
        for j, beta, T, fresh in reqs:
            pid = pids[j] if fresh is None else srv.add_poly(pool[j].p, pool[j].exps, fresh)
            rids.append(srv.submit(pid, beta, T))
            new_ids.append(None if fresh is None else pid)
        got = [srv.wait(r, 120000) for r in rids]
        for pid in new_ids:
            if pid is not None:
                srv.remove_poly(pid)
        st = srv.stats()
        print("stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    used = len({j for j, _, _, f in reqs if f is None})
    assert st["uploads"] >= used + sum(f is not None for *_, f in reqs)
    hs = [PV.Poly(w.p, w.exps, w.coeffs) for w in pool]
    try:
        for k, ((j, beta, T, fresh), g) in enumerate(zip(reqs, got)):
            if fresh is None:
                want = hs[j].run(beta, T)
            else:
                with PV.Poly(pool[j].p, pool[j].exps, fresh) as h:
                    want = h.run(beta, T)
            assert np.array_equal(g, want), f"request {k}: poly {j} (s={pool[j].s}) T={T} new={fresh is not None}"
    finally:
        for h in hs:
            h.destroy()
    orc = Oracle()
    checked = 0
    for k, (j, beta, T, fresh) in enumerate(reqs):
        w = pool[j]
        if w.s * T <= 2e7 and checked < 4:
            coeffs = w.coeffs if fresh is None else fresh
            assert np.array_equal(got[k].astype(np.uint64), orc.evaluate(w.p, w.exps, coeffs, beta, T, threads=8))
            checked += 1
    assert checked >= 2
