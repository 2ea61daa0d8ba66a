"""Server policy on the CPU (simulated executor: no device calls)."""
import time

import numpy as np
import pytest

from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W


def _poly(seed, s, n=5, p=W.P63):
    rng = np.random.default_rng(seed)
    return W.random_small(rng, p, n, s, 1, dmax=6)


def test_simulated_requests_complete_with_stats():
    with PV.Server(1 << 30, simulate=True) as srv:
        srv.configure(slice_work=1e6, sim_rate=1e9)
        pids = [srv.add_poly(q.p, q.exps, q.coeffs) for q in (_poly(1, 2000), _poly(2, 500, p=W.P31))]
        rids = [srv.submit(pids[j % 2], np.ones(3, np.uint64), 64 + 32 * j) for j in range(10)]
        for r in rids:
            srv.wait(r, 10000)
        st = srv.stats()
        assert st["completed"] == 10 and st["rejected"] == 0 and st["queued"] == 0
        assert st["term_evals"] == sum((2000 if j % 2 == 0 else 500) * (64 + 32 * j) for j in range(10))
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        assert st["passes"] >= 1


def test_request_larger_than_budget_is_refused():
    with PV.Server(2 << 20, simulate=True) as srv:
        q = _poly(3, 3000)
        pid = srv.add_poly(q.p, q.exps, q.coeffs)
        with pytest.raises(PV.PevalError) as e:
            srv.submit(pid, np.ones(3, np.uint64), 100000)
        assert e.value.code == PV.ENOMEM
        assert srv.stats()["rejected"] == 1


def test_small_budget_queues_but_completes_in_order():
    # each request's output is ~1 MB; a 4 MB budget holds only a few at once
    with PV.Server(4 << 20, simulate=True) as srv:
        srv.configure(slice_work=1e5, sim_rate=2e8)
        q = _poly(4, 1500)
        pid = srv.add_poly(q.p, q.exps, q.coeffs)
        G = len({(a, b) for a, b in q.exps[:, :2].tolist()})
        T = (1 << 20) // (8 * G)
        rids = [srv.submit(pid, np.ones(3, np.uint64), T) for _ in range(12)]
        peak_q = 0
        for _ in range(200):
            st = srv.stats()
            peak_q = max(peak_q, st["queued"])
            if st["completed"] == 12:
                break
            time.sleep(0.01)
        for r in rids:
            srv.wait(r, 20000)
        st = srv.stats()
        assert st["completed"] == 12 and peak_q > 0
        assert st["hbm_peak"] <= 4 << 20


def test_lru_eviction_and_remove():
    with PV.Server(6 << 20, simulate=True) as srv:
        srv.configure(slice_work=1e6, sim_rate=1e9)
        qs = [_poly(10 + j, 40000, n=6) for j in range(8)]   # ~0.85 MB resident each
        pids = [srv.add_poly(q.p, q.exps, q.coeffs) for q in qs]
        for pid in pids * 2:
            srv.wait(srv.submit(pid, np.ones(4, np.uint64), 8), 20000)
        st = srv.stats()
        assert st["completed"] == 16 and st["hbm_peak"] <= 6 << 20
        assert st["evictions"] >= 1 and st["uploads"] > 8   # re-uploaded after eviction
        srv.remove_poly(pids[0])
        with pytest.raises(PV.PevalError):
            srv.submit(pids[0], np.ones(4, np.uint64), 8)


def test_bad_arguments():
    with pytest.raises(PV.PevalError):
        PV.Server(100, simulate=True)
    with PV.Server(1 << 24, simulate=True) as srv:
        with pytest.raises(PV.PevalError):
            srv.add_poly(10, np.zeros((1, 3), np.uint32), np.ones(1, np.uint64))
        q = _poly(5, 10)
        pid = srv.add_poly(q.p, q.exps, q.coeffs)
        with pytest.raises(PV.PevalError):
            srv.submit(pid, np.ones(3, np.uint64), 0)
        with pytest.raises(PV.PevalError):
            srv.wait(12345, 10)


def test_completion_queue_order():
    with PV.Server(1 << 30, simulate=True) as srv:
        srv.configure(slice_work=1e9, sim_rate=1e8)
        big, small = _poly(20, 10000), _poly(21, 100)
        pb, ps = srv.add_poly(big.p, big.exps, big.coeffs), srv.add_poly(small.p, small.exps, small.coeffs)
        r_big = srv.submit(pb, np.ones(3, np.uint64), 500)      # ~0.1 s simulated
        r_small = [srv.submit(ps, np.ones(3, np.uint64), 16) for _ in range(5)]
        order = [srv.next_done(5000) for _ in range(6)]
        assert set(order) == {r_big, *r_small}
        for r in order:
            srv.release(r)
        with pytest.raises(PV.PevalError) as e:
            srv.next_done(10)
        assert e.value.code == PV.ETIMEOUT


def test_admission_never_evicts_its_own_polynomial():
    """A request that needs room must not evict the polynomial it is about to
    use (the budget check has already counted that polynomial as resident):
    a is resident and least recently used, b resident after it; the first
    request on a that does not fit beside b must evict b, not a."""
    budget = 6 << 20
    qa, qb = _poly(20, 40000, n=6), _poly(21, 40000, n=6)
    triggered = False
    T = 1 << 14
    while T >= 8 and not triggered:
        with PV.Server(budget, simulate=True) as srv:
            srv.configure(slice_work=1e6, sim_rate=1e9)
            pa, pb = srv.add_poly(qa.p, qa.exps, qa.coeffs), srv.add_poly(qb.p, qb.exps, qb.coeffs)
            srv.wait(srv.submit(pa, np.ones(4, np.uint64), 8), 20000)
            srv.wait(srv.submit(pb, np.ones(4, np.uint64), 8), 20000)
            try:
                rid = srv.submit(pa, np.ones(4, np.uint64), T)
            except PV.PevalError:      # larger than the budget even alone
                T //= 2
                continue
            srv.wait(rid, 20000)
            st = srv.stats()
            assert st["hbm_peak"] <= budget
            if st["evictions"]:
                triggered = True
                assert st["uploads"] == 2, st   # b was evicted; a was neither evicted nor uploaded again
        T //= 2
    assert triggered, "no request size needed an eviction"


def test_poly_info_reports_the_library_group_count():
    """The binding takes the output shape from the library (no second
    definition of the group count): G is the number of distinct (x1, x2)
    pairs, the width follows p, and nothing is resident before a request."""
    with PV.Server(1 << 30, simulate=True) as srv:
        for seed, p, s, n in ((11, W.P63, 3000, 6), (12, W.P31, 700, 4), (13, W.P50, 1, 3)):
            q = _poly(seed, s, n=n, p=p)
            pid = srv.add_poly(q.p, q.exps, q.coeffs)
            inf = srv.poly_info(pid)
            want_G = len(np.unique(q.exps[:, :2], axis=0))
            assert inf["G"] == want_G and srv._meta[pid] == (p, n, want_G)
            assert inf["s"] == s and inf["n"] == n and inf["p"] == p
            assert inf["elem_bytes"] == (4 if p < 2**31 else 8)
            assert inf["device_bytes"] == 0
            assert inf["max_exp"] == [int(x) for x in q.exps.max(axis=0)]
        with pytest.raises(PV.PevalError) as e:
            srv.poly_info(10**9)
        assert e.value.code == PV.EINVAL
