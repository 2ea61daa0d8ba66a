"""Autotuner: picks a valid tuning, the cache steers later runs, results unchanged."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_and_cache(tmp_path):
    orc = Oracle()
    PV.tune_clear()
    w = W.make_poly(W.workload_seed(2, 7), W.P63, 6, 20000, 64, 40, 20)
    with PV.Poly(w.p, w.exps, w.coeffs) as q:
        heur = q.get_tuning(w.T)
        K, P, C, ms = q.autotune(w.beta, w.T)
        print("heuristic", heur, "tuned", (K, P, C), ms, flush=True)
        assert K in (1, 2, 4, 8, 16) and P in (8, 16, 32) and 1 <= C <= w.T and ms > 0
        assert q.get_tuning(w.T) == (K, P, C)
        got = q.run(w.beta, w.T)
    want = orc.evaluate(w.p, w.exps, w.coeffs, w.beta, w.T, threads=8)
    assert np.array_equal(got, want)
    path = str(tmp_path / "tune.txt")
    PV.tune_save(path)
    PV.tune_clear()
    with PV.Poly(w.p, w.exps, w.coeffs) as q:
        assert q.get_tuning(w.T) == heur
        PV.tune_load(path)
        assert q.get_tuning(w.T) == (K, P, C)
    PV.tune_clear()


def test_autotune_exhaustive_small(tmp_path):
    """A run small enough for the single-launch path: the autotuner times it
    too, and its choice (K = P = C = 0 for that path) survives save / load."""
    PV.tune_clear()
    w = W.n4_s1e3_p31_T64()
    with PV.Poly(w.p, w.exps, w.coeffs) as q:
        assert q.get_tuning(w.T) == (0, 0, 0)
        K, P, C, ms = q.autotune(w.beta, w.T, exhaustive=True)
        print("tuned", (K, P, C), ms, flush=True)
        assert ms > 0
        assert (K, P, C) == (0, 0, 0) or (K in (1, 2, 4, 8, 16) and P in (8, 16, 32) and C >= 1)
        assert q.get_tuning(w.T) == (K, P, C)
        assert np.array_equal(q.run(w.beta, w.T), Oracle().evaluate(w.p, w.exps, w.coeffs, w.beta, w.T))
        path = str(tmp_path / "tune.txt")
        PV.tune_save(path)
        PV.tune_clear()
        PV.tune_load(path)
        assert q.get_tuning(w.T) == (K, P, C)
    PV.tune_clear()


@pytest.mark.parametrize("exhaustive", [False, True])
def test_autotune_fp64_product(exhaustive):
    """A modulus below 2^50 takes the FP64 product by default, whose kernels
    exist only for K <= 8: the autotuner keeps to those and the result stays
    exact."""
    PV.tune_clear()
    w = W.make_poly(W.workload_seed(2, 8), W.P50, 6, 30000, 48, 40, 20)
    with PV.Poly(w.p, w.exps, w.coeffs) as q:
        assert q.arith() == "fp64"
        K, P, C, ms = q.autotune(w.beta, w.T, exhaustive=exhaustive)
        print("fp64 tuned", (K, P, C), ms, flush=True)
        assert ms > 0
        assert (K, P, C) == (0, 0, 0) or K <= 8
        got = q.run(w.beta, w.T)
    assert np.array_equal(got, Oracle().evaluate(w.p, w.exps, w.coeffs, w.beta, w.T, threads=8))
    PV.tune_clear()
