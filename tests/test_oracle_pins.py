"""The CPU oracle against pins that do not reuse its formula (see oracle_pins)."""
import pytest

import oracle_pins as P
from oracle import Oracle


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_entry_matches_table(orc):
    import numpy as np
    from paper_2004_11571_amd import workloads as W
    rng = np.random.default_rng(11)
    poly = W.random_small(rng, W.P63, 6, 50, 6, dmax=3, allow_dup=True)
    out = orc.evaluate(W.P63, poly.exps, poly.coeffs, poly.beta, 6)
    gd, ge = orc.groups(poly.exps)
    for t in range(1, 7):
        for g in range(len(gd)):
            assert orc.entry(W.P63, poly.exps, poly.coeffs, poly.beta, t, int(gd[g]), int(ge[g])) == int(out[t - 1, g])
    assert orc.entry(W.P63, poly.exps, poly.coeffs, poly.beta, 1, 999, 999) == 0


def test_threads_do_not_change_result(orc):
    import numpy as np
    from paper_2004_11571_amd import workloads as W
    rng = np.random.default_rng(12)
    poly = W.random_small(rng, W.P31, 5, 80, 13, dmax=4)
    a = orc.evaluate(W.P31, poly.exps, poly.coeffs, poly.beta, 13, threads=1)
    b = orc.evaluate(W.P31, poly.exps, poly.coeffs, poly.beta, 13, threads=4)
    assert np.array_equal(a, b)


def test_unreduced_inputs(orc):
    """Coefficients and base point are taken modulo p on entry."""
    import numpy as np
    from paper_2004_11571_amd import workloads as W
    rng = np.random.default_rng(13)
    p = 1000003
    poly = W.random_small(rng, p, 4, 20, 4, dmax=3)
    base = orc.evaluate(p, poly.exps, poly.coeffs, poly.beta, 4)
    big_c = poly.coeffs + np.uint64(p) * np.uint64(5)
    big_b = poly.beta + np.uint64(p) * np.uint64(3)
    assert np.array_equal(orc.evaluate(p, poly.exps, big_c, big_b, 4), base)
