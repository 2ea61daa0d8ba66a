"""The device modular arithmetic of the evaluation kernels, element by
element, against exact Python integers (paper, Section 3.1: the modular
product of Alg. 2 and the sums of Alg. 3, and the integer Shoup products
used in their place on gfx950).

Each operation runs through the test-only C-ABI entry ``peval_test_arith``
on 2^20 random operand pairs plus the edge operands 0, 1, 2, (p-1)/2,
(p+1)/2, p-2, p-1 and 2^32-1, 2^32, 2^32+1 (reduced), for the moduli 3,
2^31-1, 2^31+11, 2^50-27, a 50-bit modulus whose double reciprocal lies
well below 1/p, 2^63-25 and an odd composite.  Integer results must be
exactly the defined value: canonical residues, the Shoup quotient, and for
the lazy product the exact remainder a b - floor(a wq / 2^k) p of Shoup's
method; the FP64 product must be congruent and within the range its
no-correction argument claims."""
import numpy as np
import pytest

from paper_2004_11571_amd import peval as PV

pytestmark = pytest.mark.gpu

P_LOW_RECIP = 1123934916484611
P_COMPOSITE = 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23 * 29 * 31 * 37 * 41 * 43 * 47   # odd, < 2^63
MODULI_64 = [3, (1 << 31) - 1, (1 << 31) + 11, (1 << 50) - 27, P_LOW_RECIP, (1 << 63) - 25, P_COMPOSITE]
MODULI_32 = [3, 97, 65537, (1 << 31) - 1, P_COMPOSITE % (1 << 31) | 1]
MODULI_F64 = [(1 << 31) + 11, (1 << 40) - 87, (1 << 50) - 27, (1 << 50) - 1, P_LOW_RECIP]
N_RANDOM = 1 << 20
M64 = 1 << 64


def _say(*a):
    print(*a, flush=True)


def _edges(p):
    vals = [0, 1, 2, (p - 1) // 2, (p + 1) // 2, p - 2, p - 1, (M64 >> 32) - 1, M64 >> 32, (M64 >> 32) + 1]
    return sorted({v % p for v in vals})


def _operands(p, seed, lazy_a=False, bits_a=64):
    """Random canonical pairs plus every pair of edge operands.  lazy_a:
    the left operand may be any word of bits_a bits (the lazy product's
    input), with the lazy edges 2p-1 and 2^bits_a - 1 added."""
    rng = np.random.default_rng(seed)
    hi = min(p, M64 - 1)
    a = rng.integers(0, hi, size=N_RANDOM, dtype=np.uint64)
    b = rng.integers(0, hi, size=N_RANDOM, dtype=np.uint64)
    ea = _edges(p)
    if lazy_a:
        a[: N_RANDOM // 2] = rng.integers(0, (1 << bits_a) - 1, size=N_RANDOM // 2, dtype=np.uint64,
                                          endpoint=True)
        ea = ea + [2 * p - 1, (1 << bits_a) - 1]
    eb = _edges(p)
    ga, gb = np.meshgrid(np.array(ea, dtype=np.uint64), np.array(eb, dtype=np.uint64))
    return np.concatenate([a, ga.ravel()]), np.concatenate([b, gb.ravel()])


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).to("cuda")


def _run(op, p, a, b=None, count=None):
    import torch
    L = PV.lib()
    da = _dev(a)
    db = _dev(b) if b is not None else None
    n = count if count is not None else len(a)
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    rc = L.peval_test_arith(op, p, n, da.data_ptr(), db.data_ptr() if db is not None else None,
                            out.data_ptr(), None)
    PV._check(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def _objs(x):
    return np.array([int(v) for v in x], dtype=object)


def _mismatch(got, want, a, b=None):
    bad = np.nonzero(got != want)[0]
    if bad.size == 0:
        return None
    i = int(bad[0])
    return f"{bad.size} mismatches; first a={int(a[i])} b={int(b[i]) if b is not None else None} " \
           f"got={got[i]} want={want[i]}"


OPS = {"MUL64": 0, "QUOT64": 1, "SHOUP64": 2, "REDUCE96": 3, "POW64": 4, "SUM64": 5, "FOLD96": 6, "ALG2": 8, "FOLD": 9,
       "CANON_F64": 10, "PM63": 12, "PM31": 13, "MUL32": 16, "QUOT32": 17, "SHOUP32": 18, "REDUCE64_32": 19,
       "POW32": 20, "SUM32": 21, "MONT32": 22}


@pytest.mark.parametrize("p", MODULI_64)
def test_mul_quot_shoup_64(p):
    _say(f"case 64-bit products p={p}")
    a, b = _operands(p, p % 9973)
    A, B = _objs(a), _objs(b)
    got = _run(OPS["MUL64"], p, a, b)
    assert (err := _mismatch(_objs(got), A * B % p, a, b)) is None, err
    got = _run(OPS["QUOT64"], p, b)
    wq = (B * M64) // p
    assert (err := _mismatch(_objs(got), wq, b)) is None, err
    # lazy product: any 64-bit left operand; the exact Shoup remainder
    la, lb = _operands(p, p % 9973 + 1, lazy_a=True)
    LA, LB = _objs(la), _objs(lb)
    lwq = (LB * M64) // p
    want = LA * LB - ((LA * lwq) >> 64) * p
    got = _objs(_run(OPS["SHOUP64"], p, la, lb))
    assert (err := _mismatch(got, want, la, lb)) is None, err
    assert all(int(g) < 2 * p for g in got)


@pytest.mark.parametrize("p", MODULI_64)
def test_reduce96_pow_sum_64(p):
    _say(f"case 64-bit reductions p={p}")
    rng = np.random.default_rng(p % 7919)
    lo = rng.integers(0, M64 - 1, size=N_RANDOM, dtype=np.uint64, endpoint=True)
    hi = rng.integers(0, 1 << 32, size=N_RANDOM, dtype=np.uint64)
    lo[:4] = [0, M64 - 1, M64 - 1, p - 1]
    hi[:4] = [0, (1 << 32) - 1, 0, (1 << 32) - 1]
    got = _objs(_run(OPS["REDUCE96"], p, lo, hi))
    want = (_objs(hi) * M64 + _objs(lo)) % p
    assert (err := _mismatch(got, want, lo, hi)) is None, err
    # the partial coefficients' fold: congruent, any 64-bit word (the output
    # array holds 64 bits, so only congruence is left to check)
    got = _objs(_run(OPS["FOLD96"], p, lo, hi))
    assert (err := _mismatch(got % p, want, lo, hi)) is None, err
    # powers: bases canonical, exponents up to 2^64 - 1 (and 0: 0^0 = 1)
    n = 1 << 14
    base = rng.integers(0, p, size=n, dtype=np.uint64)
    ex = rng.integers(0, M64 - 1, size=n, dtype=np.uint64, endpoint=True)
    ex[: n // 2] %= np.uint64(5000)
    base[:6] = [0, 0, 1, p - 1, p - 1, 2 % p]
    ex[:6] = [0, 7, M64 - 1, M64 - 1, 2, 64]
    got = _objs(_run(OPS["POW64"], p, base, ex))
    want = np.array([pow(int(x), int(e), p) for x, e in zip(base, ex)], dtype=object)
    assert (err := _mismatch(got, want, base, ex)) is None, err
    # the evaluation kernel's sums of 16 lazy values (any 64-bit words)
    m = N_RANDOM // 16
    vals = rng.integers(0, M64 - 1, size=16 * m, dtype=np.uint64, endpoint=True)
    vals[:16] = M64 - 1
    vals[16:32] = 0
    got = _objs(_run(OPS["SUM64"], p, vals, None, count=m))
    want = _objs(vals).reshape(m, 16).sum(axis=1) % p
    assert (err := _mismatch(got, want, vals[::16])) is None, err


@pytest.mark.parametrize("p", MODULI_32)
def test_products_and_sums_32(p):
    _say(f"case 32-bit p={p}")
    a, b = _operands(p, p % 9967)
    got = _run(OPS["MUL32"], p, a, b)
    assert (err := _mismatch(got, (a * b) % np.uint64(p), a, b)) is None, err
    got = _run(OPS["QUOT32"], p, b)
    assert (err := _mismatch(got, (b << np.uint64(32)) // np.uint64(p), b)) is None, err
    la, lb = _operands(p, p % 9967 + 1, lazy_a=True, bits_a=32)
    lwq = (lb << np.uint64(32)) // np.uint64(p)
    want = (la * lb - ((la * lwq) >> np.uint64(32)) * np.uint64(p)) % np.uint64(1 << 32)  # exact: < 2p
    got = _run(OPS["SHOUP32"], p, la, lb)
    assert (err := _mismatch(got, want, la, lb)) is None, err
    assert (got < 2 * p).all()
    rng = np.random.default_rng(p)
    v = rng.integers(0, M64 - 1, size=N_RANDOM, dtype=np.uint64, endpoint=True)
    v[:2] = [0, M64 - 1]
    got = _objs(_run(OPS["REDUCE64_32"], p, v))
    assert (err := _mismatch(got, _objs(v) % p, v)) is None, err
    base = rng.integers(0, p, size=1 << 14, dtype=np.uint64)
    ex = rng.integers(0, M64 - 1, size=1 << 14, dtype=np.uint64, endpoint=True)
    base[:3] = [0, 0, p - 1]
    ex[:3] = [0, 5, M64 - 1]
    got = _objs(_run(OPS["POW32"], p, base, ex))
    want = np.array([pow(int(x), int(e), p) for x, e in zip(base, ex)], dtype=object)
    assert (err := _mismatch(got, want, base, ex)) is None, err
    m = N_RANDOM // 16
    vals = rng.integers(0, 1 << 32, size=16 * m, dtype=np.uint64)
    vals[:16] = (1 << 32) - 1
    got = _objs(_run(OPS["SUM32"], p, vals, None, count=m))
    want = _objs(vals).reshape(m, 16).sum(axis=1) % p
    assert (err := _mismatch(got, want, vals[::16])) is None, err
    # Montgomery's product: any a < 2p by any b < p gives a value below 2p
    # congruent to a b 2^-32 (edge operands first)
    ma = rng.integers(0, 2 * p, size=N_RANDOM, dtype=np.uint64)
    mb = rng.integers(0, p, size=N_RANDOM, dtype=np.uint64)
    ma[:6] = [0, 1, p - 1, p, 2 * p - 1, 2 * p - 1]
    mb[:6] = [p - 1, p - 1, p - 1, 1, p - 1, 0]
    got = _objs(_run(OPS["MONT32"], p, ma, mb))
    rinv = pow(1 << 32, -1, p)
    want = (_objs(ma) * _objs(mb) * rinv) % p
    assert (err := _mismatch(got % p, want, ma, mb)) is None, err
    assert all(int(g) < 2 * p for g in got)


def _signed(x):
    return np.array([int(v) - M64 if int(v) >> 63 else int(v) for v in x], dtype=object)


@pytest.mark.parametrize("p", MODULI_F64)
def test_fp64_product_fold_and_conversion(p):
    _say(f"case FP64 product p={p}")
    rng = np.random.default_rng(p % 9931)
    # left operand signed, |x| < p (the running values of the FP64 loop)
    xs = rng.integers(-(p - 1), p - 1, size=N_RANDOM, dtype=np.int64, endpoint=True)
    ys = rng.integers(0, p, size=N_RANDOM, dtype=np.uint64)
    edge_x = [0, 1, -1, p - 1, -(p - 1), (p - 1) // 2, -((p - 1) // 2), p - 2, -(p - 2)]
    edge_y = [0, 1, 2, p - 1, p - 2, (p - 1) // 2, (p + 1) // 2]
    gx, gy = np.meshgrid(np.array(edge_x, np.int64), np.array(edge_y, np.uint64))
    xs = np.concatenate([xs, gx.ravel()])
    ys = np.concatenate([ys, gy.ravel()])
    got = _signed(_run(OPS["ALG2"], p, xs.view(np.uint64), ys))
    X, Y = _objs(xs), _objs(ys)
    assert ((got - X * Y) % p == 0).all(), "FP64 product not congruent"
    worst = max(abs(int(g)) for g in got)
    assert 8 * worst < 7 * p, f"|g| = {worst} beyond 7p/8"
    # folds of exact sums below 2^53 (up to eight running values and more)
    s = rng.integers(-(1 << 53) + 1, (1 << 53) - 1, size=N_RANDOM, dtype=np.int64)
    s[:6] = [0, (1 << 53) - 1, -(1 << 53) + 1, p, -p, 8 * (p - 1)]
    got = _signed(_run(OPS["FOLD"], p, s.view(np.uint64)))
    S = _objs(s)
    assert ((got - S) % p == 0).all(), "fold not congruent"
    assert max(abs(int(g)) for g in got) < p
    # conversion of a signed value in (-p, p) to its canonical residue
    got = _objs(_run(OPS["CANON_F64"], p, xs.view(np.uint64)))
    assert (err := _mismatch(got, X % p, xs)) is None, err


@pytest.mark.parametrize("p", [(1 << 63) - 25, (1 << 63) - 1, (1 << 63) - (1 << 20) + 1])
def test_pseudo_mersenne_63(p):
    _say(f"case pseudo-Mersenne p={p}")
    a, b = _operands(p, p % 9901, lazy_a=True)
    got = _objs(_run(OPS["PM63"], p, a, b))
    A, B = _objs(a), _objs(b)
    assert ((got - A * B) % p == 0).all()
    assert all(int(g) < 2 * p for g in got)


@pytest.mark.parametrize("p", [(1 << 31) - 1, (1 << 31) - 4095, (1 << 31) - 19])
def test_pseudo_mersenne_31(p):
    _say(f"case pseudo-Mersenne p={p}")
    a, b = _operands(p, p % 9901, lazy_a=True, bits_a=32)
    got = _run(OPS["PM31"], p, a, b)
    assert ((got.astype(object) - _objs(a) * _objs(b)) % p == 0).all()
    assert (got < 2 * p).all()
