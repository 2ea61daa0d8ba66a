"""Seeded synthetic workloads for partial modular evaluation.

This module only draws random inputs (exponent vectors, coefficients, base
points, arrival times).  It holds none of the evaluation arithmetic, so both
the CPU oracle and the HIP path can be fed from it without sharing any of the
method's computation.

Input model (paper, Section 2.3, Eq. (1)): a sparse polynomial
``f = sum_i a_i x1^{d_i} x2^{e_i} M_i(x3..xn)`` over F_p, given as ``s`` rows
of ``n`` exponents and ``s`` coefficients, plus a base point
``beta = (beta_3..beta_n)`` drawn uniformly from F_p \\ {0} (Section 2.1
picks non-zero beta at random) and a number of evaluations ``T``.

The paper's own workload (Section 2.3: s = 5e5, n = 6, degree <= 10 per
variable, T = 1e4) and its application polynomials (Section 2.2) are not
available as data; the configurations below are synthetic stand-ins with the
shapes of the target workloads.  Exponent distributions:

* x1, x2 exponents: independent, uniform in [0, D12];
* x3..xn exponents: uniform over {e : sum(e) <= Dr} (stars and bars), or
  per-variable uniform in [0, D] when ``per_var`` is set;
* all exponent vectors distinct (rejection of duplicates);
* coefficients uniform in [0, p); beta uniform in [1, p).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

P31 = (1 << 31) - 1          # 2^31 - 1
P63 = (1 << 63) - 25         # largest prime below 2^63
P50 = (1 << 50) - 27         # largest prime below 2^50

SEED_BASE = 2004115710


def workload_seed(stream: int, instance: int = 0) -> int:
    """Seed of one input stream (a workload shape or a draw of points) and instance."""
    return SEED_BASE + 1000 * stream + instance


@dataclasses.dataclass
class Poly:
    """One polynomial plus one evaluation request."""
    p: int
    n: int
    exps: np.ndarray        # (s, n) uint32, row i = exponents of x1..xn in term i
    coeffs: np.ndarray      # (s,) uint64, in [0, p)
    beta: np.ndarray        # (n-2,) uint64, in [1, p)
    T: int
    name: str = ""

    @property
    def s(self) -> int:
        return int(self.exps.shape[0])

    def term_evals(self) -> int:
        return self.s * self.T


def _monomial_space_tail(m: int, dr: int) -> int:
    """Number of exponent vectors of m variables with total degree <= dr."""
    return math.comb(dr + m, m)


def _draw_tail_total_degree(rng: np.random.Generator, rows: int, m: int, dr: int) -> np.ndarray:
    """Uniform draw over {e in N^m : sum(e) <= dr} (stars and bars).

    A sorted m-subset c_1 < ... < c_m of {1..dr+m} maps bijectively to such e
    via gaps e_1 = c_1 - 1, e_j = c_j - c_{j-1} - 1.
    """
    if m == 0:
        return np.zeros((rows, 0), dtype=np.uint32)
    out = np.empty((rows, m), dtype=np.int64)
    todo = np.arange(rows)
    while todo.size:
        c = rng.integers(1, dr + m + 1, size=(todo.size, m))
        c.sort(axis=1)
        ok = np.all(np.diff(c, axis=1) > 0, axis=1) if m > 1 else np.ones(todo.size, dtype=bool)
        good = todo[ok]
        cg = c[ok]
        gaps = np.empty_like(cg)
        gaps[:, 0] = cg[:, 0] - 1
        if m > 1:
            gaps[:, 1:] = np.diff(cg, axis=1) - 1
        out[good] = gaps
        todo = todo[~ok]
    return out.astype(np.uint32)


def _pack_keys(exps: np.ndarray) -> np.ndarray:
    """Injective row key for duplicate detection."""
    s, n = exps.shape
    bits = [max(1, int(exps[:, k].max()).bit_length()) if s else 1 for k in range(n)]
    if sum(bits) <= 64:
        key = np.zeros(s, dtype=np.uint64)
        shift = 0
        for k in range(n):
            key |= exps[:, k].astype(np.uint64) << np.uint64(shift)
            shift += bits[k]
        return key
    return np.ascontiguousarray(exps).view(np.dtype((np.void, 4 * n))).ravel()


def draw_exponents(rng: np.random.Generator, s: int, n: int, d12: int, dr: int,
                   per_var: bool = False) -> np.ndarray:
    """s distinct exponent rows of n variables."""
    if n < 2:
        raise ValueError("n >= 2 required")
    m = n - 2
    space = (d12 + 1) ** 2 * ((dr + 1) ** m if per_var else _monomial_space_tail(m, dr))
    if space < s:
        raise ValueError(f"monomial space {space} < s={s}")

    def draw(rows: int) -> np.ndarray:
        e12 = rng.integers(0, d12 + 1, size=(rows, 2)).astype(np.uint32)
        if per_var:
            tail = rng.integers(0, dr + 1, size=(rows, m)).astype(np.uint32)
        else:
            tail = _draw_tail_total_degree(rng, rows, m, dr)
        return np.concatenate([e12, tail], axis=1)

    exps = draw(s)
    for _ in range(200):
        keys = _pack_keys(exps)
        order = np.argsort(keys)           # any order among equal keys will do
        ks = keys[order]
        dup = np.zeros(s, dtype=bool)
        dup[order[1:][ks[1:] == ks[:-1]]] = True
        ndup = int(dup.sum())
        if ndup == 0:
            break
        exps = np.concatenate([exps[~dup], draw(ndup)], axis=0)
    else:  # pragma: no cover - only for pathologically dense spaces
        raise RuntimeError("could not draw distinct exponent rows")
    # present terms in random order: the library sorts them itself
    perm = rng.permutation(s)
    return np.ascontiguousarray(exps[perm])


def raise_dr(s: int, n: int, d12: int, dr: int) -> int:
    """Smallest tail-degree bound >= dr whose monomial space holds 2s rows."""
    m = n - 2
    while (d12 + 1) ** 2 * _monomial_space_tail(m, dr) < 2 * s:
        dr += 1
    return dr


def make_poly(seed: int, p: int, n: int, s: int, T: int, d12: int, dr: int,
              per_var: bool = False, name: str = "") -> Poly:
    rng = np.random.default_rng(seed)
    exps = draw_exponents(rng, s, n, d12, dr, per_var)
    coeffs = rng.integers(0, p, size=s, dtype=np.uint64)
    beta = rng.integers(1, p, size=n - 2, dtype=np.uint64)
    return Poly(p=p, n=n, exps=exps, coeffs=coeffs, beta=beta, T=T, name=name)


# ---------------------------------------------------------------------------
# Named workloads (each named for its shape)
# ---------------------------------------------------------------------------

def n4_s1e3_p31_T64(instance: int = 0) -> Poly:
    """n=4, 1000 distinct terms, every exponent uniform in [0,10], p=2^31-1, T=64."""
    return make_poly(workload_seed(1, instance), P31, 4, 1000, 64, 10, 10, per_var=True,
                     name="n4_s1e3_p31_T64")


def n6_s1e6_p63_T1024(instance: int = 0) -> Poly:
    """n=6, 1e6 distinct terms, x1,x2 degree <= 40, x3..x6 total degree <= 20,
    p=2^63-25, T=1024."""
    return make_poly(workload_seed(2, instance), P63, 6, 1_000_000, 1024, 40, 20,
                     name="n6_s1e6_p63_T1024")


def n6_s1e6_p31_T1024(instance: int = 0) -> Poly:
    """The 1e6-term shape of n6_s1e6_p63_T1024 with the 31-bit prime 2^31-1 (32-bit
    residues)."""
    return make_poly(workload_seed(2, 500 + instance), P31, 6, 1_000_000, 1024, 40, 20,
                     name="n6_s1e6_p31_T1024")


def paper_table2(instance: int = 0) -> Poly:
    """The paper's default workload (Section 2.3; timed in Table 2): n = 6
    (4 evaluated variables), 5e5 terms, degree <= 10 in each variable,
    T = 1e4 evaluations, 64-bit integers with a prime below 2^50 (the FP64
    product of Alg. 2 needs p <= 50 bits).  The exponent distribution is not
    given in the paper: per-variable uniform in [0, 10] here."""
    return make_poly(workload_seed(6, instance), P50, 6, 500_000, 10_000, 10, 10, per_var=True,
                     name="n6_s5e5_d10_p50_T1e4")


def n8_s1e7_p63_T4096(instance: int = 0) -> Poly:
    """n=8, 1e7 distinct terms, x1,x2 degree <= 60, x3..x8 total degree <= 30,
    p=2^63-25, T=4096."""
    return make_poly(workload_seed(4, instance), P63, 8, 10_000_000, 4096, 60, 30,
                     name="n8_s1e7_p63_T4096")


def uneven_batch(count: int = 256, instance: int = 0, s_max: float = 1e6,
                 t_log2: tuple = (5, 11), moduli: tuple = None) -> List[Poly]:
    """Uneven batch: n ~ U{4..8}, s log-uniform in [1e3, s_max], T log-uniform
    in [2^5, 2^11], p in {2^31-1, 2^63-25} with probability 1/2 each (or
    uniform over ``moduli`` when given)."""
    rng = np.random.default_rng(workload_seed(3, instance))
    polys = []
    for j in range(count):
        n = int(rng.integers(4, 9))
        s = int(round(10 ** rng.uniform(3, math.log10(s_max))))
        T = int(round(2 ** rng.uniform(*t_log2)))
        if moduli is None:
            p = P31 if rng.random() < 0.5 else P63
        else:
            p = int(moduli[min(int(rng.random() * len(moduli)), len(moduli) - 1)])
        dr = raise_dr(s, n, 40, 20)
        seed = int(rng.integers(0, 2**62))
        polys.append(make_poly(seed, p, n, s, T, 40, dr, name=f"batch{j}"))
    return polys


def random_points(poly: Poly, T: int = 0, instance: int = 0) -> np.ndarray:
    """T points (x3..xn) drawn uniformly from [1, p)^(n-2), for the point
    mode (Zippel's random points, Section 2.1); T defaults to poly.T."""
    rng = np.random.default_rng(workload_seed(7, instance))
    T = T or poly.T
    return rng.integers(1, poly.p, size=(T, poly.n - 2), dtype=np.uint64)


@dataclasses.dataclass
class Request:
    arrival_s: float
    poly_index: int         # index into the pool
    T: int
    beta: np.ndarray


def serve_stream(rate_per_s: float, duration_s: float, pool: List[Poly], instance: int = 0,
                 t_log2: tuple = (6, 11)) -> List[Request]:
    """Poisson arrivals; each request picks a polynomial from ``pool``
    uniformly, T log-uniform in 2^t_log2 and a fresh base point."""
    rng = np.random.default_rng(workload_seed(5, instance))
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        j = int(rng.integers(0, len(pool)))
        T = int(round(2 ** rng.uniform(*t_log2)))
        beta = rng.integers(1, pool[j].p, size=pool[j].n - 2, dtype=np.uint64)
        reqs.append(Request(arrival_s=t, poly_index=j, T=T, beta=beta))
    return reqs


def serve_new_polys(reqs: List[Request], pool: List[Poly], fraction: float = 0.1,
                    instance: int = 0) -> dict:
    """About ``fraction`` of the requests ask for a polynomial that the server
    has not seen before the stream: the exponent rows of the request's pool
    member with fresh coefficients, uniform in [0, p).  Returns
    {request index: coefficients}."""
    rng = np.random.default_rng(workload_seed(5, 200 + instance))
    out = {}
    for i, r in enumerate(reqs):
        if rng.random() < fraction:
            w = pool[r.poly_index]
            out[i] = rng.integers(0, w.p, size=w.s, dtype=np.uint64)
    return out


def serve_pool(count: int, instance: int = 0, s_max: float = 5e6) -> List[Poly]:
    """Polynomials for the served stream: n ~ U{4..8}, s log-uniform in
    [1e3, s_max], p in {2^31-1, 2^63-25}."""
    rng = np.random.default_rng(workload_seed(5, 100 + instance))
    pool = []
    for j in range(count):
        n = int(rng.integers(4, 9))
        s = int(round(10 ** rng.uniform(3, math.log10(s_max))))
        p = P31 if rng.random() < 0.5 else P63
        dr = raise_dr(s, n, 40, 20)
        seed = int(rng.integers(0, 2**62))
        pool.append(make_poly(seed, p, n, s, 64, 40, dr, name=f"pool{j}"))
    return pool


def random_small(rng: np.random.Generator, p: int, n: int, s: int, T: int,
                 dmax: int = 6, allow_dup: bool = False) -> Poly:
    """Small random polynomial for parity and edge-case tests (exponents
    uniform per variable in [0, dmax]; duplicates allowed on request)."""
    if allow_dup:
        exps = rng.integers(0, dmax + 1, size=(s, n)).astype(np.uint32)
    else:
        exps = draw_exponents(rng, s, n, dmax, dmax, per_var=True)
    coeffs = rng.integers(0, p, size=s, dtype=np.uint64) if s else np.zeros(0, np.uint64)
    beta = rng.integers(1, p, size=n - 2, dtype=np.uint64) if p > 2 else np.ones(n - 2, np.uint64)
    return Poly(p=p, n=n, exps=np.ascontiguousarray(exps), coeffs=coeffs, beta=beta, T=T)
