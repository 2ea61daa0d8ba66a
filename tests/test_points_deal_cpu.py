"""Host-only checks of the point mode's slot dealing (which term each thread
slot of the point kernel evaluates; paper Section 2.1, random points).

Any assignment of a group's terms to its own threads gives the same images
(the group's sum does not depend on the order), so the dealing must be a
bijection between the terms and the filled slots that keeps every term in
a thread of its own group.  It also exists to spread the kernel's LDS
gathers over the banks: the second test compares the bank conflicts of one
k's gathers with those of dealing the terms sorted by their table entries,
under the gfx950 bank model (4- and 8-byte gathers served per 32 lanes over
32 banks of 4-byte or 8-byte words, 16-byte gathers per 16 lanes).  The
tables have 4-byte entries for 32-bit residues, 16-byte ones for 64-bit."""
import numpy as np
import pytest

from paper_2004_11571_amd import peval as PV


def _groups(rng, n_small, n_mid, n_large):
    sizes = np.concatenate([rng.integers(1, 6, n_small), rng.integers(30, 81, n_mid),
                            rng.integers(500, 1201, n_large)])
    rng.shuffle(sizes)
    return sizes.astype(np.uint64)


def _thread_groups(sizes, K):
    lay = PV.layout(sizes, K, 8)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    g = np.searchsorted(off, lay["thr_first"].astype(np.int64), side="right") - 1
    g[lay["thr_cnt"] == 0] = -1  # padding threads
    return g, off


@pytest.mark.parametrize("w,K,deg", [(4, 16, 100), (4, 8, 100), (8, 16, 100), (4, 16, 30), (4, 1, 100)])
def test_dealing_is_a_bijection_within_groups(w, K, deg):
    rng = np.random.default_rng(7 + K + deg + w)
    sizes = _groups(rng, 60, 40, 12)
    s = int(sizes.sum())
    ex = rng.integers(0, deg + 1, (2, s)).astype(np.uint16)
    slots = PV.deal_points(w, ex, sizes, K)
    tg, off = _thread_groups(sizes, K)
    assert slots.shape == (K, tg.size)
    filled = slots != 0xFFFFFFFF
    terms = slots[filled]
    assert terms.size == s and np.array_equal(np.sort(terms), np.arange(s))
    term_group = np.searchsorted(off, terms.astype(np.int64), side="right") - 1
    thread_of_slot = np.broadcast_to(np.arange(tg.size), slots.shape)[filled]
    assert np.array_equal(term_group, tg[thread_of_slot])
    # a group of m terms on nt threads fills slots (k, t) with k nt + t < m
    for g in range(sizes.size):
        thr = np.flatnonzero(tg == g)
        m, nt = int(sizes[g]), thr.size
        want = np.zeros((K, nt), bool)
        for q in range(m):
            want[q // nt, q % nt] = True
        assert np.array_equal(filled[:, thr], want)


def _extra_cycles(slots, e0, e1, w):
    """Bank-conflict cycles beyond one pass, summed over every (wave, k)
    gather of the first factor's value and the last factor's entry: 4-byte
    entries for 32-bit residues (both gathers: entry e in bank e mod 32),
    16-byte (value, quotient) entries for 64-bit ones (the value: 8-byte
    word 2e mod 32; the whole entry: e mod 16, per 16 lanes)."""
    K, NT = slots.shape
    lanes1, banks1 = (32, 32) if w == 4 else (16, 16)
    scale0 = 1 if w == 4 else 2
    tot = 0
    for k in range(K):
        for w0 in range(0, NT, 64):
            row = slots[k, w0:w0 + 64]
            for a in range(0, 64, 32):   # first factor's value, 32 banks per 32 lanes
                t = row[a:a + 32]
                t = t[t != 0xFFFFFFFF]
                if t.size:
                    words = np.unique(scale0 * e0[t])
                    tot += np.bincount(words % 32).max() - 1
            for a in range(0, 64, lanes1):  # last factor: whole entries
                t = row[a:a + lanes1]
                t = t[t != 0xFFFFFFFF]
                if t.size:
                    ent = np.unique(e1[t])
                    tot += np.bincount(ent % banks1).max() - 1
    return tot


@pytest.mark.parametrize("w", [4, 8])
def test_dealing_spreads_the_gathers_over_banks(w):
    rng = np.random.default_rng(11 + w)
    sizes = _groups(rng, 20, 20, 24)
    s = int(sizes.sum())
    deg = 100
    ex = rng.integers(0, deg + 1, (2, s)).astype(np.uint16)
    nf, E = PV.points_factors(w, [deg, deg])
    assert nf == 2 and E >= 2 * (deg + 1)  # x3 in the first table, x4 in the second
    e0 = ex[0].astype(np.int64)
    e1 = (deg + 1) + ex[1].astype(np.int64)
    K = 16
    slots = PV.deal_points(w, ex, sizes, K)
    # reference: each group's terms sorted by (first, last) entry, dealt k-major
    tg, off = _thread_groups(sizes, K)
    ref = np.full_like(slots, 0xFFFFFFFF)
    for g in range(sizes.size):
        thr = np.flatnonzero(tg == g)
        idx = np.arange(off[g], off[g + 1])
        idx = idx[np.lexsort((e1[idx], e0[idx]))]
        for q, i in enumerate(idx):
            ref[q // thr.size, thr[q % thr.size]] = i
    new, old = _extra_cycles(slots, e0, e1, w), _extra_cycles(ref, e0, e1, w)
    assert new <= 0.5 * old, (new, old)
