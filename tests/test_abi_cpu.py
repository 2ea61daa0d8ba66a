"""The C-ABI library on the CPU: symbols, argument validation, host layout.

No compute call is made here (there is no GPU in the build container);
argument validation happens before any device call, so it is testable."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2004_11571_amd import peval as PV

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(peval_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert "peval_create" in syms and "peval_run" in syms and "peval_destroy" in syms
    L = ctypes.CDLL(PV.LIB_PATH)
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing


@pytest.mark.parametrize("p,n,why", [
    (2, 4, "even p"), (1, 4, "p < 3"), ((1 << 63) + 1, 4, "p >= 2^63"), (10, 4, "even p"),
    (101, 1, "n < 2"), (101, 33, "n > 32"),
])
def test_create_rejects_bad_arguments(p, n, why):
    L = PV.lib()
    exps = np.zeros((1, max(n, 1)), np.uint32)
    co = np.ones(1, np.uint64)
    h = ctypes.c_void_p()
    rc = L.peval_create(p % (1 << 64), n, 1, exps.ctypes.data, co.ctypes.data, ctypes.byref(h))
    assert rc == PV.EINVAL, why
    assert h.value is None
    assert L.peval_last_error().decode()


def test_create_rejects_large_tail_exponent():
    L = PV.lib()
    exps = np.asarray([[0, 0, 65536]], np.uint32)
    co = np.ones(1, np.uint64)
    h = ctypes.c_void_p()
    assert L.peval_create(101, 3, 1, exps.ctypes.data, co.ctypes.data, ctypes.byref(h)) == PV.EUNSUPPORTED


def test_null_arguments():
    L = PV.lib()
    h = ctypes.c_void_p()
    assert L.peval_create(101, 3, 5, None, None, ctypes.byref(h)) == PV.EINVAL
    assert L.peval_create(101, 3, 0, None, None, None) == PV.EINVAL
    assert L.peval_run(None, None, 4, None) == PV.EINVAL
    assert L.peval_run_async(None, None, 1, 4, None, None) == PV.EINVAL
    assert L.peval_info(None, None) == PV.EINVAL
    assert L.peval_destroy(None) == PV.OK
    assert L.peval_set_tuning(None, 0, 0, 0) == PV.EINVAL
    assert L.peval_strerror(PV.EINVAL) == b"invalid argument"


def _check_layout(sizes, K, P):
    lay = PV.layout(sizes, K, P)
    NT, NW = lay["NT"], lay["NW"]
    assert NT % 64 == 0 and NW * 64 == NT
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    # every term is covered exactly once, runs of <= K terms inside one group
    covered = np.zeros(int(off[-1]), np.int64)
    grp_of_thread = np.full(NT, -1)
    for j in range(NT):
        c = int(lay["thr_cnt"][j])
        if c == 0:
            continue
        f = int(lay["thr_first"][j])
        assert 1 <= c <= K
        g = int(np.searchsorted(off, f, side="right") - 1)
        assert f + c <= off[g + 1]
        covered[f:f + c] += 1
        grp_of_thread[j] = g
    assert (covered == 1).all()
    # threads of a group are contiguous and in group order
    real = grp_of_thread[grp_of_thread >= 0]
    assert (np.diff(real) >= 0).all()
    # segment ends: group boundaries and wave ends; slots per group contiguous
    slots = []
    last = -1
    for w in range(NW):
        assert int(lay["slot_base"][w]) == len(slots)
        m = int(lay["endmask"][w])
        for l in range(64):
            j = w * 64 + l
            g = grp_of_thread[j] if grp_of_thread[j] >= 0 else len(sizes) - 1
            last = g
            if (m >> l) & 1:
                slots.append(g)
            if l == 63:
                assert (m >> l) & 1          # a segment never leaves its wave open
            elif (m >> l) & 1:
                g2 = grp_of_thread[j + 1] if grp_of_thread[j + 1] >= 0 else len(sizes) - 1
                assert g2 != g                # only group changes end a segment inside a wave
            if j + 1 < NT:
                g2 = grp_of_thread[j + 1] if grp_of_thread[j + 1] >= 0 else len(sizes) - 1
                if g2 != g:
                    assert (m >> l) & 1
    assert len(slots) == lay["nslots"]
    so = lay["slot_off"]
    for g in range(len(sizes)):
        assert all(s == g for s in slots[so[g]:so[g + 1]])
        assert so[g + 1] > so[g]
    assert so[-1] == len(slots)


@pytest.mark.parametrize("K", [1, 2, 4, 8, 16, 32])
@pytest.mark.parametrize("P", [8, 16, 32])
def test_layout_invariants(K, P):
    rng = np.random.default_rng(K * 100 + P)
    sizes = np.concatenate([rng.integers(1, 5, 40), rng.integers(50, 400, 6), [1, 1, 1000]])
    _check_layout(sizes, K, P)


def test_layout_edges():
    _check_layout(np.asarray([1]), 8, 16)
    _check_layout(np.asarray([64 * 8]), 8, 16)
    _check_layout(np.asarray([1] * 130), 1, 32)
    with pytest.raises(PV.PevalError):
        PV.layout(np.asarray([3, 0, 2]), 4, 16)
    with pytest.raises(PV.PevalError):
        PV.layout(np.asarray([3]), 3, 16)


def test_tune_file_validation(tmp_path):
    bad = tmp_path / "bad.txt"
    bad.write_text("8 10 4 20 3 16 5 0.1\n")  # K = 3 is not a kernel
    with pytest.raises(PV.PevalError):
        PV.tune_load(str(bad))
    for partial in ("8 10 4 20 0 16 5 0.1\n", "8 10 4 20 0 0 5 0.1\n", "8 10 4 20 8 16 0 0.1\n"):
        bad.write_text(partial)  # only K = P = C = 0 together (the single-launch path) is valid
        with pytest.raises(PV.PevalError):
            PV.tune_load(str(bad))
    good = tmp_path / "good.txt"
    good.write_text("# comment\n8 10 4 20 8 16 5 0.1\n4 6 2 12 1 8 64 0.02\n4 19 7 12 0 0 0 0.01\n")
    PV.tune_load(str(good))
    out = tmp_path / "out.txt"
    PV.tune_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 3
    assert "4 19 7 12 0 0 0 0.010000" in lines
    PV.tune_clear()
    PV.tune_save(str(out))
    assert [l for l in out.read_text().splitlines() if not l.startswith("#")] == []


def test_batch_rejects_bad_arguments():
    L = PV.lib()
    b = ctypes.c_void_p()
    assert L.peval_batch_create(0, None, None, 0, ctypes.byref(b)) == PV.EINVAL
    assert L.peval_batch_run(None, None, None, None, None) == PV.EINVAL
    assert L.peval_batch_destroy(None) == PV.OK
    assert L.peval_batch_kinds(None, None, None) == PV.EINVAL


# --- point mode: factor-table planner (host only) ---------------------------

@pytest.mark.parametrize("w,maxdeg,want", [
    (8, [20, 20, 20, 20], (2, 882)),            # 1e6-term shape: two tables of 21 x 21
    (8, [30] * 6, (4, 1984)),                   # 1e7-term shape: 31^2, 31^2, 31, 31
    (8, [10] * 4, (2, 242)),                    # Table 2 shape: 11^2 + 11^2
    (4, [30] * 6, (3, 2884)),                   # 32-bit residues: twice the entries fit (3 x 961, padded to 4)
    (8, [100, 100, 100], (3, 304)),             # 101 + 101 + 101, padded to even
    (8, [65535], (2, 512)),                     # split into two base-256 digits
    (8, [300], (1, 512)),                       # digits of radix 256 and 2 in one table
    (8, [0, 0, 0], (1, 2)),                     # no tail variable occurs: one entry, 1
    (8, [], (1, 2)),                            # n = 2
])
def test_points_factor_plans(w, maxdeg, want):
    nf, E = PV.points_factors(w, maxdeg)
    assert nf == want[0]
    # every plan fits one point's tables in 32 KiB of LDS (entries of 2w
    # bytes at most), in whole 16-byte pieces (4-byte entries for w = 4,
    # 16-byte ones for w = 8)
    assert E * 2 * w <= 32768 and E % (4 if w == 4 else 2) == 0
    if want[1] is not None:
        assert E == want[1]


def test_points_factor_plan_unsupported():
    with pytest.raises(PV.PevalError) as ei:
        PV.points_factors(8, [10] * 30)
    assert ei.value.code == PV.EUNSUPPORTED


def test_points_factor_plan_bad_arguments():
    for w, d in ((5, [3]), (8, [70000])):
        with pytest.raises(PV.PevalError) as ei:
            PV.points_factors(w, d)
        assert ei.value.code == PV.EINVAL
    L = PV.lib()
    assert L.peval_run_points(None, None, 1, None) == PV.EINVAL
    assert L.peval_run_points_async(None, None, 1, None, None) == PV.EINVAL
    assert L.peval_points_tuning(None, 1, None, None, None) == PV.EINVAL


def test_interpolate_null_arguments():
    L = PV.lib()
    assert L.peval_interpolate(None, None, 1, None, None) == PV.EINVAL
    assert L.peval_interpolate_async(None, None, 1, None, None, None, None) == PV.EINVAL
    assert L.peval_strerror(PV.ESINGULAR) == b"singular system"


def test_testing_entries_validate_before_any_device_call():
    L = PV.lib()
    top_mul32, top_alg2, top_pm63 = 16, 8, 12
    assert L.peval_test_arith(top_mul32, (1 << 31) + 11, 0, None, None, None, None) == PV.EINVAL
    assert L.peval_test_arith(top_alg2, (1 << 50) + 1, 0, None, None, None, None) == PV.EINVAL
    assert L.peval_test_arith(top_alg2, (1 << 31) - 1, 0, None, None, None, None) == PV.EINVAL
    assert L.peval_test_arith(top_pm63, (1 << 63) - (1 << 21) + 1, 0, None, None, None, None) == PV.EINVAL
    assert L.peval_test_arith(99, 101, 0, None, None, None, None) == PV.EINVAL
    assert L.peval_test_arith(0, 101, 5, None, None, None, None) == PV.EINVAL   # null arrays
    assert L.peval_test_arith(0, 101, 0, None, None, None, None) == PV.OK       # empty: nothing to do
    ms, work = ctypes.c_double(), ctypes.c_double()
    assert L.peval_bench_product(7, 101, 1, 1, ctypes.byref(ms), ctypes.byref(work)) == PV.EINVAL
    assert L.peval_bench_product(0, 100, 1, 1, ctypes.byref(ms), ctypes.byref(work)) == PV.EINVAL
    assert L.peval_bench_product(1, (1 << 31) + 11, 1, 1, ctypes.byref(ms), ctypes.byref(work)) == PV.EINVAL
    assert L.peval_bench_product(16, 0, 0, 1, ctypes.byref(ms), ctypes.byref(work)) == PV.EINVAL
