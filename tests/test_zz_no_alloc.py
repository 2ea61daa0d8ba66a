"""The allocation-free entry point (peval_run_async_noalloc) against
peval_run_async, element by element (bit-exact), through the C ABI."""
import numpy as np
import pytest

from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _buf(poly, T, fill=-1):
    import torch
    dt = torch.int64 if poly.elem_bytes == 8 else torch.int32
    return torch.full((T, max(poly.G, 1)), fill, dtype=dt, device="cuda")


def _host(poly, buf):
    return buf.cpu().numpy().view(poly.dtype)[:, :poly.G].copy()


def _reference(poly, beta, T, t0=1):
    import torch
    ref = _buf(poly, T, fill=0)
    poly.run_async(beta, T, ref, t0=t0, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    return _host(poly, ref)


def test_two_calls_in_a_row_second_smaller():
    """A larger run, then a smaller one on another handle, both through the
    fixed region (the second finds the first's leftovers there)."""
    import torch
    a = W.make_poly(W.workload_seed(9, 1), W.P63, 6, 200_000, 700, 40, 20)
    b = W.make_poly(W.workload_seed(9, 2), W.P63, 5, 20_000, 150, 40, 20)
    _say(f"case noalloc pair: s={a.s} T={a.T}, then s={b.s} T={b.T}")
    with PV.Poly(a.p, a.exps, a.coeffs) as pa, PV.Poly(b.p, b.exps, b.coeffs) as pb:
        ref_a = _reference(pa, a.beta, a.T)
        ref_b = _reference(pb, b.beta, b.T)
        got_a, got_b = _buf(pa, a.T), _buf(pb, b.T)
        st = torch.cuda.current_stream()
        pa.run_async_noalloc(a.beta, a.T, got_a, stream=st)
        pb.run_async_noalloc(b.beta, b.T, got_b, stream=st)
        torch.cuda.synchronize()
        assert np.array_equal(_host(pa, got_a), ref_a)
        assert np.array_equal(_host(pb, got_b), ref_b)
        # and again in the other order, starting past t = 1
        got_b2, got_a2 = _buf(pb, 40), _buf(pa, 64)
        pb.run_async_noalloc(b.beta, 40, got_b2, t0=77, stream=st)
        pa.run_async_noalloc(a.beta, 64, got_a2, t0=600, stream=st)
        torch.cuda.synchronize()
        assert np.array_equal(_host(pb, got_b2), ref_b[76:116])
        assert np.array_equal(_host(pa, got_a2), ref_a[599:663])


def test_region_limits_chains_and_chunks():
    """1e6 terms of 64-bit residues, T = 2048: the tuning's chains and the
    partial sums of the whole run do not fit the region at once, so the call
    takes fewer chains and several stretches of T."""
    import torch
    w = W.n6_s1e6_p63_T1024()
    T = 2048
    _say(f"case noalloc large: s={w.s} T={T}")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        K, P, C = poly.get_tuning(T)
        assert K and C > 1, (K, P, C)
        ref = _reference(poly, w.beta, T)
        got = _buf(poly, T)
        poly.run_async_noalloc(w.beta, T, got, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert np.array_equal(_host(poly, got), ref)


@pytest.mark.parametrize("p,n,s,T", [
    (W.P31, 6, 100_000, 300),     # 32-bit residues
    (W.P50, 6, 100_000, 300),     # the FP64 product
    (W.P31, 4, 1000, 64),         # single-launch path (no scratch at all)
    (W.P63, 3, 5000, 1),          # one evaluation
])
def test_matches_run_async(p, n, s, T):
    import torch
    w = W.make_poly(W.workload_seed(9, 10 + n), p, n, s, T, 40, 20)
    _say(f"case noalloc p={p} n={n} s={s} T={T}")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        ref = _reference(poly, w.beta, T)
        for _ in range(2):
            got = _buf(poly, T)
            poly.run_async_noalloc(w.beta, T, got, stream=torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert np.array_equal(_host(poly, got), ref)


def test_missing_layout_is_refused():
    w = W.make_poly(W.workload_seed(9, 30), W.P63, 5, 30_000, 100, 40, 20)
    _say("case noalloc missing layout")
    with PV.Poly(w.p, w.exps, w.coeffs) as poly:
        poly.set_tuning(4, 8, 2)
        buf = _buf(poly, w.T)
        with pytest.raises(PV.PevalError) as ei:
            poly.run_async_noalloc(w.beta, w.T, buf)
        assert ei.value.code == PV.EUNSUPPORTED and "layout" in str(ei.value)


def test_too_many_terms_is_refused():
    """6e6 terms of 64-bit residues need more than the region holds."""
    import torch
    s = 6_000_000
    exps = np.zeros((s, 3), np.uint32)
    exps[:, 2] = np.arange(s, dtype=np.uint32) % 7
    coeffs = np.arange(s, dtype=np.uint64)
    _say(f"case noalloc too large: s={s}")
    with PV.Poly(W.P63, exps, coeffs) as poly:
        buf = _buf(poly, 4)
        poly.run_async(np.asarray([3], np.uint64), 4, buf, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        with pytest.raises(PV.PevalError) as ei:
            poly.run_async_noalloc(np.asarray([3], np.uint64), 4, buf)
        assert ei.value.code == PV.EUNSUPPORTED and "scratch" in str(ei.value)
