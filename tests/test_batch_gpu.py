"""Batched persistent launch: every member equals its own plain run (and the
oracle), for graph replays and direct launches, across replays."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2004_11571_amd import peval as PV
from paper_2004_11571_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _outs(polys, Ts):
    import torch
    return [torch.empty((T, q.G), dtype=torch.int32 if q.elem_bytes == 4 else torch.int64, device="cuda")
            for q, T in zip(polys, Ts)]


def _host(q, buf):
    return buf.cpu().numpy().view(q.dtype)


def _mixed(count, s_max, seed):
    return W.uneven_batch(count=count, instance=seed, s_max=s_max, t_log2=(0, 9))


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_plain_runs(graph):
    import torch
    ws = _mixed(24, 2e4, 1)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    _say("batch members", [(q.s, q.G, T, q.elem_bytes) for q, T in zip(polys, Ts)])
    try:
        with PV.Batch(polys, Ts, graph=graph) as b:
            _say("info", b.info())
            outs = _outs(polys, Ts)
            for rep in range(3):
                betas = [np.asarray((w.beta.astype(object) * (rep + 1)) % w.p, np.uint64) for w in ws]
                b.run(betas, outs, stream=torch.cuda.current_stream())
                torch.cuda.synchronize()
                for q, w, beta, o in zip(polys, ws, betas, outs):
                    want = q.run(beta, w.T)  # eager work between replays
                    assert np.array_equal(_host(q, o), want), (rep, w.name)
    finally:
        for q in polys:
            q.destroy()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_fp64_members(graph):
    """Members with 2^31 <= p < 2^50 take the FP64 product in the batch as in
    their plain runs (a third queue and kernel), mixed with 32- and 64-bit
    integer members; one such member forced to the integer product."""
    import torch
    orc = Oracle()
    ws = W.uneven_batch(count=18, instance=5, s_max=2e4, t_log2=(0, 9), moduli=(W.P31, W.P50, W.P63))
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    fp = [j for j, w in enumerate(ws) if w.p == W.P50]
    assert len(fp) >= 3 and all(polys[j].arith() == "fp64" for j in fp)
    polys[fp[0]].set_arith("int")
    Ts = [w.T for w in ws]
    try:
        with PV.Batch(polys, Ts, graph=graph) as b:
            outs = _outs(polys, Ts)
            for rep in range(2):
                betas = [np.asarray((w.beta.astype(object) * (rep + 2)) % w.p, np.uint64) for w in ws]
                b.run(betas, outs, stream=torch.cuda.current_stream())
                torch.cuda.synchronize()
                for j, (q, w, beta, o) in enumerate(zip(polys, ws, betas, outs)):
                    got = _host(q, o)
                    assert np.array_equal(got, q.run(beta, w.T)), (rep, j, w.p)
                    if j in fp:
                        want = orc.evaluate(w.p, w.exps, w.coeffs, beta, w.T, threads=8)
                        assert np.array_equal(got.astype(np.uint64), want), (rep, j)
    finally:
        for q in polys:
            q.destroy()


def test_batch_against_oracle_and_offsets():
    import torch
    orc = Oracle()
    ws = _mixed(10, 3e3, 2)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    try:
        with PV.Batch(polys, Ts) as b:
            outs = _outs(polys, Ts)
            t0s = [1 + 37 * j for j in range(len(ws))]
            b.run([w.beta for w in ws], outs, t0s=t0s)
            torch.cuda.synchronize()
            for q, w, o, t0 in zip(polys, ws, outs, t0s):
                want = orc.evaluate(w.p, w.exps, w.coeffs, w.beta, w.T, t0=t0, threads=8)
                assert np.array_equal(_host(q, o).astype(np.uint64), want), w.name
    finally:
        for q in polys:
            q.destroy()


def test_batch_edge_members():
    """Single-term and single-group members, T = 1, n = 2, 32-bit and 64-bit."""
    import torch
    orc = Oracle()
    rng = np.random.default_rng(5)
    ws = [W.random_small(rng, W.P31, 2, 1, 1, dmax=3),
          W.random_small(rng, W.P63, 3, 1, 7, dmax=3),
          W.random_small(rng, 97, 5, 300, 17, dmax=4),
          W.random_small(rng, W.P63, 8, 2000, 33, dmax=3)]
    ws[3].exps[:, :2] = 0  # one group
    ws[3].exps = np.unique(ws[3].exps, axis=0)
    ws[3].coeffs = ws[3].coeffs[:ws[3].exps.shape[0]]
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    try:
        with PV.Batch(polys, [w.T for w in ws]) as b:
            outs = _outs(polys, [w.T for w in ws])
            b.run([w.beta for w in ws], outs)
            torch.cuda.synchronize()
            for q, w, o in zip(polys, ws, outs):
                want = orc.evaluate(w.p, w.exps, w.coeffs, w.beta, w.T, threads=4)
                assert np.array_equal(_host(q, o).astype(np.uint64), want)
    finally:
        for q in polys:
            q.destroy()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_runs_pipeline_across_streams(graph):
    """Six runs enqueued back to back, alternating between two streams, with
    no host synchronisation in between: each run's outputs equal the plain
    runs at its own base points (runs share scratch, so they must be ordered
    on the device)."""
    import torch
    ws = _mixed(12, 2e4, 3)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    try:
        with PV.Batch(polys, Ts, graph=graph) as b:
            runs = []
            for rep in range(6):
                betas = [np.asarray((w.beta.astype(object) * (rep + 2)) % w.p, np.uint64) for w in ws]
                outs = _outs(polys, Ts)
                b.run(betas, outs, stream=streams[rep % 2])
                runs.append((betas, outs))
            torch.cuda.synchronize()
            for rep, (betas, outs) in enumerate(runs):
                for q, w, beta, o in zip(polys, ws, betas, outs):
                    assert np.array_equal(_host(q, o), q.run(beta, w.T)), (rep, w.name)
    finally:
        for q in polys:
            q.destroy()


def test_batch_tuned_tiles_equal_plain_runs():
    """A batch whose tiles were tuned on the device (members' K moved per
    class, items resized) gives every member's plain-run images; the members'
    reported K and kernel kinds are consistent with their moduli."""
    import torch
    moduli = (W.P31, W.P63, W.P50)
    ws = W.uneven_batch(count=30, instance=7, s_max=2e5, t_log2=(3, 9), moduli=moduli)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    _say("tuned batch members", [(q.s, q.G, T, q.elem_bytes) for q, T in zip(polys, Ts)])
    try:
        with PV.Batch(polys, Ts, graph=True, tune=True) as b:
            mi = b.members()
            _say("members", mi)
            assert mi["tune_trials"] >= 3 and mi["tuned_ms"] > 0
            kinds = b.kinds()
            present = set(int(k) for k in mi["kind"])
            for kd in range(5):  # every present kind has its pass size and blocks
                assert (kinds["P"][kd] in (8, 16)) == (kd in present), kinds
                assert (kinds["blocks"][kd] > 0) == (kd in present), kinds
            for q, w, k, kd in zip(polys, ws, mi["K"], mi["kind"]):
                assert k in (1, 2, 4, 8, 16, 32)
                if q.elem_bytes == 4:
                    assert kd in (3, 4) and (kd == 3) == (k == 32)
                elif w.p == W.P50:
                    assert kd == 2 and k <= 8
                else:
                    assert kd in (0, 1) and (kd == 0) == (k == 16)
            outs = _outs(polys, Ts)
            for rep in range(2):
                betas = [np.asarray((w.beta.astype(object) * (rep + 2)) % w.p, np.uint64) for w in ws]
                b.run(betas, outs, stream=torch.cuda.current_stream())
                torch.cuda.synchronize()
                for q, w, beta, o in zip(polys, ws, betas, outs):
                    assert np.array_equal(_host(q, o), q.run(beta, w.T)), (rep, w.name)
    finally:
        for q in polys:
            q.destroy()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_eight_per_pass_equals_plain_runs(graph):
    """Every kind's kernel staging 8 evaluations per pass (the tuner's other
    choice) gives the members' plain-run images; kinds report P = 8."""
    import torch
    moduli = (W.P31, W.P63, W.P50)
    ws = W.uneven_batch(count=24, instance=11, s_max=1e5, t_log2=(3, 9), moduli=moduli)
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    Ts = [w.T for w in ws]
    _say("pass8 batch members", [(q.s, q.G, T, q.elem_bytes) for q, T in zip(polys, Ts)], "graph", graph)
    try:
        with PV.Batch(polys, Ts, graph=graph, pass8=True) as b:
            kinds = b.kinds()
            present = set(int(k) for k in b.members()["kind"])
            assert all(kinds["P"][kd] == (8 if kd in present else 0) for kd in range(5)), kinds
            outs = _outs(polys, Ts)
            b.run([w.beta for w in ws], outs, stream=torch.cuda.current_stream())
            torch.cuda.synchronize()
            for q, w, o in zip(polys, ws, outs):
                assert np.array_equal(_host(q, o), q.run(w.beta, w.T)), w.name
    finally:
        for q in polys:
            q.destroy()
