"""Benchmark: partial modular evaluation (matrix method) on one MI355X.

One step = one pass of the whole evaluation path (power tables, monomial
values and chain starts, Hadamard products with coefficient reductions,
combine) for one resident polynomial and one base point, i.e. one
``peval_run_async`` of T evaluations.  The polynomial is ingested once before
timing (its data is resident in HBM when the timed region starts).

Default workload: the largest single polynomial, n = 8 variables, 1e7
distinct terms, x1/x2 degree <= 60, x3..x8 total degree <= 30,
p = 2^63 - 25, T = 4096 evaluations.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "term-evals/s mod p (terms×points) vs oracle; %roofline; p99 latency"

# MI355X: 256 CUs x 64 lanes x 2.4 GHz; 32-bit integer multiplies (mul_lo,
# mul_hi, mad_u64_u32) issue at the full VALU rate on gfx950.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12

# Algorithmic VALU operations per term-evaluation: one lazy Shoup product
# on 32-bit limbs plus one lazy addition into the coefficient sum, counting
# each gfx950 integer instruction of the shortest sequence as one op (a
# 32x32->64 multiply-add, a 32-bit add/sub with carry, a three-input add or a
# 64-bit add each count once):
#   64-bit residues: high half of x*w' (mul_hi + 3 mad_u64_u32, the middle
#   one's carry-out turned into the last one's addend by one select) = 5;
#   the remainder x*w - q*p mod 2^64 as x*w + q*(2^64 - p) (four
#   cross-product mads into one pair, a 64-bit shift, two mads) = 7; the
#   lazy sum (the value's two 32-bit halves into two 64-bit sums, one mad
#   each) = 2; total 14.
#   32-bit residues: mul_hi, and the remainder as the low word of
#   x*w + q*(2^32 - p) by two mads = 3; the lazy 64-bit sum by one mad = 1;
#   total 4.
#   FP64 product (Alg. 2, p < 2^50, signed running values, the quotient
#   rounded to nearest so that no correction follows): mul, fma, mul,
#   rint, fma, add = 6; the double sum (add) = 1; total 7.
ALGO_OPS = {8: 14, 4: 4, "fp64": 7}
# Point mode (arbitrary points): a term's contribution takes one lazy Shoup
# product per factor table (NF - 1 for the monomial, one for the
# coefficient) plus the lazy sum: NF * 12 + 2 ops (64-bit residues; the
# product alone is 14 - 2 = 12), NF * 3 + 1 (32-bit residues), NF * 6 + 1
# (the FP64 product).
def points_ops(w: int, nf: int, arith: str = "int") -> int:
    if arith == "fp64":
        return nf * 6 + 1
    return nf * 12 + 2 if w == 8 else nf * 3 + 1
# Algorithmic HBM bytes per run: resident term data read once (coefficient
# and n-2 16-bit exponents per term) plus the dense output written once.


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (0: enough for about 2 s of timed work, at least 20)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="n8_s1e7_p63_T4096",
                    choices=["n4_s1e3_p31_T64", "n6_s1e6_p63_T1024", "n6_s1e6_p31_T1024", "n8_s1e7_p63_T4096",
                             "paper_table2", "batch", "serve", "modarith",
                             "n6_s1e6_p63_T1024_points", "n6_s1e6_p31_T1024_points", "paper_table2_points",
                             "n6_s1e6_p63_T1024_interp", "paper_table2_interp"])
    ap.add_argument("--rate", type=float, default=2000.0, help="served stream: mean arrivals per second")
    ap.add_argument("--duration", type=float, default=3.0, help="served stream: seconds of arrivals")
    ap.add_argument("--pool", type=int, default=20, help="served stream: resident polynomials")
    ap.add_argument("--new-fraction", type=float, default=0.1,
                    help="served stream: share of requests for a polynomial the server has not seen")
    ap.add_argument("--oracle-requests", type=int, default=24, help="served stream: requests checked by the oracle")
    ap.add_argument("--oracle-max-work", type=float, default=1e8,
                    help="served stream: largest s*T of a request in the oracle sample")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--sweep", default="250,500,1000,4000", help="served stream: other arrival rates (paced)")
    ap.add_argument("--tight-gb", type=float, default=2.0, help="served stream: a run under this HBM budget (0: skip)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-smax", type=float, default=1e6)
    ap.add_argument("--no-batch-tune", action="store_true", help="batch: heuristic tiles, no tuning at create")
    ap.add_argument("--tuning", default="", help="K,P,C override")
    ap.add_argument("--no-autotune", action="store_true",
                    help="power mode: the heuristic's K, P, C instead of timing candidates first")
    ap.add_argument("--arith", default="auto", choices=["auto", "int", "fp64", "pm"],
                    help="modular product of the evaluation kernel (fp64: the paper's Alg. 2, p < 2^50)")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="oracle sample: images checked (half the first rows, half the last; "
                         "0: about 1.6e8 term-evaluations of oracle work)")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    return ap.parse_args()


def profile_traffic(kernel_sha: str, workload: str, kernel: str = "eval_kernel", tuning=None):
    """HBM bytes per launch of the evaluation kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and (when the summary names one) with the run's own tiles: the chain
    count changes what the kernel re-reads."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != kernel_sha:
        return None
    if tuning is not None:  # the bytes counted with these tiles, if any were
        for m in re.finditer(r"traffic_for_tuning:\s*K=(\d+) P=(\d+) C=(\d+) bytes=([0-9.eE+]+)", text):
            if tuple(int(x) for x in m.groups()[:3]) == tuple(tuning):
                return float(m.group(4))
    m_t = re.search(r"counted_tuning:\s*K=(\d+) P=(\d+) C=(\d+)", text)
    if m_t and tuning is not None and tuple(int(x) for x in m_t.groups()) != tuple(tuning):
        return None
    return float(m_b.group(1))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Headers each profiled kernel is compiled from.
KERNEL_SOURCES = {
    "eval_kernel": ("kernels.hpp", "modarith.hpp"),
    "small_run_kernel": ("kernels.hpp", "modarith.hpp", "small_kernels.hpp"),
    "points_eval_kernel": ("kernels.hpp", "modarith.hpp", "points_kernels.hpp"),
    "batch_pass": ("kernels.hpp", "modarith.hpp", "batch_kernels.hpp", "batch_types.hpp"),
}


def kernel_source_sha(kernel: str = "eval_kernel", sources=None) -> str:
    """Hash of one kernel's code (the headers it is compiled from):
    comments and whitespace are dropped, so that only a change of the
    compiled code invalidates the counter profiles taken on it."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        text = sources[f] if sources else open(os.path.join(ROOT, "paper_2004_11571_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]

# Microbenchmark kinds (include/peval_testing.h): product forms, with the
# modulus each is measured at and its counted operations per product and
# addition; then single instructions.
MB_PRODUCTS = [("shoup64", 0, (1 << 63) - 25, 14), ("shoup32", 1, (1 << 31) - 1, 4),
               ("fp64_alg2_rounded", 2, (1 << 50) - 27, 7), ("pseudo_mersenne63", 3, (1 << 63) - 25, None),
               ("pseudo_mersenne31", 4, (1 << 31) - 1, None)]
MB_INSNS = [("v_add_u32", 16), ("v_mul_lo_u32", 17), ("v_mul_hi_u32", 18), ("v_mad_u64_u32", 19),
            ("v_fma_f64", 20)]
MB_BLOCKS = 256 * 8   # eight 256-thread workgroups per CU


def bench_product(kind: int, p: int, target_ms: float = 80.0):
    """(work per second, ms) of one microbenchmark kind, its iteration count
    scaled so that the timed launch takes about target_ms."""
    import ctypes

    from paper_2004_11571_amd import peval as PV
    L = PV.lib()
    ms, work = ctypes.c_double(), ctypes.c_double()
    iters = 64
    for _ in range(4):
        PV._check(L.peval_bench_product(kind, p, iters, MB_BLOCKS, ctypes.byref(ms), ctypes.byref(work)))
        if ms.value >= 0.5 * target_ms:
            break
        iters = int(min(1 << 24, iters * max(2.0, target_ms / max(ms.value, 1e-3))))
    return work.value / (ms.value / 1e3), ms.value


def modarith_main(args):
    """Modular products at full occupancy (every thread 16 running values, 8
    for the FP64 product, each added into the thread's sum and multiplied by
    its fixed multiplier per iteration) and the issue rates of the
    instructions they are built from; rates per CU per clock at 2.4 GHz."""
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    per_clk = 256 * 2.4e9
    products = {}
    for name, kind, p, ops in MB_PRODUCTS:
        rate, ms = bench_product(kind, p)
        products[name] = {"p": p, "products_per_s": rate, "per_cu_per_clock": rate / per_clk,
                          "lane_cycles_per_product": 64 * per_clk / rate, "ms": ms,
                          "counted_ops": ops, "frac_of_valu_peak": (rate * ops / VALU_PEAK_OPS) if ops else None}
    insns = {}
    for name, kind in MB_INSNS:
        rate, ms = bench_product(kind, 0)
        insns[name] = {"lane_ops_per_s": rate, "per_cu_per_clock": rate / per_clk, "ms": ms}
    best = products["shoup64"]["products_per_s"]
    res = {"metric": "modular products with additions per second (full occupancy)", "value": best,
           "unit": "products/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": products["shoup64"]["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "modarith_microbenchmark", "blocks": MB_BLOCKS, "threads_per_block": 256},
           "products": products, "instructions": insns}
    print(json.dumps(res), flush=True)


def interp_main(args):
    """Coefficients back from the images (the interpolation that follows the
    evaluations): one step = one solve of every group's transposed
    Vandermonde system from images already in HBM."""
    import torch

    from paper_2004_11571_amd import peval as PV
    from paper_2004_11571_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    base = args.workload[: -len("_interp")]
    w = {"n6_s1e6_p63_T1024": W.n6_s1e6_p63_T1024, "paper_table2": W.paper_table2}[base]()
    _, sizes = np.unique(w.exps[:, :2], axis=0, return_counts=True)
    T = int(sizes.max())
    poly = PV.Poly(w.p, w.exps, w.coeffs)
    dt = torch.int64 if poly.elem_bytes == 8 else torch.int32
    img = torch.empty((T, poly.G), dtype=dt, device=dev)
    out = torch.empty(w.s, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    poly.run_async(w.beta, T, img, stream=stream)
    args.steps = args.steps or 200
    for _ in range(args.warmup):
        poly.interpolate_async(w.beta, T, img, out, status, stream=stream)
    torch.cuda.synchronize()
    PV.prof_read()
    PV.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        poly.interpolate_async(w.beta, T, img, out, status, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    PV.prof_enable(False)
    kern = PV.prof_read()
    # the two solve kernels: per-group polynomials, then per-term evaluation
    solve_s = sum(kern[k][0] / max(kern[k][1], 1) for k in ("eval", "combine")) / 1e3
    # algorithmic work: per group of m terms, 3 m^2 modular multiply-adds
    # (Q, the b_l, and the two Horner evaluations) plus the Fermat inversion
    # of each term (2 log2 p products, each with its quotient computed: 2),
    # each priced as one lazy Shoup product and sum (ALGO_OPS: 14 ops,
    # 64-bit residues; 4 for 32-bit); under the FP64 product the two Horner
    # evaluations (2 m^2 steps) take its product, an addition and a fold
    # per step (6 + 1 + 3 ops), and the b_l sums (m^2 / 2) its product, an
    # addition, a quarter of a fold and the conversion of q (6 + 1 + 1 + 3)
    bits = int(w.p).bit_length()
    m2 = float((sizes.astype(np.float64) ** 2).sum())
    mac = 3 * m2 + 4 * bits * w.s
    fp = poly.arith() == "fp64"
    horner_ops = 10 if fp else ALGO_OPS[poly.elem_bytes]
    bsum_ops = 11 if fp else ALGO_OPS[poly.elem_bytes]
    ops = ((m2 / 2 + 4 * bits * w.s) * ALGO_OPS[poly.elem_bytes] + (m2 / 2) * bsum_ops
           + 2 * m2 * horner_ops)
    achieved = ops / solve_s
    ok = int(status.item()) == 0 and bool(np.array_equal(out.cpu().numpy().view(np.uint64), w.coeffs))
    res = {
        "metric": "interpolated coefficients/s mod p", "value": w.s * args.steps / elapsed,
        "unit": "coefficients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64" if poly.elem_bytes == 8 else "u32", "data": "synthetic",
        "config": {"workload": w.name + "_interpolate", "s": w.s, "G": poly.G, "p": w.p,
                   "largest_group": T, "mean_group": float(sizes.mean()), "images": T},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "interp_group_kernel + interp_solve_kernel", "solve_launch_ms": solve_s * 1e3,
                     "multiply_adds": mac},
        "kernels_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in kern.items()},
        "round_trip_exact": ok,
    }
    if not args.no_cpu and T <= 1500:   # elimination is O(m^3) per group
        from oracle import Oracle
        orc = Oracle()
        gd, ge = poly.groups()
        ng = 3
        sel = np.zeros(w.s, bool)
        for g in range(ng):
            sel |= (w.exps[:, 0] == gd[g]) & (w.exps[:, 1] == ge[g])
        imgs = img.cpu().numpy().view(poly.dtype)[:, :ng].astype(np.uint64)
        c0 = time.perf_counter()
        ref = orc.interpolate(w.p, w.exps[sel], w.beta, imgs)
        csec = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": int(sel.sum()) / csec, "unit": "coefficients/s", "cores": 1,
                               "kind": "oracle", "seconds": csec,
                               "sample": f"the {ng} largest-key groups ({int(sel.sum())} terms) by elimination"}
        res["parity_sample"] = bool(np.array_equal(ref, w.coeffs[sel]))
    poly.destroy()
    print(json.dumps(res), flush=True)


def batch_main(args):
    """Uneven batch of polynomials: one persistent hipGraph launch per step,
    compared with the same members launched one after another."""
    import torch

    from paper_2004_11571_amd import peval as PV
    from paper_2004_11571_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy_mib:  # a plain device copy of known size (counter calibration)
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    t_gen = time.time()
    ws = W.uneven_batch(count=args.batch_count, s_max=args.batch_smax)
    gen_s = time.time() - t_gen
    t_c = time.time()
    polys = [PV.Poly(w.p, w.exps, w.coeffs) for w in ws]
    create_s = time.time() - t_c
    Ts = [w.T for w in ws]
    te = sum(w.s * w.T for w in ws)
    outs = [torch.empty((w.T, q.G), dtype=torch.int32 if q.elem_bytes == 4 else torch.int64, device="cuda")
            for w, q in zip(ws, polys)]
    betas = [w.beta for w in ws]
    stream = torch.cuda.current_stream()
    # the batch's tiles are tuned on the device before anything is timed
    t_tune = time.time()
    b = PV.Batch(polys, Ts, graph=True, tune=not args.no_batch_tune)
    tune_s = time.time() - t_tune
    info = b.info()
    mi = b.members()
    kinds = b.kinds()
    kind_names = ["w64_k16", "w64_k<=8", "fp64", "w32_k32", "w32_k<=16"]
    tiles = {}
    for w, k, c, kd in zip(ws, mi["K"], mi["C"], mi["kind"]):
        e = tiles.setdefault(kind_names[int(kd)], {"members": 0, "term_evals": 0, "K": {},
                                                   "P": int(kinds["P"][int(kd)]),
                                                   "blocks": int(kinds["blocks"][int(kd)])})
        e["members"] += 1
        e["term_evals"] += w.s * w.T
        e["K"][str(int(k))] = e["K"].get(str(int(k)), 0) + 1
    steps = args.steps or 20
    # the first replays of a newly instantiated graph can run far slower
    # (up to the eighth or so); at least twenty untimed ones
    warm = max(20, args.warmup)
    for _ in range(warm):
        b.run(betas, outs, stream=stream)
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(steps):
        b.run(betas, outs, stream=stream)
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    spread = {"min": step_ms[0], "median": step_ms[len(step_ms) // 2], "max": step_ms[-1]}
    batched = [o.cpu().numpy().view(q.dtype).copy() for o, q in zip(outs, polys)]

    # the same members as plain launches, one after another on one stream
    for q, w, o in zip(polys, ws, outs):
        q.run_async(w.beta, w.T, o, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        for q, w, o in zip(polys, ws, outs):
            q.run_async(w.beta, w.T, o, stream=stream)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1
    # device -> page-locked host bandwidth, for context (results must cross it)
    big = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    hb = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    hb.copy_(big)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(3):
        hb.copy_(big)
    torch.cuda.synchronize()
    d2h_gbps = 3 * (1 << 30) / (time.perf_counter() - tb) / 1e9
    del big, hb
    same = all(np.array_equal(o.cpu().numpy().view(q.dtype), x) for o, q, x in zip(outs, polys, batched))
    value = te * steps / el
    ops = sum(ALGO_OPS[q.elem_bytes] * w.s * w.T for q, w in zip(polys, ws))
    achieved = ops * steps / el
    # term data read once and images written once, every member
    algo_bytes = sum(w.s * (q.elem_bytes + 2 * (w.n - 2)) + w.T * q.G * q.elem_bytes for q, w in zip(polys, ws))
    res = {
        "metric": METRIC, "value": value, "unit": "term-evals/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": el / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32+u64", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}_uneven_s1e3-{args.batch_smax:.0e}_T32-2048_p31p63",
                   "members": len(ws), "term_evals_per_step": te, **info},
        "tiles": {"tuned": not args.no_batch_tune, "tune_trials": mi["tune_trials"], "tuned_pass_ms": mi["tuned_ms"],
                  "create_and_tune_s": tune_s, "by_kernel": tiles},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": profile_traffic(kernel_source_sha("batch_pass"), f"batch{len(ws)}_uneven", "batch_pass"),
                     # the counters are taken on the heuristic tiles (the same plan in every counter run)
                     "traffic_tiles": "heuristic",
                     "kernel_source_sha256": kernel_source_sha("batch_pass"),
                     "kernel": "whole batched pass (graph replay), all kernels",
                     "frac_at_median_step": ops / (spread["median"] / 1e3) / VALU_PEAK_OPS,
                     "hbm_algorithmic_bytes_per_step": algo_bytes,
                     "hbm_frac": algo_bytes / (el / steps) / HBM_PEAK},
        "step_ms_spread": spread,
        "sequential_plain": {"value": te * steps / el_seq, "ms_per_step": el_seq / steps * 1e3,
                             "batched_over_sequential": el_seq / el, "identical_outputs": same},
        "generate_s": gen_s, "create_s": create_s,
    }
    b.destroy()
    for q in polys:
        q.destroy()
    print(json.dumps(res), flush=True)


class PinnedSlots:
    """Page-locked host memory carved into one result buffer per request
    (chunks of 1 GiB), so that every served result is still there when the
    stream has ended."""

    def __init__(self, sizes, chunk=1 << 30):
        import torch
        self.chunks, self.where = [], []
        used = chunk
        for nb in sizes:
            nb = (nb + 255) & ~255
            if used + nb > chunk:
                self.chunks.append(torch.empty(max(chunk, nb), dtype=torch.uint8, pin_memory=True).numpy())
                used = 0
            self.where.append((len(self.chunks) - 1, used))
            used += nb

    def view(self, i, nbytes):
        c, off = self.where[i]
        return self.chunks[c][off:off + nbytes]


def serve_main(args):
    """Poisson stream of evaluation requests against the server (about 10%
    of them for polynomials it has not seen before); p50/p99 latency and
    throughput; every served result compared with the same request run
    alone; an oracle-checked sample; then the same requests one at a time."""
    import threading

    import torch

    from paper_2004_11571_amd import peval as PV
    from paper_2004_11571_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.time()
    pool = W.serve_pool(args.pool)
    reqs = W.serve_stream(args.rate, args.duration, pool)
    new_coeffs = W.serve_new_polys(reqs, pool, args.new_fraction)
    gen_s = time.time() - t_gen
    print(f"serve: {len(pool)} pool polynomials, {len(reqs)} requests, {len(new_coeffs)} for new polynomials "
          f"({gen_s:.1f} s to generate)", file=sys.stderr, flush=True)
    wb = [4 if w.p < 2**31 else 8 for w in pool]
    dts = [np.uint32 if b == 4 else np.uint64 for b in wb]

    srv = PV.Server(int(args.budget_gb * (1 << 30)))
    pids = [srv.add_poly(w.p, w.exps, w.coeffs) for w in pool]
    G = [srv.poly_info(pid)["G"] for pid in pids]
    for j in range(len(pool)):  # the pool is resident before the stream: one request each
        rid = srv.submit(pids[j], pool[j].beta, 64)
        srv.wait(rid, 600000)
        srv.release(rid)

    def register_new(s):
        """The stream's new polynomials, registered (host copies) but not
        resident: each is uploaded when its request is admitted."""
        t0 = time.perf_counter()
        m = {i: s.add_poly(pool[reqs[i].poly_index].p, pool[reqs[i].poly_index].exps, c)
             for i, c in new_coeffs.items()}
        return m, time.perf_counter() - t0

    def nbytes(r):
        return r.T * G[r.poly_index] * wb[r.poly_index]

    def as_image(r, buf):
        return buf[: nbytes(r)].view(dts[r.poly_index]).reshape(r.T, G[r.poly_index])

    # client-side buffers: a pool of page-locked buffers reused once a result
    # has been consumed, or one buffer per request (the verified run)
    max_bytes = max(2048 * G[j] * wb[j] for j in range(len(pool)))  # T <= 2^11 in every stream
    n_buf = 256
    bufs = [torch.empty(max_bytes, dtype=torch.uint8, pin_memory=True).numpy() for _ in range(n_buf)]

    def stream(paced, reqs=reqs, srv=srv, new_pid=None, keep=None):
        """Submit every request (at its arrival time if paced, else at once)
        into a free buffer (or its own slot of `keep`); a collector thread
        takes results in completion order, releases them and drops each new
        polynomial once its request is done."""
        new_pid = new_pid or {}
        srv.reset_stats()
        lock = threading.Lock()
        owner = {}
        free_bufs = list(range(n_buf))
        n_sub = [0]
        finished = threading.Event()
        errors = []

        def collector():
            n_done = 0
            try:
                while True:
                    with lock:
                        if finished.is_set() and n_done == n_sub[0]:
                            return
                    try:
                        rid = srv.next_done(50)
                    except PV.PevalError as e:
                        if e.code == PV.ETIMEOUT:
                            continue
                        raise
                    srv.wait(rid, 0)  # raises if the request failed
                    srv.release(rid)
                    with lock:
                        i, bi = owner.pop(rid)
                        if bi is not None:
                            free_bufs.append(bi)
                        n_done += 1
                    if i in new_pid:
                        srv.remove_poly(new_pid[i])
            except Exception as e:  # surface it to the submitting thread
                errors.append(e)

        col = threading.Thread(target=collector, daemon=True)
        col.start()
        t0 = time.perf_counter()
        lag = 0.0
        refused = 0
        try:
            for i, r in enumerate(reqs):
                if paced:
                    delay = r.arrival_s - (time.perf_counter() - t0)
                    if delay > 0:
                        time.sleep(delay)
                    else:
                        lag = max(lag, -delay)
                if keep is not None:
                    bi, out = None, as_image(r, keep.view(i, nbytes(r)))
                else:
                    t_wait = time.perf_counter()
                    while True:
                        with lock:
                            bi = free_bufs.pop() if free_bufs else None
                        if bi is not None:
                            break
                        if errors:
                            raise errors[0]
                        if time.perf_counter() - t_wait > 120:
                            raise RuntimeError("no result buffer came back within 120 s")
                        time.sleep(0.0001)
                    out = as_image(r, bufs[bi])
                pid = new_pid.get(i, pids[r.poly_index])
                with lock:
                    try:
                        rid = srv.submit(pid, r.beta, r.T, out=out)
                    except PV.PevalError as e:
                        if e.code != PV.ENOMEM:
                            raise
                        refused += 1          # cannot fit the budget even alone: refused at submit
                        if bi is not None:
                            free_bufs.append(bi)
                        continue
                    owner[rid] = (i, bi)
                    n_sub[0] += 1
        finally:
            finished.set()
        submit_s = time.perf_counter() - t0
        col.join(timeout=300)
        if col.is_alive():
            raise RuntimeError("results did not all come back within 300 s")
        if errors:
            raise errors[0]
        st = srv.stats()
        st["submit_s"] = submit_s
        st["max_submit_lag_s"] = lag
        st["refused_at_submit"] = refused
        return st

    te = sum(pool[r.poly_index].s * r.T for r in reqs)
    # the verified run: paced, every result kept
    keep = PinnedSlots([nbytes(r) for r in reqs])
    new_pid, reg_s = register_new(srv)
    st = stream(paced=True, new_pid=new_pid, keep=keep)
    print(f"serve: paced stream done ({st['uploads']} uploads)", file=sys.stderr, flush=True)
    new_pid, _ = register_new(srv)
    sat = stream(paced=False, new_pid=new_pid)
    print("serve: saturated stream done", file=sys.stderr, flush=True)
    # the knee: the pool alone at other arrival rates
    sweep = []
    for rate in [float(x) for x in args.sweep.split(",") if x]:
        rq = W.serve_stream(rate, args.duration, pool)
        sr = stream(paced=True, reqs=rq)
        sweep.append({"rate_per_s": rate, "requests": len(rq),
                      "offered_term_evals_per_s": sum(pool[r.poly_index].s * r.T for r in rq) / args.duration,
                      "value": sr["term_evals"] / sr["wall_s"], "p50_ms": sr["p50_ms"], "p99_ms": sr["p99_ms"],
                      "max_ms": sr["max_ms"]})
        print(f"serve: rate {rate:g} done", file=sys.stderr, flush=True)
    srv.destroy()
    # a tight HBM budget: residency by eviction and upload, admission by memory
    tight = None
    if args.tight_gb > 0:
        srv2 = PV.Server(int(args.tight_gb * (1 << 30)))
        pids_save = list(pids)
        pids[:] = [srv2.add_poly(w.p, w.exps, w.coeffs) for w in pool]
        new_pid2, _ = register_new(srv2)
        s2 = stream(paced=True, srv=srv2, new_pid=new_pid2)
        pids[:] = pids_save
        tight = {"budget_gb": args.tight_gb, "value": s2["term_evals"] / s2["wall_s"], "p50_ms": s2["p50_ms"],
                 "p99_ms": s2["p99_ms"], "max_ms": s2["max_ms"], "uploads": s2["uploads"],
                 "evictions": s2["evictions"], "hbm_peak_gb": s2["hbm_peak"] / 2**30,
                 "completed": s2["completed"], "refused_at_submit": s2["refused_at_submit"]}
        srv2.destroy()
        print("serve: tight budget done", file=sys.stderr, flush=True)

    # the same requests one at a time: a plain run into device memory (a new
    # polynomial is created first and destroyed after), then the result
    # copied to the same kind of page-locked buffer
    hs = [PV.Poly(w.p, w.exps, w.coeffs) for w in pool]
    dev = torch.empty(max_bytes, dtype=torch.uint8, device="cuda")
    dev2 = torch.empty(max_bytes, dtype=torch.uint8, device="cuda")
    pin = torch.from_numpy(bufs[0])
    for j, h in enumerate(hs):
        h.run_async(pool[j].beta, 16, dev)
    torch.cuda.synchronize()

    def alone(i, r):
        w = pool[r.poly_index]
        if i in new_coeffs:
            h = PV.Poly(w.p, w.exps, new_coeffs[i])
            h.run_async(r.beta, r.T, dev)
            return h
        hs[r.poly_index].run_async(r.beta, r.T, dev)
        return None

    t1 = time.perf_counter()
    for i, r in enumerate(reqs):
        h = alone(i, r)
        pin[: nbytes(r)].copy_(dev[: nbytes(r)])
        if h is not None:
            h.destroy()
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1
    print("serve: sequential plain runs done", file=sys.stderr, flush=True)

    # alone vs in the mix: every element of every served result of the
    # verified run against the same request run alone (compared on the device)
    v0 = time.perf_counter()
    mismatch = []
    for i, r in enumerate(reqs):
        h = alone(i, r)
        nb = nbytes(r)
        dev2[:nb].copy_(torch.from_numpy(keep.view(i, nb)), non_blocking=True)
        if not torch.equal(dev[:nb], dev2[:nb]):
            mismatch.append(i)
        if h is not None:
            h.destroy()
    verify_s = time.perf_counter() - v0
    print(f"serve: alone vs mix checked ({len(mismatch)} differ)", file=sys.stderr, flush=True)
    # the oracle on a seeded sample of the verified run's requests (both kinds)
    from oracle import Oracle
    orc = Oracle()
    rng = np.random.default_rng(W.workload_seed(5, 300))
    small = [i for i, r in enumerate(reqs) if pool[r.poly_index].s * r.T <= args.oracle_max_work]
    small_new = [i for i in small if i in new_coeffs]
    small_old = [i for i in small if i not in new_coeffs]
    n_new = min(len(small_new), args.oracle_requests // 4)
    pick = sorted(list(rng.choice(small_new, n_new, replace=False)) +
                  list(rng.choice(small_old, min(len(small_old), args.oracle_requests - n_new), replace=False)))
    o0 = time.perf_counter()
    ok = 0
    o_te = 0
    for i in pick:
        r = reqs[i]
        w = pool[r.poly_index]
        want = orc.evaluate(w.p, w.exps, new_coeffs.get(i, w.coeffs), r.beta, r.T, threads=args.cpu_threads)
        ok += int(np.array_equal(as_image(r, keep.view(i, nbytes(r))).astype(np.uint64), want))
        o_te += w.s * r.T
    oracle_s = time.perf_counter() - o0
    print(f"serve: oracle sample {ok}/{len(pick)}", file=sys.stderr, flush=True)
    for h in hs:
        h.destroy()
    # device -> page-locked host bandwidth, for context (results must cross it)
    big = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    hb = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    hb.copy_(big)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(3):
        hb.copy_(big)
    torch.cuda.synchronize()
    d2h_gbps = 3 * (1 << 30) / (time.perf_counter() - tb) / 1e9
    del big, hb
    te_seq = sum(pool[r.poly_index].s * r.T for r in reqs)
    res = {
        "metric": METRIC, "value": st["term_evals"] / st["wall_s"], "unit": "term-evals/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": len(pool), "ms_per_step": st["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+u64", "data": "synthetic",
        "config": {"workload": f"served_poisson{args.rate:g}_s1e3-5e6_T64-2048_p31p63_new{args.new_fraction:g}",
                   "rate_per_s": args.rate, "duration_s": args.duration, "requests": len(reqs),
                   "pool": len(pool), "new_poly_requests": len(new_coeffs), "budget_gb": args.budget_gb,
                   "offered_term_evals_per_s": te / args.duration},
        "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"], "max": st["max_ms"], "mean": st["mean_ms"]},
        "server": st,
        "new_poly_registration_s": reg_s,
        "alone_vs_mix": {"requests": len(reqs), "identical": len(reqs) - len(mismatch),
                         "first_mismatches": mismatch[:10], "seconds": verify_s,
                         "how": "every element of every served result against the same request run alone "
                                "(peval_run_async; a new polynomial created for it), compared on the device"},
        "alone_vs_mix_identical": not mismatch,
        "oracle_sample": {"n": len(pick), "ok": ok, "new_poly_requests": n_new, "term_evals": o_te,
                          "seconds": oracle_s, "threads": args.cpu_threads,
                          "selection": f"seeded, among requests with s*T <= {args.oracle_max_work:.0e}"},
        "saturated": {"value": sat["term_evals"] / sat["wall_s"], "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"],
                      "passes": sat["passes"], "slices": sat["slices"], "uploads": sat["uploads"],
                      "host_pass_s": sat["host_pass_s"], "gpu_pass_s": sat["gpu_pass_s"], "wall_s": sat["wall_s"]},
        "d2h_pinned_GBps": d2h_gbps,
        "output_GB": sum(nbytes(r) for r in reqs) / 1e9,
        "sequential_plain": {"requests": len(reqs), "value": te_seq / el_seq, "seconds": el_seq,
                             "saturated_served_over_sequential": (sat["term_evals"] / sat["wall_s"]) / (te_seq / el_seq)},
        "generate_s": gen_s,
        "rate_sweep": sweep,
        "tight_budget": tight,
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding over several GPUs is described "
                          "in the design notes, not implemented"}), flush=True)
        sys.exit(2)

    if args.workload == "batch":
        return batch_main(args)
    if args.workload == "serve":
        return serve_main(args)
    if args.workload == "modarith":
        return modarith_main(args)
    if args.workload.endswith("_interp"):
        return interp_main(args)

    import torch

    from paper_2004_11571_amd import peval as PV
    from paper_2004_11571_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    points_mode = args.workload.endswith("_points")
    base = args.workload[: -len("_points")] if points_mode else args.workload
    w = {"n4_s1e3_p31_T64": W.n4_s1e3_p31_T64, "n6_s1e6_p63_T1024": W.n6_s1e6_p63_T1024, "n6_s1e6_p31_T1024": W.n6_s1e6_p31_T1024,
         "n8_s1e7_p63_T4096": W.n8_s1e7_p63_T4096, "paper_table2": W.paper_table2}[base]()
    t_gen = time.time()
    poly = PV.Poly(w.p, w.exps, w.coeffs)
    create_s = time.time() - t_gen
    poly.set_arith(args.arith)
    tuned = None
    if args.tuning:
        poly.set_tuning(*[int(x) for x in args.tuning.split(",")])
    elif not args.no_autotune and not points_mode:
        # the evaluation kernel's K, P and C timed on the device for this
        # polynomial before anything is timed (the tuning cache then serves
        # every run of this shape)
        heur = poly.get_tuning(w.T)
        t_tune = time.time()
        tk, tp, tc, tms = poly.autotune(w.beta, w.T)
        tuned = {"K": tk, "P": tp, "C": tc, "tuned_run_ms": tms, "tune_s": time.time() - t_tune,
                 "heuristic": dict(zip("KPC", heur))}
    K, P, C = poly.points_tuning(w.T) if points_mode else poly.get_tuning(w.T)
    single = (K, P, C) == (0, 0, 0) and not points_mode  # one kernel for the whole run
    dt = torch.int64 if poly.elem_bytes == 8 else torch.int32
    out = torch.empty((w.T, poly.G), dtype=dt, device=dev)
    stream = torch.cuda.current_stream(dev)
    if points_mode:
        pts = W.random_points(w)
        dpts = torch.from_numpy(pts.view(np.int64)).to(dev)
        nf, E = PV.points_factors(poly.elem_bytes, poly.info()["max_exp"][2:w.n])

        def step():
            poly.run_points_async(dpts, w.T, out, stream=stream)
    else:
        def step():
            poly.run_async(w.beta, w.T, out, stream=stream)

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not args.steps:  # about 2 s of timed work, at least 20 steps
        t_est = time.perf_counter()
        step()
        torch.cuda.synchronize()
        args.steps = int(min(5000, max(20, 2.0 / max(time.perf_counter() - t_est, 1e-6))))
    # timed steps.  The library records a HIP event pair around every kernel
    # launch on the launch stream (the per-kernel times and the roofline come
    # from these same steps), and one torch event per step on the same stream
    # gives the spread of the step times.
    PV.prof_read()  # drop anything recorded so far
    PV.prof_enable(True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(args.steps):
        step()
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    PV.prof_enable(False)
    kern = PV.prof_read()
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps))
    spread = {"min": step_ms[0], "median": step_ms[len(step_ms) // 2], "max": step_ms[-1]}
    # the same steps without the per-kernel events (host cost of the events)
    ust = min(args.steps, 500)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(ust):
        step()
    torch.cuda.synchronize()
    unprof_ms = (time.perf_counter() - t1) / ust * 1e3

    te = w.s * w.T
    value = te * args.steps / elapsed
    eval_ms, eval_n = kern["eval"]
    eval_avg_s = eval_ms / max(eval_n, 1) / 1e3
    te_per_launch = te * args.steps / max(eval_n, 1)
    # the boundary's host form: peval_run into a page-locked host buffer
    # (the rate including the device-to-host copy of the images)
    host_out = None
    if not points_mode:
        hb = torch.empty((w.T, poly.G), dtype=dt, pin_memory=True).numpy().view(poly.dtype)
        poly.run(w.beta, w.T, out=hb)
        hsteps = min(args.steps, 200)
        t3 = time.perf_counter()
        for _ in range(hsteps):
            poly.run(w.beta, w.T, out=hb)
        hel = time.perf_counter() - t3
        host_out = {"ms_per_step": hel / hsteps * 1e3, "value": te * hsteps / hel, "steps": hsteps,
                    "output_MB": w.T * poly.G * poly.elem_bytes / 1e6}
    # the whole pass as one replay of a captured graph (a batch of one): no
    # per-kernel launch cost on the host
    graph = None
    if not points_mode:
        b = PV.Batch([poly], [w.T])
        for _ in range(3):
            b.run([w.beta], [out], stream=stream)
        torch.cuda.synchronize()
        gsteps = min(args.steps, 500)
        t2 = time.perf_counter()
        for _ in range(gsteps):
            b.run([w.beta], [out], stream=stream)
        torch.cuda.synchronize()
        gel = time.perf_counter() - t2
        b.destroy()
        graph = {"ms_per_step": gel / gsteps * 1e3, "value": te * gsteps / gel, "steps": gsteps}
    arith = poly.arith()
    if points_mode:
        ops = points_ops(poly.elem_bytes, nf, arith)
        kname = "points_eval_kernel"
    else:
        ops = ALGO_OPS["fp64" if arith == "fp64" else poly.elem_bytes]
        kname = "small_run_kernel" if single else "eval_kernel"
    achieved = ops * te_per_launch / eval_avg_s
    sha = kernel_source_sha(kname)
    traffic = profile_traffic(sha, args.workload, kname, None if (single or points_mode) else (K, P, C))
    # algorithmic HBM bytes of one step: the resident term data read once
    # (coefficient and n-2 16-bit exponents per term) and the images written
    # once; against the HBM peak they give the step's bandwidth fraction
    algo_bytes = w.s * (poly.elem_bytes + 2 * (w.n - 2)) + w.T * poly.G * poly.elem_bytes
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (int32 lane-ops)", "frac": achieved / VALU_PEAK_OPS,
            "traffic": traffic, "kernel": kname, "ops_per_term_eval": ops,
            "eval_launch_ms": eval_avg_s * 1e3, "kernel_source_sha256": sha,
            "hbm_algorithmic_bytes_per_step": algo_bytes,
            "hbm_frac": algo_bytes / (elapsed / args.steps) / HBM_PEAK,
            "traffic_frac": (traffic / eval_avg_s / HBM_PEAK) if traffic else None}
    if points_mode:
        roof["factor_tables"] = {"nf": nf, "entries_per_point": E}
    else:
        # the same product and sum alone at full occupancy (microbenchmark):
        # the rate of the evaluation loop without its stage, walk and memory
        mb_kind = {"fp64": 2, "pm": 3 if poly.elem_bytes == 8 else 4}.get(arith, 0 if poly.elem_bytes == 8 else 1)
        mb_rate, _ = bench_product(mb_kind, w.p, target_ms=40.0)
        roof["measured_product_ceiling"] = {"kind": [k for k in MB_PRODUCTS if k[1] == mb_kind][0][0],
                                            "products_per_s": mb_rate,
                                            "frac": te_per_launch / eval_avg_s / mb_rate}

    got = out.cpu().numpy().view(poly.dtype)
    res = {
        "metric": METRIC, "value": value, "unit": "term-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak",
        # the paper's Table 2 times this exact workload shape (best: 1411 ms on
        # one AVX-512 core = 3.54e9 term-evals/s); other configurations have no
        # published number
        "vs_baseline": (value / (5e9 / 1.411)) if args.workload == "paper_table2" else None,
        "dtype": "f64" if arith == "fp64" else ("u64" if poly.elem_bytes == 8 else "u32"),
        "data": "synthetic",
        "config": {"workload": w.name + ("_random_points" if points_mode else ""), "n": w.n, "s": w.s,
                   "T": w.T, "p": w.p, "G": poly.G,
                   "tuning": "single_launch" if single else {"K": K, "P": P, "C": C},
                   "tuning_source": "explicit" if args.tuning else ("autotuned" if tuned else "heuristic"),
                   "autotune": tuned,
                   "arith": arith,
                   "points": "uniform random in [1,p)^(n-2)" if points_mode else "powers of one base point"},
        "roofline": roof,
        "kernels_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in kern.items()},
        "step_ms_spread": spread,
        "unprofiled_ms_per_step": unprof_ms,
        "graph_replay": graph,
        "host_output": host_out,
        "create_s": create_s,
    }

    if not args.no_cpu:
        from oracle import Oracle
        orc = Oracle()
        # the sample: half the images from the start of the run, half from its
        # end (the last rows come from the far end of every chain)
        rows = min(args.cpu_rows or max(8, int(round(1.6e8 / max(w.s, 1)))), w.T)
        head = (rows + 1) // 2
        tail_t0 = w.T - (rows - head) + 1
        threads = min(args.cpu_threads, rows)
        c0 = time.perf_counter()
        if points_mode:
            ref = np.concatenate([orc.evaluate_points(w.p, w.exps, w.coeffs, pts[:head], threads=threads),
                                  orc.evaluate_points(w.p, w.exps, w.coeffs, pts[tail_t0 - 1:], threads=threads)])
        else:
            ref = np.concatenate([orc.evaluate(w.p, w.exps, w.coeffs, w.beta, head, t0=1, threads=threads),
                                  orc.evaluate(w.p, w.exps, w.coeffs, w.beta, rows - head, t0=tail_t0,
                                               threads=threads)])
        csec = time.perf_counter() - c0
        # one thread on a few images: the per-core rate (comparable with the
        # paper's single-core timings)
        rows1 = min(2, rows)
        c1 = time.perf_counter()
        if points_mode:
            orc.evaluate_points(w.p, w.exps, w.coeffs, pts[:rows1], threads=1)
        else:
            orc.evaluate(w.p, w.exps, w.coeffs, w.beta, rows1, t0=1, threads=1)
        csec1 = time.perf_counter() - c1
        res["cpu_baseline"] = {"value": w.s * rows / csec, "unit": "term-evals/s", "cores": threads,
                               "kind": "oracle", "seconds": csec,
                               "sample": f"images 1..{head} and {tail_t0}..{w.T} of the same polynomial "
                                         f"(all {w.s} terms), {threads} threads over the points",
                               "single_thread_value": w.s * rows1 / csec1,
                               "single_thread_sample": f"the first {rows1} images, one thread",
                               "cpu_model": cpu_model(), "host_threads": os.cpu_count()}
        sel = np.r_[0:head, tail_t0 - 1:w.T]
        res["parity_sample"] = bool(np.array_equal(got[sel].astype(np.uint64), ref))
        res["parity_rows"] = int(rows)
    poly.destroy()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
