"""ctypes binding of libpeval (include/peval.h).  Argument marshalling only:
every step of the evaluation runs in the HIP library.

PyTorch is used by callers only for device memory and streams; this module
accepts raw device pointers or torch tensors (``.data_ptr()``) and raw
stream handles or torch streams (``.cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpeval.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY, ETIMEOUT, ESINGULAR = 0, -1, -2, -3, -4, -5, -6, -7


class PevalError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"peval error {code}: {msg}")
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("n", ctypes.c_uint32), ("elem_bytes", ctypes.c_uint32),
                ("s", ctypes.c_uint64), ("G", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("max_exp", ctypes.c_uint32 * 32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "queued", "active",
                                                "passes", "term_evals", "uploads", "evictions", "slices",
                                                "hbm_in_use", "hbm_peak")] + \
               [(n, ctypes.c_double) for n in ("wall_s", "p50_ms", "p99_ms", "max_ms", "mean_ms", "host_pass_s",
                                               "gpu_pass_s")]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the built library (never builds, never falls back)."""
    global _lib
    if _lib is not None:
        return _lib
    # The library must share PyTorch's HIP runtime (PyTorch ships its own
    # libamdhip64 with the same soname): load torch first so that the dynamic
    # loader binds libpeval to that runtime instead of a second copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_2004_11571_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    sig = {
        "peval_create": ([u64, u32, u64, vp, vp, ctypes.POINTER(vp)], i32),
        "peval_info": ([vp, ctypes.POINTER(_Info)], i32),
        "peval_groups": ([vp, vp, vp], i32),
        "peval_run": ([vp, vp, u32, vp], i32),
        "peval_run_async": ([vp, vp, u64, u32, vp, vp], i32),
        "peval_run_async_noalloc": ([vp, vp, u64, u32, vp, vp], i32),
        "peval_run_points": ([vp, vp, u32, vp], i32),
        "peval_run_points_async": ([vp, vp, u32, vp, vp], i32),
        "peval_points_factors": ([u32, u32, vp, vp, vp], i32),
        "peval_interpolate": ([vp, vp, u32, vp, vp], i32),
        "peval_interpolate_async": ([vp, vp, u32, vp, vp, vp, vp], i32),
        "peval_destroy": ([vp], i32),
        "peval_set_tuning": ([vp, u32, u32, u32], i32),
        "peval_get_tuning": ([vp, u32, vp, vp, vp], i32),
        "peval_points_tuning": ([vp, u32, vp, vp, vp], i32),
        "peval_prof_enable": ([i32], i32),
        "peval_prof_read": ([vp, vp], i32),
        "peval_layout": ([vp, u64, u32, u32, vp, vp, vp, vp, vp, vp], i32),
        "peval_autotune": ([vp, vp, u32, u32, vp, vp, vp, vp], i32),
        "peval_set_arith": ([vp, u32], i32),
        "peval_get_arith": ([vp, vp], i32),
        "peval_server_create": ([u64, u32, ctypes.POINTER(vp)], i32),
        "peval_server_configure": ([vp, ctypes.c_double, ctypes.c_double, u32, ctypes.c_double], i32),
        "peval_server_add_poly": ([vp, u64, u32, u64, vp, vp, ctypes.POINTER(u64)], i32),
        "peval_server_remove_poly": ([vp, u64], i32),
        "peval_server_poly_info": ([vp, u64, ctypes.POINTER(_Info)], i32),
        "peval_server_submit": ([vp, u64, vp, u32, vp, ctypes.POINTER(u64)], i32),
        "peval_server_poll": ([vp, u64, ctypes.POINTER(ctypes.c_int)], i32),
        "peval_server_wait": ([vp, u64, ctypes.c_int64], i32),
        "peval_server_release": ([vp, u64], i32),
        "peval_server_next_done": ([vp, ctypes.c_int64, ctypes.POINTER(u64)], i32),
        "peval_server_stats": ([vp, ctypes.POINTER(_ServerStats)], i32),
        "peval_server_reset_stats": ([vp], i32),
        "peval_server_destroy": ([vp], i32),
        "peval_batch_create": ([u32, vp, vp, u32, ctypes.POINTER(vp)], i32),
        "peval_batch_run": ([vp, vp, vp, vp, vp], i32),
        "peval_batch_info": ([vp, vp], i32),
        "peval_batch_members": ([vp, vp, vp, vp, vp, vp], i32),
        "peval_batch_kinds": ([vp, vp, vp], i32),
        "peval_batch_destroy": ([vp], i32),
        "peval_tune_clear": ([], i32),
        "peval_tune_save": ([ctypes.c_char_p], i32),
        "peval_tune_load": ([ctypes.c_char_p], i32),
        "peval_test_arith": ([u32, u64, u64, vp, vp, vp, vp], i32),
        "peval_bench_product": ([u32, u64, u32, u32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)], i32),
        "peval_test_deal_points": ([u32, u32, u64, vp, u64, vp, u32, vp, u64], i32),
        "peval_strerror": ([i32], ctypes.c_char_p),
        "peval_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        L = lib()
        raise PevalError(rc, f"{L.peval_strerror(rc).decode()}: {L.peval_last_error().decode()}")


def _ptr(x) -> int:
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    return int(x)


def _stream(st) -> int:
    if st is None:
        return 0
    if hasattr(st, "cuda_stream"):
        return int(st.cuda_stream)
    return int(st)


def out_dtype(p: int):
    return np.uint32 if p < (1 << 31) else np.uint64


class Poly:
    """A polynomial resident on the current HIP device (peval_create)."""

    def __init__(self, p: int, exps, coeffs):
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        if exps.ndim != 2 or coeffs.shape != (exps.shape[0],):
            raise ValueError("exps must be (s, n) and coeffs (s,)")
        s, n = exps.shape
        h = ctypes.c_void_p()
        _check(lib().peval_create(p, n, s, exps.ctypes.data, coeffs.ctypes.data, ctypes.byref(h)))
        self._h = h
        inf = self.info()
        self.p, self.n, self.s, self.G = inf["p"], inf["n"], inf["s"], inf["G"]
        self.elem_bytes = inf["elem_bytes"]
        self.dtype = np.uint32 if self.elem_bytes == 4 else np.uint64

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("polynomial destroyed")
        return self._h

    def info(self) -> dict:
        inf = _Info()
        _check(lib().peval_info(self.handle, ctypes.byref(inf)))
        return {"p": inf.p, "n": inf.n, "elem_bytes": inf.elem_bytes, "s": inf.s, "G": inf.G,
                "device_bytes": inf.device_bytes, "max_exp": list(inf.max_exp)[: inf.n]}

    def groups(self) -> Tuple[np.ndarray, np.ndarray]:
        d = np.zeros(max(self.G, 1), np.uint32)
        e = np.zeros(max(self.G, 1), np.uint32)
        _check(lib().peval_groups(self.handle, d.ctypes.data, e.ctypes.data))
        return d[: self.G], e[: self.G]

    def _beta(self, beta) -> np.ndarray:
        b = np.ascontiguousarray(beta, dtype=np.uint64)
        if b.shape != (self.n - 2,):
            raise ValueError(f"beta must have n-2 = {self.n - 2} entries")
        return b

    def run(self, beta, T: int, out=None) -> np.ndarray:
        """(T, G) images b_1..b_T in host memory (``out``: a C-contiguous
        (T, G) array of the handle's dtype to fill, e.g. page-locked)."""
        b = self._beta(beta)
        if out is None:
            out = np.zeros((T, self.G), self.dtype)
        elif out.shape != (T, self.G) or out.dtype != self.dtype or not out.flags.c_contiguous:
            raise ValueError(f"out must be a C-contiguous ({T}, {self.G}) {np.dtype(self.dtype).name} array")
        _check(lib().peval_run(self.handle, b.ctypes.data if b.size else None, T,
                               out.ctypes.data if out.size else None))
        return out

    def run_async(self, beta, T: int, dev_out, t0: int = 1, stream=None):
        """Enqueue b_{t0}..b_{t0+T-1} into device memory ``dev_out``."""
        b = self._beta(beta)
        _check(lib().peval_run_async(self.handle, b.ctypes.data if b.size else None, t0, T,
                                     _ptr(dev_out), _stream(stream)))

    def run_async_noalloc(self, beta, T: int, dev_out, t0: int = 1, stream=None):
        """run_async without device allocation: the scratch is the library's
        fixed per-GPU region (the handle needs a thread layout for the run's
        tuning, made by an earlier run_async)."""
        b = self._beta(beta)
        _check(lib().peval_run_async_noalloc(self.handle, b.ctypes.data if b.size else None, t0, T,
                                             _ptr(dev_out), _stream(stream)))

    def _points(self, points):
        pts = np.ascontiguousarray(points, dtype=np.uint64)
        if pts.ndim != 2 or pts.shape[1] != self.n - 2:
            raise ValueError(f"points must be (T, {self.n - 2})")
        return pts

    def run_points(self, points) -> np.ndarray:
        """(T, G) images at the T rows of ``points`` (x3..xn each), host memory."""
        pts = self._points(points)
        T = pts.shape[0]
        out = np.zeros((T, self.G), self.dtype)
        _check(lib().peval_run_points(self.handle, pts.ctypes.data if pts.size else None, T,
                                      out.ctypes.data if out.size else None))
        return out

    def run_points_async(self, points_dev, T: int, dev_out, stream=None):
        """Enqueue the images at T points held in device memory (T x (n-2)
        uint64, e.g. a torch tensor) into device memory ``dev_out``."""
        _check(lib().peval_run_points_async(self.handle, _ptr(points_dev) or None, T, _ptr(dev_out),
                                            _stream(stream)))

    def interpolate(self, beta, images) -> np.ndarray:
        """Coefficients (s,) uint64, in the order of the rows given at
        creation, recovered from the images b_1..b_T (a (T, G) array) taken
        at base point ``beta``; raises PevalError(ESINGULAR) if a group's
        system is singular."""
        b = self._beta(beta)
        img = np.ascontiguousarray(images, dtype=self.dtype)
        if img.ndim != 2 or img.shape[1] != self.G:
            raise ValueError(f"images must be (T, {self.G})")
        out = np.zeros(self.s, np.uint64)
        _check(lib().peval_interpolate(self.handle, b.ctypes.data if b.size else None, img.shape[0],
                                       img.ctypes.data if img.size else None, out.ctypes.data if out.size else None))
        return out

    def interpolate_async(self, beta, T: int, dev_images, dev_coeffs, dev_status, stream=None):
        """Device-memory form: images (T, G), coefficients (s,) uint64 and a
        device int32 status word (set to 1 if some group is singular)."""
        b = self._beta(beta)
        _check(lib().peval_interpolate_async(self.handle, b.ctypes.data if b.size else None, T, _ptr(dev_images),
                                             _ptr(dev_coeffs), _ptr(dev_status), _stream(stream)))

    def set_arith(self, mode: str = "auto"):
        """'auto' / 'int' (Shoup products), 'fp64' (the paper's Alg. 2, 2^31 <= p < 2^50) or
        'pm' (pseudo-Mersenne folding, p = 2^63 - c or 2^31 - c with small c)."""
        _check(lib().peval_set_arith(self.handle, {"auto": 0, "int": 1, "fp64": 2, "pm": 3}[mode]))

    def arith(self) -> str:
        """The product the evaluation kernel uses now: 'int' or 'fp64'."""
        m = ctypes.c_uint32()
        _check(lib().peval_get_arith(self.handle, ctypes.byref(m)))
        return {2: "fp64", 3: "pm"}.get(m.value, "int")

    def set_tuning(self, K: int = 0, P: int = 0, C: int = 0):
        _check(lib().peval_set_tuning(self.handle, K, P, C))

    def get_tuning(self, T: int) -> Tuple[int, int, int]:
        """(K, P, C) of the next run of T evaluations; (0, 0, 0) for the single-launch path."""
        k, p, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().peval_get_tuning(self.handle, T, ctypes.byref(k), ctypes.byref(p), ctypes.byref(c)))
        return k.value, p.value, c.value

    def points_tuning(self, T: int) -> Tuple[int, int, int]:
        """(K, P, C) of the next point-mode run with T points."""
        k, p, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().peval_points_tuning(self.handle, T, ctypes.byref(k), ctypes.byref(p), ctypes.byref(c)))
        return k.value, p.value, c.value

    def autotune(self, beta, T: int, exhaustive: bool = False):
        """Time candidate (K, P, C) for this polynomial and T; returns (K, P, C, ms),
        with K = P = C = 0 if the single-launch path was fastest."""
        b = self._beta(beta)
        k, pp, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        ms = ctypes.c_float()
        _check(lib().peval_autotune(self.handle, b.ctypes.data if b.size else None, T, int(exhaustive),
                                    ctypes.byref(k), ctypes.byref(pp), ctypes.byref(c), ctypes.byref(ms)))
        return k.value, pp.value, c.value, ms.value

    def destroy(self):
        if self._h is not None:
            _check(lib().peval_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


BATCH_NO_GRAPH = 1
BATCH_TUNE = 2
BATCH_PASS8 = 4


class Batch:
    """A planned batched pass over resident polynomials (peval_batch_*)."""

    def __init__(self, polys, Ts, graph: bool = True, tune: bool = False, pass8: bool = False):
        self.polys = list(polys)
        self.Ts = [int(t) for t in Ts]
        if len(self.polys) != len(self.Ts) or not self.polys:
            raise ValueError("polys and Ts must be non-empty and of equal length")
        hs = (ctypes.c_void_p * len(self.polys))(*[q.handle.value for q in self.polys])
        ts = np.ascontiguousarray(self.Ts, dtype=np.uint32)
        b = ctypes.c_void_p()
        flags = (0 if graph else BATCH_NO_GRAPH) | (BATCH_TUNE if tune else 0) | (BATCH_PASS8 if pass8 else 0)
        _check(lib().peval_batch_create(len(self.polys), hs, ts.ctypes.data, flags, ctypes.byref(b)))
        self._b = b

    def members(self) -> dict:
        """Per member: terms per thread K, chains C and kernel kind; the
        tuner's pass time (ms) and number of timed candidates (0: untuned)."""
        n = len(self.polys)
        K, C, kind = (np.zeros(n, np.uint32) for _ in range(3))
        ms, trials = ctypes.c_float(), ctypes.c_uint32()
        _check(lib().peval_batch_members(self._b, K.ctypes.data, C.ctypes.data, kind.ctypes.data,
                                         ctypes.byref(ms), ctypes.byref(trials)))
        return {"K": K, "C": C, "kind": kind, "tuned_ms": ms.value, "tune_trials": trials.value}

    def kinds(self) -> dict:
        """Per kind of member (0..4): evaluations per pass P and persistent
        blocks of its kernel (0 where the batch has no such member)."""
        P, blocks = np.zeros(5, np.uint32), np.zeros(5, np.uint32)
        _check(lib().peval_batch_kinds(self._b, P.ctypes.data, blocks.ctypes.data))
        return {"P": P, "blocks": blocks}

    def info(self) -> dict:
        v = np.zeros(5, np.uint64)
        _check(lib().peval_batch_info(self._b, v.ctypes.data))
        return {"members": int(v[0]), "items": int(v[1]), "blocks": int(v[2]),
                "scratch_bytes": int(v[3]), "term_evals": int(v[4])}

    def run(self, betas, dev_outs, t0s=None, stream=None):
        n = len(self.polys)
        bs = [np.ascontiguousarray(b, dtype=np.uint64) for b in betas]
        self._keep = bs
        bp = (ctypes.c_void_p * n)(*[b.ctypes.data if b.size else None for b in bs])
        op = (ctypes.c_void_p * n)(*[_ptr(o) for o in dev_outs])
        t0 = None
        if t0s is not None:
            t0 = np.ascontiguousarray(t0s, dtype=np.uint64)
        _check(lib().peval_batch_run(self._b, bp, t0.ctypes.data if t0 is not None else None, op, _stream(stream)))

    def destroy(self):
        if getattr(self, "_b", None) is not None:
            _check(lib().peval_batch_destroy(self._b))
            self._b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


SERVER_SIMULATE = 1


class Server:
    """Request loop over resident polynomials (peval_server_*)."""

    def __init__(self, hbm_budget_bytes: int, simulate: bool = False):
        s = ctypes.c_void_p()
        _check(lib().peval_server_create(int(hbm_budget_bytes), SERVER_SIMULATE if simulate else 0, ctypes.byref(s)))
        self._s = s
        self._outs = {}
        self._meta = {}

    def configure(self, slice_work: float = 2e9, pass_work: float = 1.5e10, max_members: int = 512,
                  sim_rate: float = 1e12):
        _check(lib().peval_server_configure(self._s, float(slice_work), float(pass_work), int(max_members),
                                            float(sim_rate)))

    def add_poly(self, p: int, exps, coeffs) -> int:
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        s, n = exps.shape
        pid = ctypes.c_uint64()
        _check(lib().peval_server_add_poly(self._s, p, n, s, exps.ctypes.data if s else None,
                                           coeffs.ctypes.data if s else None, ctypes.byref(pid)))
        inf = self.poly_info(pid.value)
        self._meta[pid.value] = (inf["p"], inf["n"], inf["G"])
        return pid.value

    def poly_info(self, pid: int) -> dict:
        """Modulus, sizes and output columns G of a registered polynomial."""
        inf = _Info()
        _check(lib().peval_server_poly_info(self._s, pid, ctypes.byref(inf)))
        return {"p": inf.p, "n": inf.n, "elem_bytes": inf.elem_bytes, "s": inf.s, "G": inf.G,
                "device_bytes": inf.device_bytes, "max_exp": list(inf.max_exp)[: inf.n]}

    def remove_poly(self, pid: int):
        _check(lib().peval_server_remove_poly(self._s, pid))
        self._meta.pop(pid, None)

    def submit(self, pid: int, beta, T: int, out: Optional[np.ndarray] = None) -> int:
        if pid not in self._meta:  # not registered (or removed): the library refuses it
            rid = ctypes.c_uint64()
            _check(lib().peval_server_submit(self._s, pid, None, T, None, ctypes.byref(rid)))
        p, n, G = self._meta[pid]
        if out is None:
            out = np.zeros((T, G), out_dtype(p))
        b = np.ascontiguousarray(beta, dtype=np.uint64)
        rid = ctypes.c_uint64()
        _check(lib().peval_server_submit(self._s, pid, b.ctypes.data if b.size else None, T,
                                         out.ctypes.data if out.size else None, ctypes.byref(rid)))
        self._outs[rid.value] = out
        return rid.value

    def poll(self, rid: int) -> bool:
        d = ctypes.c_int()
        _check(lib().peval_server_poll(self._s, rid, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid: int, timeout_ms: int = -1) -> np.ndarray:
        _check(lib().peval_server_wait(self._s, rid, timeout_ms))
        return self._outs[rid]

    def next_done(self, timeout_ms: int = -1) -> int:
        """Id of the next finished request (completion order)."""
        rid = ctypes.c_uint64()
        _check(lib().peval_server_next_done(self._s, timeout_ms, ctypes.byref(rid)))
        return rid.value

    def release(self, rid: int):
        _check(lib().peval_server_release(self._s, rid))
        self._outs.pop(rid, None)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().peval_server_stats(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def reset_stats(self):
        _check(lib().peval_server_reset_stats(self._s))

    def destroy(self):
        if getattr(self, "_s", None) is not None:
            _check(lib().peval_server_destroy(self._s))
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tune_clear():
    _check(lib().peval_tune_clear())


def tune_save(path: str):
    _check(lib().peval_tune_save(path.encode()))


def tune_load(path: str):
    _check(lib().peval_tune_load(path.encode()))


def prof_enable(on: bool = True):
    _check(lib().peval_prof_enable(1 if on else 0))


KERNEL_KINDS = ("power_table", "monomial", "eval", "combine")


def prof_read() -> dict:
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_uint64 * 4)()
    _check(lib().peval_prof_read(ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_KINDS)}


def points_factors(w: int, maxdeg) -> Tuple[int, int]:
    """Host-only plan of the point mode's tables: (factors, entries per point)."""
    d = np.ascontiguousarray(maxdeg, dtype=np.uint32)
    nf, E = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().peval_points_factors(w, d.size, d.ctypes.data if d.size else None, ctypes.byref(nf),
                                      ctypes.byref(E)))
    return nf.value, E.value


def layout(group_sizes, K: int, P: int) -> dict:
    """Host-only thread layout of the evaluation kernel (peval_layout)."""
    gs = np.ascontiguousarray(group_sizes, dtype=np.uint64)
    sizes = np.zeros(3, np.uint64)
    L = lib()
    _check(L.peval_layout(gs.ctypes.data if gs.size else None, gs.size, K, P, sizes.ctypes.data,
                          None, None, None, None, None))
    NT, NW, ns = (int(x) for x in sizes)
    thr_first = np.zeros(NT, np.uint32)
    thr_cnt = np.zeros(NT, np.uint8)
    endmask = np.zeros(NW, np.uint64)
    slot_base = np.zeros(NW, np.uint32)
    slot_off = np.zeros(gs.size + 1, np.uint32)
    _check(L.peval_layout(gs.ctypes.data if gs.size else None, gs.size, K, P, sizes.ctypes.data,
                          thr_first.ctypes.data, thr_cnt.ctypes.data, endmask.ctypes.data,
                          slot_base.ctypes.data, slot_off.ctypes.data))
    return {"NT": NT, "NW": NW, "nslots": ns, "thr_first": thr_first, "thr_cnt": thr_cnt,
            "endmask": endmask, "slot_base": slot_base, "slot_off": slot_off}


def deal_points(w: int, tail_exps, group_sizes, K: int) -> np.ndarray:
    """Host-only: the point kernel's term of each thread slot, [K][NT]
    (peval_test_deal_points; tail_exps is (n - 2) x s, variable-major)."""
    ex = np.ascontiguousarray(tail_exps, dtype=np.uint16)
    gs = np.ascontiguousarray(group_sizes, dtype=np.uint64)
    ntail, s = (int(x) for x in ex.shape)
    NT = layout(gs, K, 8)["NT"]
    out = np.zeros((K, NT), np.uint32)
    _check(lib().peval_test_deal_points(w, ntail, s, ex.ctypes.data if ex.size else None, gs.size,
                                        gs.ctypes.data if gs.size else None, K, out.ctypes.data, out.size))
    return out
