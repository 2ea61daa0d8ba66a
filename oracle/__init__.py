"""CPU oracle for partial modular polynomial evaluation (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the HIP path.

The C source ``peval_oracle.c`` evaluates the plain definition of the
bivariate images (paper, Section 2.1 and Section 2.3, Eq. (1)):

    out[t - t0][g] = sum_{i in group g} a_i * prod_{k>=3} (beta_k^t)^{g_ik}  mod p

with groups = distinct (x1, x2) exponent pairs in descending lexicographic
order, and the same images at T arbitrary points x_t in place of beta^t
(``evaluate_points``), and the inverse step: the coefficients recovered
from the images by solving each group's Vandermonde system
(``interpolate``).  Parity status of each function is recorded in the test suite's pins
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "peval_oracle.c")
_LIB = os.path.join(_HERE, "libpeval_oracle.so")


def build(out_path: str = _LIB, src: str = _SRC, extra_flags=()) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", *extra_flags,
           src, "-o", out_path]
    subprocess.run(cmd, check=True)
    return out_path


def load(path: str = _LIB) -> ctypes.CDLL:
    if not os.path.exists(path) or (path == _LIB and os.path.getmtime(path) < os.path.getmtime(_SRC)):
        build(path)
    lib = ctypes.CDLL(path)
    u64, u32, ptr = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    lib.oracle_groups.argtypes = [u64, u32, ptr, ptr, ptr, ptr]
    lib.oracle_groups.restype = ctypes.c_int
    lib.oracle_eval.argtypes = [u64, u32, u64, ptr, ptr, ptr, u64, u64, ptr, u32]
    lib.oracle_eval.restype = ctypes.c_int
    lib.oracle_entry.argtypes = [u64, u32, u64, ptr, ptr, ptr, u64, u32, u32]
    lib.oracle_entry.restype = u64
    lib.oracle_eval_points.argtypes = [u64, u32, u64, ptr, ptr, ptr, u64, ptr, u32]
    lib.oracle_eval_points.restype = ctypes.c_int
    lib.oracle_interpolate.argtypes = [u64, u32, u64, ptr, ptr, u64, ptr, ptr]
    lib.oracle_interpolate.restype = ctypes.c_int
    return lib


class SingularError(ArithmeticError):
    pass


class Oracle:
    """Thin ctypes wrapper; every array is converted to a contiguous copy."""

    def __init__(self, path: str = _LIB):
        self.lib = load(path)

    @staticmethod
    def _prep(exps, coeffs, beta):
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        if exps.ndim != 2:
            raise ValueError("exps must be (s, n)")
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        beta = np.ascontiguousarray(beta, dtype=np.uint64)
        s, n = exps.shape
        if coeffs.shape != (s,) or beta.shape != (max(n - 2, 0),):
            raise ValueError("shape mismatch")
        return exps, coeffs, beta, s, n

    def groups(self, exps):
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        s, n = exps.shape
        gd = np.zeros(max(s, 1), np.uint32)
        ge = np.zeros(max(s, 1), np.uint32)
        G = ctypes.c_uint64(0)
        rc = self.lib.oracle_groups(s, n, exps.ctypes.data, gd.ctypes.data, ge.ctypes.data,
                                    ctypes.byref(G))
        if rc != 0:
            raise MemoryError("oracle_groups failed")
        return gd[:G.value].copy(), ge[:G.value].copy()

    def evaluate(self, p, exps, coeffs, beta, T, t0=1, threads=1):
        """(T, G) uint64 array, row j = b_{t0+j}."""
        exps, coeffs, beta, s, n = self._prep(exps, coeffs, beta)
        gd, _ = self.groups(exps)
        G = gd.size
        out = np.zeros((T, G), np.uint64)
        if T and G:
            rc = self.lib.oracle_eval(p, n, s, exps.ctypes.data, coeffs.ctypes.data,
                                      beta.ctypes.data, t0, T, out.ctypes.data, threads)
            if rc != 0:
                raise RuntimeError(f"oracle_eval failed ({rc})")
        return out

    def evaluate_points(self, p, exps, coeffs, points, threads=1):
        """(T, G) uint64 array, row t = the images at the point points[t]
        (T rows of n-2 values for x3..xn)."""
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint64)
        s, n = exps.shape
        points = np.ascontiguousarray(points, dtype=np.uint64)
        if points.ndim != 2 or points.shape[1] != n - 2:
            raise ValueError("points must be (T, n-2)")
        if coeffs.shape != (s,):
            raise ValueError("shape mismatch")
        T = points.shape[0]
        gd, _ = self.groups(exps)
        G = gd.size
        out = np.zeros((T, G), np.uint64)
        if T and G:
            rc = self.lib.oracle_eval_points(p, n, s, exps.ctypes.data, coeffs.ctypes.data,
                                             points.ctypes.data, T, out.ctypes.data, threads)
            if rc != 0:
                raise RuntimeError(f"oracle_eval_points failed ({rc})")
        return out

    def interpolate(self, p, exps, beta, images):
        """Coefficients (s,) uint64 of the support ``exps`` from the images
        b_1..b_T (a (T, G) array in the column order of ``groups``), solving
        each group's Vandermonde system by elimination.  Raises
        ``SingularError`` when a group's system is singular."""
        exps = np.ascontiguousarray(exps, dtype=np.uint32)
        s, n = exps.shape
        beta = np.ascontiguousarray(beta, dtype=np.uint64)
        images = np.ascontiguousarray(images, dtype=np.uint64)
        if beta.shape != (n - 2,) or images.ndim != 2:
            raise ValueError("shape mismatch")
        out = np.zeros(s, np.uint64)
        rc = self.lib.oracle_interpolate(p, n, s, exps.ctypes.data, beta.ctypes.data, images.shape[0],
                                         images.ctypes.data, out.ctypes.data)
        if rc == -3:
            raise SingularError("a group's Vandermonde system is singular")
        if rc != 0:
            raise RuntimeError(f"oracle_interpolate failed ({rc})")
        return out

    def entry(self, p, exps, coeffs, beta, t, d, e):
        exps, coeffs, beta, s, n = self._prep(exps, coeffs, beta)
        return int(self.lib.oracle_entry(p, n, s, exps.ctypes.data, coeffs.ctypes.data,
                                         beta.ctypes.data, t, d, e))
