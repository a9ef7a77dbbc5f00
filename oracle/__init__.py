"""TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it.

``cr_oracle.c`` implements block cyclic reduction for Hermitian positive
definite block-tridiagonal systems from the paper (arXiv 1807.00370): the
one-sided reduction (``solve_cr``), Algorithm 1 as printed with recursion on
both half systems (``solve_pcr``), the one-sided reduction finished by
Algorithm 1 below a block count (``solve_hybrid``), a block Cholesky cross-check
(``solve_thomas``), one split of Eq. (Formulas) (``split``), the residual of
Eq. (Axb) and the adjoint (gradient) formulas.  All arithmetic is FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cr_oracle.c")
_LIB = os.path.join(_HERE, "libcr_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over independent blocks of a level)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-fcx-limited-range", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("level", ctypes.c_int32), ("block", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for name in ("cro_solve_cr", "cro_solve_pcr", "cro_solve_thomas"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.POINTER(_Info)]
            f.restype = ctypes.c_int
        lib.cro_solve_hybrid.argtypes = [ctypes.c_int] * 4 + [P] * 4 + [ctypes.POINTER(_Info)]
        lib.cro_solve_hybrid.restype = ctypes.c_int
        lib.cro_split.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [P] * 9
        lib.cro_split.restype = ctypes.c_int
        lib.cro_residual.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [P] * 5
        lib.cro_residual.restype = None
        lib.cro_backward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [P] * 4
        lib.cro_backward.restype = None
        lib.cro_num_threads.argtypes = []
        lib.cro_num_threads.restype = ctypes.c_int
        lib.cro_set_num_threads.argtypes = [ctypes.c_int]
        lib.cro_set_num_threads.restype = None
        _lib = lib
    return _lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _shape(A, B, y):
    A, B, y = _c(A), _c(B), _c(y)
    N, m, m2 = A.shape
    if m != m2 or y.shape[:2] != (N, m) or B.shape != (max(N - 1, 0), m, m):
        raise ValueError("shape mismatch: A %s B %s y %s" % (A.shape, B.shape, y.shape))
    if B.size == 0:
        B = np.zeros((1, m, m), np.complex128)
    return A, B, y, N, m, y.shape[2]


def _solve(name, A, B, y):
    A, B, y, N, m, k = _shape(A, B, y)
    x = np.empty((N, m, k), np.complex128)
    info = _Info()
    rc = getattr(_load(), name)(N, m, k, _ptr(A), _ptr(B), _ptr(y), _ptr(x), ctypes.byref(info))
    if rc != 0:
        raise ValueError("%s: invalid arguments" % name)
    return x, dict(status=int(info.status), level=int(info.level), block=int(info.block))


def solve_cr(A, B, y):
    """One-sided cyclic reduction; returns (x, info)."""
    return _solve("cro_solve_cr", A, B, y)


def solve_pcr(A, B, y):
    """Algorithm 1 (recursion on both half systems); returns (x, info)."""
    return _solve("cro_solve_pcr", A, B, y)


def solve_hybrid(A, B, y, tail_blocks):
    """One-sided reduction until a level holds at most ``tail_blocks`` blocks,
    then Algorithm 1 on that level's system; returns (x, info)."""
    A, B, y, N, m, k = _shape(A, B, y)
    x = np.empty((N, m, k), np.complex128)
    info = _Info()
    rc = _load().cro_solve_hybrid(N, m, k, int(tail_blocks), _ptr(A), _ptr(B), _ptr(y), _ptr(x),
                                  ctypes.byref(info))
    if rc != 0:
        raise ValueError("cro_solve_hybrid: invalid arguments")
    return x, dict(status=int(info.status), level=int(info.level), block=int(info.block))


def solve_thomas(A, B, y):
    """Block Cholesky of the block-tridiagonal matrix; returns (x, info)."""
    return _solve("cro_solve_thomas", A, B, y)


def split(A, B, y):
    """One split (Eq. (Formulas)) of an even-sized system.

    Returns (U, E, u, V, F, v, failed)."""
    A, B, y, N, m, k = _shape(A, B, y)
    h = N // 2
    U = np.zeros((h, m, m), np.complex128); V = np.zeros_like(U)
    E = np.zeros((max(h, 1), m, m), np.complex128); F = np.zeros_like(E)
    u = np.zeros((h, m, k), np.complex128); v = np.zeros_like(u)
    rc = _load().cro_split(N, m, k, _ptr(A), _ptr(B), _ptr(y), _ptr(U), _ptr(E), _ptr(u),
                           _ptr(V), _ptr(F), _ptr(v))
    if rc < 0:
        raise ValueError("split needs an even N >= 2")
    return U, E[:h - 1], u, V, F[:h - 1], v, bool(rc)


def residual(A, B, x, y):
    """r = y - A x (Eq. (Axb), Hermitian reading of the diagonal blocks)."""
    A, B, y, N, m, k = _shape(A, B, y)
    x = _c(x)
    r = np.empty_like(y)
    _load().cro_residual(N, m, k, _ptr(A), _ptr(B), _ptr(x), _ptr(y), _ptr(r))
    return r


def rel_residual(A, B, x, y) -> float:
    r = residual(A, B, x, y)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(np.asarray(y).ravel()))


def backward(x, lam, B_shape=None):
    """Block gradients (gA, gB) of a real loss given x and lam = A^{-1} dL/dx."""
    x, lam = _c(x), _c(lam)
    N, m, k = x.shape
    gA = np.empty((N, m, m), np.complex128)
    gB = np.empty((max(N - 1, 1), m, m), np.complex128)
    _load().cro_backward(N, m, k, _ptr(x), _ptr(lam), _ptr(gA), _ptr(gB))
    return gA, gB[:N - 1]


def num_threads() -> int:
    return int(_load().cro_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel regions (CPU-baseline timing)."""
    _load().cro_set_num_threads(int(n))
