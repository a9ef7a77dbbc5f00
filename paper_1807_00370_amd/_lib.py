"""ctypes binding of the C ABI in ``include/crsolve.h`` (marshalling only).

Every numerical step runs in the HIP library; this module only passes device
pointers, sizes and the stream.  It raises if the library is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrsolve.so")

C128, C64, R64, R32 = 0, 1, 2, 3
PREC_NATIVE, PREC_FP32_REFINE = 0, 1
SCHED_CR, SCHED_PCR = 0, 1

OK, EINVAL, EHIP, EWORKSPACE, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5

EXPORTS = ("crsolve_plan_create", "crsolve_workspace_size", "crsolve_factor", "crsolve_check_hpd",
           "crsolve_solve",
           "crsolve_factor_solve", "crsolve_factor_solve_noalloc", "crsolve_backward", "crsolve_residual", "crsolve_set_graphs",
           "crsolve_autotune", "crsolve_set_tuning", "crsolve_timing_enable",
           "crsolve_timing_read", "crsolve_plan_destroy", "crsolve_error_string")


class Desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32),
                ("N", ctypes.POINTER(ctypes.c_int32)),
                ("m", ctypes.POINTER(ctypes.c_int32)),
                ("k", ctypes.POINTER(ctypes.c_int32)),
                ("dtype", ctypes.c_int),
                ("precision", ctypes.c_int),
                ("schedule", ctypes.c_int),
                ("rtol", ctypes.c_double),
                ("max_refine", ctypes.c_int32),
                ("fp64_tail_blocks", ctypes.c_int32),
                ("pcr_tail_blocks", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("level", ctypes.c_int32), ("block", ctypes.c_int64),
                ("refine_iters", ctypes.c_int32), ("fp64_fallback", ctypes.c_int32),
                ("rel_residual", ctypes.c_double)]


INFO_DTYPE = np.dtype([("status", "<i4"), ("level", "<i4"), ("block", "<i8"),
                       ("refine_iters", "<i4"), ("fp64_fallback", "<i4"),
                       ("rel_residual", "<f8")])
assert INFO_DTYPE.itemsize == ctypes.sizeof(Info) == 32


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32),
                ("total_ms", ctypes.c_double)]


class CrsolveError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s failed: %d (%s)" % (fn, code, error_string(code)))
        self.code = code


_lib = None


def load():
    """Load the HIP library; raise if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcrsolve.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.c_void_p, ctypes.c_size_t
    lib.crsolve_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(P)]
    lib.crsolve_workspace_size.argtypes = [P, ctypes.POINTER(S)]
    lib.crsolve_factor.argtypes = [P, P, P, P, S, P, P]
    lib.crsolve_check_hpd.argtypes = [P, P, P, P, S, P, P]
    lib.crsolve_solve.argtypes = [P, P, S, P, P, P, P, P, P]
    lib.crsolve_factor_solve.argtypes = [P, P, P, P, P, S, P, P, P]
    lib.crsolve_factor_solve_noalloc.argtypes = [P, P, P, P, P, P, P]
    lib.crsolve_backward.argtypes = [P, P, S, P, P, P, P, P, P]
    lib.crsolve_residual.argtypes = [P, P, S, P, P, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.crsolve_set_graphs.argtypes = [P, ctypes.c_int]
    lib.crsolve_autotune.argtypes = [P, P, P, P, P, S, P, P, ctypes.c_char_p, S]
    lib.crsolve_set_tuning.argtypes = [P, ctypes.c_char_p]
    lib.crsolve_timing_enable.argtypes = [P, ctypes.c_int]
    lib.crsolve_timing_read.argtypes = [P, ctypes.POINTER(KernelTime), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]
    lib.crsolve_plan_destroy.argtypes = [P]
    lib.crsolve_error_string.argtypes = [ctypes.c_int]
    lib.crsolve_error_string.restype = ctypes.c_char_p
    for n in EXPORTS[:-1]:
        getattr(lib, n).restype = ctypes.c_int
    _lib = lib
    return lib


def error_string(code: int) -> str:
    return load().crsolve_error_string(int(code)).decode()


def check(fn: str, rc: int):
    if rc != OK:
        raise CrsolveError(fn, rc)


class Plan:
    """Owns a ``crsolve_plan`` (host metadata only)."""

    def __init__(self, Ns, ms, ks, dtype=C128, precision=PREC_NATIVE, schedule=SCHED_CR,
                 rtol=1e-12, max_refine=30, fp64_tail_blocks=8, pcr_tail_blocks=0):
        lib = load()
        self.Ns = [int(v) for v in Ns]
        self.ms = [int(v) for v in ms]
        self.ks = [int(v) for v in ks]
        self.batch = len(self.Ns)
        arr = ctypes.c_int32 * self.batch
        self._N, self._m, self._k = arr(*self.Ns), arr(*self.ms), arr(*self.ks)
        d = Desc(self.batch, self._N, self._m, self._k, dtype, precision, schedule, rtol,
                 max_refine, fp64_tail_blocks, pcr_tail_blocks)
        self.dtype, self.precision, self.schedule = dtype, precision, schedule
        h = ctypes.c_void_p()
        check("crsolve_plan_create", lib.crsolve_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        sz = ctypes.c_size_t()
        check("crsolve_workspace_size", lib.crsolve_workspace_size(h, ctypes.byref(sz)))
        self.ws_bytes = int(sz.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            load().crsolve_plan_destroy(h)
            self._h = None

    def factor(self, A, B, ws, info, stream):
        check("crsolve_factor", load().crsolve_factor(self._h, A, B, ws, self.ws_bytes, info,
                                                      stream))

    def check_hpd(self, A, B, ws, info, stream):
        check("crsolve_check_hpd", load().crsolve_check_hpd(self._h, A, B, ws, self.ws_bytes, info,
                                                            stream))

    def solve(self, ws, A, B, y, x, info, stream):
        check("crsolve_solve", load().crsolve_solve(self._h, ws, self.ws_bytes, A, B, y, x, info,
                                                    stream))

    def factor_solve(self, A, B, y, ws, x, info, stream):
        check("crsolve_factor_solve", load().crsolve_factor_solve(self._h, A, B, y, ws,
                                                                  self.ws_bytes, x, info, stream))

    def factor_solve_noalloc(self, A, B, y, x, info, stream):
        """factor_solve in the library's own device scratch array (no
        workspace argument, nothing allocated)."""
        check("crsolve_factor_solve_noalloc",
              load().crsolve_factor_solve_noalloc(self._h, A, B, y, x, info, stream))

    def residual(self, ws, A, B, x, y, stream):
        """Per-system FP64 relative residuals (synchronizes)."""
        out = (ctypes.c_double * self.batch)()
        check("crsolve_residual", load().crsolve_residual(self._h, ws, self.ws_bytes, A, B, x, y,
                                                          out, stream))
        return [float(v) for v in out]

    def set_graphs(self, enable: bool):
        check("crsolve_set_graphs", load().crsolve_set_graphs(self._h, int(enable)))

    def autotune(self, A, B, y, ws, x, stream) -> str:
        buf = ctypes.create_string_buffer(4096)
        check("crsolve_autotune", load().crsolve_autotune(self._h, A, B, y, ws, self.ws_bytes, x,
                                                          stream, buf, 4096))
        return buf.value.decode()

    def set_tuning(self, choice: str):
        check("crsolve_set_tuning", load().crsolve_set_tuning(self._h, choice.encode()))

    def timing(self, enable: bool):
        check("crsolve_timing_enable", load().crsolve_timing_enable(self._h, int(enable)))

    def timing_read(self) -> dict:
        """{kernel name: (launches, total ms)} since timing was enabled."""
        buf = (KernelTime * 16)()
        n = ctypes.c_int()
        check("crsolve_timing_read", load().crsolve_timing_read(self._h, buf, 16, ctypes.byref(n)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                for i in range(min(n.value, 16))}

    def backward(self, ws, x, gx, gy, gA, gB, stream):
        check("crsolve_backward", load().crsolve_backward(self._h, ws, self.ws_bytes, x, gx, gy,
                                                          gA, gB, stream))
