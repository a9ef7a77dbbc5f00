"""PyTorch front end of the HIP block cyclic reduction library.

PyTorch provides device memory and the stream; every step of the method runs
in ``libcrsolve.so`` (see ``include/crsolve.h``).  Arrays follow the paper's
problem statement (Section 1, Eq. (Axb)): ``A`` holds A_1..A_N (Hermitian,
lower triangle read), ``B`` holds B_1..B_{N-1} (B_j at block row j+1,
column j), ``y`` holds y_1..y_N.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_DT = {torch.complex128: _lib.C128, torch.complex64: _lib.C64, torch.float64: _lib.R64,
       torch.float32: _lib.R32}
PCR_TAIL_DEFAULT = 64


def pcr_tail_default(ms) -> int:
    """Block count at which the default schedule switches from one-sided
    levels to Algorithm 1, by the largest block size of the plan: 64 for
    m <= 32, 16 for m <= 64, 8 above (the fastest switch points measured at
    N = 65536, m = 32, k = 16; N = 16384, m = 64, k = 32; N = 4096, m = 256,
    k = 1: the larger the blocks, the dearer a level of Algorithm 1, which
    keeps every block of its system)."""
    mx = max(int(m) for m in ms)
    return PCR_TAIL_DEFAULT if mx <= 32 else (16 if mx <= 64 else 8)
_PREC = {"native": _lib.PREC_NATIVE, "fp32_refine": _lib.PREC_FP32_REFINE}
_SCHED = {"cr": _lib.SCHED_CR, "pcr": _lib.SCHED_PCR}


def _ptr(t):
    if t is None or t.numel() == 0:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(t, name, dtype, numel, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError("%s must be on %s" % (name, device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


class Solver:
    """A plan plus its workspace: factor once, then solve / backward many times.

    ``Ns, ms, ks`` give the batch (one entry per independent system); tensors
    are packed back to back (for one system the natural shapes
    ``[N, m, m]``, ``[N-1, m, m]``, ``[N, m, k]`` are packed already).
    """

    def __init__(self, Ns, ms, ks, dtype=torch.complex128, precision="native", schedule="cr",
                 device="cuda", rtol=1e-12, max_refine=30, fp64_tail_blocks=8,
                 pcr_tail_blocks=None):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        if pcr_tail_blocks is None:
            # one-sided levels down to pcr_tail_default(ms) blocks, then
            # Algorithm 1; the mixed form stays one-sided
            pcr_tail_blocks = (pcr_tail_default(ms) if (precision == "native" and schedule == "cr")
                               else 0)
        self.pcr_tail_blocks = pcr_tail_blocks
        self.plan = _lib.Plan(Ns, ms, ks, _DT[dtype], _PREC[precision], _SCHED[schedule], rtol,
                              max_refine, fp64_tail_blocks, pcr_tail_blocks)
        self.Ns, self.ms, self.ks = self.plan.Ns, self.plan.ms, self.plan.ks
        self.batch = self.plan.batch
        self.nA = sum(N * m * m for N, m in zip(self.Ns, self.ms))
        self.nB = sum((N - 1) * m * m for N, m in zip(self.Ns, self.ms))
        self.ny = sum(N * m * k for N, m, k in zip(self.Ns, self.ms, self.ks))
        raw = torch.empty(self.plan.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + self.plan.ws_bytes]
        self.info = torch.zeros(self.batch * _lib.INFO_DTYPE.itemsize, dtype=torch.uint8,
                                device=self.device)
        self.factored = False

    # -- checks -------------------------------------------------------------
    def _mat(self, A, B):
        _check(A, "A", self.dtype, self.nA, self.device)
        _check(B, "B", self.dtype, self.nB, self.device)

    def _rhs(self, y, name="y"):
        _check(y, name, self.dtype, self.ny, self.device)

    def _out(self, x, like):
        if x is None:
            return torch.empty_like(like)
        self._rhs(x, "x")
        return x

    # -- calls ----------------------------------------------------------------
    def factor(self, A, B):
        self._mat(A, B)
        self.plan.factor(_ptr(A), _ptr(B), _ptr(self.ws), _ptr(self.info), _stream(self.device))
        self.factored = True

    def check_hpd(self, A, B) -> np.ndarray:
        """Positive-definiteness test of every system of the batch (the
        factorization's breakdown flag; the factors stay usable for solves).
        Synchronizes; returns one bool per system."""
        self._mat(A, B)
        self.plan.check_hpd(_ptr(A), _ptr(B), _ptr(self.ws), _ptr(self.info), _stream(self.device))
        self.factored = True
        return self.info_host()["status"] == 0

    def solve(self, y, x=None, A=None, B=None):
        """Solve with the stored factors.  The mixed-precision form also needs
        the FP64 matrix (A, B) for its residuals."""
        if not self.factored:
            raise RuntimeError("solve before factor")
        self._rhs(y)
        if self.plan.precision == _lib.PREC_FP32_REFINE:
            self._mat(A, B)
        x = self._out(x, y)
        self.plan.solve(_ptr(self.ws), _ptr(A), _ptr(B), _ptr(y), _ptr(x), _ptr(self.info),
                        _stream(self.device))
        return x

    def factor_solve(self, A, B, y, x=None):
        self._mat(A, B)
        self._rhs(y)
        x = self._out(x, y)
        self.plan.factor_solve(_ptr(A), _ptr(B), _ptr(y), _ptr(self.ws), _ptr(x),
                               _ptr(self.info), _stream(self.device))
        self.factored = self.plan.schedule == _lib.SCHED_CR
        return x

    def residual(self, A, B, x, y):
        """FP64 relative residuals ||y - A x||_F / ||y||_F per system, computed
        by the library on the device (synchronizes)."""
        self._mat(A, B)
        self._rhs(x, "x")
        self._rhs(y)
        return self.plan.residual(_ptr(self.ws), _ptr(A), _ptr(B), _ptr(x), _ptr(y),
                                  _stream(self.device))

    def set_graphs(self, enable=True):
        """Record each distinct call once into a HIP graph and replay it."""
        self.plan.set_graphs(enable)

    def autotune(self, A, B, y, cache=None):
        """Pick the faster kernel variant per (role, block-size class,
        precision) on this data (overwrites the workspace and a scratch x).
        With ``cache`` (a JSON file path, default $CRSOLVE_TUNE_CACHE) a
        previous choice for the same classes is reused and new ones are
        stored."""
        import json
        import os
        cache = cache or os.environ.get("CRSOLVE_TUNE_CACHE")
        key = "|".join(sorted({"m%d_k%d" % (m, k) for m, k in zip(self.ms, self.ks)})) + \
            "|%s|%s" % (self.dtype, self.plan.precision)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
            if key in table:
                self.plan.set_tuning(table[key])
                return table[key]
        self._mat(A, B)
        self._rhs(y)
        x = torch.empty_like(y)
        choice = self.plan.autotune(_ptr(A), _ptr(B), _ptr(y), _ptr(self.ws), _ptr(x),
                                    _stream(self.device))
        if cache:
            table[key] = choice
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1)
        return choice

    def timing(self, enable=True):
        """Per-kernel HIP-event timing of this solver's launches."""
        self.plan.timing(enable)

    def timing_read(self):
        return self.plan.timing_read()

    def backward(self, x, gx):
        """Returns (grad_A, grad_B, grad_y) for the factored matrix."""
        if not self.factored:
            raise RuntimeError("backward before factor")
        self._rhs(x, "x")
        self._rhs(gx, "grad_x")
        gy = torch.empty_like(gx)
        gA = torch.empty(self.nA, dtype=self.dtype, device=self.device)
        gB = torch.empty(max(self.nB, 0), dtype=self.dtype, device=self.device)
        self.plan.backward(_ptr(self.ws), _ptr(x), _ptr(gx), _ptr(gy), _ptr(gA), _ptr(gB),
                           _stream(self.device))
        return gA, gB, gy

    def info_host(self) -> np.ndarray:
        """Synchronizes and returns the per-system crsolve_info records."""
        raw = self.info.cpu().numpy()
        return raw.view(_lib.INFO_DTYPE)


def _shape_of(A, B, y):
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be [N, m, m]")
    N, m = A.shape[0], A.shape[1]
    if y.dim() != 3 or y.shape[0] != N or y.shape[1] != m:
        raise ValueError("y must be [N, m, k]")
    if B.shape != (max(N - 1, 0), m, m):
        raise ValueError("B must be [N-1, m, m]")
    return N, m, y.shape[2]


def solve(A, B, y, schedule="cr", pcr_tail_blocks=None):
    """Solve one system; returns (x, info_record).  Synchronizes for info."""
    N, m, k = _shape_of(A, B, y)
    s = Solver([N], [m], [k], dtype=A.dtype, schedule=schedule, device=A.device,
               pcr_tail_blocks=pcr_tail_blocks)
    x = s.factor_solve(A, B, y)
    return x, s.info_host()[0]


def check_hpd(A, B):
    """Is the Hermitian block-tridiagonal matrix (A_1..A_N on the diagonal,
    B_j at block row j+1, column j) positive definite?  Returns (bool,
    info_record): the first failing (level, block) when it is not.
    Synchronizes."""
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be [N, m, m]")
    N, m = A.shape[0], A.shape[1]
    if B.shape != (max(N - 1, 0), m, m):
        raise ValueError("B must be [N-1, m, m]")
    s = Solver([N], [m], [1], dtype=A.dtype, device=A.device)
    ok = s.check_hpd(A.contiguous(), B.contiguous())
    return bool(ok[0]), s.info_host()[0]


class CRSolve(torch.autograd.Function):
    """x = A^{-1} y for one system, differentiable in A, B and y.

    The backward pass reuses the stored factors to solve A lam = dL/dx and
    forms grad y = lam, grad A_j = -lam_j x_j^H,
    grad B_j = -(lam_{j+1} x_j^H + x_{j+1} lam_j^H) in the library.
    Raises ``torch.linalg.LinAlgError`` when A is not positive definite.

    grad A_j is the block of the dense gradient -lam x^H, which is the
    gradient of the loss for Hermitian perturbations of A_j.  The forward
    pass reads only the lower triangle and the real diagonal of the tensor
    A_j, so for a raw, unconstrained leaf tensor A the gradient of what the
    solver actually computes is tril(G, -1) + tril(G^H, -1) + diag(Re G)
    with G = grad A_j (upper triangle zero), not G itself: build A_j from a
    Hermitian parametrization (e.g. (M + M^H) / 2) when differentiating
    through A, or project the returned gradient that way.
    """

    @staticmethod
    def forward(ctx, A, B, y):
        N, m, k = _shape_of(A, B, y)
        s = Solver([N], [m], [k], dtype=A.dtype, device=A.device)
        A, B, y = A.contiguous(), B.contiguous(), y.contiguous()
        x = s.factor_solve(A, B, y)
        info = s.info_host()[0]
        if info["status"] != 0:
            raise torch.linalg.LinAlgError(
                "matrix is not positive definite: Cholesky breakdown at level %d, block %d"
                % (info["level"], info["block"]))
        ctx.solver = s
        ctx.shape = (N, m, k)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        N, m, k = ctx.shape
        gA, gB, gy = ctx.solver.backward(x, gx.contiguous())
        return gA.view(N, m, m), gB.view(max(N - 1, 0), m, m), gy.view(N, m, k)


def cr_solve(A, B, y):
    """Differentiable solve (see ``CRSolve``)."""
    return CRSolve.apply(A, B, y)
