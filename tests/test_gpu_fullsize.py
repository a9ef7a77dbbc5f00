"""Parity at the full sizes of the precision and differentiation workloads
(GPU), in the launch configuration bench.py times, against the FP64 oracle.

* precision form: N = 65536, m = 32, k = 16, complex128 inputs, FP32 levels,
  FP64 tail (<= 8 blocks), FP64 residual refinement to 1e-12 -- the
  well-conditioned generator and the stated ill variant;
* differentiation form: N = 16384, m = 64, k = 32, loss
  sum_j Re tr(W_j^H x_j), gradients for A, B, y in complex128 and complex64.

Tolerances are those of the smaller parity tests: 1e-11 on x (FP64 and
refined), 1e-10 on the FP64 gradients (one more solve and an outer product),
1e-3 on the complex64 gradients (kappa * 6e-8 with kappa <= 10 and the
reduction depth).
"""
import numpy as np
import pytest

import oracle
from paper_1807_00370_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev(cuda_ok):
    import torch
    from paper_1807_00370_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("ill", [False, True])
def test_refine_full_size(tdev, ill):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    print("case refine full N=65536 m=32 k=16 ill=%s" % ill, flush=True)
    s = W.random_hpd(**W.LARGE, seed=W.config_seed(2), ill=ill)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([s.N], [s.m], [s.k], precision="fp32_refine", device=dev, rtol=1e-12,
                 max_refine=30, fp64_tail_blocks=8)
    sol.set_graphs(True)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    rec = sol.info_host()[0]
    assert int(rec["status"]) == 0 and int(rec["fp64_fallback"]) == 0
    res = oracle.rel_residual(s.A, s.B, x, s.y)
    assert res <= 1e-12
    assert abs(float(rec["rel_residual"]) - res) <= 0.1 * res + 1e-16
    xo, io = oracle.solve_cr(s.A, s.B, s.y)
    assert io["status"] == 0
    assert _rel(x, xo) <= 1e-11


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_full_size(tdev, dt):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import cr_solve
    print("case adjoint full N=16384 m=64 k=32 %s" % dt, flush=True)
    dtype = torch.complex128 if dt == "c128" else torch.complex64
    s = W.random_hpd(**W.DIFF, seed=W.config_seed(4), with_W=True)
    A, B, y, Wt = (torch.from_numpy(v).to(dev).to(dtype) for v in (s.A, s.B, s.y, s.W))
    for t in (A, B, y):
        t.requires_grad_(True)
    x = cr_solve(A, B, y)
    (Wt.conj() * x).real.sum().backward()
    xo, _ = oracle.solve_cr(s.A, s.B, s.y)
    lam, _ = oracle.solve_cr(s.A, s.B, s.W)
    gA, gB = oracle.backward(xo, lam)
    tol = 1e-10 if dt == "c128" else 1e-3
    assert _rel(x.detach().cpu().numpy().astype(np.complex128), xo) <= (1e-11 if dt == "c128" else 2e-4)
    assert _rel(A.grad.cpu().numpy(), gA) <= tol
    assert _rel(B.grad.cpu().numpy(), gB) <= tol
    assert _rel(y.grad.cpu().numpy(), lam) <= tol


def test_pcr_full_size(tdev):
    """Algorithm 1 at the full large-system size N = 65536, m = 32, k = 16
    (every level above 1024 blocks runs the populated-level kernels)."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    print("case pcr full N=65536 m=32 k=16", flush=True)
    s = W.random_hpd(**W.LARGE, seed=W.config_seed(1))
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([s.N], [s.m], [s.k], device=dev, schedule="pcr")
    x = sol.factor_solve(A, B, y).cpu().numpy()
    rec = sol.info_host()[0]
    assert int(rec["status"]) == 0
    assert oracle.rel_residual(s.A, s.B, x, s.y) <= 1e-12
    xo, io = oracle.solve_cr(s.A, s.B, s.y)
    assert io["status"] == 0
    assert _rel(x, xo) <= 1e-11


def _kappa_rec():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kappa_shifts.json")
    with open(path) as fh:
        return json.load(fh)


def _kappa_shift(kappa):
    return _kappa_rec()["shifts"]["%g" % kappa]


@pytest.mark.parametrize("kappa", [1e5, 1e6])
def test_refine_calibrated_kappa_full_size(tdev, kappa):
    """The precision workload shifted to kappa = 1e5 and 1e6 (shift from
    tests/golden/kappa_shifts.json, computed with the oracle only): the
    mixed form certifies ||y - A x|| / ||y|| <= 1e-12, either by refinement
    or by its FP64 fallback, and x agrees with the FP64 oracle within
    kappa * 200 u (both are backward stable; forward errors scale with
    kappa)."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    c = _kappa_shift(kappa)
    print("case refine kappa=%g shift=%.15g" % (kappa, c), flush=True)
    s = W.random_hpd(**W.LARGE, seed=W.config_seed(2), diag_shift=c)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([s.N], [s.m], [s.k], precision="fp32_refine", device=dev, rtol=1e-12,
                 max_refine=30, fp64_tail_blocks=8)
    sol.set_graphs(True)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    rec = sol.info_host()[0]
    print("kappa=%g: refine_iters=%d fp64_fallback=%d rel_residual=%.3e" % (
        kappa, rec["refine_iters"], rec["fp64_fallback"], rec["rel_residual"]), flush=True)
    assert int(rec["status"]) == 0
    res = oracle.rel_residual(s.A, s.B, x, s.y)
    assert res <= 1e-12
    # the library's and the oracle's residuals differ by their own rounding,
    # |fl(r) - r| <~ m u ||A||_2 ||x|| (||A||_2 = lambda_max - c), which at
    # kappa = 1e6 is no longer small against ||r||
    normA = _kappa_rec()["lambda_max"] - c
    slack = s.m * 2.0 ** -53 * normA * np.linalg.norm(x) / np.linalg.norm(s.y)
    assert abs(float(rec["rel_residual"]) - res) <= 0.1 * res + slack
    assert int(rec["fp64_fallback"]) == 1 or int(rec["refine_iters"]) >= 1
    xo, io = oracle.solve_cr(s.A, s.B, s.y)
    assert io["status"] == 0
    assert _rel(x, xo) <= kappa * 200 * 2.0 ** -53
