"""The real symmetric dtypes (GPU): real A, B, y, x arrays (the real case of
Section 1).  Checked against the FP64 oracle on the same data (its solution
of a real system is real), against the closed form of the block 2D Poisson
system, and bit for bit against the complex path on the same data (for real
data the complex arithmetic is the real arithmetic plus exact zeros, and the
real path's single-MFMA products give the same values)."""
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


def _rec(r):
    return dict(status=int(r["status"]), level=int(r["level"]), block=int(r["block"]))


CASES = [(1000, 4, 1), (777, 16, 4), (513, 32, 16), (300, 64, 8), (200, 80, 2), (64, 256, 1),
         (1, 8, 2), (2049, 8, 3)]


@pytest.mark.parametrize("N,m,k", CASES)
def test_real_matches_oracle_and_complex_path(tdev, N, m, k):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver, pcr_tail_default
    print("case real N=%d m=%d k=%d" % (N, m, k), flush=True)
    s = W.random_spd(N, m, k, 9300 + N + m + k)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([N], [m], [k], dtype=torch.float64, device=dev)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    assert x.dtype == np.float64
    xo, io = oracle.solve_hybrid(s.A, s.B, s.y, pcr_tail_default([m]))
    assert _rec(sol.info_host()[0]) == io
    assert np.all(xo.imag == 0.0)
    assert _rel(x, xo.real) <= 1e-11
    assert oracle.rel_residual(s.A, s.B, x, s.y) <= 1e-12
    # the complex path on the same data
    Ac, Bc, yc = (t.to(torch.complex128) for t in (A, B, y))
    solc = Solver([N], [m], [k], dtype=torch.complex128, device=dev)
    xc = solc.factor_solve(Ac, Bc, yc).cpu().numpy()
    assert np.all(xc.imag == 0.0)
    assert np.array_equal(x, xc.real)
    # single precision
    A32, B32, y32 = (t.to(torch.float32) for t in (A, B, y))
    sol32 = Solver([N], [m], [k], dtype=torch.float32, device=dev)
    x32 = sol32.factor_solve(A32, B32, y32).cpu().numpy()
    assert _rel(x32.astype(np.float64), xo.real) <= 2e-4


def test_real_factor_then_solve_and_breakdown(tdev):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver, solve, pcr_tail_default
    s = W.random_spd(600, 40, 3, 77)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([600], [40], [3], dtype=torch.float64, device=dev)
    sol.factor(A, B)
    y2 = np.ascontiguousarray(s.y[::-1])
    x2 = sol.solve(torch.from_numpy(y2).to(dev)).cpu().numpy()
    xo2, _ = oracle.solve_cr(s.A, s.B, y2)
    assert _rel(x2, xo2.real) <= 1e-11
    t = W.random_spd(300, 12, 2, 78, shift_scale=2.0)
    x, rec = solve(*(torch.from_numpy(v).to(dev) for v in (t.A, t.B, t.y)))
    _, io = oracle.solve_hybrid(t.A, t.B, t.y, pcr_tail_default([12]))
    assert _rec(rec) == io == dict(status=1, level=0, block=1)
    assert np.isnan(x.cpu().numpy()).all()


def test_real_poisson_full_size(tdev):
    """N = 4096, m = 256, k = 1 in float64: the closed-form solution y /
    lambda, within the bounds of the complex Poisson test."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    print("case real poisson N=4096 m=256 k=1", flush=True)
    s = W.poisson(W.POISSON["N"], W.POISSON["m"], real=True)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([s.N], [s.m], [s.k], dtype=torch.float64, device=dev)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    assert int(sol.info_host()[0]["status"]) == 0
    lam = s.meta["lam"]
    u = np.finfo(np.float64).eps / 2
    x_exact = s.y / lam
    assert _rel(x, x_exact) <= 16 * u * 8.0 / lam
    res = oracle.rel_residual(s.A, s.B, x, s.y)
    res_rounded_exact = oracle.rel_residual(s.A, s.B, x_exact, s.y)
    print("residual %.3e, of the rounded exact solution %.3e" % (res, res_rounded_exact))
    assert res <= 4 * res_rounded_exact


def test_real_unsupported_combinations(tdev):
    torch, dev = tdev
    from paper_1807_00370_amd import _lib
    for kw in (dict(precision=_lib.PREC_FP32_REFINE), dict(schedule=_lib.SCHED_PCR)):
        with pytest.raises(_lib.CrsolveError) as e:
            _lib.Plan([16], [4], [1], dtype=_lib.R64, **kw)
        assert e.value.code == _lib.EUNSUPPORTED
