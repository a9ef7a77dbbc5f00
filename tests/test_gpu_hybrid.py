"""The one-sided reduction finished by Algorithm 1 (GPU): once a level holds
at most `pcr_tail_blocks` blocks, the rest of the system is solved in place by
both half systems at every level, without back substitution for those levels
(Section 3, "Time-Complexity").  Compared with the oracle's hybrid schedule on
the same seeded inputs: records bit-exact, x element by element within 1e-11
max |x_ref|, residual <= 1e-12."""
import numpy as np
import pytest

import oracle
from paper_1807_00370_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


@pytest.fixture(scope="module")
def tdev(cuda_ok):
    import torch
    from paper_1807_00370_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


def _gpu(torch, dev, *arrs):
    return [torch.from_numpy(np.array(a, order="C", copy=True)).to(dev) for a in arrs]


def _rec(r):
    return dict(status=int(r["status"]), level=int(r["level"]), block=int(r["block"]))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# switch levels with odd and even block counts, at level 0 (N <= H), in the
# one-wave classes, the work-group classes and the tiled ones
CASES = [(1000, 16, 4, 256), (777, 32, 16, 100), (300, 8, 1, 300), (5000, 80, 2, 64),
         (513, 3, 7, 40), (2049, 32, 16, 256), (1, 4, 1, 8), (96, 64, 4, 5)]


@pytest.mark.parametrize("N,m,k,H", CASES)
def test_hybrid_matches_oracle(tdev, N, m, k, H):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    print("case hybrid N=%d m=%d k=%d H=%d" % (N, m, k, H), flush=True)
    s = W.random_hpd(N, m, k, 9100 + N + m + H)
    A, B, y = _gpu(torch, dev, s.A, s.B, s.y)
    sol = Solver([N], [m], [k], device=dev, pcr_tail_blocks=H)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    xo, io = oracle.solve_hybrid(s.A, s.B, s.y, H)
    assert _rec(sol.info_host()[0]) == io
    assert _rel(x, xo) <= TOL64
    assert oracle.rel_residual(s.A, s.B, x, s.y) <= 1e-12
    # the factors stay usable: a second right-hand side through crsolve_solve
    y2 = s.y[::-1].copy()
    x2 = sol.solve(_gpu(torch, dev, y2)[0]).cpu().numpy()
    xo2, _ = oracle.solve_hybrid(s.A, s.B, y2, H)
    assert _rel(x2, xo2) <= TOL64


def test_hybrid_full_size(tdev):
    """N = 65536, m = 32, k = 16 with the switch at 256 blocks."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    print("case hybrid full N=65536 m=32 k=16 H=256", flush=True)
    s = W.random_hpd(**W.LARGE, seed=W.config_seed(1))
    A, B, y = _gpu(torch, dev, s.A, s.B, s.y)
    sol = Solver([s.N], [s.m], [s.k], device=dev, pcr_tail_blocks=256)
    sol.set_graphs(True)
    x = sol.factor_solve(A, B, y).cpu().numpy()
    assert int(sol.info_host()[0]["status"]) == 0
    assert oracle.rel_residual(s.A, s.B, x, s.y) <= 1e-12
    xo, io = oracle.solve_hybrid(s.A, s.B, s.y, 256)
    assert io["status"] == 0
    assert _rel(x, xo) <= TOL64


@pytest.mark.parametrize("H", [16, 32, 64])
def test_hybrid_breakdown_records(tdev, H):
    """The scalar system A_j = 1, B_j = 0.55, N = 64 (positive blocks,
    indefinite matrix) and the shifted generator: the (level, block) record
    of the switched schedule equals the oracle's."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import solve
    N = 64
    A = np.ones((N, 1, 1), np.complex128)
    B = np.full((N - 1, 1, 1), 0.55, np.complex128)
    y = np.ones((N, 1, 1), np.complex128)
    x, rec = solve(*_gpu(torch, dev, A, B, y), pcr_tail_blocks=H)
    _, io = oracle.solve_hybrid(A, B, y, H)
    assert _rec(rec) == io and io["status"] == 1
    assert np.isnan(x.cpu().numpy()).all()
    t = W.random_hpd(600, 8, 2, W.config_seed(0, 7), shift_scale=2.0)
    x, rec = solve(*_gpu(torch, dev, t.A, t.B, t.y), pcr_tail_blocks=H)
    _, io = oracle.solve_hybrid(t.A, t.B, t.y, H)
    assert _rec(rec) == io == dict(status=1, level=0, block=1)


def test_hybrid_backward_matches_oracle(tdev):
    """The adjoint reuses the factors of the switched schedule."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    s = W.random_hpd(500, 16, 4, 4321, with_W=True)
    A, B, y, gx = _gpu(torch, dev, s.A, s.B, s.y, s.W)
    sol = Solver([500], [16], [4], device=dev, pcr_tail_blocks=50)
    x = sol.factor_solve(A, B, y)
    gA, gB, gy = sol.backward(x, gx)
    xo, _ = oracle.solve_cr(s.A, s.B, s.y)
    lam, _ = oracle.solve_cr(s.A, s.B, s.W)
    oA, oB = oracle.backward(xo, lam)
    assert _rel(gy.cpu().numpy(), lam) <= 1e-10
    assert _rel(gA.cpu().numpy().reshape(oA.shape), oA) <= 1e-10
    assert _rel(gB.cpu().numpy().reshape(oB.shape), oB) <= 1e-10
