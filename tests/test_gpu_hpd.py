"""The positive-definiteness test (GPU): crsolve_check_hpd against the
smallest eigenvalue of the assembled dense matrix, and its (level, block)
against the oracle's, for the three kernel families (m <= 8, 8 < m <= 32
with its four-group and two-group Cholesky, tiled m > 32).  Each matrix is shifted by c I so that its smallest
eigenvalue is +0.05 or -0.05: far enough from zero for the verdict to be
exact (the flag near the boundary is rounding-dependent)."""
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


def _dense(A, B):
    N, m = A.shape[0], A.shape[1]
    M = np.zeros((N * m, N * m), np.complex128)
    for j in range(N):
        M[j * m:(j + 1) * m, j * m:(j + 1) * m] = A[j]
    for j in range(N - 1):
        M[(j + 1) * m:(j + 2) * m, j * m:(j + 1) * m] = B[j]
        M[j * m:(j + 1) * m, (j + 1) * m:(j + 2) * m] = B[j].conj().T
    return M


@pytest.mark.parametrize("N,m", [(12, 3), (9, 12), (10, 24), (8, 32), (7, 40)])
@pytest.mark.parametrize("sign", [1, -1])
def test_check_hpd_matches_eigenvalues(tdev, N, m, sign):
    torch, dev = tdev
    from paper_1807_00370_amd.solver import check_hpd
    print("case check_hpd N=%d m=%d sign=%d" % (N, m, sign), flush=True)
    s = W.random_hpd(N, m, 1, 7700 + m)
    lam_min = np.linalg.eigvalsh(_dense(s.A, s.B))[0]
    A = s.A - (lam_min - sign * 0.05) * np.eye(m)[None]
    lam_new = np.linalg.eigvalsh(_dense(A, s.B))[0]
    assert abs(lam_new - sign * 0.05) < 1e-9
    At, Bt = (torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (A, s.B))
    ok, rec = check_hpd(At, Bt)
    assert ok == (sign > 0)
    # the default schedule: one-sided levels, then Algorithm 1 from the
    # block-size dependent switch point
    from paper_1807_00370_amd.solver import pcr_tail_default
    _, io = oracle.solve_hybrid(A, s.B, s.y, pcr_tail_default([m]))
    assert (int(rec["status"]), int(rec["level"]), int(rec["block"])) == \
        (io["status"], io["level"], io["block"])


def test_check_hpd_then_solve(tdev):
    """The test leaves the factors in the workspace: a solve may follow."""
    torch, dev = tdev
    from paper_1807_00370_amd.solver import Solver
    s = W.random_hpd(300, 24, 5, 7800)
    A, B, y = (torch.from_numpy(v).to(dev) for v in (s.A, s.B, s.y))
    sol = Solver([s.N], [s.m], [s.k], device=dev)
    assert sol.check_hpd(A, B).tolist() == [True]
    x = sol.solve(y).cpu().numpy()
    xo, _ = oracle.solve_cr(s.A, s.B, s.y)
    assert np.max(np.abs(x - xo)) <= 1e-11 * np.max(np.abs(xo))
