"""crsolve_factor_solve_noalloc (GPU): the variant of crsolve_factor_solve
whose workspace is the library's own device scratch array.  Called through
the C ABI and compared with crsolve_factor_solve on a caller workspace, for
two calls in a row (the second with a smaller system, which must not see the
first call's leftovers): the same kernels on the same data, so x and the
info record are bit for bit equal."""
import ctypes

import numpy as np
import pytest

from paper_1807_00370_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev(cuda_ok):
    import torch
    from paper_1807_00370_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


def _run_both(torch, dev, s, **plan_kw):
    from paper_1807_00370_amd import _lib
    plan = _lib.Plan([s.N], [s.m], [s.k], **plan_kw)
    A, B, y = (torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (s.A, s.B, s.y))
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t.numel() else None
    # the existing entry point on a caller-owned workspace
    raw = torch.empty(plan.ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws = ctypes.c_void_p(raw.data_ptr() + (-raw.data_ptr()) % 256)
    x_ref = torch.empty_like(y)
    info_ref = torch.zeros(32, dtype=torch.uint8, device=dev)
    plan.factor_solve(P(A), P(B), P(y), ws, P(x_ref), P(info_ref), st)
    # the no-allocation entry point (output buffers poisoned first)
    x = torch.full_like(y, float("nan"))
    info = torch.full((32,), 255, dtype=torch.uint8, device=dev)
    plan.factor_solve_noalloc(P(A), P(B), P(y), P(x), P(info), st)
    torch.cuda.synchronize()
    return (x.cpu().numpy(), info.cpu().numpy().view(_lib.INFO_DTYPE)[0],
            x_ref.cpu().numpy(), info_ref.cpu().numpy().view(_lib.INFO_DTYPE)[0])


def test_noalloc_matches_factor_solve_twice(tdev):
    torch, dev = tdev
    import oracle
    for N, m, k, seed in ((2048, 16, 4, 61), (300, 8, 2, 62)):
        print("case noalloc N=%d m=%d k=%d" % (N, m, k), flush=True)
        s = W.random_hpd(N, m, k, seed)
        x, rec, x_ref, rec_ref = _run_both(torch, dev, s, pcr_tail_blocks=64)
        assert rec.tobytes() == rec_ref.tobytes() and int(rec["status"]) == 0
        assert np.array_equal(x, x_ref)
        assert oracle.rel_residual(s.A, s.B, x, s.y) <= 1e-12


def test_noalloc_breakdown_record(tdev):
    """A not positive definite system: the same (level, block) record and
    NaN solution as the existing entry point."""
    torch, dev = tdev
    t = W.random_hpd(500, 12, 3, 63, shift_scale=2.0)
    x, rec, x_ref, rec_ref = _run_both(torch, dev, t)
    assert rec.tobytes() == rec_ref.tobytes() and int(rec["status"]) == 1
    assert np.isnan(x).all() and np.isnan(x_ref).all()
