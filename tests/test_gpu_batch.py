"""Batching form (GPU): ragged batches in one launch per level and class,
HIP graph replay of the launch sequence, and the autotuner's kernel-variant
choice.  Every result is compared with the FP64 oracle."""
import re

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


def _pack(systems):
    A = np.concatenate([s.A.ravel() for s in systems])
    B = np.concatenate([s.B.ravel() for s in systems])
    y = np.concatenate([s.y.ravel() for s in systems])
    return A, B, y


def _split(x, systems):
    out, off = [], 0
    for s in systems:
        out.append(x[off:off + s.y.size].reshape(s.y.shape))
        off += s.y.size
    return out


def _solver(torch, dev, systems, **kw):
    from paper_1807_00370_amd.solver import Solver
    return Solver([s.N for s in systems], [s.m for s in systems], [s.k for s in systems],
                  device=dev, **kw)


def _check_all(systems, xs, tol=1e-11, res=1e-12):
    for i, (s, x) in enumerate(zip(systems, xs)):
        xo, io = oracle.solve_cr(s.A, s.B, s.y)
        assert io["status"] == 0
        assert np.abs(x - xo).max() <= tol * np.abs(xo).max(), i
        assert oracle.rel_residual(s.A, s.B, x, s.y) <= res, i


SHAPES = [(256, 8, 1), (300, 16, 4), (258, 32, 16), (130, 64, 4), (512, 8, 16), (2, 4, 1),
          (1, 16, 4), (777, 3, 2), (260, 64, 1), (1024, 16, 16), (99, 32, 1)]


def test_graph_replay_matches_eager(tdev):
    """Replays of the recorded graph, with eager work and synchronizations in
    between and new data in the same buffers, equal the eager results bit
    for bit."""
    torch, dev = tdev
    systems = [W.random_hpd(N, m, k, 2100 + i) for i, (N, m, k) in enumerate(SHAPES)]
    A, B, y = _pack(systems)
    At, Bt, yt = (torch.from_numpy(v).to(dev) for v in (A, B, y))
    eager = _solver(torch, dev, systems)
    xe = eager.factor_solve(At, Bt, yt).cpu().numpy()
    _check_all(systems, _split(xe, systems))
    g = _solver(torch, dev, systems)
    g.set_graphs(True)
    xg = torch.empty_like(yt)
    for rep in range(4):
        if rep == 2:
            # new right-hand sides in the same buffer: the graph reads them
            yt.copy_(torch.flip(yt, [0]))
            xe = eager.factor_solve(At, Bt, yt).cpu().numpy()
        g.factor_solve(At, Bt, yt, xg)
        torch.cuda.synchronize()
        junk = torch.ones(1000, device=dev).cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(xg.cpu().numpy(), xe), rep
        del junk
    info = g.info_host()
    assert (info["status"] == 0).all()


def test_refine_graphs_match_eager(tdev):
    torch, dev = tdev
    systems = [W.random_hpd(N, m, k, 2200 + i) for i, (N, m, k) in enumerate(SHAPES)]
    A, B, y = _pack(systems)
    At, Bt, yt = (torch.from_numpy(v).to(dev) for v in (A, B, y))
    kw = dict(precision="fp32_refine", rtol=1e-12, max_refine=30, fp64_tail_blocks=8)
    eager = _solver(torch, dev, systems, **kw)
    xe = eager.factor_solve(At, Bt, yt).cpu().numpy()
    g = _solver(torch, dev, systems, **kw)
    g.set_graphs(True)
    for rep in range(3):
        xg = g.factor_solve(At, Bt, yt).cpu().numpy()
        assert np.array_equal(xg, xe), rep
    _check_all(systems, _split(xe, systems))
    rec = g.info_host()
    assert (rec["rel_residual"] <= 1e-12).all()


def test_autotune_choice_and_both_variants(tdev):
    """The tuner returns one token per (role, class, precision) present, and
    both kernel variants of every class agree with the oracle."""
    torch, dev = tdev
    systems = [W.random_hpd(N, m, k, 2300 + i) for i, (N, m, k) in enumerate(SHAPES)]
    A, B, y = _pack(systems)
    At, Bt, yt = (torch.from_numpy(v).to(dev) for v in (A, B, y))
    s = _solver(torch, dev, systems)
    choice = s.autotune(At, Bt, yt)
    toks = choice.strip(";").split(";")
    classes = {0 if m <= 4 else 1 if m <= 8 else 2 if m <= 16 else 3 if m <= 32 else 4
               for m in s.ms}
    # launch shapes of the few-block levels (blocks of 9..32 are present)
    shape = [t for t in toks if t.startswith("tw=") or t.startswith("tb=")]
    assert len(shape) == 2 and re.fullmatch(r"tw=(1024|2048|4096)", shape[0]) and \
        re.fullmatch(r"tb=(512|1024|2048)", shape[1]), shape
    toks = [t for t in toks if t not in shape]
    # blocks above 32 (class 4) tune only the reduced-system role
    assert len(toks) == sum(1 if c >= 4 else 3 for c in classes)
    for t in toks:
        assert re.fullmatch(r"r[0-2]c[0-4]f1=[01]", t), t
    # the choice applies to another plan of the same batch
    s2 = _solver(torch, dev, systems)
    s2.plan.set_tuning(choice)
    x2 = s2.factor_solve(At, Bt, yt).cpu().numpy()
    _check_all(systems, _split(x2, systems))
    x = s.factor_solve(At, Bt, yt).cpu().numpy()
    _check_all(systems, _split(x, systems))
    for v in (0, 1):
        s.plan.set_tuning("".join("r%dc%df1=%d;" % (r, c, v) for r in range(3) for c in classes))
        x = s.factor_solve(At, Bt, yt).cpu().numpy()
        _check_all(systems, _split(x, systems))


def test_batch_512_ragged_mixed_precision_graphs(tdev):
    """512 systems with the batch workload's (m, k) mix, N = 2 U{8..64}
    (reduced from 2 U{128..4096} so that the oracle checks all of them),
    complex128 inputs, FP32 levels + FP64 refinement, replayed graphs."""
    torch, dev = tdev
    shapes = W.batch_shapes(512, W.config_seed(3), n_half_range=(8, 64))
    systems = W.batch_systems(shapes, W.config_seed(3))
    A, B, y = _pack(systems)
    At, Bt, yt = (torch.from_numpy(v).to(dev) for v in (A, B, y))
    s = _solver(torch, dev, systems, precision="fp32_refine", rtol=1e-12, max_refine=30,
                fp64_tail_blocks=8)
    s.set_graphs(True)
    for _ in range(2):
        x = s.factor_solve(At, Bt, yt).cpu().numpy()
    rec = s.info_host()
    assert (rec["status"] == 0).all() and (rec["fp64_fallback"] == 0).all()
    assert (rec["rel_residual"] <= 1e-12).all()
    _check_all(systems, _split(x, systems), tol=1e-10)


@pytest.mark.parametrize("form", ["fp32_refine", "fp64"])
def test_stated_range_batch(tdev, form):
    """The first 32 systems of the stated batch (N = 2 U{128..4096}, m in
    {8, 16, 32, 64}, k in {1, 4, 16}, the same seeds as the benchmark), one
    plan, graph replay: every system against the FP64 oracle element by
    element and by its residual."""
    torch, dev = tdev
    shapes = W.batch_shapes(W.BATCH_COUNT, W.config_seed(3))[:32]
    print("case stated batch %s, %d systems, %d block rows" % (
        form, len(shapes), sum(q[0] for q in shapes)), flush=True)
    systems = W.batch_systems(shapes, W.config_seed(3))
    A, B, y = (torch.from_numpy(v).to(dev) for v in _pack(systems))
    kw = dict(precision="fp32_refine", rtol=1e-12, max_refine=30, fp64_tail_blocks=8) \
        if form == "fp32_refine" else {}
    sol = _solver(torch, dev, systems, **kw)
    sol.set_graphs(True)
    x = sol.factor_solve(A, B, y)
    x = sol.factor_solve(A, B, y)  # a replay of the recorded graph
    torch.cuda.synchronize()
    info = sol.info_host()
    assert (info["status"] == 0).all()
    if form == "fp32_refine":
        assert (info["rel_residual"] <= 1e-12).all()
    _check_all(systems, _split(x.cpu().numpy(), systems))
