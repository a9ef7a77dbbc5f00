"""Throughput benchmark: block rows solved per second on one MI355X.

Workload: one Hermitian positive definite block-tridiagonal system with
N = 65536 block rows, m = 32, k = 16, complex128 inputs (seeded synthetic
inputs from ``paper_1807_00370_amd.workloads``), resident in HBM.  A step
solves the system to a certified FP64 relative residual
||y - A x||_F / ||y||_F <= 1e-12 in one of two forms:

* fp64: one fused factor + solve pass of the one-sided block cyclic
  reduction (all levels down, then the back substitution of every level);
* fp32_refine: complex FP32 reduction levels with the last levels (at most 8
  blocks) in FP64, then FP64 residuals and corrections until the residual
  bound holds.

Both forms are timed; ``value`` is the faster one (``config.form``), the other
is reported under ``forms``.  The roofline entry is for the kernel that takes
the most time per step of the reported form: algorithmic bytes (or flops) per
launch from the model below over its HIP-event-measured average launch time.

Algorithmic model per block, s bytes per complex element of the level
(16 FP64, 8 FP32), complex multiply-add = 8 real flops, T = m (m + 1) / 2:
  k_elim   matrix part: read A_p (lower, T), B_p, B_{p-1}; write L (packed T),
           P, Q.  rhs part: read y_p (and L if alone), write g.
           flops 8 (m^3/6 + m^3 [P, Q] + m^2 k / 2)
  k_reduce matrix part: read A_q (lower), P_l, Q_r, P_r; write A'_q (lower),
           B'_q.  rhs part: read y_q, g_l, g_r (and P_l, Q_r if alone),
           write y'_q.  flops 8 (m^3 [two Hermitian products] + m^3 + 2 m^2 k)
  k_back   read L, P, Q, g, x_{p-1}, x_{p+1}; write x_p.  flops 8 (5/2 m^2 k)
  k_residual (FP64) read A_j (lower), B_j, x_j, y_j; write r_j.
           flops 8 (3 m^2 k)
Blocks without a neighbour skip the missing terms.  Blocks above 64 split
the elimination into k_potrf_big (Cholesky) and k_trsm_big (substitutions).

Other workloads (one JSON line each, same keys; the default run above is the
one the contract names):
  --workload poisson   block 2D Poisson, N=4096, m=256, k=1, eigenvector
                       right-hand side (residual bound 16 u kappa, see the
                       design notes)
  --workload diff      forward solve + adjoint, N=16384, m=64, k=32, c128
                       (and c64 under forms)
  --workload batch     512 ragged systems, N = 2 U{128..--batch-half-max}
  --schedule pcr       Algorithm 1 on the default workload (FP64)
Profiling runs add --no-autotune (default kernel variants), --calib-copy
(a device copy of A of known size for counter calibration) and
--no-box-peaks.  After the timed steps the roofline entry also reports the
GPU's achievable peaks measured with library kernels (peak_measured: a 1 GiB
device copy, 8192^3 FP64 / FP32 GEMMs) and the fraction of those, with the
one-directional HBM rates (a 1 GiB reduction and fill) beside the copy's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_FP64_TFS = 78.6         # MI355X FP64 (vector = matrix), TFLOP/s
PEAK_FP32_TFS = 157.3        # MI355X FP32, TFLOP/s
METRIC = "Block-rows solved/s & % roofline: FP32+refine vs FP64 at rel. residual ≤1e-12"
RTOL = 1e-12
TAIL = 8


def levels(N: int):
    """Per level of the one-sided schedule: (n, eliminated, kept, eliminated
    with a previous block, eliminated with a next block, kept with a right
    neighbour, kept with a reduced off-diagonal block)."""
    out = []
    n = N
    while n > 0:
        ne, nk = (n + 1) // 2, n // 2
        k_right = sum(1 for q in range(1, n, 2) if q + 1 < n)
        k_f = sum(1 for q in range(1, n, 2) if q + 2 < n)
        out.append((n, ne, nk, ne - 1, nk, k_right, k_f))
        n //= 2
    return out


def pass_model(N, m, k, s_of_level, mat, rhs, s_in0=None, upd=0):
    """Algorithmic bytes and flops of one pass over the levels, per kernel.
    Blocks above 64 split the elimination into the tiled Cholesky
    (k_potrf_big: read A_p lower, write L lower) and the tiled substitutions
    (k_trsm_big: read L, B_p, B_{p-1}, y_p; write P, Q, g).  s_in0: bytes per
    element of the level-0 inputs A, B, y when they differ from the level's
    own precision (the mixed form's FP32 level 0 reads the FP64 arrays);
    upd: the mixed form's level-0 back substitution writes the FP64 x
    (1: x = d, 2: x += d, which also reads x), for the eliminated and the
    kept blocks."""
    mm, mk, T = m * m, m * k, m * (m + 1) // 2
    big = m > 64
    names = ("k_potrf_big", "k_trsm_big") if big else ("k_elim", "k_elim")
    tot = {kn: [0.0, 0.0] for kn in set(names) | {"k_reduce", "k_back"}}
    for lvl, (n, ne, nk, e_prev, e_next, k_right, k_f) in enumerate(levels(N)):
        s = s_of_level(n)
        si = s_in0 if (lvl == 0 and s_in0) else s
        if mat:
            tot[names[0]][0] += ne * T * (si + s)
            tot[names[0]][1] += 8 * ne * mm * m / 6
        b = f = 0.0
        if mat:
            b += (e_prev + e_next) * mm * (si + s) + (ne * T * s if big else 0)
            f += (e_prev + e_next) * mm * m / 2
        if rhs:
            b += ne * (mk * (si + s) + (0 if mat else T * s))
            f += ne * mk * m / 2
        tot[names[1]][0] += b
        tot[names[1]][1] += 8 * f
        b = f = 0.0
        if mat:
            b += nk * (T * (si + s) + mm * s) + k_right * mm * s + k_f * 2 * mm * s
            f += nk * mm * m / 2 + k_right * mm * m / 2 + k_f * mm * m
        if rhs:
            b += nk * mk * (si + s) + nk * mk * s + k_right * mk * s + \
                (0 if mat else (nk + k_right) * mm * s)
            f += nk * mk * m + k_right * mk * m
        tot["k_reduce"][0] += b
        tot["k_reduce"][1] += 8 * f
        if rhs:
            b = (ne * (T + mk) + (e_prev + e_next) * (mm + mk)) * s
            if lvl == 0 and upd:
                # x_p and the kept neighbour's x_{p+1} in FP64 (read too when x += d)
                b += (ne + nk) * mk * 16 * (2 if upd == 2 else 1)
            else:
                b += ne * mk * s
            f = (e_prev + e_next) * mk * m + ne * mk * m / 2
            tot["k_back"][0] += b
            tot["k_back"][1] += 8 * f
    return tot


def add(a, b, scale=1.0):
    for kn, v in b.items():
        if kn not in a:
            a[kn] = [0.0, 0.0]
        a[kn][0] += scale * v[0]
        a[kn][1] += scale * v[1]
    return a


def step_model(form, N, m, k, iters=0, real=False):
    """Per-kernel algorithmic [bytes, flops] of one step of a form.  The mixed
    form: the fused factor + first solve (level 0 reads the FP64 A, B, y and
    assigns x), `iters` correction passes (level 0 reads the FP64 residual
    and adds to x), and one FP64 residual per solve (read A_j lower, B_j,
    x_j, y_j; write r_j in FP64)."""
    if form == "fp64":
        tot = pass_model(N, m, k, lambda n: 16, True, True, s_in0=8 if real else None)
        if real:
            # real data: a real multiply-add (2 flops) per complex one (8)
            for v in tot.values():
                v[1] /= 4.0
        return tot
    s_lvl = lambda n: 16 if n <= TAIL else 8
    tot = {}
    add(tot, pass_model(N, m, k, s_lvl, True, True, s_in0=16, upd=1))
    if iters:
        add(tot, pass_model(N, m, k, s_lvl, False, True, s_in0=16, upd=2), iters)
    mm, mk, T = m * m, m * k, m * (m + 1) // 2
    add(tot, {"k_residual": [N * (T + mm + 3 * mk) * 16, 8 * N * 3 * mm * k]}, 1 + iters)
    return tot


def pcr_model(N, m, k):
    """Algorithm 1 in place: at level l (distance d = 2^l) every block is
    eliminated and every block is reduced; the last level only factors and
    solves its uncoupled blocks.  Per-kernel algorithmic [bytes, flops], FP64."""
    mm, mk, T, s = m * m, m * k, m * (m + 1) // 2, 16
    tot = {"k_elim": [0.0, 0.0], "k_reduce": [0.0, 0.0], "k_back": [0.0, 0.0]}
    D = 0
    while (1 << D) < N:
        D += 1
    for lvl in range(D + 1):
        d = 1 << lvl
        nb = max(N - d, 0)       # blocks with a neighbour at distance d on one side
        nf = max(N - 2 * d, 0)   # kept blocks with a reduced off-diagonal block
        tot["k_elim"][0] += (N * (2 * T + 2 * mk) + 2 * nb * 2 * mm) * s
        tot["k_elim"][1] += 8 * (N * mm * m / 6 + 2 * nb * mm * m / 2 + N * mk * m / 2)
        if lvl < D:
            tot["k_reduce"][0] += (N * (2 * T + 2 * mk) + 2 * nb * (mm + mk) + nf * 2 * mm) * s
            tot["k_reduce"][1] += 8 * (2 * nb * mm * m / 2 + nf * mm * m + 2 * nb * mk * m)
        else:
            tot["k_back"][0] += N * (T + 2 * mk) * s
            tot["k_back"][1] += 8 * N * mk * m / 2
    return tot


def adjoint_model(N, m, k, s):
    """Backward pass: the rhs-only levels and back substitution for lam, then
    the gradient blocks (read lam_j, x_j, lam_{j+1}, x_{j+1}; write gA_j, gB_j)."""
    tot = pass_model(N, m, k, lambda n: s, False, True)
    mm, mk = m * m, m * k
    add(tot, {"k_grad": [(N * (4 * mk + mm) + (N - 1) * mm) * s,
                         8 * (N * mm * k + (N - 1) * 2 * mm * k)]})
    return tot


def host_cpu():
    """CPU model name and logical CPU count of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def banded_lower(A, B):
    """LAPACK lower band storage of the Hermitian block-tridiagonal matrix
    (half-bandwidth 2m - 1): ab[i - j, j] = D[i, j] for i >= j."""
    N, m, _ = A.shape
    ab = np.zeros((2 * m, N * m), np.complex128)
    for r in range(m):
        for q in range(r + 1):
            v = A[:, r, q]
            ab[r - q, q::m] = v.real if r == q else v
        if N > 1:
            for q in range(m):
                ab[m + r - q, q:(N - 1) * m:m] = B[:, r, q]
    return ab


def cpu_extras(m, k, seed):
    """Per-block-row CPU rates on an N=4096 sample of the same block shape:
    the oracle on one core, and LAPACK's banded Hermitian solver (zpbsv via
    scipy.linalg.solveh_banded) as a library reference."""
    import oracle
    import scipy.linalg
    from paper_1807_00370_amd import workloads as W
    smp = W.random_hpd(4096, m, k, seed)
    nt = oracle.num_threads()
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.solve_cr(smp.A, smp.B, smp.y)
    t1 = time.perf_counter()
    oracle.set_num_threads(nt)
    ab = banded_lower(smp.A, smp.B)
    t2 = time.perf_counter()
    scipy.linalg.solveh_banded(ab, smp.y.reshape(-1, k), lower=True, check_finite=False)
    t3 = time.perf_counter()
    return {"value_1core": {"value": smp.N / (t1 - t0), "unit": "block-rows/s", "cores": 1,
                            "sample": "oracle, N=4096 sample (m=%d, k=%d), one solve in %.2f s"
                                      % (m, k, t1 - t0)},
            "lapack_banded": {"value": smp.N / (t3 - t2), "unit": "block-rows/s",
                              "sample": "scipy.linalg.solveh_banded (LAPACK zpbsv, band "
                                        "Cholesky, half-bandwidth %d), N=4096 sample, one solve "
                                        "in %.2f s" % (2 * m - 1, t3 - t2)}}


def cpu_baseline(s, budget_s: float, what: str = "full workload", solver: str = "cr",
                 extras=True):
    """The oracle's one-sided reduction (or Algorithm 1) on the host cores (at
    least one solve, repeated until the budget is spent); also returns the
    oracle's x of the last solve."""
    import oracle
    oracle.build(force=False)
    fn = oracle.solve_pcr if solver == "pcr" else oracle.solve_cr
    reps, t0 = 0, time.perf_counter()
    while True:
        x, info = fn(s.A, s.B, s.y)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 8:
            break
    assert info["status"] == 0
    out = {"value": s.N * reps / el, "unit": "block-rows/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": "%s (N=%d, m=%d, k=%d, complex128), FP64 %s, %d solve(s) in %.1f s" % (
               what, s.N, s.m, s.k, "Algorithm 1" if solver == "pcr" else
               "one-sided cyclic reduction", reps, el)}
    out.update(host_cpu())
    if extras:
        out.update(cpu_extras(s.m, s.k, 180700370 + 97))
    return out, x


def timed_steps(torch, sol, A, B, y, x, steps, warmup):
    return time_steps(torch, lambda: sol.factor_solve(A, B, y, x), steps, warmup)


def time_form(torch, sol, A, B, y, x, steps, warmup):
    """Step time with the launch sequence replayed as a HIP graph, the eager
    step time, and per-kernel event timings of eager steps."""
    sol.set_graphs(True)
    ms = timed_steps(torch, sol, A, B, y, x, steps, warmup)
    _STEP_STATS["graph_mean"] = _STEP_STATS["mean"]
    sol.set_graphs(False)
    ms_eager = timed_steps(torch, sol, A, B, y, x, steps, 1)
    # per-kernel durations from HIP events bracketing each launch
    sol.timing(True)
    for _ in range(steps):
        sol.factor_solve(A, B, y, x)
    kt = sol.timing_read()
    sol.timing(False)
    torch.cuda.synchronize()
    return ms, ms_eager, {kn: (cnt / steps, tot / steps) for kn, (cnt, tot) in kt.items()}


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1807_00370_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(form, kernel, shape=(65536, 32, 16)):
    """HBM bytes per launch from the committed counter summary of this
    workload, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s_N%d_m%d_k%d.json" % ((form,) + shape))
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes_per_launch"]


def roofline(per_step, mod, prec_f64, form="fp64", shape=(65536, 32, 16)):
    timed = [kn for kn in mod if kn in per_step]
    dom = max(timed, key=lambda kn: per_step[kn][1])
    launches, kms = per_step[dom]
    avg_ms = kms / launches
    byts, flops = mod[dom]
    peak_f = PEAK_FP64_TFS if prec_f64 else PEAK_FP32_TFS
    if flops / max(byts, 1.0) < peak_f * 1e12 / (PEAK_HBM_GBS * 1e9):
        ach = byts / launches / (avg_ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        ach = flops / launches / (avg_ms * 1e-3) / 1e12
        r = {"bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = measured_traffic(form, dom, shape)
    r["kernel"] = dom
    r["avg_launch_ms"] = avg_ms
    r["launches_per_step"] = launches
    r["algorithmic_bytes_per_launch"] = byts / launches
    r["algorithmic_flops_per_launch"] = flops / launches
    return r


_STEP_STATS = {}


def time_steps(torch, step, steps, warmup):
    """Median step time (ms) over `steps` steps, each bracketed by HIP events on
    the current stream; the mean over the same steps is kept in _STEP_STATS."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    _STEP_STATS["mean"] = ev[0].elapsed_time(ev[-1]) / steps
    _STEP_STATS["min"] = min(per)
    return float(np.median(per))


def kernel_times(torch, sol, step, steps):
    sol.timing(True)
    for _ in range(steps):
        step()
    kt = sol.timing_read()
    sol.timing(False)
    torch.cuda.synchronize()
    return {kn: (cnt / steps, tot / steps) for kn, (cnt, tot) in kt.items()}


_BOX = {}


def box_peaks():
    """Achievable peaks of this GPU, measured with library kernels after the
    timed region: a 1 GiB device-to-device copy (read + written bytes) for
    HBM, and 8192^3 FP64 and FP32 GEMMs for the matrix cores.  Context for
    the published peaks, not a replacement for them."""
    if _BOX:
        return _BOX
    import torch
    dev = torch.device("cuda:0")

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    nb = a.numel() * 8
    _BOX["hbm_GBs"] = 2 * nb / timed(lambda: b.copy_(a), 10) / 1e9
    # one-directional rates beside the copy's mixed one (a reduction reads,
    # a fill writes)
    s = torch.empty((), dtype=torch.float64, device=dev)
    _BOX["hbm_read_GBs"] = nb / timed(lambda: torch.sum(a, dim=0, out=s), 10) / 1e9
    _BOX["hbm_write_GBs"] = nb / timed(lambda: b.fill_(2.0), 10) / 1e9
    del a, b, s
    M = 8192
    for dt, key in ((torch.float64, "fp64_TFs"), (torch.float32, "fp32_TFs")):
        g = torch.Generator(device=dev)
        g.manual_seed(1)
        x = torch.randn(M, M, dtype=dt, device=dev, generator=g)
        yv = torch.randn(M, M, dtype=dt, device=dev, generator=g)
        z = torch.empty_like(x)
        _BOX[key] = 2.0 * M ** 3 / timed(lambda: torch.matmul(x, yv, out=z), 5) / 1e12
        del x, yv, z
    torch.cuda.empty_cache()
    return _BOX


def add_measured_peak(roof):
    pk = box_peaks()
    if roof["unit"] == "GB/s":
        ref = pk["hbm_GBs"]
    else:
        ref = pk["fp64_TFs"] if roof["peak"] == PEAK_FP64_TFS else pk["fp32_TFs"]
    roof["peak_measured"] = ref
    roof["frac_of_measured"] = roof["achieved"] / ref
    roof["peak_measured_how"] = ("1 GiB device copy, read + written bytes" if roof["unit"] == "GB/s"
                                 else "8192^3 GEMM through torch.matmul")
    if roof["unit"] == "GB/s":
        roof["peak_measured_read"] = pk["hbm_read_GBs"]
        roof["peak_measured_write"] = pk["hbm_write_GBs"]


def emit(args, value, ms, dtype, config, forms, roof, cpu, model=None):
    if not args.no_box_peaks and roof is not None:
        add_measured_peak(roof)
    out = {"metric": METRIC, "value": value, "unit": "block-rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    if model is not None:
        out["step_model"] = model
    out.update({"roofline": roof, "forms": forms, "cpu_baseline": cpu})
    print(json.dumps(out), flush=True)


def run_diff(args, torch, W, dev):
    """Differentiation workload: forward solve plus the adjoint (lam = A^{-1}
    dL/dx from the stored factors, gradient blocks) for L = sum_j Re tr(W_j^H
    x_j), so dL/dx = W; N=16384, m=64, k=32 in complex128 and complex64."""
    import oracle
    from paper_1807_00370_amd.solver import Solver
    N, m, k = W.DIFF["N"], W.DIFF["m"], W.DIFF["k"]
    s = W.random_hpd(N, m, k, W.config_seed(4), with_W=True)
    forms = {}
    for name, dt, es in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        A, B, y, gx = (torch.from_numpy(v).to(dev).to(dt) for v in (s.A, s.B, s.y, s.W))
        x = torch.empty_like(y)
        sol = Solver([N], [m], [k], dtype=dt, device=dev)

        def step():
            sol.factor_solve(A, B, y, x)
            return sol.backward(x, gx)

        ms = time_steps(torch, step, args.steps, args.warmup)
        per_step = kernel_times(torch, sol, step, args.steps)
        info = sol.info_host()[0]
        if info["status"] != 0:
            raise SystemExit("diff %s: factorization failed" % name)
        mod = add(pass_model(N, m, k, lambda n: es, True, True), adjoint_model(N, m, k, es))
        forms[name] = {"ms_per_step": ms, "value": N / (ms * 1e-3),
                       "kernel_ms_per_step": {kn: round(v[1], 4) for kn, v in per_step.items()},
                       "roofline": roofline(per_step, mod, es == 16, "diff_" + name),
                       "model_bytes": sum(v[0] for v in mod.values()),
                       "model_flops": sum(v[1] for v in mod.values())}
        if name == "c128":
            forms[name]["rel_residual"] = sol.residual(A, B, x, y)[0]
        print("diff %s: %.3f ms/step (forward + adjoint), %s" % (
            name, ms, json.dumps(forms[name]["kernel_ms_per_step"])), file=sys.stderr, flush=True)
        del sol, A, B, y, gx, x
        torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline:
        oracle.build(force=False)
        smp = W.random_hpd(1024, m, k, W.config_seed(4, 1), with_W=True)
        reps, t0 = 0, time.perf_counter()
        while True:
            xo, _ = oracle.solve_cr(smp.A, smp.B, smp.y)
            lam, _ = oracle.solve_cr(smp.A, smp.B, smp.W)
            oracle.backward(xo, lam)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_budget or reps >= 8:
                break
        cpu = {"value": smp.N * reps / el, "unit": "block-rows/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "N=1024 sample of the differentiation workload (m=%d, "
               "k=%d, complex128): forward solve, adjoint solve and gradient blocks, %d time(s) "
               "in %.1f s" % (m, k, reps, el)}
    f = forms["c128"]
    emit(args, f["value"], f["ms_per_step"], "c128",
         {"workload": "differentiation: forward solve + adjoint of one HPD system, N=%d, m=%d, "
                      "k=%d, complex128 (complex64 under forms)" % (N, m, k),
          "N": N, "m": m, "k": k, "form": "c128"}, forms, f["roofline"], cpu)


def run_batch(args, torch, W, dev):
    """Batching workload: 512 independent systems of uneven N, m, k in one
    plan (one launch per level, block-size class and precision), the launch
    sequence replayed as a HIP graph; complex128 inputs solved by the
    FP32 + FP64-refinement form (the stated form) and, when its workspace
    fits beside the inputs, by the FP64 form."""
    import oracle
    from paper_1807_00370_amd import _lib
    from paper_1807_00370_amd.solver import Solver
    t0 = time.perf_counter()
    shapes = W.batch_shapes(W.BATCH_COUNT, W.config_seed(3), n_half_range=(128, args.batch_half_max))
    # generator processes forked before this process touches the GPU
    stream = W.BatchStream(shapes, W.config_seed(3), workers=min(16, os.cpu_count() or 1))
    Ns, ms_, ks = [q[0] for q in shapes], [q[1] for q in shapes], [q[2] for q in shapes]
    rows = sum(Ns)
    nA, nB, ny = stream.offA[-1], stream.offB[-1], stream.offy[-1]
    A = torch.empty(nA, dtype=torch.complex128, device=dev)
    B = torch.empty(max(nB, 1), dtype=torch.complex128, device=dev)[:nB]
    y = torch.empty(ny, dtype=torch.complex128, device=dev)
    done = 0
    for i, a_, b_, y_ in stream:
        A[stream.offA[i]:stream.offA[i + 1]].copy_(torch.from_numpy(a_.ravel()))
        B[stream.offB[i]:stream.offB[i + 1]].copy_(torch.from_numpy(b_.ravel()))
        y[stream.offy[i]:stream.offy[i + 1]].copy_(torch.from_numpy(y_.ravel()))
        done += 1
        if done % 64 == 0:
            print("batch inputs: %d of %d systems on the GPU (%.0f s)" % (
                done, len(shapes), time.perf_counter() - t0), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print("batch inputs generated in %.1f s: %d block rows, %.1f GB" % (
        time.perf_counter() - t0, rows, (nA + nB + ny) * 16 / 1e9), file=sys.stderr, flush=True)
    x = torch.empty_like(y)
    # oracle reference for the first 16 systems (error against FP64 per result)
    ref = W.batch_systems(shapes[:16], W.config_seed(3))
    xo_ref = [oracle.solve_cr(q.A, q.B, q.y)[0] for q in ref]
    forms = {}
    for form in ("fp32_refine", "fp64"):
        prec = _lib.PREC_FP32_REFINE if form != "fp64" else _lib.PREC_NATIVE
        ws = _lib.Plan(Ns, ms_, ks, precision=prec).ws_bytes
        free, _ = torch.cuda.mem_get_info(dev)
        if ws + (2 << 30) > free:
            forms[form] = {"skipped": "workspace of %.1f GB exceeds the %.1f GB of device memory "
                                      "left beside the %.1f GB of inputs and x" % (
                                          ws / 1e9, free / 1e9, (nA + nB + 2 * ny) * 16 / 1e9),
                           "workspace_bytes": ws}
            print("batch %s: %s" % (form, forms[form]["skipped"]), file=sys.stderr, flush=True)
            continue
        if form == "fp64":
            sol = Solver(Ns, ms_, ks, device=dev)
            tuning = sol.autotune(A, B, y)
        else:
            sol = Solver(Ns, ms_, ks, precision="fp32_refine", device=dev, rtol=RTOL,
                         max_refine=30, fp64_tail_blocks=TAIL)
            tuning = None
        sol.set_graphs(True)
        step = lambda: sol.factor_solve(A, B, y, x)
        ms = time_steps(torch, step, args.steps, args.warmup)
        mean = _STEP_STATS["mean"]
        sol.set_graphs(False)
        per_step = kernel_times(torch, sol, step, args.steps)
        info = sol.info_host()
        if (info["status"] != 0).any():
            raise SystemExit("batch %s: a factorization failed" % form)
        rel = sol.residual(A, B, x, y)
        xh = x[:stream.offy[16]].cpu().numpy()
        err = max(float(np.max(np.abs(xh[stream.offy[i]:stream.offy[i + 1]].reshape(q.y.shape) - xo))
                        / np.max(np.abs(xo))) for i, (q, xo) in enumerate(zip(ref, xo_ref)))
        mod = {}
        for i, (N, m, k) in enumerate(zip(Ns, ms_, ks)):
            add(mod, step_model(form, N, m, k, int(info["refine_iters"][i]) if form != "fp64" else 0))
        forms[form] = {"ms_per_step": ms, "ms_per_step_mean": mean, "value": rows / (ms * 1e-3),
                       "tuning": tuning, "workspace_bytes": ws,
                       "max_rel_residual": float(np.max(rel)),
                       "certified": bool(np.max(rel) <= RTOL),
                       "max_refine_iters": int(np.max(info["refine_iters"])),
                       "fp64_fallbacks": int(np.sum(info["fp64_fallback"])),
                       "err_vs_oracle_first16": err,
                       "kernel_ms_per_step": {kn: round(v[1], 4) for kn, v in per_step.items()},
                       "roofline": roofline(per_step, mod, form == "fp64", "batch_" + form),
                       "model_bytes": sum(v[0] for v in mod.values()),
                       "model_flops": sum(v[1] for v in mod.values())}
        print("batch %s: %.3f ms/step, max rel residual %.2e, err %.2e, %s" % (
            form, ms, np.max(rel), err, json.dumps(forms[form]["kernel_ms_per_step"])),
            file=sys.stderr, flush=True)
        del sol
        torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline:
        oracle.build(force=False)
        reps, done, t0 = 0, 0, time.perf_counter()
        for q in ref:
            oracle.solve_cr(q.A, q.B, q.y)
            done += q.N
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        el = time.perf_counter() - t0
        cpu = {"value": done / el, "unit": "block-rows/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "the first %d systems of the batch (%d block rows), "
               "FP64 one-sided cyclic reduction, in %.1f s" % (reps, done, el)}
        cpu.update(host_cpu())
    best = min((f for f in forms if forms[f].get("certified")), key=lambda f: forms[f]["ms_per_step"])
    f = forms[best]
    emit(args, f["value"], f["ms_per_step"], "c64+f64" if best != "fp64" else "c128",
         {"workload": "batch of %d independent HPD systems, N = 2 U{128..%d}, m in {8,16,32,64}, "
                      "k in {1,4,16}, complex128 inputs, %d block rows, solved to rel. residual "
                      "<= 1e-12 (%s form, graph replay)" % (len(shapes), args.batch_half_max,
                                                            rows, best),
          "systems": len(shapes), "block_rows": rows, "form": best,
          "n_half_range": [128, args.batch_half_max]}, forms, f["roofline"], cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--forms", default=None,
                    help="default: fp64,fp64_onesided,fp32_refine (poisson: fp64,r64,fp32_refine)")
    ap.add_argument("--schedule", choices=("cr", "pcr"), default="cr",
                    help="cr: one-sided reduction (default); pcr: Algorithm 1 as printed (fp64)")
    ap.add_argument("--batch-half-max", type=int, default=4096,
                    help="batch workload: N = 2 U{128..this} (the stated range is 4096)")
    ap.add_argument("--workload", choices=("random", "poisson", "diff", "batch"), default="random",
                    help="random: the HPD generator at --N/--m/--k; poisson: the block 2D "
                         "Poisson system N=4096, m=256, k=1 with an eigenvector right-hand side")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kappa", action="store_true",
                    help="skip the calibrated kappa = 1e5 / 1e6 instances of the precision "
                         "workload (default run only)")
    ap.add_argument("--no-box-peaks", action="store_true",
                    help="skip the measured copy / GEMM peaks reported beside the published ones")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel variants (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="one plain device copy of A (known size) before timing, to calibrate "
                         "HBM byte counters")
    args = ap.parse_args()
    if args.forms is None:
        args.forms = ("fp64,r64,fp32_refine" if args.workload == "poisson"
                      else "fp64,fp64_onesided,fp32_refine")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs each system on a single "
              "device and this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1807_00370_amd import workloads as W
    from paper_1807_00370_amd.solver import Solver

    dev = torch.device("cuda:0")
    if args.workload == "diff":
        return run_diff(args, torch, W, dev)
    if args.workload == "batch":
        return run_batch(args, torch, W, dev)
    t0 = time.perf_counter()
    if args.workload == "poisson":
        s = W.poisson(W.POISSON["N"], W.POISSON["m"])
        # y is the lowest eigenvector: ||A|| ||x|| / ||y|| = kappa ~ 8 / lambda_min, and even
        # the rounded exact solution has a residual near u kappa; the bound is 16 u kappa
        rtol = 16 * 2.0 ** -53 * 8.0 / s.meta["lam"]
    else:
        s = W.random_hpd(args.N, args.m, args.k, W.config_seed(1))
        rtol = RTOL
    print("inputs generated in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    A = torch.from_numpy(s.A).to(dev)
    B = torch.from_numpy(s.B).to(dev)
    y = torch.from_numpy(s.y).to(dev)
    x = torch.empty_like(y)
    if args.calib_copy:
        dst = torch.empty_like(A)
        dst.copy_(A)
        torch.cuda.synchronize()
        print("calibration copy: %d bytes read, %d bytes written" % (A.numel() * 16, A.numel() * 16),
              file=sys.stderr, flush=True)
        del dst

    forms = {}
    xs = {}
    pcr = args.schedule == "pcr"

    def run_form(form, s, A, B, y, x, rtol, steps, warmup, tag):
        if form == "r64":
            # the real symmetric dtype on the real arrays of the same system
            A, B, y = (t.real.contiguous() for t in (A, B, y))
            x = torch.empty_like(y)
            s = W.System(s.A.real.copy(), s.B.real.copy(), s.y.real.copy(), None, s.meta)
            sol = Solver([s.N], [s.m], [s.k], dtype=torch.float64, device=dev)
        elif form in ("fp64", "fp64_onesided"):
            # fp64: one-sided levels, then Algorithm 1 below 64 blocks (the
            # library default); fp64_onesided: one-sided throughout
            sol = Solver([s.N], [s.m], [s.k], dtype=torch.complex128, device=dev,
                         schedule=args.schedule,
                         pcr_tail_blocks=0 if form == "fp64_onesided" else None)
        else:
            sol = Solver([s.N], [s.m], [s.k], dtype=torch.complex128, precision="fp32_refine",
                         device=dev, rtol=rtol, max_refine=30, fp64_tail_blocks=TAIL)
        tuning = (sol.autotune(A, B, y) if form != "fp32_refine" and s.m <= 64 and not pcr
                  and not args.no_autotune else None)
        ms, ms_eager, per_step = time_form(torch, sol, A, B, y, x, steps, warmup)
        mean = _STEP_STATS["graph_mean"]
        info = sol.info_host()[0]
        if info["status"] != 0:
            raise SystemExit("%s: factorization failed: %s" % (tag, info))
        if form == "r64":  # no device residual for the real dtypes: the oracle's
            import oracle
            rel = oracle.rel_residual(s.A, s.B, x.cpu().numpy(), s.y)
        else:
            rel = sol.residual(A, B, x, y)[0]
        iters = int(info["refine_iters"]) if form == "fp32_refine" else 0
        mod = pcr_model(s.N, s.m, s.k) if pcr else step_model(
            "fp64" if form != "fp32_refine" else form, s.N, s.m, s.k, iters,
            real=form == "r64")
        rec = {
            "pcr_tail_blocks": sol.pcr_tail_blocks,
            "ms_per_step": ms,
            "ms_per_step_mean": mean,
            "ms_per_step_eager": ms_eager,
            "tuning": tuning,
            "value": s.N / (ms * 1e-3),
            "rel_residual": rel,
            "certified": bool(rel <= rtol),
            "refine_iters": iters,
            "fp64_fallback": int(info["fp64_fallback"]) if form == "fp32_refine" else 0,
            "workspace_bytes": sol.plan.ws_bytes,
            "kernel_ms_per_step": {kn: round(v[1], 4) for kn, v in per_step.items()},
            "kernel_launches_per_step": {kn: v[0] for kn, v in per_step.items()},
            "roofline": roofline(per_step, mod, form != "fp32_refine",
                                 ("pcr_" if pcr else "") + form, (s.N, s.m, s.k)),
            "model_bytes": sum(v[0] for v in mod.values()),
            "model_flops": sum(v[1] for v in mod.values()),
        }
        print("%s: %.3f ms/step, rel residual %.2e, %s" % (tag, ms, rel, json.dumps(
            rec["kernel_ms_per_step"])), file=sys.stderr, flush=True)
        xh = x.cpu().numpy()
        del sol
        torch.cuda.synchronize()
        return rec, xh

    for form in args.forms.split(","):
        if pcr and form != "fp64":
            continue  # Algorithm 1 runs in FP64 only
        forms[form], xs[form] = run_form(form, s, A, B, y, x, rtol, args.steps, args.warmup, form)

    certified = [f for f in forms if forms[f]["certified"]]
    if not certified:
        raise SystemExit("no form reached the residual bound: %s" % json.dumps(forms))
    best = min(certified, key=lambda f: forms[f]["ms_per_step"])
    xo = None
    if args.no_cpu_baseline:
        cpu = None
    elif args.workload == "poisson":
        # bounded sample: the same Poisson blocks with N = 256 (per block row the
        # reduction costs about the same at any N)
        cpu, _ = cpu_baseline(W.poisson(256, W.POISSON["m"]), args.cpu_budget,
                              "sample of the Poisson workload", extras=False)
    elif pcr:
        cpu, _ = cpu_baseline(W.random_hpd(4096, s.m, s.k, W.config_seed(1, 1)), args.cpu_budget,
                              "N=4096 sample of the workload, Algorithm 1", solver="pcr",
                              extras=False)
    else:
        cpu, xo = cpu_baseline(s, args.cpu_budget)
    # error of every form against the FP64 oracle (the closed form for Poisson)
    if args.workload == "poisson":
        xref = s.y / s.meta["lam"]
        for f in forms:
            forms[f]["err_vs_exact"] = float(np.max(np.abs(xs[f] - xref)) / np.max(np.abs(xref)))
    else:
        if xo is None and not args.no_cpu_baseline:
            import oracle
            xo, _ = oracle.solve_cr(s.A, s.B, s.y)
        if xo is not None:
            for f in forms:
                forms[f]["err_vs_oracle"] = float(np.max(np.abs(xs[f] - xo)) / np.max(np.abs(xo)))
    del xs

    # the precision workload at calibrated condition numbers (shifts from the
    # oracle-only calibration in tests/golden/kappa_shifts.json)
    if (args.workload == "random" and not pcr and not args.no_kappa
            and (s.N, s.m, s.k) == (W.LARGE["N"], W.LARGE["m"], W.LARGE["k"])):
        import oracle
        with open(os.path.join(ROOT, "tests", "golden", "kappa_shifts.json")) as fh:
            shifts = json.load(fh)["shifts"]
        del A, B, y
        t0 = time.perf_counter()
        base = W.random_hpd(**W.LARGE, seed=W.config_seed(2))
        print("precision workload generated in %.1f s" % (time.perf_counter() - t0),
              file=sys.stderr, flush=True)
        A0 = torch.from_numpy(base.A).to(dev)
        B = torch.from_numpy(base.B).to(dev)
        y = torch.from_numpy(base.y).to(dev)
        idx = np.arange(base.m)
        for kap, c in sorted(shifts.items(), key=lambda kv: float(kv[0])):
            A = A0.clone()
            A.diagonal(dim1=1, dim2=2).sub_(c)
            sk = W.System(base.A.copy(), base.B, base.y)
            sk.A[:, idx, idx] -= c
            xo_k, io_k = oracle.solve_cr(sk.A, sk.B, sk.y)
            assert io_k["status"] == 0
            for form in [f for f in args.forms.split(",") if f != "fp64_onesided"]:
                tag = "%s_kappa%s" % (form, kap)
                rec, xh = run_form(form, sk, A, B, y, x, rtol, min(args.steps, 5), 2, tag)
                rec["kappa"] = float(kap)
                rec["diag_shift"] = c
                rec["err_vs_oracle"] = float(np.max(np.abs(xh - xo_k)) / np.max(np.abs(xo_k)))
                forms[tag] = rec
            del A, sk
        del A0

    fb = forms[best]
    if not args.no_box_peaks:
        add_measured_peak(fb["roofline"])
    model_ms = max(fb["model_bytes"] / (PEAK_HBM_GBS * 1e9),
                   fb["model_flops"] / (PEAK_FP64_TFS * 1e12)) * 1e3
    out = {
        "metric": METRIC,
        "value": fb["value"],
        "unit": "block-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_refine": "c64+f64", "r64": "f64"}.get(best, "c128"),
        "data": "synthetic",
        "config": {"workload": "%s, N=%d block rows, m=%d, k=%d, complex128 inputs, solved "
                               "to rel. residual <= %.3g (%s, %s form)" % (
                                   "block 2D Poisson system, eigenvector right-hand side"
                                   if args.workload == "poisson" else
                                   "one HPD block-tridiagonal system", s.N, s.m, s.k, rtol,
                                   "Algorithm 1 in place" if pcr else
                                   "one-sided block cyclic reduction", best),
                   "schedule": args.schedule, "N": s.N, "m": s.m, "k": s.k, "form": best, "rtol": rtol,
                   "timing": "median of %d steps (HIP events per step), graph replay" % args.steps},
        "step_model": {"bytes": fb["model_bytes"], "flops": fb["model_flops"],
                       "roofline_ms": model_ms, "frac_of_step_roofline": model_ms / fb["ms_per_step"]},
        "roofline": fb["roofline"],
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
