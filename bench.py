"""Throughput benchmark: block rows solved per second on one MI355X.

Workload: one Hermitian positive definite block-tridiagonal system with
N = 65536 block rows, m = 32, k = 16, complex128 (seeded synthetic inputs from
``paper_1807_00370_amd.workloads``).  A step is one fused factor + solve pass
of the one-sided block cyclic reduction (every reduction level, then the
back substitution of every level) on inputs already resident in HBM.

Prints one JSON line with the throughput, a roofline entry for the kernel
that takes the most time per step (algorithmic bytes or flops from the model
below, divided by its event-measured average launch duration) and the FP64
CPU oracle timed on this host as a reported baseline.

Algorithmic model, per eliminated block of the fused pass, s bytes per complex
element (16 for complex128), complex multiply-add = 8 real flops:
  k_elim   (Cholesky + three triangular solves)
           bytes (6 m^2 + 2 m k) s: read A_p, B_p, B_{p-1}, y_p, write L, P, Q, g
           flops 8 (m^3/6 + m^3 + m^2 k/2)
  k_reduce (per kept block: two Hermitian products, one product, two rhs products)
           bytes (6 m^2 + 4 m k) s: read A_q, P_l, Q_r, P_r, y_q, g_l, g_r,
           write A'_q, B'_q, y'_q
           flops 8 (2 m^3 + 2 m^2 k)
  k_back   bytes (3 m^2 + 4 m k) s: read L, P, Q, g, x_{p-1}, x_{p+1}, write x_p
           flops 8 (5/2 m^2 k)
Blocks without a neighbour (ends of each level) skip the missing terms.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_FP64_TFS = 78.6         # MI355X FP64 (vector = matrix), TFLOP/s
PEAK_FP32_TFS = 157.3        # MI355X FP32, TFLOP/s
METRIC = "Block-rows solved/s & % roofline: FP32+refine vs FP64 at rel. residual ≤1e-12"


def level_counts(N: int):
    """(n, eliminated, kept, eliminated-with-prev, eliminated-with-next,
    kept-with-right) per level of the one-sided schedule."""
    out = []
    n = N
    while n > 0:
        ne, nk = (n + 1) // 2, n // 2
        e_prev = ne - 1                      # p = 0 has no previous block
        e_next = nk                          # p + 1 < n
        k_right = sum(1 for q in range(1, n, 2) if q + 1 < n)
        k_f = sum(1 for q in range(1, n, 2) if q + 2 < n)
        out.append((n, ne, nk, e_prev, e_next, k_right, k_f))
        n //= 2
    return out


def model(N: int, m: int, k: int, s: int):
    """Algorithmic bytes and flops per fused factor + solve pass, per kernel."""
    mm, mk = m * m, m * k
    tot = {"k_elim": [0, 0], "k_reduce": [0, 0], "k_back": [0, 0]}
    for (n, ne, nk, e_prev, e_next, k_right, k_f) in level_counts(N):
        # k_elim: A, y in; L, g out; B_{p-1} in + Q out if prev; B_p in + P out if next
        b = ne * (2 * mm + 2 * mk) + (e_prev + e_next) * 2 * mm
        f = ne * (mm * m / 6 + mk * m / 2) + (e_prev + e_next) * mm * m / 2
        tot["k_elim"][0] += b * s
        tot["k_elim"][1] += 8 * f
        # k_reduce: A_q, y_q in, outputs A', y'; P_l, g_l always; Q_r, g_r if right;
        # F = -P_r^H Q_r when the right block has both
        b = nk * (2 * mm + 2 * mk) + nk * (mm + mk) + k_right * (mm + mk) + k_f * (mm + mm + mm)
        f = nk * (mm * m / 2 + mk * m) + k_right * (mm * m / 2 + mk * m) + k_f * mm * m
        tot["k_reduce"][0] += b * s
        tot["k_reduce"][1] += 8 * f
        # k_back: L, g, x in; x out; Q, x_{p-1} if prev; P, x_{p+1} if next
        b = ne * (mm + 2 * mk) + (e_prev + e_next) * (mm + mk)
        f = (e_prev + e_next) * mk * m + ne * mk * m / 2
        tot["k_back"][0] += b * s
        tot["k_back"][1] += 8 * f
    return {kname: {"bytes": v[0], "flops": v[1]} for kname, v in tot.items()}


def cpu_baseline(s, budget_s: float):
    import oracle
    oracle.build(force=False)
    reps, t0 = 0, time.perf_counter()
    while True:
        x, info = oracle.solve_cr(s.A, s.B, s.y)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 8:
            break
    assert info["status"] == 0
    return {"value": s.N * reps / el, "unit": "block-rows/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "full workload (N=%d, m=%d, k=%d, complex128), FP64 one-sided cyclic "
                      "reduction, %d solve(s) in %.1f s" % (s.N, s.m, s.k, reps, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs each system on a single "
              "device and this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1807_00370_amd import workloads as W
    from paper_1807_00370_amd.solver import Solver

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    s = W.random_hpd(args.N, args.m, args.k, W.config_seed(1))
    print("inputs generated in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    A = torch.from_numpy(s.A).to(dev)
    B = torch.from_numpy(s.B).to(dev)
    y = torch.from_numpy(s.y).to(dev)
    sol = Solver([s.N], [s.m], [s.k], dtype=torch.complex128, device=dev)
    x = torch.empty_like(y)

    for _ in range(args.warmup):
        sol.factor_solve(A, B, y, x)
    torch.cuda.synchronize()
    info = sol.info_host()[0]
    if info["status"] != 0:
        raise SystemExit("factorization failed: %s" % (info,))

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        sol.factor_solve(A, B, y, x)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    print("timed %d steps: %.3f ms/step" % (args.steps, ms), file=sys.stderr, flush=True)

    # per-kernel durations from HIP events bracketing each launch, same steps again
    sol.plan.timing(True)
    for _ in range(args.steps):
        sol.factor_solve(A, B, y, x)
    kt = sol.plan.timing_read()
    sol.plan.timing(False)
    torch.cuda.synchronize()
    mod = model(s.N, s.m, s.k, 16)
    per_step = {kn: (cnt / args.steps, tot / args.steps) for kn, (cnt, tot) in kt.items()}
    print("kernel times per step: %s" % json.dumps(
        {kn: {"launches": v[0], "ms": round(v[1], 4)} for kn, v in per_step.items()}),
        file=sys.stderr, flush=True)
    dom = max((kn for kn in mod), key=lambda kn: per_step.get(kn, (0, 0))[1])
    launches, kms = per_step[dom]
    avg_launch_ms = kms / launches
    byts, flops = mod[dom]["bytes"], mod[dom]["flops"]
    ai = flops / byts
    balance = PEAK_FP64_TFS * 1e12 / (PEAK_HBM_GBS * 1e9)
    if ai < balance:
        achieved = byts / launches / (avg_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        achieved = flops / launches / (avg_launch_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_launch_ms
    roof["launches_per_step"] = launches
    roof["algorithmic_bytes_per_launch"] = byts / launches
    roof["algorithmic_flops_per_launch"] = flops / launches
    tot_b = sum(v["bytes"] for v in mod.values())
    tot_f = sum(v["flops"] for v in mod.values())
    step_roof_ms = max(tot_b / (PEAK_HBM_GBS * 1e9), tot_f / (PEAK_FP64_TFS * 1e12)) * 1e3

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s, args.cpu_budget)
    del np

    out = {
        "metric": METRIC,
        "value": s.N / (ms * 1e-3),
        "unit": "block-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "one HPD block-tridiagonal system, N=%d block rows, m=%d, "
                               "k=%d, complex128, FP64 fused factor+solve (one-sided cyclic "
                               "reduction)" % (s.N, s.m, s.k),
                   "N": s.N, "m": s.m, "k": s.k, "form": "fp64"},
        "step_model": {"bytes": tot_b, "flops": tot_f, "roofline_ms": step_roof_ms,
                       "frac_of_step_roofline": step_roof_ms / ms},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
