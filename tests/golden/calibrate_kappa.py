"""Writes kappa_shifts.json: diagonal shifts c that give the precision
workload (N=65536, m=32, k=16, the random HPD generator with the seed of the
precision workload) a prescribed condition number kappa once every diagonal
block is replaced by A_j - c I.

Calls only the CPU oracle (test infrastructure):
* lambda_min(A) by bisection on the oracle's breakdown flag (Section 2,
  "Determination of Positive Definiteness": A - c I is positive definite iff
  every Cholesky factorization of the reduction succeeds, i.e. iff
  c < lambda_min);
* lambda_max(A) by power iteration with the products A v = -r(A, B, v, 0)
  of the oracle's residual of Eq. (Axb), with the Rayleigh quotient.
Then c = lambda_min - (lambda_max - lambda_min) / (kappa - 1), so that
(lambda_max - c) / (lambda_min - c) = kappa.

Run: python tests/golden/calibrate_kappa.py   (about 5 minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1807_00370_amd import workloads as W  # noqa: E402

N, M, K = 65536, 32, 16
KAPPAS = (1e5, 1e6)
OUT = os.path.join(HERE, "kappa_shifts.json")


def shifted(A, c):
    As = A.copy()
    idx = np.arange(A.shape[1])
    As[:, idx, idx] -= c
    return As


def is_pd(A, B, y1, c):
    _, info = oracle.solve_cr(shifted(A, c), B, y1)
    return info["status"] == 0


def main():
    t0 = time.time()
    s = W.random_hpd(N, M, 1, W.config_seed(2))
    A, B, y1 = s.A, s.B, s.y
    # bracket: the generator makes A block diagonally dominant with margin 1,
    # so lambda_min >= 1 - (rounding); lambda_min <= min_j lambda_min(A_j)
    lo = 0.5
    hi = float(np.min(np.linalg.eigvalsh(A[:4096])[:, 0]))
    assert is_pd(A, B, y1, lo) and not is_pd(A, B, y1, hi)
    steps = 0
    while hi - lo > 1e-13 * hi:
        mid = 0.5 * (lo + hi)
        if is_pd(A, B, y1, mid):
            lo = mid
        else:
            hi = mid
        steps += 1
    lam_min = lo
    print("lambda_min %.15g after %d bisection steps (%.0f s)" % (lam_min, steps, time.time() - t0),
          flush=True)
    rng = np.random.default_rng(2024)
    v = rng.standard_normal((N, M, 1)) + 1j * rng.standard_normal((N, M, 1))
    v /= np.linalg.norm(v)
    zero = np.zeros_like(v)
    rq_prev, rq = 0.0, 0.0
    for it in range(400):
        av = -oracle.residual(A, B, v, zero)
        rq = float(np.vdot(v, av).real)
        v = av / np.linalg.norm(av)
        if it > 20 and abs(rq - rq_prev) <= 1e-10 * rq:
            break
        rq_prev = rq
    lam_max = rq
    print("lambda_max %.12g after %d power steps (%.0f s)" % (lam_max, it + 1, time.time() - t0),
          flush=True)
    rec = {"workload": "random HPD generator, N=%d, m=%d, seed %d (precision workload)"
                       % (N, M, W.config_seed(2)),
           "lambda_min": lam_min, "lambda_max": lam_max,
           "kappa_unshifted": lam_max / lam_min, "bisection_steps": steps,
           "power_steps": it + 1, "shifts": {}}
    for kap in KAPPAS:
        c = lam_min - (lam_max - lam_min) / (kap - 1.0)
        assert is_pd(A, B, y1, c)
        rec["shifts"]["%g" % kap] = c
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
