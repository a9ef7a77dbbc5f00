"""Seeded synthetic inputs for block-tridiagonal Hermitian positive definite systems.

This module only draws inputs; it holds none of the solver's arithmetic, so both
the CPU oracle and the HIP path can take their inputs from here.

Problem shape (paper, Section 1, Eq. (Axb) and Eq. (Data)): blocks
``A_1..A_N`` (m x m), ``B_1..B_{N-1}`` (m x m) and right-hand sides
``y_1..y_N`` (m x k), all complex.  Arrays use 0-based numpy storage:

* ``A[j-1]``  is ``A_j``            shape ``[N, m, m]``
* ``B[j-1]``  is ``B_j``            shape ``[N-1, m, m]``  (block row j+1, column j)
* ``y[j-1]``  is ``y_j``            shape ``[N, m, k]``

Every array is C-contiguous complex128.  Only the lower triangle and the real
part of the diagonal of each ``A_j`` carry meaning for the solver; the
generators still return exactly Hermitian blocks.

Recipes (the synthetic stand-ins for the paper's unspecified workloads):

* ``random_hpd``: ``B_j`` iid complex normal with standard deviation
  ``1/sqrt(m)``; ``A_j = M_j M_j^H / m + (||B_{j-1}||_2 + ||B_j||_2 + margin) I``
  with ``M_j`` iid complex normal, which makes the matrix block diagonally
  dominant and hence Hermitian positive definite.  ``||B_0|| = ||B_N|| = 0``.
  ``shift`` subtracts ``shift_scale * (||B_{j-1}|| + ||B_j|| + margin) I``
  (``shift_scale=2`` makes every diagonal block indefinite).
  ``ill=True`` replaces the margin 1 by ``1e-5 (||B_{j-1}|| + ||B_j||)``.
  ``diag_shift=c`` subtracts ``c I`` from every ``A_j`` afterwards (the
  calibrated condition numbers of the precision workload use the shifts in
  ``tests/golden/kappa_shifts.json``, computed from the oracle's extreme
  eigenvalues by the script beside it).
* ``poisson``: the real 2D five-point Laplacian on an m x N grid,
  ``A_j = tridiag(-1, 4, -1)``, ``B_j = -I``, with ``y`` an eigenvector
  ``y[j, a] = sin(p a pi/(m+1)) sin(q j pi/(N+1))`` (1-based a, j).
* ``batch_shapes``: ragged batch of (N, m, k) triples.

Complex normal draws with standard deviation s put ``N(0, s^2/2)`` in the real
and in the imaginary part, so that ``E|z|^2 = s^2``.  Draw order per system:
``B``, then ``M``, then ``y``, then ``W``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 180700370


def config_seed(config_index: int, instance: int = 0) -> int:
    """Seed of instance ``instance`` of workload ``config_index``."""
    return SEED_BASE + 10 * config_index + instance


def _cnormal(rng: np.random.Generator, shape, std: float) -> np.ndarray:
    z = rng.standard_normal((2,) + tuple(shape))
    out = np.empty(shape, dtype=np.complex128)
    out.real = z[0]
    out.imag = z[1]
    out *= std / math.sqrt(2.0)
    return out


def spectral_norms(B: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """2-norm of every block of ``B`` (largest singular value)."""
    out = np.empty(B.shape[0], dtype=np.float64)
    for s in range(0, B.shape[0], chunk):
        blk = B[s:s + chunk]
        # largest eigenvalue of B^H B equals ||B||_2^2
        g = np.conj(np.swapaxes(blk, 1, 2)) @ blk
        out[s:s + chunk] = np.sqrt(np.maximum(np.linalg.eigvalsh(g)[:, -1], 0.0))
    return out


@dataclass
class System:
    A: np.ndarray
    B: np.ndarray
    y: np.ndarray
    W: np.ndarray | None = None
    meta: dict | None = None

    @property
    def N(self) -> int:
        return self.A.shape[0]

    @property
    def m(self) -> int:
        return self.A.shape[1]

    @property
    def k(self) -> int:
        return self.y.shape[2]


def random_hpd(N: int, m: int, k: int, seed: int, *, margin: float = 1.0,
               shift_scale: float = 0.0, ill: bool = False, diag_shift: float = 0.0,
               with_W: bool = False, chunk: int = 8192) -> System:
    """The block diagonally dominant Hermitian positive definite generator."""
    if N < 1 or m < 1 or k < 1:
        raise ValueError("N, m, k must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    B = _cnormal(rng, (max(N - 1, 0), m, m), 1.0 / math.sqrt(m))
    nb = spectral_norms(B) if N > 1 else np.zeros(0)
    left = np.zeros(N)
    right = np.zeros(N)
    if N > 1:
        left[1:] = nb       # ||B_{j-1}||
        right[:-1] = nb     # ||B_j||
    if ill:
        diag = (1.0 + 1e-5) * (left + right)
    else:
        diag = left + right + margin
    if shift_scale:
        diag = diag - shift_scale * (left + right + margin)
    A = np.empty((N, m, m), dtype=np.complex128)
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        M = _cnormal(rng, (e - s, m, m), 1.0)
        blk = M @ np.conj(np.swapaxes(M, 1, 2))
        blk /= m
        blk = 0.5 * (blk + np.conj(np.swapaxes(blk, 1, 2)))
        idx = np.arange(m)
        blk[:, idx, idx] = blk[:, idx, idx].real + diag[s:e, None] - diag_shift
        A[s:e] = blk
    y = _cnormal(rng, (N, m, k), 1.0)
    W = _cnormal(rng, (N, m, k), 1.0) if with_W else None
    return System(A, B, y, W, dict(kind="random_hpd", N=N, m=m, k=k, seed=seed,
                                   margin=margin, shift_scale=shift_scale, ill=ill,
                                   diag_shift=diag_shift))


def random_spd(N: int, m: int, k: int, seed: int, *, margin: float = 1.0,
               shift_scale: float = 0.0) -> System:
    """The real case of the generator: ``B_j`` iid normal with standard
    deviation ``1/sqrt(m)``, ``A_j = M_j M_j^T / m + (||B_{j-1}||_2 +
    ||B_j||_2 + margin) I``, ``y`` iid normal; real float64 arrays.
    ``shift_scale`` as in ``random_hpd``.  Draw order B, M, y."""
    if N < 1 or m < 1 or k < 1:
        raise ValueError("N, m, k must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.standard_normal((max(N - 1, 0), m, m)) / math.sqrt(m)
    nb = spectral_norms(B.astype(np.complex128)) if N > 1 else np.zeros(0)
    left = np.zeros(N)
    right = np.zeros(N)
    if N > 1:
        left[1:] = nb
        right[:-1] = nb
    diag = left + right + margin
    if shift_scale:
        diag = diag - shift_scale * (left + right + margin)
    M = rng.standard_normal((N, m, m))
    A = M @ np.swapaxes(M, 1, 2) / m
    A = 0.5 * (A + np.swapaxes(A, 1, 2))
    idx = np.arange(m)
    A[:, idx, idx] += diag[:, None]
    y = rng.standard_normal((N, m, k))
    return System(np.ascontiguousarray(A), np.ascontiguousarray(B), y, None,
                  dict(kind="random_spd", N=N, m=m, k=k, seed=seed, margin=margin,
                       shift_scale=shift_scale))


def poisson(N: int, m: int, p: int = 1, q: int = 1, real: bool = False) -> System:
    """Block 2D Poisson system with an eigenvector right-hand side (k = 1).

    Returns the eigenvalue as ``meta['lam']``; the exact solution is
    ``y / lam``.  ``real``: float64 arrays instead of complex128.
    """
    dt = np.float64 if real else np.complex128
    A1 = 4.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    A = np.broadcast_to(A1, (N, m, m)).astype(dt)
    B = np.broadcast_to(-np.eye(m), (max(N - 1, 0), m, m)).astype(dt)
    a = np.arange(1, m + 1)
    j = np.arange(1, N + 1)
    ya = np.sin(p * a * math.pi / (m + 1))
    yj = np.sin(q * j * math.pi / (N + 1))
    y = (yj[:, None] * ya[None, :])[:, :, None].astype(dt)
    lam = 4.0 - 2.0 * math.cos(p * math.pi / (m + 1)) - 2.0 * math.cos(q * math.pi / (N + 1))
    return System(np.ascontiguousarray(A), np.ascontiguousarray(B), y, None,
                  dict(kind="poisson", N=N, m=m, k=1, p=p, q=q, lam=lam))


def batch_shapes(count: int, seed: int, n_half_range=(128, 4096),
                 m_choices=(8, 16, 32, 64), k_choices=(1, 4, 16)):
    """Ragged batch: N = 2*U{lo..hi}, m and k uniform over the choices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = 2 * rng.integers(n_half_range[0], n_half_range[1] + 1, size=count)
    ms = rng.choice(np.asarray(m_choices), size=count)
    ks = rng.choice(np.asarray(k_choices), size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(Ns, ms, ks)]


def batch_systems(shapes, seed: int, **kw):
    """One ``random_hpd`` system per (N, m, k), each with its own seed."""
    return [random_hpd(N, m, k, seed * 1000 + i, **kw) for i, (N, m, k) in enumerate(shapes)]


_PACK = {}


def _pack_one(i):
    from multiprocessing import shared_memory
    from threadpoolctl import threadpool_limits
    st = _PACK
    N, m, k = st["shapes"][i]
    with threadpool_limits(1):  # one BLAS thread per worker process
        q = random_hpd(N, m, k, st["seed"] * 1000 + i)
    for name, arr, off in (("A", q.A, st["offA"][i]), ("B", q.B, st["offB"][i]),
                           ("y", q.y, st["offy"][i])):
        shm = shared_memory.SharedMemory(name=st["shm"][name])
        dst = np.ndarray((st["tot"][name],), dtype=np.complex128, buffer=shm.buf)
        dst[off:off + arr.size] = arr.ravel()
        del dst
        shm.close()
    return i


def batch_packed(shapes, seed: int, workers: int = 1, shared: bool = False):
    """The systems of ``batch_systems(shapes, seed)`` packed back to back:
    flat (A, B, y) arrays in the library's batch layout.  With ``workers`` > 1
    the systems are drawn by forked worker processes into shared memory
    (same values: every system has its own generator).  Fork only from a
    process that has not initialised a GPU.  With ``shared`` (and workers >
    1) the arrays are views of the shared-memory segments, returned with a
    ``release()`` callable that frees them (no copy of the inputs)."""
    offA, offB, offy = [0], [0], [0]
    for N, m, k in shapes:
        offA.append(offA[-1] + N * m * m)
        offB.append(offB[-1] + (N - 1) * m * m)
        offy.append(offy[-1] + N * m * k)
    tot = {"A": offA[-1], "B": offB[-1], "y": offy[-1]}
    if workers <= 1:
        out = {n: np.empty(tot[n], np.complex128) for n in tot}
        for i, (N, m, k) in enumerate(shapes):
            q = random_hpd(N, m, k, seed * 1000 + i)
            out["A"][offA[i]:offA[i + 1]] = q.A.ravel()
            out["B"][offB[i]:offB[i + 1]] = q.B.ravel()
            out["y"][offy[i]:offy[i + 1]] = q.y.ravel()
        return out["A"], out["B"], out["y"]
    import multiprocessing as mp
    from multiprocessing import shared_memory
    shms = {n: shared_memory.SharedMemory(create=True, size=max(tot[n], 1) * 16) for n in tot}
    try:
        _PACK.clear()
        _PACK.update(shapes=list(shapes), seed=seed, offA=offA, offB=offB, offy=offy, tot=tot,
                     shm={n: shms[n].name for n in shms})
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_pack_one, range(len(shapes))):
                pass
        if shared:
            views = [np.ndarray((tot[n],), dtype=np.complex128, buffer=shms[n].buf)
                     for n in ("A", "B", "y")]

            def release():
                views.clear()
                for sh in shms.values():
                    sh.close()
                    sh.unlink()
            _PACK.clear()
            return views[0], views[1], views[2], release
        out = [np.ndarray((tot[n],), dtype=np.complex128, buffer=shms[n].buf).copy()
               for n in ("A", "B", "y")]
    except BaseException:
        for sh in shms.values():
            sh.close()
            sh.unlink()
        _PACK.clear()
        raise
    for sh in shms.values():
        sh.close()
        sh.unlink()
    _PACK.clear()
    return tuple(out)


def _draw_one(args):
    from threadpoolctl import threadpool_limits
    i, N, m, k, seed = args
    with threadpool_limits(1):
        q = random_hpd(N, m, k, seed * 1000 + i)
    return i, q.A, q.B, q.y


class BatchStream:
    """The systems of ``batch_systems(shapes, seed)`` drawn by forked worker
    processes and handed to the caller one by one (``for i, A, B, y in
    stream``), so that a batch larger than host memory can be copied into
    packed device arrays system by system.  Create it before the calling
    process initialises a GPU (the workers are forked at construction)."""

    def __init__(self, shapes, seed: int, workers: int):
        import multiprocessing as mp
        self.shapes = list(shapes)
        self.seed = seed
        self.pool = mp.get_context("fork").Pool(max(1, workers))
        self.offA, self.offB, self.offy = [0], [0], [0]
        for N, m, k in self.shapes:
            self.offA.append(self.offA[-1] + N * m * m)
            self.offB.append(self.offB[-1] + (N - 1) * m * m)
            self.offy.append(self.offy[-1] + N * m * k)

    def __iter__(self):
        jobs = [(i, N, m, k, self.seed) for i, (N, m, k) in enumerate(self.shapes)]
        try:
            for rec in self.pool.imap_unordered(_draw_one, jobs):
                yield rec
        finally:
            self.pool.close()
            self.pool.join()


# The named workloads (sizes as the paper's problem statement instantiates them)
TINY = dict(N=64, m=4, k=1)                 # one system, plus an indefinite twin
LARGE = dict(N=65536, m=32, k=16)           # large single system
POISSON = dict(N=4096, m=256, k=1)          # real block 2D Poisson
DIFF = dict(N=16384, m=64, k=32)            # adjoint workload
BATCH_COUNT = 512                           # ragged batch size
