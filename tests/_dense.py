"""Test helper: assemble the dense matrix of Eq. (Axb) from block arrays."""
import numpy as np


def herm_block(a: np.ndarray) -> np.ndarray:
    """Hermitian reading of a diagonal block: lower triangle, real diagonal."""
    m = a.shape[0]
    h = np.tril(a) + np.conj(np.tril(a, -1)).T
    h[np.diag_indices(m)] = h[np.diag_indices(m)].real
    return h


def dense(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    N, m, _ = A.shape
    D = np.zeros((N * m, N * m), dtype=np.complex128)
    for j in range(N):
        D[j * m:(j + 1) * m, j * m:(j + 1) * m] = herm_block(A[j])
    for j in range(N - 1):
        D[(j + 1) * m:(j + 2) * m, j * m:(j + 1) * m] = B[j]
        D[j * m:(j + 1) * m, (j + 1) * m:(j + 2) * m] = np.conj(B[j]).T
    return D


def stack(x: np.ndarray) -> np.ndarray:
    """[N, m, k] -> [N*m, k]."""
    return x.reshape(-1, x.shape[2])


def rel_err(a, b) -> float:
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
