"""Block cyclic reduction for Hermitian positive definite block-tridiagonal
systems on AMD Instinct MI355X (arXiv 1807.00370).

``solver`` holds the PyTorch front end (device memory and streams only);
``_lib`` the ctypes binding of ``include/crsolve.h``; ``workloads`` the seeded
synthetic inputs.  Importing the package does not load the HIP library.
"""
__all__ = ["solver", "workloads"]
