"""Gradient of a loss of the solution z of A z = b with respect to A's nonzeros.

With z = A^{-1} b and a scalar loss L(z), differentiating A z = b gives
dz = -A^{-1} dA z, so dL/dA_ij = -lambda_i z_j with A^T lambda = dL/dz.
Only the stored entries (the sparsity pattern of A, in CSR order) receive a
gradient.  Exact sparse solves (SuperLU) are used here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    return spla.splu(sp.csc_matrix(A)).solve(b)


def pattern_grad(A: sp.csr_matrix, lam: np.ndarray, z: np.ndarray) -> np.ndarray:
    """-lambda[i_k] * z[j_k] for every stored entry k of A (CSR order)."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    if lam.ndim == 1:
        return -lam[rows] * z[A.indices]
    return -np.sum(lam[rows, :] * z[A.indices, :], axis=1)


def loss_and_grad(A: sp.csr_matrix, b: np.ndarray, zstar: np.ndarray):
    """L = ||z - z*||^2 with z = A^{-1} b; returns (L, z, lambda, dL/dvals)."""
    lu = spla.splu(sp.csc_matrix(A))
    z = lu.solve(b)
    gz = 2.0 * (z - zstar)
    lam = lu.solve(gz, trans="T")
    return float(np.sum((z - zstar) ** 2)), z, lam, pattern_grad(A, lam, z)
