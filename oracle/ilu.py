"""Threshold incomplete LU of a diagonal block (the ilu() of Algorithm 4), oracle side.

The paper builds ILU factors of every B_i and C_i with a dropping threshold
of 1e-2 (Algorithm 4; Sec. 4, Tables 1-3).  This is the row-oriented
threshold ILU of Saad (ILUT, Numer. Linear Algebra Appl. 1, 1994; Iterative
Methods for Sparse Linear Systems, 2nd ed., Sec. 10.4) with the dropping
threshold only (no cap on the entries kept per row), in the block's own row
order and without pivoting.  The row's reference size is the mean modulus of
its stored entries (||a_i||_1 / nnz(a_i), as in Saad's SPARSKIT ILUT): with
it the fill factor of Table 1 (2.68 at s = 5 on the 50^3 problem) is
reproduced, while the 2-norm gives about 1.55.

  for each row i:  w = a_i;  tau_i = drop * ||a_i||_1 / nnz(a_i)
    for each k < i with w_k != 0, in increasing k:
      w_k = w_k / u_kk;  if |w_k| < tau_i: drop it (no update from row k)
      else: w = w - w_k * u_k            (u_k: row k of U right of the diagonal)
    l_i = the kept w_k (k < i);  u_i = w_i and every w_j (j > i) with |w_j| >= tau_i

drop = 0 gives the exact LU factorisation without pivoting.  Pure Python
loops: meant for the small blocks of the tests.
"""
from __future__ import annotations

import heapq

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def ilut(M, drop: float):
    """Return (L, U): L unit lower triangular (diagonal stored), U upper, both CSR."""
    M = sp.csr_matrix(M)
    M.sort_indices()
    n = M.shape[0]
    Lrows = []
    Urows = []          # row k of U right of the diagonal: list of (j, u_kj), ascending j
    diag = np.zeros(n)
    for i in range(n):
        cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
        vals = M.data[M.indptr[i]:M.indptr[i + 1]]
        w = {}
        nrm1 = 0.0
        for j, v in zip(cols.tolist(), vals.tolist()):
            w[j] = v
            nrm1 = nrm1 + abs(v)
        tau_i = drop * (nrm1 / len(cols)) if len(cols) else 0.0
        heap = [j for j in w if j < i]
        heapq.heapify(heap)
        lrow = []
        while heap:
            k = heapq.heappop(heap)
            wk = w.pop(k) / diag[k]
            if abs(wk) < tau_i:
                continue
            lrow.append((k, wk))
            for j, ukj in Urows[k]:
                if j not in w:
                    w[j] = 0.0
                    if j < i:
                        heapq.heappush(heap, j)
                w[j] = w[j] - wk * ukj
        if w.get(i, 0.0) == 0.0:
            raise ZeroDivisionError("zero pivot in the incomplete factorisation at row %d" % i)
        diag[i] = w[i]
        Urows.append(sorted((j, v) for j, v in w.items() if j > i and abs(v) >= tau_i))
        Lrows.append(sorted(lrow))
    L = _csr([[(k, v) for k, v in r] + [(i, 1.0)] for i, r in enumerate(Lrows)], n)
    U = _csr([[(i, diag[i])] + r for i, r in enumerate(Urows)], n)
    return L, U


def _csr(rows, n):
    ptr = np.zeros(n + 1, dtype=np.int64)
    idx, val = [], []
    for i, r in enumerate(rows):
        r = sorted(r)
        idx.extend(j for j, _ in r)
        val.extend(v for _, v in r)
        ptr[i + 1] = len(idx)
    return sp.csr_matrix((np.array(val, dtype=np.float64), np.array(idx, dtype=np.int64), ptr),
                         shape=(n, n))


class IlutSolver:
    """Solves with the incomplete factors: M^{-1} r ~ U^{-1} L^{-1} r (or its transpose)."""

    def __init__(self, M, drop: float):
        self.L, self.U = ilut(M, drop)
        self.LT = sp.csr_matrix(self.L.T)
        self.UT = sp.csr_matrix(self.U.T)

    def solve(self, r, trans="N"):
        if trans == "T":
            y = spla.spsolve_triangular(self.UT, r, lower=True)
            return spla.spsolve_triangular(self.LT, y, lower=False, unit_diagonal=True)
        y = spla.spsolve_triangular(self.L, r, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)

    @property
    def nnz(self):
        """Entries of L + U (the unit diagonal of L not counted)."""
        return int(self.L.nnz - self.L.shape[0] + self.U.nnz)
