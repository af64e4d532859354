"""PSLR preconditioner, oracle side (paper Sec. 3, Algorithms 3 and 4).

Notation follows the paper: after reordering, A = [[B, E], [F, C]] with
B (p x p) and E, F block diagonal by subdomain (eq. resystem),
S = C - F B^{-1} E (Schur complement, eq. solve), C0 = blkdiag(C_i) and
E_s = C0 - S = (C0 - C) + F B^{-1} E (eq. matrixS), C_g = C - C0.

P_m := sum_{i=0}^{m} (C0^{-1} E_s)^i C0^{-1}            (eq. approx1)
E_rr(m) := I - S P_m                                     (eqs. err1, err0)
Arnoldi on E_rr(m): E_rr ~ V H V^T                       (eq. schur)
G = (I - H)^{-1} - I                                     (eqs. Sinv0)
S_app^{-1} = P_m (I + V G V^T)                           (eq. Sinv)

Preconditioner application (Algorithm 3, eq. application):
    y = g - F B^{-1} f;  y += V G V^T y;  y = P_m y;  x = B^{-1}(f - E y).

The local solves use exact sparse LU (scipy's SuperLU) of every B_i and C_i,
or the paper's threshold ILU (oracle.ilu).  All arithmetic is FP64.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ilu as oilu
from . import partition as opart


# --------------------------------------------------------------------------
# Blocks (paper Sec. 2, eq. resystem; Sec. 3.1 for C0 and C_g)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Blocks:
    n: int
    p: int
    q: int
    perm: np.ndarray      # perm[new] = old
    int_ptr: np.ndarray   # interior ranges per part (in 0..p)
    if_ptr: np.ndarray    # interface ranges per part (in 0..q)
    B: sp.csr_matrix
    E: sp.csr_matrix
    F: sp.csr_matrix
    C: sp.csr_matrix
    C0: sp.csr_matrix
    Cg: sp.csr_matrix

    @property
    def nparts(self):
        return len(self.int_ptr) - 1


def make_blocks(A: sp.csr_matrix, label: np.ndarray) -> Blocks:
    A = sp.csr_matrix(A)
    perm, p, q, int_ptr, if_ptr = opart.reorder(A, label)
    Ap = A[perm][:, perm].tocsr()
    B = Ap[:p, :p].tocsr()
    E = Ap[:p, p:].tocsr()
    F = Ap[p:, :p].tocsr()
    C = Ap[p:, p:].tocsr()
    # C0 = block-diagonal part of C by subdomain
    owner = np.repeat(np.arange(len(if_ptr) - 1), np.diff(if_ptr))
    Ccoo = C.tocoo()
    same = owner[Ccoo.row] == owner[Ccoo.col]
    C0 = sp.csr_matrix((Ccoo.data[same], (Ccoo.row[same], Ccoo.col[same])), shape=(q, q))
    Cg = sp.csr_matrix((Ccoo.data[~same], (Ccoo.row[~same], Ccoo.col[~same])), shape=(q, q))
    blk = Blocks(A.shape[0], p, q, perm, int_ptr, if_ptr, B, E, F, C, C0, Cg)
    _assert_block_diagonal(blk)
    return blk


def _assert_block_diagonal(blk: Blocks):
    """B, E, F are block diagonal by subdomain (paper Sec. 2)."""
    iown = np.repeat(np.arange(blk.nparts), np.diff(blk.int_ptr))
    fown = np.repeat(np.arange(blk.nparts), np.diff(blk.if_ptr))
    for M, ro, co in ((blk.B, iown, iown), (blk.E, iown, fown), (blk.F, fown, iown)):
        c = M.tocoo()
        assert np.all(ro[c.row] == co[c.col])


# --------------------------------------------------------------------------
# Local exact LU factors (Algorithm 4, with exact LU in place of ILU)
# --------------------------------------------------------------------------


class BlockDiagSolver:
    """Block-diagonal solve with one factorisation per diagonal block: exact
    sparse LU (SuperLU) or the threshold ILU of Algorithm 4 (oracle.ilu)."""

    def __init__(self, M: sp.csr_matrix, ptr: np.ndarray, factor: str = "lu", drop: float = 1e-2):
        self.ptr = ptr
        self.lu = []
        for i in range(len(ptr) - 1):
            a, b = int(ptr[i]), int(ptr[i + 1])
            if b > a:
                blk = M[a:b, a:b]
                self.lu.append(spla.splu(sp.csc_matrix(blk)) if factor == "lu"
                               else oilu.IlutSolver(blk, drop))
            else:
                self.lu.append(None)

    def solve(self, r: np.ndarray, trans: bool = False) -> np.ndarray:
        out = np.empty_like(r)
        for i, lu in enumerate(self.lu):
            a, b = int(self.ptr[i]), int(self.ptr[i + 1])
            if lu is not None:
                out[a:b] = lu.solve(np.ascontiguousarray(r[a:b]), trans="T" if trans else "N")
        return out


# --------------------------------------------------------------------------
# Dense closed forms (small inputs only)
# --------------------------------------------------------------------------


def dense_forms(blk: Blocks, m: int):
    """S, E_s, P_m and E_rr(m) as dense matrices (eqs. matrixS, approx1, err1)."""
    B = blk.B.toarray(); E = blk.E.toarray(); F = blk.F.toarray()
    C = blk.C.toarray(); C0 = blk.C0.toarray()
    S = C - F @ np.linalg.solve(B, E)
    Es = C0 - S
    C0inv = np.linalg.inv(C0)
    K = C0inv @ Es
    Pm = np.zeros_like(S)
    term = C0inv.copy()
    for _ in range(m + 1):
        Pm += term
        term = K @ term
    Err = np.eye(blk.q) - S @ Pm
    return S, Es, Pm, Err


# --------------------------------------------------------------------------
# Arnoldi and the low-rank correction (eqs. schur, Sinv0)
# --------------------------------------------------------------------------


def arnoldi(op, v0: np.ndarray, rank: int, breakdown_tol: float = 1e-14):
    """rank-step Arnoldi on op, modified Gram-Schmidt with one full re-orthogonalisation.

    Returns (V, H, Hbar, vnext): V (q x r) orthonormal, H = Hbar[:r, :r] the
    square Hessenberg matrix of eq. schur, Hbar ((r+1) x r) and the next basis
    vector (or None after a breakdown).  A breakdown (h_{j+1,j} below
    breakdown_tol * ||op v_j||) stops with r = j + 1 vectors: the Krylov space
    is then invariant.
    """
    q = v0.shape[0]
    rank = min(rank, q)
    V = np.zeros((q, rank + 1))
    Hbar = np.zeros((rank + 1, rank))
    V[:, 0] = v0 / np.linalg.norm(v0)
    r = rank
    for j in range(rank):
        w = op(V[:, j])
        wnorm = np.linalg.norm(w)
        for _pass in range(2):
            for i in range(j + 1):
                c = V[:, i] @ w
                Hbar[i, j] += c
                w = w - c * V[:, i]
        h = np.linalg.norm(w)
        Hbar[j + 1, j] = h
        if h <= breakdown_tol * wnorm:
            r = j + 1
            return V[:, :r].copy(), Hbar[:r, :r].copy(), Hbar[:r + 1, :r].copy(), None
        V[:, j + 1] = w / h
    return V[:, :r].copy(), Hbar[:r, :r].copy(), Hbar.copy(), V[:, r].copy()


def g_matrix(H: np.ndarray) -> np.ndarray:
    """G = (I - H)^{-1} - I (eq. Sinv0)."""
    k = H.shape[0]
    I = np.eye(k)
    return np.linalg.solve(I - H, I) - I


# --------------------------------------------------------------------------
# The preconditioner
# --------------------------------------------------------------------------


class PSLR:
    """Matrix-free PSLR preconditioner (Algorithm 4 setup, Algorithm 3 apply)."""

    def __init__(self, A: sp.csr_matrix, label: np.ndarray, m: int, rank: int,
                 v0: np.ndarray | None = None, V: np.ndarray | None = None,
                 H: np.ndarray | None = None, factor: str = "lu", drop: float = 1e-2):
        """factor: "lu" (exact local factors) or "ilut" (threshold ILU, drop tolerance drop)."""
        self.A = sp.csr_matrix(A)
        self.m = int(m)
        self.blk = make_blocks(self.A, label)
        b = self.blk
        self.Bs = BlockDiagSolver(b.B, b.int_ptr, factor, drop)
        self.C0s = BlockDiagSolver(b.C0, b.if_ptr, factor, drop)
        if V is not None:
            self.set_lowrank(V, H)
        elif rank > 0 and b.q > 0:
            if v0 is None:
                v0 = np.ones(b.q)
            self.V, self.H, self.Hbar, _ = arnoldi(self.err_op, v0, rank)
            self.G = g_matrix(self.H)
        else:
            self.set_lowrank(np.zeros((b.q, 0)), np.zeros((0, 0)))

    def set_lowrank(self, V, H):
        self.V = np.asarray(V, dtype=np.float64)
        self.H = np.asarray(H, dtype=np.float64)
        self.G = g_matrix(self.H) if self.H.size else np.zeros((0, 0))

    # -- pieces --------------------------------------------------------------
    def Es(self, u):
        """E_s u = (C0 - C) u + F B^{-1} E u = -C_g u + F B^{-1} E u."""
        b = self.blk
        return -(b.Cg @ u) + b.F @ self.Bs.solve(b.E @ u)

    def EsT(self, u):
        b = self.blk
        return -(b.Cg.T @ u) + b.E.T @ self.Bs.solve(b.F.T @ u, trans=True)

    def err_op(self, v):
        """E_rr(m) v = (E_s C0^{-1})^{m+1} v (Theorem t2, eq. err)."""
        for _ in range(self.m + 1):
            v = self.Es(self.C0s.solve(v))
        return v

    def power_series(self, y):
        """P_m y via u_0 = C0^{-1} y, u_i = C0^{-1}(y + E_s u_{i-1}), i = 1..m."""
        u = self.C0s.solve(y)
        for _ in range(self.m):
            u = self.C0s.solve(y + self.Es(u))
        return u

    def power_series_T(self, y):
        """P_m^T y = C0^{-T} sum_i (E_s^T C0^{-T})^i y, by the same recurrence transposed."""
        u = self.C0s.solve(y, trans=True)
        for _ in range(self.m):
            u = self.C0s.solve(y + self.EsT(u), trans=True)
        return u

    def lowrank(self, y):
        if self.V.shape[1] == 0:
            return y
        return y + self.V @ (self.G @ (self.V.T @ y))

    def lowrank_T(self, y):
        if self.V.shape[1] == 0:
            return y
        return y + self.V @ (self.G.T @ (self.V.T @ y))

    # -- Algorithm 3 --------------------------------------------------------
    def apply(self, bvec: np.ndarray) -> np.ndarray:
        """z = PSLR(b), b and z in the ORIGINAL ordering (1-D or n x nrhs)."""
        if bvec.ndim == 2:
            return np.column_stack([self.apply(bvec[:, j]) for j in range(bvec.shape[1])])
        b = self.blk
        bp = bvec[b.perm]
        f, g = bp[:b.p], bp[b.p:]
        y = g - b.F @ self.Bs.solve(f)           # line 2 (read as g - F (B^{-1} f))
        y = self.lowrank(y)                      # line 3
        y = self.power_series(y)                 # line 4
        x = self.Bs.solve(f - b.E @ y)           # line 5
        z = np.empty_like(bvec)
        z[b.perm] = np.concatenate([x, y])       # line 6, back to original order
        return z

    def apply_transpose(self, bvec: np.ndarray) -> np.ndarray:
        """z = M^{-T} b where M^{-1} is the operator of Algorithm 3."""
        if bvec.ndim == 2:
            return np.column_stack([self.apply_transpose(bvec[:, j]) for j in range(bvec.shape[1])])
        b = self.blk
        bp = bvec[b.perm]
        f, g = bp[:b.p], bp[b.p:]
        y = g - b.E.T @ self.Bs.solve(f, trans=True)
        y = self.power_series_T(y)
        y = self.lowrank_T(y)
        x = self.Bs.solve(f - b.F.T @ y, trans=True)
        z = np.empty_like(bvec)
        z[b.perm] = np.concatenate([x, y])
        return z

    # -- dense forms of this operator (small inputs) ------------------------
    def dense_sapp_inv(self):
        S, Es, Pm, Err = dense_forms(self.blk, self.m)
        k = self.V.shape[1]
        return Pm @ (np.eye(self.blk.q) + self.V @ self.G @ self.V.T) if k else Pm

    def delta(self):
        """Delta(m, r_k) = ||X||_F ||Z^{-1}||_F with X = E_rr(m) - V H V^T and
        Z = I - V H V^T, the bound of Prop. l3 (Sec. 3.2.3), from the dense forms
        (small inputs).  Returns (delta, ||X||_F, ||Z^{-1}||_F)."""
        S, Es, Pm, Err = dense_forms(self.blk, self.m)
        VHV = self.V @ self.H @ self.V.T if self.V.shape[1] else np.zeros_like(Err)
        X = Err - VHV
        Zi = np.linalg.inv(np.eye(self.blk.q) - VHV)
        nx, nz = np.linalg.norm(X), np.linalg.norm(Zi)
        return nx * nz, nx, nz

    def dense_inverse(self):
        """M^{-1} in the permuted ordering from the block LDU inverse with S_app."""
        b = self.blk
        B = b.B.toarray(); E = b.E.toarray(); F = b.F.toarray()
        Sai = self.dense_sapp_inv()
        Bi = np.linalg.inv(B)
        top = np.hstack([Bi + Bi @ E @ Sai @ F @ Bi, -Bi @ E @ Sai])
        bot = np.hstack([-Sai @ F @ Bi, Sai])
        return np.vstack([top, bot])
