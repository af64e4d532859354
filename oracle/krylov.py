"""Right-preconditioned flexible GMRES in FP64 (the paper's accelerator, Sec. 4).

Flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993): the preconditioned
vectors z_j = M^{-1} v_j are kept, and the update is x = x0 + Z_j y_j.  The
paper counts "its" as iterations needed to reduce the initial residual norm by
1e8 from x0 = 0, failing above 500; this oracle uses the same rule with the
residual measured relative to ||b|| (identical for x0 = 0).
"""
from __future__ import annotations

import numpy as np


def fgmres(A, b, precond=None, x0=None, restart=40, maxit=500, tol=1e-8):
    """Returns (x, iterations, true relative residual, converged)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    M = (lambda v: v) if precond is None else precond
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0, True
    its = 0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm or its >= maxit:
            break
        V = np.zeros((n, restart + 1))
        Z = np.zeros((n, restart))
        Hh = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[:, j] = M(V[:, j])
            w = A @ Z[:, j]
            for i in range(j + 1):              # modified Gram-Schmidt
                Hh[i, j] = V[:, i] @ w
                w = w - Hh[i, j] * V[:, i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] > 0:
                V[:, j + 1] = w / Hh[j + 1, j]
            for i in range(j):                  # apply previous Givens rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            d = np.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j] = Hh[j, j] / d
            sn[j] = Hh[j + 1, j] / d
            Hh[j, j] = d
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            if abs(g[j + 1]) <= tol * bnorm or its >= maxit:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):     # back substitution
            y[i] = (g[i] - Hh[i, i + 1:j_done] @ y[i + 1:]) / Hh[i, i]
        x = x + Z[:, :j_done] @ y
    rel = np.linalg.norm(b - A @ x) / bnorm
    return x, its, rel, rel <= tol
