"""Deflated low-rank correction: Krylov-Schur on E_rr(m), oracle side.

The paper builds V and H from an r_k-step Arnoldi process on
E_rr(m) = (E_s C0^{-1})^{m+1} (eq. schur, Thm. t2) and motivates the low-rank
term as a deflation of the eigenvalues of modulus above 1 (Sec. 1, advantage
1; Sec. 3.2.2, Figs. 4-5; Prop. l3 needs r_k above their count).  A raw
r_k-step Arnoldi basis only approximates that invariant subspace.  This
variant converges it: Stewart's Krylov-Schur restarting (SIAM J. Matrix Anal.
Appl. 23, 2001) expands the basis to r_k + p vectors, takes the real Schur
form of the projected matrix with the r_k Ritz values of largest modulus
first, truncates to those r_k Schur vectors and expands again, until the
coupling of the kept space to the rest is below tol.  The result keeps the
paper's form: V orthonormal (q x r_k) and H = V^T E_rr V, now with
E_rr V = V H + O(tol), so S_app^{-1} = P_m (I + V G V^T) with
G = (I - H)^{-1} - I as in eq. Sinv0.  With an exact invariant subspace the
preconditioned Schur complement has r_k eigenvalues equal to 1 and the others
equal to 1 - theta for the eigenvalues theta of E_rr outside it
(lambda(S_app^{-1} S) = 1 - lambda(Z^{-1} X), Sec. 3.2.3).

Selection rule (both sides implement it): the kept Ritz values are the r_k of
largest modulus; when the cut would split a complex-conjugate pair, the pair
is dropped and r_k - 1 are kept.

The dense real Schur decomposition with a selected leading block is SciPy's
(LAPACK gees with a selection callable), used here as a library primitive.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def select_count(evals: np.ndarray, k: int) -> tuple[int, float]:
    """Number kept and the modulus threshold: the k largest |theta|, dropping a
    complex pair that the cut would split."""
    mod = np.abs(evals)
    order = np.argsort(-mod, kind="stable")
    k = min(k, len(evals))
    if k == 0:
        return 0, np.inf
    if k < len(evals):
        a, b = evals[order[k - 1]], evals[order[k]]
        if abs(a.imag) > 0 and abs(a - np.conj(b)) <= 1e-12 * max(1.0, abs(a)):
            k -= 1
    if k == 0:
        return 0, np.inf
    return k, float(mod[order[k - 1]])


def sorted_schur(Hm: np.ndarray, k: int):
    """Real Schur form Hm = Z T Z^T with the k largest-modulus eigenvalues first.

    Returns (Z, T, kept)."""
    ev = np.linalg.eigvals(Hm)
    kept, thr = select_count(ev, k)
    if kept == 0:
        return np.eye(Hm.shape[0]), Hm.copy(), 0
    # modulus threshold slightly below the kept one so rounding cannot drop it
    cut = thr * (1.0 - 1e-10)
    T, Z, sdim = sla.schur(Hm, output="real", sort=lambda re, im: np.hypot(re, im) >= cut)
    return Z, T, int(sdim)


def krylov_schur(op, v0: np.ndarray, k: int, p: int | None = None, tol: float = 1e-9,
                 max_restarts: int = 60, grow: bool = False, kmax: int = 256):
    """Converged r_k-dimensional invariant subspace of op for its largest-modulus eigenvalues.

    op: v -> E_rr(m) v on the interface (length q).  Returns (V, H, info) with
    V (q x kept) orthonormal, H = V^T op(V) and info = dict(restarts,
    applies, residual) where residual = ||op(V) - V H||_2 bound from the
    Krylov-Schur coupling row.

    grow: the paper's case for the correction is the deflation of every
    eigenvalue of modulus above 1 (Sec. 3.2.2; Prop. l3 needs r_k above their
    count).  When a cycle has converged with every kept Ritz value outside the
    unit circle, k is raised to 16 more than the number of Ritz values of the
    whole projected matrix outside it (at least k + 16, at most kmax) and the
    iteration continues from the kept space, with p = max(k, 16) again.
    """
    q = v0.shape[0]
    k = min(k, q)
    kmax = min(kmax, q)
    if p is None:
        p = max(k, 16)
    m = min(k + p, q)
    if m <= k:  # the whole space: one Arnoldi pass is exact
        m = k
    width = max(m, min(kmax + max(kmax, 16), q)) if grow else m
    V = np.zeros((q, width + 1))
    H = np.zeros((width + 1, width))
    V[:, 0] = v0 / np.linalg.norm(v0)
    j0 = 0
    applies = 0
    kept = k
    res = np.inf
    for restart in range(max_restarts + 1):
        # Arnoldi expansion of columns j0 .. m-1 (Gram-Schmidt, two passes)
        breakdown = False
        for j in range(j0, m):
            w = op(V[:, j])
            applies += 1
            for _pass in range(2):
                c = V[:, :j + 1].T @ w
                H[:j + 1, j] += c
                w = w - V[:, :j + 1] @ c
            h = np.linalg.norm(w)
            H[j + 1, j] = h
            if h <= 1e-14 * max(1.0, np.abs(H[:j + 1, j]).max()):
                # invariant subspace of dimension j + 1
                m_eff = j + 1
                breakdown = True
                break
            V[:, j + 1] = w / h
        m_eff = m_eff if breakdown else m
        Hm = H[:m_eff, :m_eff]
        Z, T, kept = sorted_schur(Hm, min(k, m_eff))
        # coupling of the kept Schur vectors to the next basis vector
        b = H[m_eff, :m_eff] @ Z[:, :kept] if not breakdown else np.zeros(kept)
        scale = np.abs(np.diag(T)[:kept]).min() if kept else 1.0
        res = float(np.linalg.norm(b))
        done = breakdown or m_eff == q or res <= tol * max(scale, 1e-300) or restart == max_restarts
        if (done and grow and not breakdown and m_eff < q and restart < max_restarts and kept
                and kept_min_modulus(T, kept) > 1.0 and k < kmax):
            above = int(np.sum(np.abs(np.linalg.eigvals(Hm)) > 1.0))
            k = min(kmax, max(k + 16, above + 16))
            p = max(k, 16)
            done = False
        if done:
            Vk = V[:, :m_eff] @ Z[:, :kept]
            Hk = T[:kept, :kept].copy()
            return Vk, Hk, dict(restarts=restart, applies=applies, residual=res)
        # truncate to the kept Krylov-Schur decomposition and expand again
        Vk = V[:, :m_eff] @ Z[:, :kept]
        vnext = V[:, m_eff].copy()
        V[:] = 0.0
        V[:, :kept] = Vk
        V[:, kept] = vnext
        Hn = np.zeros_like(H)
        Hn[:kept, :kept] = T[:kept, :kept]
        Hn[kept, :kept] = b
        H = Hn
        j0 = kept
        m = min(max(kept, k) + p, q, width)
    raise AssertionError("unreachable")


def kept_min_modulus(T: np.ndarray, kept: int) -> float:
    """Smallest modulus among the eigenvalues of the leading kept x kept block
    of a real Schur form."""
    return float(np.abs(np.linalg.eigvals(T[:kept, :kept])).min())
