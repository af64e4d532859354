"""Pins of the oracle's deflated low-rank correction (Krylov-Schur on E_rr(m)), no GPU.

Each check compares the oracle with something outside it: the dense
eigen-decomposition of E_rr (LAPACK geev through numpy, a different routine
from the sorted real Schur step the oracle uses on its small projected
matrix), the inertia count of the shifted symmetric case, and the closed-form
spectrum of the deflated preconditioned Schur complement
(lambda(S_app^{-1} S) = 1 - lambda(Z^{-1} X), Sec. 3.2.3).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2002_00917_amd import workloads as wl
from oracle import partition as opart
from oracle import pslr as opslr
from oracle import deflation as odefl


def cases():
    out = []
    # cases and ranks chosen with a gap in |eigenvalue| right after the kept ones
    A = wl.laplacian2d(12, wl.sigma_for_negatives(wl.laplacian_eigs((12, 12)), 10))
    out.append(("lap2d_12_10neg", A.to_scipy(), opart.geometric_labels((12, 12), (2, 2)), 2, 10))
    A = wl.laplacian3d(8, wl.sigma_for_negatives(wl.laplacian_eigs((8, 8, 8)), 11))
    out.append(("lap3d_8_11neg", A.to_scipy(), opart.geometric_labels((8, 8, 8), (2, 2, 2)), 3, 12))
    A = wl.convdiff3d(7, 10.0, 0.8)
    As = A.to_scipy()
    out.append(("convdiff_7_rg", As, opart.region_growing_labels(As, 5, 7), 2, 8))
    return out


CASES = cases()
IDS = [c[0] for c in CASES]


def dense_err(pre):
    S, Es, Pm, Err = opslr.dense_forms(pre.blk, pre.m)
    return S, Pm, Err


def top_invariant_basis(M, k):
    """Orthonormal real basis of M's invariant subspace for its k largest-modulus
    eigenvalues, from the dense eigenvectors (conjugate pairs give Re and Im)."""
    ev, X = np.linalg.eig(M)
    order = np.argsort(-np.abs(ev), kind="stable")[:k]
    cols = []
    for i in order:
        cols.append(X[:, i].real)
        if abs(ev[i].imag) > 0:
            cols.append(X[:, i].imag)
    Q, R = np.linalg.qr(np.column_stack(cols))
    rank = int(np.sum(np.abs(np.diag(R)) > 1e-8 * np.abs(np.diag(R)).max()))
    return Q[:, :rank], ev[order]


def test_selection_rule():
    ev = np.array([5.0, 3 + 1j, 3 - 1j, 2.0, -1.5, 0.5])
    assert odefl.select_count(ev, 1)[0] == 1
    assert odefl.select_count(ev, 2)[0] == 1        # the cut would split 3 +- i: dropped
    assert odefl.select_count(ev, 3)[0] == 3
    assert odefl.select_count(ev, 5)[0] == 5
    k, thr = odefl.select_count(ev, 4)
    assert k == 4 and thr == 2.0


@pytest.mark.parametrize("name,A,lab,m,k", CASES, ids=IDS)
def test_krylov_schur_finds_dominant_invariant_subspace(name, A, lab, m, k):
    pre = opslr.PSLR(A, lab, m, 0)
    q = pre.blk.q
    S, Pm, Err = dense_err(pre)
    V, H, info = odefl.krylov_schur(pre.err_op, wl.start_vector(q, 3), k, tol=1e-11)
    kk = V.shape[1]
    print(name, "q", q, "kept", kk, "restarts", info["restarts"], "applies", info["applies"],
          "residual", info["residual"])
    assert kk in (k, k - 1)
    # orthonormal, H the Rayleigh quotient, and the space invariant under E_rr
    assert np.abs(V.T @ V - np.eye(kk)).max() < 1e-12
    EV = np.column_stack([pre.err_op(V[:, j]) for j in range(kk)])
    nE = np.linalg.norm(Err, 2)
    assert np.abs(H - V.T @ EV).max() < 1e-11 * nE
    assert np.linalg.norm(EV - V @ H, 2) < 1e-9 * nE
    # the same space and eigenvalues as the dense eigen-decomposition's dominant part
    Qd, evd = top_invariant_basis(Err, kk)
    assert Qd.shape[1] == kk
    gap = np.sort(np.abs(np.linalg.eigvals(Err)))[::-1]
    assert gap[kk - 1] > 1.01 * gap[kk], "cases are chosen with a gap after the kept values"
    assert np.abs(V @ V.T - Qd @ Qd.T).max() < 1e-7
    np.testing.assert_allclose(np.sort(np.abs(np.linalg.eigvals(H))), np.sort(np.abs(evd)), rtol=1e-9)


def test_deflated_spectrum_closed_form():
    """With the converged invariant subspace, S_app^{-1} S has kept eigenvalues
    equal to 1 and the others equal to 1 - theta for the remaining eigenvalues
    theta of E_rr (Sec. 3.2.3 with X V = 0)."""
    name, A, lab, m, k = CASES[1]
    pre = opslr.PSLR(A, lab, m, 0)
    S, Pm, Err = dense_err(pre)
    V, H, info = odefl.krylov_schur(pre.err_op, wl.start_vector(pre.blk.q, 3), k, tol=1e-12)
    pre.set_lowrank(V, H)
    Sapp_inv = pre.dense_sapp_inv()
    lam = np.linalg.eigvals(Sapp_inv @ S)
    theta = np.linalg.eigvals(Err)
    order = np.argsort(-np.abs(theta), kind="stable")
    rest = theta[order[V.shape[1]:]]
    expect = np.concatenate([np.ones(V.shape[1]), 1.0 - rest])
    # match the two multisets greedily (eigenvalues of a nonsymmetric product)
    lam = list(lam)
    for e in expect:
        d = [abs(e - x) for x in lam]
        j = int(np.argmin(d))
        assert d[j] < 1e-6 * max(1.0, abs(e)), (e, lam[j])
        lam.pop(j)


def test_inertia_count_of_deflated_values():
    """Shifted symmetric case: E_s C0^{-1} is similar to a symmetric matrix, and
    the number of its eigenvalues above 1 equals neg(A) - neg(B) (Haynsworth +
    Sylvester); Krylov-Schur with enough rank keeps exactly those outside the
    unit circle in E_rr = (E_s C0^{-1})^{m+1} first."""
    A = wl.laplacian3d(8, wl.sigma_for_negatives(wl.laplacian_eigs((8, 8, 8)), 11))
    As = A.to_scipy()
    lab = opart.geometric_labels((8, 8, 8), (2, 2, 2))
    pre = opslr.PSLR(As, lab, 2, 0)
    negA = int(np.sum(np.linalg.eigvalsh(As.toarray()) < 0))
    negB = int(np.sum(np.linalg.eigvalsh(pre.blk.B.toarray()) < 0))
    S, Pm, Err = dense_err(pre)
    lam = np.linalg.eigvals(Err)
    n_out = int(np.sum(np.abs(lam) > 1.0))
    assert n_out >= negA - negB
    k = n_out + 4
    V, H, info = odefl.krylov_schur(pre.err_op, wl.start_vector(pre.blk.q, 9), k, tol=1e-11)
    th = np.linalg.eigvals(H)
    assert int(np.sum(np.abs(th) > 1.0)) == n_out
    C0 = pre.blk.C0.toarray()
    K = (C0 - S) @ np.linalg.inv(C0)      # E_s C0^{-1}
    assert int(np.sum(np.linalg.eigvals(K).real > 1.0)) == negA - negB


def test_raw_arnoldi_is_not_invariant_but_deflation_is():
    """The paper's raw r_k-step Arnoldi basis leaves a residual E_rr V - V H
    of the size of h_{r+1,r}; the Krylov-Schur basis of the same rank does not."""
    name, A, lab, m, k = CASES[0]
    pre = opslr.PSLR(A, lab, m, 0)
    v0 = wl.start_vector(pre.blk.q, 3)
    Va, Ha, Hbar, _ = opslr.arnoldi(pre.err_op, v0, k)
    Vk, Hk, info = odefl.krylov_schur(pre.err_op, v0, k, tol=1e-11)
    ra = np.linalg.norm(np.column_stack([pre.err_op(Va[:, j]) for j in range(Va.shape[1])]) - Va @ Ha)
    rk = np.linalg.norm(np.column_stack([pre.err_op(Vk[:, j]) for j in range(Vk.shape[1])]) - Vk @ Hk)
    np.testing.assert_allclose(ra, abs(Hbar[-1, -1]), rtol=1e-8)
    assert rk < 1e-6 * ra


def test_growth_keeps_every_eigenvalue_outside_the_unit_circle():
    """grow=True (Sec. 3.2.2): started with a rank below the count, the kept
    space grows until it holds every eigenvalue of E_rr of modulus above 1; in
    the shifted symmetric case that count is neg(A) - neg(B) (inertia), and
    the kept space contains the dense invariant subspace of those eigenvalues
    (E_s C0^{-1} may also have eigenvalues below -1, so the count outside the
    unit circle is at least neg(A) - neg(B))."""
    A = wl.laplacian3d(8, wl.sigma_for_negatives(wl.laplacian_eigs((8, 8, 8)), 11))
    As = A.to_scipy()
    lab = opart.geometric_labels((8, 8, 8), (2, 2, 2))
    pre = opslr.PSLR(As, lab, 2, 0)
    negA = int(np.sum(np.linalg.eigvalsh(As.toarray()) < 0))
    negB = int(np.sum(np.linalg.eigvalsh(pre.blk.B.toarray()) < 0))
    S, Pm, Err = dense_err(pre)
    lam = np.linalg.eigvals(Err)
    n_out = int(np.sum(np.abs(lam) > 1.0))
    assert n_out >= negA - negB and n_out > 4
    V, H, info = odefl.krylov_schur(pre.err_op, wl.start_vector(pre.blk.q, 9), 4, tol=1e-11,
                                    grow=True)
    th = np.linalg.eigvals(H)
    assert V.shape[1] >= n_out + 1
    assert int(np.sum(np.abs(th) > 1.0)) == n_out
    assert np.abs(th).min() <= 1.0
    Qd, _ = top_invariant_basis(Err, n_out)
    assert np.linalg.norm(Qd - V @ (V.T @ Qd)) < 1e-7
    # without growth the same start keeps only 4
    V4, _, _ = odefl.krylov_schur(pre.err_op, wl.start_vector(pre.blk.q, 9), 4, tol=1e-11)
    assert V4.shape[1] == 4
