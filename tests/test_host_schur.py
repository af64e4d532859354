"""Host-only Krylov-Schur truncation step of the library (pslr_host_schur_select),
no GPU: an orthonormal basis of the invariant subspace of a small real matrix
for its k eigenvalues of largest modulus.  Checked against the definition
(H W = W Hk, W^T W = I, eig(Hk) = the kept eigenvalues), against numpy's
eigenvalues, and against the oracle's selection rule and its sorted real
Schur basis (SciPy), on random, Hessenberg-with-coupling-row, defective and
degenerate matrices."""
import numpy as np
import pytest

from paper_2002_00917_amd import pslr as P
from oracle import deflation as odefl


def _check(H, k, tol=1e-11, evtol=1e-9):
    n = H.shape[0]
    W, Hk, ritz = P.pslr_host_schur_select(H, k)
    ev = np.linalg.eigvals(H)
    # the oracle's kept count: the selection rule plus values tied at the cut
    kept_o = odefl.sorted_schur(H, k)[2] if k > 0 else 0
    kept = W.shape[1]
    assert kept == kept_o
    # all eigenvalues, by decreasing modulus
    assert np.allclose(np.sort(np.abs(ritz))[::-1], np.sort(np.abs(ev))[::-1],
                       rtol=evtol, atol=1e-12 * max(1.0, np.abs(ev).max()))
    if kept == 0:
        return W, Hk
    nrm = max(np.linalg.norm(H, 2), 1e-300)
    assert np.linalg.norm(W.T @ W - np.eye(kept)) <= 1e-13 * kept
    assert np.linalg.norm(H @ W - W @ Hk) <= tol * nrm
    # the kept eigenvalues are the kept_o of largest modulus
    top = np.sort(np.abs(ev))[::-1][:kept]
    assert np.allclose(np.sort(np.abs(np.linalg.eigvals(Hk)))[::-1], top, rtol=max(evtol, 1e-8),
                       atol=1e-10 * nrm)
    return W, Hk


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,k", [(8, 3), (40, 12), (96, 40)])
def test_random(seed, n, k):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n, n))
    W, _ = _check(H, k)
    # the same subspace as the oracle's sorted real Schur basis, when the cut has a gap
    ev = np.linalg.eigvals(H)
    mods = np.sort(np.abs(ev))[::-1]
    kept = W.shape[1]
    if kept < n and mods[kept - 1] - mods[kept] > 1e-3 * mods[0]:
        Z, T, sdim = odefl.sorted_schur(H, k)
        Zk = Z[:, :sdim]
        assert sdim == kept
        assert np.linalg.norm(W @ W.T - Zk @ Zk.T) <= 1e-8


def test_krylov_schur_shape():
    """Leading triangular block, a full coupling row, then Hessenberg columns."""
    rng = np.random.default_rng(7)
    n, k = 60, 20
    H = np.triu(rng.standard_normal((n, n)), -1)
    H[:k, :k] = np.triu(rng.standard_normal((k, k)))
    H[k, :k] = rng.standard_normal(k)
    _check(H, k)


def test_complex_pair_at_cut():
    # eigenvalues 5, 3 +- 1i, 2, -1.5, 0.5 in a random real basis
    B = np.zeros((6, 6))
    B[0, 0] = 5.0
    B[1:3, 1:3] = [[3.0, 1.0], [-1.0, 3.0]]
    B[3, 3], B[4, 4], B[5, 5] = 2.0, -1.5, 0.5
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((6, 6)))
    H = Q @ B @ Q.T
    for k, want in ((1, 1), (2, 1), (3, 3), (4, 4), (6, 6)):
        W, Hk = _check(H, k)
        assert W.shape[1] == want


def test_defective_and_degenerate():
    # a 3 x 3 Jordan block (eigenvalues perturbed by ~eps^(1/3)) above four
    # simple eigenvalues; the cut after the block keeps its invariant subspace
    n = 7
    J = np.diag([2.0, 2.0, 2.0, 0.5, 0.4, 0.3, 0.2]) + np.diag([1.0, 1.0, 0, 0, 0, 0], 1)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((n, n)))
    W, Hk = _check(Q @ J @ Q.T, 3, tol=1e-9, evtol=1e-4)
    assert W.shape[1] == 3
    X = Q[:, :3]  # the exact invariant subspace of the block
    assert np.linalg.norm(W @ W.T - X @ X.T) <= 1e-8
    I6 = np.eye(6) * 3.0
    W, Hk = _check(I6, 4)       # all six tie at the cut: all are kept
    assert np.allclose(Hk, 3.0 * np.eye(6))
    # a tie at the cut between +-2 (E_rr with odd powers keeps signs)
    D = np.diag([5.0, 2.0, -2.0, 1.0, 0.5])
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((5, 5)))
    W, Hk = _check(Q @ D @ Q.T, 2)
    assert W.shape[1] == 3


def test_edge_sizes():
    _check(np.array([[4.0]]), 1)
    _check(np.zeros((5, 5)), 2)
    _check(np.random.default_rng(3).standard_normal((7, 7)), 7)
    _check(np.random.default_rng(4).standard_normal((7, 7)), 20)
    W, Hk, ritz = P.pslr_host_schur_select(np.eye(3), 0)
    assert W.shape[1] == 0
