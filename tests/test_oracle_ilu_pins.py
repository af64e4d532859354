"""Pins of the oracle's threshold ILU (the ilu() of Algorithm 4), no GPU.

* drop = 0 is the exact LU factorisation without pivoting: L U = A, and the
  solve equals SuperLU's (a library routine);
* drop > 0: by the definition of the row-oriented threshold ILU, A - L U
  vanishes on the kept pattern of L + U; every entry of A - L U off that
  pattern is a dropped one, below tau_i (times |u_jj| for an L entry, which is
  dropped after division by the pivot); every kept off-diagonal entry is at
  least tau_i, with tau_i = drop * ||a_i||_1 / nnz(a_i) (the mean modulus of
  the row's stored entries);
* a hand-worked 3 x 3 case where that rule and the 2-norm rule differ;
* more dropping keeps fewer entries (monotone fill in the threshold).
The fill factor against the paper's Table 1 is checked on the library's ILUT
(test_host_library.py), which keeps exactly the oracle's entries.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2002_00917_amd import workloads as wl
from oracle import ilu as oilu


def mats():
    return [("lap2d_15_shift", wl.laplacian2d(15, 0.3).to_scipy()),
            ("lap3d_7_shift", wl.laplacian3d(7, wl.sigma_for_negatives(wl.laplacian_eigs((7, 7, 7)), 4)).to_scipy()),
            ("convdiff_6", wl.convdiff3d(6, 10.0, 0.2).to_scipy())]


@pytest.mark.parametrize("name,A", mats(), ids=[m[0] for m in mats()])
def test_drop_zero_is_exact_lu(name, A):
    L, U = oilu.ilut(A, 0.0)
    Ad = A.toarray()
    assert np.allclose(np.tril(L.toarray(), -1), L.toarray() - np.eye(A.shape[0]))
    assert np.allclose(np.diag(L.toarray()), 1.0)
    assert np.allclose(np.tril(U.toarray(), -1), 0.0)
    np.testing.assert_allclose((L @ U).toarray(), Ad, atol=1e-13 * np.abs(Ad).max())
    b = np.sin(np.arange(A.shape[0]) + 1.0)
    s = oilu.IlutSolver(A, 0.0)
    ref = spla.splu(sp.csc_matrix(A)).solve(b)
    np.testing.assert_allclose(s.solve(b), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(s.solve(b, trans="T"), spla.splu(sp.csc_matrix(A)).solve(b, trans="T"),
                               rtol=1e-11, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("drop", [1e-3, 1e-2, 5e-2])
@pytest.mark.parametrize("name,A", mats(), ids=[m[0] for m in mats()])
def test_dropping_rule_invariants(name, A, drop):
    L, U = oilu.ilut(A, drop)
    n = A.shape[0]
    Ad = A.toarray()
    R = Ad - (L @ U).toarray()
    tau = drop * np.abs(Ad).sum(axis=1) / np.diff(sp.csr_matrix(A).indptr)
    kept = (np.abs(L.toarray() - np.eye(n)) > 0) | (np.abs(U.toarray()) > 0)
    np.fill_diagonal(kept, True)
    # zero on the kept pattern
    assert np.abs(R[kept]).max() <= 1e-13 * np.abs(Ad).max()
    # dropped entries: below tau_i (U side) or tau_i |u_jj| (L side)
    Ud = np.diag(U.toarray())
    ii, jj = np.nonzero(~kept & (np.abs(R) > 0))
    lim = np.where(jj < ii, tau[ii] * np.abs(Ud[jj]), tau[ii])
    assert np.all(np.abs(R[ii, jj]) < lim * (1 + 1e-12))
    # kept off-diagonal entries pass the threshold
    Lo = sp.tril(L, -1).tocoo()
    Uo = sp.triu(U, 1).tocoo()
    assert np.all(np.abs(Lo.data) >= tau[Lo.row])
    assert np.all(np.abs(Uo.data) >= tau[Uo.row])


def test_fill_decreases_with_the_threshold():
    A = wl.laplacian3d(9, 0.2).to_scipy()
    nnz = [oilu.IlutSolver(A, d).nnz for d in (0.0, 1e-3, 1e-2, 1e-1)]
    assert nnz[0] > nnz[1] > nnz[2] > nnz[3] >= A.nnz - 0.5 * A.nnz


def test_mean_modulus_rule_by_hand():
    """Row 1 of [[4, 1, 0], [1, 4, .05], [0, .05, 4]] at drop .02: tau_1 = .02 * 5.05 / 3
    = .0337, so u_12 = .05 is kept (the 2-norm rule, .02 * 4.12 = .0825, would drop it).
    Row 2: l_21 = .05 / u_11 = .05 / 3.75 = .0133 < tau_2 = .02 * 4.05 / 2 = .0405 is
    dropped, so u_22 = 4 exactly."""
    A = sp.csr_matrix(np.array([[4.0, 1.0, 0.0], [1.0, 4.0, 0.05], [0.0, 0.05, 4.0]]))
    L, U = oilu.ilut(A, 0.02)
    Ld, Ud = L.toarray(), U.toarray()
    np.testing.assert_allclose(Ld, [[1, 0, 0], [0.25, 1, 0], [0, 0, 1]], atol=1e-15)
    np.testing.assert_allclose(Ud, [[4, 1, 0], [0, 3.75, 0.05], [0, 0, 4]], atol=1e-15)
