"""Host-side logic of the HIP library, checked on the CPU (no GPU calls).

* the C ABI exports every function include/pslr.h declares;
* partition labels and the reordering are bit-exact with the oracle;
* the exact LU factors and the packed level-scheduled solve layouts solve the
  diagonal blocks to rounding (host execution of the device layouts).
"""
import os
import re

import numpy as np
import pytest

from paper_2002_00917_amd import workloads as wl
from paper_2002_00917_amd import pslr as P
from oracle import partition as opart

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="libpslr.so not built")


def test_header_symbols_exported():
    with open(os.path.join(ROOT, "include", "pslr.h")) as fh:
        src = fh.read()
    names = set(re.findall(r"^\s*(?:pslr_status|void|const char\*)\s+(\w+)\s*\(", src, re.M))
    assert {"pslr_setup", "pslr_apply", "pslr_apply_transpose", "fgmres_solve"} <= names
    L = P.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(P.EXPORTED) == names


def test_geometric_partition_bit_exact():
    for dims, parts in (((64, 64), (2, 2)), ((64, 64, 64), (4, 4, 4)), ((37, 23), (3, 5)),
                        ((11, 7, 5), (2, 3, 1)), ((256, 256), (4, 4))):
        assert np.array_equal(P.pslr_partition_geometric(dims, parts),
                              opart.geometric_labels(dims, parts))


def test_region_growing_bit_exact():
    cases = [(wl.laplacian2d(40, 0.0, Ny=31), 9, 3), (wl.convdiff3d(14, 10.0, 0.1), 17, 4),
             (wl.laplacian2d(130, 0.0), 23, 3003)]
    for A, s, seed in cases:
        lab, nl = P.pslr_partition_region_growing(A.rowptr, A.colind, s, seed)
        olab = opart.region_growing_labels(A.to_scipy(), s, seed)
        assert nl == s and np.array_equal(lab, olab)


def test_region_growing_disconnected_graph():
    # two disconnected grids and one seed: the unreached part gets a new label
    import scipy.sparse as sp
    a = wl.laplacian2d(6, 0.0).to_scipy()
    A = wl.CSR.from_scipy(sp.block_diag([a, a]))
    lab, nl = P.pslr_partition_region_growing(A.rowptr, A.colind, 1, 1)
    olab = opart.region_growing_labels(A.to_scipy(), 1, 1)
    assert np.array_equal(lab, olab) and nl == 2 and len(set(lab.tolist())) == 2


def test_reorder_bit_exact():
    rng = np.random.default_rng(3)
    for A, lab in ((wl.c1().A, opart.geometric_labels((64, 64), (2, 2))),
                   (wl.laplacian3d(20, 0.1), opart.geometric_labels((20,) * 3, (3, 2, 2))),
                   (wl.laplacian2d(30, 0.0), rng.integers(0, 5, size=900).astype(np.int32))):
        perm, p, q = P.pslr_reorder(A.rowptr, A.colind, lab, int(lab.max()) + 1)
        operm, op, oq, _, _ = opart.reorder(A.to_scipy(), lab)
        assert (p, q) == (op, oq) and np.array_equal(perm, operm)


@pytest.mark.parametrize("case", ["c1", "lap3d", "convdiff_rg", "random_labels", "c5_like"])
def test_block_factor_layouts_solve(case):
    rng = np.random.default_rng(0)
    if case == "c1":
        A = wl.c1().A
        lab = opart.geometric_labels((64, 64), (2, 2))
    elif case == "lap3d":
        A = wl.laplacian3d(18, wl.SIGMA_C2)
        lab = opart.geometric_labels((18,) * 3, (2, 2, 2))
    elif case == "convdiff_rg":
        A = wl.convdiff3d(16, 10.0, 0.2)
        lab = opart.region_growing_labels(A.to_scipy(), 6, 4)
    elif case == "random_labels":
        A = wl.laplacian2d(25, 0.3)
        lab = rng.integers(0, 7, size=A.n).astype(np.int32)
    else:
        w, kappa, kref, sigma = wl.c5(48)
        A = w.A
        lab = opart.geometric_labels((48, 48), (4, 4))
    fr, sr = P.pslr_host_selfcheck(A.rowptr, A.colind, A.vals, lab, int(lab.max()) + 1,
                                   want_transpose=True, nthreads=4)
    assert fr < 1e-13, fr
    assert sr < 1e-10, sr


def test_singular_block_reported():
    # a 1-D Laplacian block shifted exactly onto one of its eigenvalues is singular
    N = 9
    lam = 2.0 - 2.0 * np.cos(np.pi / (N + 1))
    import scipy.sparse as sp
    T = sp.diags([-np.ones(N - 1), (2.0 - lam) * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    A = wl.CSR.from_scipy(T)
    lab = np.zeros(N, dtype=np.int32)
    with pytest.raises(P.PslrError) as ei:
        P.pslr_host_selfcheck(A.rowptr, A.colind, A.vals, lab, 1)
    assert ei.value.status == P.PSLR_ESINGULAR


def test_invalid_arguments():
    A = wl.laplacian2d(5, 0.0)
    bad = np.full(A.n, 3, dtype=np.int32)
    with pytest.raises(P.PslrError) as ei:
        P.pslr_reorder(A.rowptr, A.colind, bad, 2)
    assert ei.value.status == P.PSLR_EINVAL
    with pytest.raises(P.PslrError):
        P.pslr_partition_geometric((4, 4), (5, 1))


@pytest.mark.parametrize("case", ["lap3d", "convdiff_rg", "c1"])
def test_level_schedules_are_valid(case):
    """Every packed factor (exact LU and ILU, forward and transposed): each
    position scheduled once, a supernode on one level, every dependency solved
    before the row that needs it."""
    if case == "lap3d":
        A = wl.laplacian3d(14, wl.SIGMA_C2)
        lab = opart.geometric_labels((14,) * 3, (2, 2, 2))
    elif case == "convdiff_rg":
        A = wl.convdiff3d(12, 10.0, 0.2)
        lab = opart.region_growing_labels(A.to_scipy(), 6, 4)
    else:
        A = wl.c1().A
        lab = opart.geometric_labels((64, 64), (2, 2))
    for factor in ("lu", "ilut"):
        st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, int(lab.max()) + 1,
                               want_transpose=True, nthreads=4, factor=factor)
        print(case, factor, st)
        assert st["levels_valid"] == 1
        assert st["solve_residual"] < 1e-12
        assert st["factor_residual"] < (1e-13 if factor == "lu" else 1e-14)


@pytest.mark.parametrize("case", ["lap2d", "lap3d", "convdiff_rg"])
def test_ilut_keeps_the_oracles_entries(case):
    """The library's threshold ILU of every B_i and C_i keeps exactly as many
    entries as the oracle's (the dropping decisions are integer results taken
    in FP64 by the same sequence of operations on both sides)."""
    from oracle import pslr as opslr
    from oracle import ilu as oilu
    if case == "lap2d":
        A = wl.laplacian2d(30, wl.sigma20_2d(30))
        lab = opart.geometric_labels((30, 30), (2, 3))
    elif case == "lap3d":
        A = wl.laplacian3d(12, wl.sigma_for_negatives(wl.laplacian_eigs((12,) * 3), 8))
        lab = opart.geometric_labels((12,) * 3, (2, 2, 2))
    else:
        A = wl.convdiff3d(10, 10.0, 0.3)
        lab = opart.region_growing_labels(A.to_scipy(), 5, 4)
    blk = opslr.make_blocks(A.to_scipy(), lab)
    for drop in (1e-2, 1e-3):
        st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, int(lab.max()) + 1,
                               want_transpose=False, factor="ilut", drop_tol=drop)
        nB = sum(oilu.IlutSolver(blk.B[a:b, a:b], drop).nnz
                 for a, b in zip(blk.int_ptr[:-1], blk.int_ptr[1:]) if b > a)
        nC = sum(oilu.IlutSolver(blk.C0[a:b, a:b], drop).nnz
                 for a, b in zip(blk.if_ptr[:-1], blk.if_ptr[1:]) if b > a)
        print(case, drop, "library", st["nnz_LU_B"], st["nnz_LU_C0"], "oracle", nB, nC)
        assert (st["nnz_LU_B"], st["nnz_LU_C0"]) == (nB, nC)


def test_ilut_fill_matches_table1():
    """The paper's Table 1 (50^3 Laplacian, shift .05, drop 1e-2) prints fill(ILU)
    2.68, 2.45, 2.30, 2.23, 2.17, 2.11 for s = 5 .. 55 (METIS parts).  The library's
    ILUT with region-grown parts (nnz of L + U, L's unit diagonal counted as
    stored) is within 6% of each, and decreases with s as printed."""
    A = wl.laplacian3d(50, 0.05)
    fills = []
    for s, printed in ((5, 2.68), (15, 2.45), (25, 2.30), (35, 2.23), (45, 2.17), (55, 2.11)):
        lab, nl = P.pslr_partition_region_growing(A.rowptr, A.colind, s, 35)
        st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, nl, want_transpose=False,
                               factor="ilut", drop_tol=1e-2)
        fill = (st["nnz_LU_B"] + st["nnz_LU_C0"] + A.n) / A.nnz
        print("s", s, "fill(ILU) %.3f printed %.2f" % (fill, printed))
        assert abs(fill - printed) <= 0.06 * printed
        fills.append(fill)
    assert all(fills[i + 1] < fills[i] for i in range(len(fills) - 1))


@pytest.mark.parametrize("team", [2, 3, 4, 8])
def test_team_split_structure_and_host_solve(team):
    """The team split of every B_i: each position in one group, subtree groups
    reach only their own rows or the top group, and the groups applied in turn
    on the host equal the plain packed solve."""
    A = wl.laplacian3d(16, 0.1)
    lab = opart.geometric_labels((16,) * 3, (2, 2, 2))
    st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, 8, want_transpose=False, team=team)
    assert st["team"] == team and st["team_valid"] == 1 and st["levels_valid"] == 1
    assert st["team_residual"] < 1e-14
    A = wl.convdiff3d(12, 10.0, 0.2)
    lab, nl = P.pslr_partition_region_growing(A.rowptr, A.colind, 6, 4)
    st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, nl, want_transpose=False, team=team)
    assert st["team_valid"] == 1 and st["team_residual"] < 1e-14
    # parts without interior unknowns keep the team layout (empty groups)
    A2 = wl.laplacian2d(9, 0.1)
    lab2 = opart.geometric_labels((9, 9), (4, 4))
    st = P.pslr_host_stats(A2.rowptr, A2.colind, A2.vals, lab2, 16, want_transpose=False, team=team)
    assert st["team"] == team and st["team_valid"] == 1
    # blocks of very different sizes: each is cut into groups in proportion to
    # its share of the largest block (the smallest into one group and an
    # empty top group)
    A3 = wl.laplacian2d(40, 0.1)
    col = np.arange(A3.n) // 40
    lab3 = np.where(col < 30, 0, np.where(col < 36, 1, 2)).astype(np.int32)
    st = P.pslr_host_stats(A3.rowptr, A3.colind, A3.vals, lab3, 3, want_transpose=False, team=team)
    assert st["team"] == team and st["team_valid"] == 1 and st["team_residual"] < 1e-14
    p = [1200 - 40, 240 - 80, 160 - 40]  # interior rows: parts minus their lines next to a cut
    share = [max(1, min(32, int(np.floor(team * pi / max(p) + 0.5)))) for pi in p]
    assert st["team_groups_max_B"] == team and st["team_items_B"] == sum(share), (st, share)
    # blocks above 2048 rows get at least one group per 2048 rows, whatever `team`
    A4 = wl.laplacian2d(150, 0.05, Ny=150)
    lab4 = opart.geometric_labels((150, 150), (2, 1))
    st = P.pslr_host_stats(A4.rowptr, A4.colind, A4.vals, lab4, 2, want_transpose=False, team=team)
    pi = int(np.sum(lab4 == 0)) - 150
    assert st["team_valid"] == 1 and st["team_residual"] < 1e-12
    assert st["team_groups_max_B"] == max(team, -(-pi // 2048)) and st["team_items_B"] == 2 * st["team_groups_max_B"]
    # threshold ILU has no team split
    st = P.pslr_host_stats(A.rowptr, A.colind, A.vals, lab, nl, want_transpose=False, team=team,
                           factor="ilut")
    assert st["team"] == 0
