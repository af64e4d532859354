"""Batched handles (many uneven systems in one handle) and the global-memory
working-vector mode, on the GPU, through the C ABI.

* rank 0: every system's block of the batched apply equals the oracle's
  preconditioner of that system (FP64 bound as in test_gpu_parity);
* rank > 0: each system's Arnoldi basis and hence its apply equal those of a
  single-system handle built with the same start vector (to 1e-10: the
  partial sums of V^T y are chunked per system, so rounding differs);
* FGMRES runs one Krylov space per (system, right-hand side) and each reaches
  the tolerance with the iteration count of the single-system solve;
* global working vectors give the same apply as LDS ones.
"""
import numpy as np
import pytest

from paper_2002_00917_amd import workloads as wl
from paper_2002_00917_amd import pslr as P
from oracle import partition as opart
from oracle import pslr as opslr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64, device=_dev())


def _cols(t):
    return t.cpu().numpy().T.copy()


def small_systems():
    """Uneven 2D/3D systems, each with its own partition (labels local to the system)."""
    out = []
    A = wl.laplacian2d(23, 0.2, Ny=17)
    out.append((A, opart.region_growing_labels(A.to_scipy(), 5, 31)))
    A = wl.laplacian3d(7, 0.3)
    out.append((A, opart.geometric_labels((7, 7, 7), (2, 2, 1))))
    A = wl.laplacian2d(40, wl.sigma20_2d(40))
    out.append((A, opart.region_growing_labels(A.to_scipy(), 9, 32)))
    A = wl.convdiff3d(8, 10.0, 0.2)
    out.append((A, opart.region_growing_labels(A.to_scipy(), 4, 33)))
    A = wl.laplacian2d(12, 0.05)
    out.append((A, opart.geometric_labels((12, 12), (3, 2))))
    return out


def build_union(systems):
    class W:
        pass
    ws = []
    for A, _ in systems:
        w = W()
        w.A = A
        ws.append(w)
    U, sys_ptr = wl.union(ws)
    labels, off = [], 0
    for A, lab in systems:
        labels.append(lab + off)
        off += int(lab.max()) + 1
    return U, sys_ptr, np.concatenate(labels).astype(np.int32), off


def test_batched_rank0_matches_oracle_per_system():
    systems = small_systems()
    U, sys_ptr, lab, nparts = build_union(systems)
    h = P.pslr_setup_batched(U.rowptr, U.colind, U.vals, lab, nparts, sys_ptr, m=3, rank=0,
                             want_transpose=True)
    assert P.pslr_info(h)["nsys"] == len(systems)
    b = wl.normal_rhs(U.n, 3, 12)
    z = torch.zeros((3, U.n), dtype=torch.float64, device=_dev())
    zt = torch.zeros_like(z)
    P.pslr_apply(h, _t(b), z)
    P.pslr_apply_transpose(h, _t(b), zt)
    torch.cuda.synchronize()
    zc, ztc = _cols(z), _cols(zt)
    for s, (A, labs) in enumerate(systems):
        a0, a1 = sys_ptr[s], sys_ptr[s + 1]
        pre = opslr.PSLR(A.to_scipy(), labs, 3, 0)
        ref = pre.apply(b[a0:a1])
        reft = pre.apply_transpose(b[a0:a1])
        e = np.linalg.norm(zc[a0:a1] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        et = np.linalg.norm(ztc[a0:a1] - reft, axis=0) / np.linalg.norm(reft, axis=0)
        print("system", s, "n", a1 - a0, "apply", e, "transpose", et)
        assert np.all(e <= 1e-11) and np.all(et <= 1e-11)


def test_batched_matches_single_handles_and_fgmres():
    systems = small_systems()
    U, sys_ptr, lab, nparts = build_union(systems)
    v0s = []
    for s, (A, labs) in enumerate(systems):
        q = opslr.make_blocks(A.to_scipy(), labs).q
        v0s.append(wl.start_vector(q, 100 + s))
    hb = P.pslr_setup_batched(U.rowptr, U.colind, U.vals, lab, nparts, sys_ptr, m=2, rank=6,
                              v0=np.concatenate(v0s))
    b = wl.normal_rhs(U.n, 2, 13)
    z = torch.zeros((2, U.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(hb, _t(b), z)
    torch.cuda.synchronize()
    zc = _cols(z)
    x = torch.zeros((2, U.n), dtype=torch.float64, device=_dev())
    st, its, rel = P.fgmres_solve(hb, _t(b), x, restart=30, maxit=400, tol=1e-10)
    assert st == P.PSLR_OK and np.all(rel <= 1e-10)
    ns = len(systems)
    xs = _cols(x)
    Us = U.to_scipy()
    for s, (A, labs) in enumerate(systems):
        a0, a1 = sys_ptr[s], sys_ptr[s + 1]
        h1 = P.pslr_setup(A.rowptr, A.colind, A.vals, labs, int(labs.max()) + 1, m=2, rank=6, v0=v0s[s])
        z1 = torch.zeros((2, A.n), dtype=torch.float64, device=_dev())
        P.pslr_apply(h1, _t(b[a0:a1]), z1)
        x1 = torch.zeros_like(z1)
        st1, its1, rel1 = P.fgmres_solve(h1, _t(b[a0:a1]), x1, restart=30, maxit=400, tol=1e-10)
        torch.cuda.synchronize()
        ref = _cols(z1)
        e = np.linalg.norm(zc[a0:a1] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        bits = [int(its[r * ns + s]) for r in range(2)]
        print("system", s, "apply vs single handle", e, "its batched", bits, "single", list(its1))
        # same Arnoldi process; the V^T y partial sums are chunked per system in the
        # batched handle, and G amplifies that rounding difference
        assert np.all(e <= 1e-10)
        assert all(abs(bits[r] - int(its1[r])) <= 1 for r in range(2))
        for r in range(2):
            res = b[a0:a1, r] - A.to_scipy() @ xs[a0:a1, r]
            assert np.linalg.norm(res) <= 1.01e-10 * np.linalg.norm(b[a0:a1, r])
    assert np.linalg.norm(b - Us @ xs) <= 1.01e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("precision", [0, 1])
def test_global_working_vectors_match_lds(precision):
    A = wl.laplacian3d(12, 0.2)
    lab = opart.geometric_labels((12, 12, 12), (2, 2, 2))
    blk = opslr.make_blocks(A.to_scipy(), lab)
    v0 = wl.start_vector(blk.q, 5)
    hl = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 8, m=3, rank=8, v0=v0, precision=precision,
                      want_transpose=True)
    hg = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 8, m=3, rank=8, v0=v0, precision=precision,
                      want_transpose=True, working_vectors=1)
    assert P.pslr_info(hg)["global_vectors"] == 1 and P.pslr_info(hl)["global_vectors"] == 0
    b = wl.normal_rhs(A.n, 3, 14)
    out = []
    for h in (hl, hg):
        z = torch.zeros((3, A.n), dtype=torch.float64, device=_dev())
        zt = torch.zeros_like(z)
        P.pslr_apply(h, _t(b), z)
        P.pslr_apply_transpose(h, _t(b), zt)
        torch.cuda.synchronize()
        out.append((_cols(z), _cols(zt)))
    tol = 1e-13 if precision == 0 else 1e-6
    for a, c in zip(out[0], out[1]):
        assert np.all(np.linalg.norm(a - c, axis=0) / np.linalg.norm(a, axis=0) <= tol)
    V, H = P.pslr_get_lowrank(hg)
    pre = opslr.PSLR(A.to_scipy(), lab, 3, 0, V=V, H=H)
    ref = pre.apply(b)
    e = np.linalg.norm(out[1][0] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.all(e <= (1e-12 if precision == 0 else 1e-5))


def test_autotuned_tile_width_gives_the_same_apply():
    """The setup autotuner may narrow the right-hand-side tiles; the apply is unchanged."""
    systems = small_systems()
    U, sys_ptr, lab, nparts = build_union(systems)
    h8 = P.pslr_setup_batched(U.rowptr, U.colind, U.vals, lab, nparts, sys_ptr, m=3, rank=0)
    ht = P.pslr_setup_batched(U.rowptr, U.colind, U.vals, lab, nparts, sys_ptr, m=3, rank=0,
                              autotune=True)
    assert P.pslr_info(h8)["max_tile"] == 8
    assert P.pslr_info(ht)["max_tile"] in (1, 2, 4, 8)
    print("autotuned tile width", P.pslr_info(ht)["max_tile"])
    for nr in (8, 3):
        b = wl.normal_rhs(U.n, nr, 40 + nr)
        out = []
        for h in (h8, ht):
            z = torch.zeros((nr, U.n), dtype=torch.float64, device=_dev())
            P.pslr_apply(h, _t(b), z)
            torch.cuda.synchronize()
            out.append(_cols(z))
        e = np.linalg.norm(out[0] - out[1], axis=0) / np.linalg.norm(out[0], axis=0)
        assert np.all(e <= 1e-12), e
