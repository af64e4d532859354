"""Parity of the HIP library (through the C ABI) with the CPU oracle, on the GPU.

Every comparison imports the oracle's V and H into the library (never the
other way), so both sides apply the same operator of Algorithm 3.

Bounds, checked per right-hand side both normwise (||z - z_o|| / ||z_o||) and
elementwise (max_i |z_i - z_o,i| / max_i |z_o,i|):
  FP64 apply and transposed apply   1e-12
  FP32 apply (FP32 V)               1e-5
  FP32 apply with BF16 V            1e-5 against the oracle run with the same
                                    BF16-rounded V; against the exact-V oracle
                                    a per-case bound (BF16_VS_EXACT)
  FGMRES                            true relative residual <= tol
except the cases in TOL64 / TOL32, whose diagonal blocks are ill conditioned:
there both sides are backward stable and may differ by the forward-error
bound kappa * eps (kappa = largest 2-norm condition number of the B_i, C_i),
and the bound is at most three times the error measured on the MI355X:
  2D 64^2, sigma 4.7e-5 from an eigenvalue of the 31 x 31 subdomain operator,
    kappa(B_i) = 1.7e5: kappa * eps64 = 3.7e-11 (measured up to 4.9e-11),
    kappa * eps32 = 1.0e-2 (measured up to 1.1e-2);
  3D 9^3, kappa = 1.6e2: kappa * eps32 = 9.2e-6 (measured up to 4.4e-5; the
    FP32 solves also round the factors, so a few times kappa * eps32);
  the 24^3 upwind case (C4-shaped), kappa = 2.6e3: kappa * eps32 = 1.5e-4
    (measured up to 1.6e-4 over runs: the atomic adds change the summation
    order from run to run, and the FP32 solves also round the factors).
"""
import numpy as np
import pytest

from paper_2002_00917_amd import workloads as wl
from paper_2002_00917_amd import pslr as P
from oracle import partition as opart
from oracle import pslr as opslr
from oracle import krylov as okry
from oracle import adjoint as oadj

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# per-case bounds where kappa * eps exceeds the stated 1e-12 (FP64) / 1e-5 (FP32)
TOL64 = {"c1": 1.5e-10}
TOL32 = {"c1": 3.3e-2, "lap3d_9_2x2x2": 8.4e-5, "c4_shaped": 4.5e-4}
# BF16 storage of V (8 significant bits) against the exact-V preconditioner,
# where the library keeps it (pslr_info.v_bf16): the rounding breaks V's
# orthonormality, and the change of the low-rank term is amplified by the
# conditioning of the rest of the preconditioner.  Three times the measured
# difference.  On the 2D 64^2 workload (kappa(B_i) = 1.7e5) the difference is
# O(10): the setup probe withdraws BF16 there and V stays in FP32.
BF16_VS_EXACT = {"lap2d_10_2x2": 2.1e-2, "lap2d_37x23_3x5": 2.4e-3, "lap3d_9_2x2x2": 2.7e-2,
                 "convdiff_11_rg7": 7.5e-4}
BF16_WITHDRAWN = {"c1"}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _cols(t):
    """(nrhs, n) device tensor -> n x nrhs numpy."""
    return t.detach().cpu().numpy().T.copy()


def _tens(x):
    return torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64, device=_dev())


def relerr(a, b):
    """Normwise relative error per column."""
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def maxerr(a, b):
    """Elementwise error per column: max |a - b| over max |b|."""
    return np.abs(a - b).max(axis=0) / np.abs(b).max(axis=0)


def _fmt(a):
    return "[" + " ".join("%.2e" % v for v in np.ravel(a)) + "]"


def check(name, what, z, ref, tol):
    e2, ei = relerr(z, ref), maxerr(z, ref)
    print("%s %s: normwise %s elementwise %s (max %.2e / %.2e) bound %.1e"
          % (name, what, _fmt(e2), _fmt(ei), e2.max(), ei.max(), tol), flush=True)
    assert np.all(e2 <= tol), (what, e2, tol)
    assert np.all(ei <= tol), (what, ei, tol)


def tiny_cases():
    out = []
    A = wl.laplacian2d(10, wl.sigma_for_negatives(wl.laplacian_eigs((10, 10)), 6))
    out.append(("lap2d_10_2x2", A, opart.geometric_labels((10, 10), (2, 2)), 3, 6))
    A = wl.laplacian2d(37, 0.05, Ny=23)
    out.append(("lap2d_37x23_3x5", A, opart.geometric_labels((37, 23), (3, 5)), 2, 8))
    A = wl.laplacian3d(9, wl.sigma_for_negatives(wl.laplacian_eigs((9, 9, 9)), 10))
    out.append(("lap3d_9_2x2x2", A, opart.geometric_labels((9, 9, 9), (2, 2, 2)), 4, 10))
    A = wl.convdiff3d(11, 10.0, 0.25)
    out.append(("convdiff_11_rg7", A, opart.region_growing_labels(A.to_scipy(), 7, 4), 3, 12))
    A = wl.laplacian2d(64, wl.SIGMA_C1)
    out.append(("c1", A, opart.geometric_labels((64, 64), (2, 2)), 3, 16))
    return out


CASES = tiny_cases()
IDS = [c[0] for c in CASES]


def _pair(A, lab, m, rank, precision=0, want_T=True, **kw):
    """Library handle with the oracle's Arnoldi V, H imported, and the oracle preconditioner."""
    nparts = int(lab.max()) + 1
    blk = opslr.make_blocks(A.to_scipy(), lab)
    v0 = wl.start_vector(blk.q, 17)
    pre = opslr.PSLR(A.to_scipy(), lab, m, rank, v0=v0)
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, nparts, m=m, rank=0, precision=precision,
                     want_transpose=want_T, **kw)
    P.pslr_set_lowrank(h, pre.V, pre.H)
    return h, pre


@pytest.mark.parametrize("name,A,lab,m,rank", CASES, ids=IDS)
def test_apply_fp64_matches_oracle(name, A, lab, m, rank):
    print("case", name, flush=True)
    h, pre = _pair(A, lab, m, rank)
    b = wl.normal_rhs(A.n, 3, 5)
    z = torch.zeros((3, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    zt = torch.zeros_like(z)
    P.pslr_apply_transpose(h, _tens(b), zt)
    torch.cuda.synchronize()
    tol = TOL64.get(name, 1e-12)
    check(name, "fp64 apply", _cols(z), pre.apply(b), tol)
    check(name, "fp64 apply_transpose", _cols(zt), pre.apply_transpose(b), tol)


@pytest.mark.parametrize("name,A,lab,m,rank", CASES, ids=IDS)
def test_apply_fp32_matches_oracle(name, A, lab, m, rank):
    print("case", name, flush=True)
    h, pre = _pair(A, lab, m, rank, precision=1)
    b = wl.normal_rhs(A.n, 2, 6)
    z = torch.zeros((2, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    zt = torch.zeros_like(z)
    P.pslr_apply_transpose(h, _tens(b), zt)
    torch.cuda.synchronize()
    tol = TOL32.get(name, 1e-5)
    check(name, "fp32 apply", _cols(z), pre.apply(b), tol)
    check(name, "fp32 apply_transpose", _cols(zt), pre.apply_transpose(b), tol)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even) via float32, as the library stores V."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


@pytest.mark.parametrize("name,A,lab,m,rank", CASES, ids=IDS)
def test_apply_bf16_lowrank_matches_oracle(name, A, lab, m, rank):
    print("case", name, flush=True)
    h, pre = _pair(A, lab, m, rank, precision=2)
    info = P.pslr_info(h)
    print(name, "v_bf16", info["v_bf16"], "bf16_probe %.2e" % info["bf16_probe"], flush=True)
    b = wl.normal_rhs(A.n, 2, 7)
    z = torch.zeros((2, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    torch.cuda.synchronize()
    exact = pre.apply(b)
    if name in BF16_WITHDRAWN:
        assert info["v_bf16"] == 0 and info["bf16_probe"] > 2.5e-2
        check(name, "precision-2 apply (V kept in FP32) vs exact-V oracle", _cols(z), exact,
              TOL32.get(name, 1e-5))
        return
    assert info["v_bf16"] == 1 and info["bf16_probe"] <= 2.5e-2
    pre.set_lowrank(bf16_round(pre.V), pre.H)
    check(name, "bf16-V apply vs rounded-V oracle", _cols(z), pre.apply(b), TOL32.get(name, 1e-5))
    check(name, "bf16-V apply vs exact-V oracle", _cols(z), exact, BF16_VS_EXACT[name])


@pytest.mark.parametrize("name,A,lab,m,rank", CASES, ids=IDS)
def test_library_arnoldi_invariants(name, A, lab, m, rank):
    """The library's own FP64 Arnoldi basis satisfies the Arnoldi invariants of eq. schur."""
    nparts = int(lab.max()) + 1
    blk = opslr.make_blocks(A.to_scipy(), lab)
    v0 = wl.start_vector(blk.q, 17)
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, nparts, m=m, rank=rank, v0=v0)
    V, H = P.pslr_get_lowrank(h)
    k = V.shape[1]
    assert k == min(rank, blk.q) or h.status == P.PSLR_EBREAKDOWN
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-12
    pre = opslr.PSLR(A.to_scipy(), lab, m, 0)
    EV = np.column_stack([pre.err_op(V[:, j]) for j in range(k)])
    scale = max(1.0, np.abs(EV).max())
    assert np.abs(H - V.T @ EV).max() < 1e-10 * scale
    assert np.allclose(np.tril(H, -2), 0.0)
    # the library's V spans the oracle's Krylov space: projector agreement
    Vo, Ho, _, _ = opslr.arnoldi(pre.err_op, v0, k)
    Pl, Po = V @ V.T, Vo @ Vo.T
    print(name, "projector difference", np.abs(Pl - Po).max())
    assert np.abs(Pl - Po).max() < 1e-6


def test_fgmres_c1_converges_like_oracle():
    name, A, lab, m, rank = CASES[-1]
    h, pre = _pair(A, lab, m, rank)
    b = wl.c1().b
    x = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
    st, its, rel = P.fgmres_solve(h, _tens(b), x, restart=40, maxit=500, tol=1e-8)
    xo, ito, relo, oko = okry.fgmres(A.to_scipy(), b[:, 0], pre.apply, restart=40, tol=1e-8)
    print("c1 fgmres its lib", its, "oracle", ito, "relres", rel, relo)
    assert st == P.PSLR_OK and rel[0] <= 1e-8
    # the two preconditioners agree to kappa(B_i) * eps ~ 5e-11 here (kappa = 1.7e5),
    # which moves the iteration where the residual estimate crosses 1e-8 by up to two
    assert abs(int(its[0]) - ito) <= 2
    xs = _cols(x)[:, 0]
    assert np.abs(xs - 1.0).max() < 1e-5          # b = A * ones
    # FP32 apply inside FP64 FGMRES still reaches the FP64 tolerance
    h32, _ = _pair(A, lab, m, rank, precision=1)
    x32 = torch.zeros_like(x)
    st32, its32, rel32 = P.fgmres_solve(h32, _tens(b), x32, restart=40, maxit=500, tol=1e-8)
    print("c1 mixed fgmres its", its32, "relres", rel32)
    assert st32 == P.PSLR_OK and rel32[0] <= 1e-8


def test_fgmres_multi_rhs_and_transpose():
    name, A, lab, m, rank = CASES[2]
    h, pre = _pair(A, lab, m, rank)
    b = wl.normal_rhs(A.n, 4, 8)
    x = torch.zeros((4, A.n), dtype=torch.float64, device=_dev())
    st, its, rel = P.fgmres_solve(h, _tens(b), x, restart=20, maxit=500, tol=1e-10)
    assert st == P.PSLR_OK and np.all(rel <= 1e-10)
    As = A.to_scipy()
    xr = _cols(x)
    for j in range(4):
        assert np.linalg.norm(b[:, j] - As @ xr[:, j]) <= 1.01e-10 * np.linalg.norm(b[:, j])
        _, ito, _, _ = okry.fgmres(As, b[:, j], pre.apply, restart=20, tol=1e-10)
        print("multi-rhs column", j, "its lib", its[j], "oracle", ito)
        assert abs(int(its[j]) - ito) <= 1
    xt = torch.zeros_like(x)
    st, its, rel = P.fgmres_solve(h, _tens(b), xt, restart=20, maxit=500, tol=1e-10, transpose=True)
    assert st == P.PSLR_OK and np.all(rel <= 1e-10)
    xtr = _cols(xt)
    for j in range(4):
        assert np.linalg.norm(b[:, j] - As.T @ xtr[:, j]) <= 1.01e-10 * np.linalg.norm(b[:, j])


def test_fgmres_reports_no_convergence():
    name, A, lab, m, rank = CASES[-1]
    h, pre = _pair(A, lab, m, rank)
    b = wl.c1().b
    x = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
    st, its, rel = P.fgmres_solve(h, _tens(b), x, restart=40, maxit=3, tol=1e-8)
    assert st == P.PSLR_ENOCONV and its[0] == 3 and rel[0] > 1e-8


def test_sddmm_gradient_matches_oracle():
    w, kappa, kref, sigma = wl.c5(32)
    A = w.A
    lab = opart.geometric_labels((32, 32), (4, 4))
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 16, m=3, rank=8)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal((A.n, 2))
    zz = rng.standard_normal((A.n, 2))
    g = torch.zeros(A.nnz, dtype=torch.float64, device=_dev())
    P.pslr_sddmm_grad(h, _tens(lam), _tens(zz), g)
    torch.cuda.synchronize()
    go = oadj.pattern_grad(A.to_scipy(), lam, zz)
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-14 * np.abs(go).max()
    # a gradient buffer of the wrong length or type is rejected before any launch
    with pytest.raises(ValueError):
        P.pslr_sddmm_grad(h, _tens(lam), _tens(zz), torch.zeros(A.nnz - 1, dtype=torch.float64, device=_dev()))
    with pytest.raises(ValueError):
        P.pslr_sddmm_grad(h, _tens(lam), _tens(zz), torch.zeros(A.nnz, dtype=torch.float32, device=_dev()))


def test_edge_cases():
    # one part: no interface, the preconditioner is B^{-1} = A^{-1}
    A = wl.laplacian2d(12, 0.3)
    lab = np.zeros(A.n, dtype=np.int32)
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 1, m=2, rank=4)
    b = wl.normal_rhs(A.n, 1, 1)
    z = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    torch.cuda.synchronize()
    import scipy.sparse.linalg as spla
    xs = spla.spsolve(A.to_scipy().tocsc(), b[:, 0])
    assert relerr(_cols(z), xs[:, None])[0] < 1e-12
    # zero right-hand side gives zero
    z0 = torch.ones((2, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, torch.zeros((2, A.n), dtype=torch.float64, device=_dev()), z0)
    torch.cuda.synchronize()
    assert float(z0.abs().max()) == 0.0
    # many small parts, some without interior unknowns; a rank above q is capped
    A = wl.laplacian2d(9, 0.1)
    lab = opart.geometric_labels((9, 9), (4, 4))
    nparts = 16
    blk = opslr.make_blocks(A.to_scipy(), lab)
    v0 = wl.start_vector(blk.q, 3)
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, nparts, m=2, rank=500, v0=v0)
    assert P.pslr_info(h)["rank"] <= min(blk.q, 256)
    # parity there with the oracle's own Arnoldi basis imported
    pre = opslr.PSLR(A.to_scipy(), lab, 2, 500, v0=v0)
    P.pslr_set_lowrank(h, pre.V, pre.H)
    b = wl.normal_rhs(A.n, 2, 9)
    z = torch.zeros((2, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    torch.cuda.synchronize()
    check("lap2d_9_4x4", "fp64 apply, full rank", _cols(z), pre.apply(b), 1e-12)
    # invalid arguments are rejected
    with pytest.raises(P.PslrError) as ei:
        P.pslr_setup(A.rowptr, A.colind, A.vals, lab, nparts, m=-1, rank=2)
    assert ei.value.status == P.PSLR_EINVAL
    with pytest.raises(P.PslrError) as ei:
        P.pslr_setup(A.rowptr, A.colind, A.vals, lab, nparts, m=2, rank=2, threads=256)
    assert ei.value.status == P.PSLR_EINVAL


def test_lr_expand_slices_512_threads_rank96_8rhs():
    """Regression: with 512-thread workgroups and k x R between 513 and 1024
    (rank 96, tiles of 8 right-hand sides) the low-rank expansion once had
    zero slices; it must match the oracle like any other launch shape."""
    A = wl.laplacian3d(9, wl.sigma_for_negatives(wl.laplacian_eigs((9, 9, 9)), 10))
    lab = opart.geometric_labels((9, 9, 9), (2, 2, 2))
    blk = opslr.make_blocks(A.to_scipy(), lab)
    assert blk.q >= 96
    pre = opslr.PSLR(A.to_scipy(), lab, 2, 96, v0=wl.start_vector(blk.q, 5))
    assert pre.V.shape[1] == 96
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 8, m=2, rank=0, threads=512)
    P.pslr_set_lowrank(h, pre.V, pre.H)
    assert P.pslr_info(h)["threads"] == 512
    b = wl.normal_rhs(A.n, 8, 31)
    z = torch.zeros((8, A.n), dtype=torch.float64, device=_dev())
    P.pslr_apply(h, _tens(b), z)
    torch.cuda.synchronize()
    check("lap3d_9 rank 96, 512 threads", "fp64 apply, 8 rhs", _cols(z), pre.apply(b), 1e-12)


def c4_shaped():
    """A small instance of the 3D upwind workload: region-grown uneven parts."""
    N = 24
    sigma = wl.sigma_for_negatives(wl.convdiff_eigs(N, 10.0), 20)
    A = wl.convdiff3d(N, 10.0, sigma)
    lab = opart.region_growing_labels(A.to_scipy(), 16, 4)
    return A, lab


@pytest.mark.parametrize("working_vectors", [0, 1], ids=["lds", "global"])
def test_c4_shaped_32rhs_parity(working_vectors):
    """Upwind convection-diffusion on 24^3 (20 negative eigenvalues), 16
    region-grown uneven parts, m = 4, r_k = 16, 32 right-hand sides: FP64,
    FP32 and BF16-V applies in tiles of 8 right-hand sides, with working
    vectors in LDS and in the global workspace."""
    A, lab = c4_shaped()
    sizes = np.bincount(lab)
    print("c4-shaped part sizes", sizes.min(), "..", sizes.max(), flush=True)
    b = wl.normal_rhs(A.n, 32, 40)
    pre = None
    for prec, tol in ((0, 1e-12), (1, TOL32["c4_shaped"]), (2, TOL32["c4_shaped"])):
        h, pre = _pair(A, lab, 4, 16, precision=prec, want_T=True, working_vectors=working_vectors)
        info = P.pslr_info(h)
        if prec == 2:
            print("c4-shaped v_bf16", info["v_bf16"], "bf16_probe %.2e" % info["bf16_probe"])
            if info["v_bf16"]:
                pre.set_lowrank(bf16_round(pre.V), pre.H)
        z = torch.zeros((32, A.n), dtype=torch.float64, device=_dev())
        P.pslr_apply(h, _tens(b), z)
        zt = torch.zeros_like(z)
        P.pslr_apply_transpose(h, _tens(b), zt)
        torch.cuda.synchronize()
        name = "c4-shaped %s precision %d (max tile %d, global vectors %d)" % (
            ["lds", "global"][working_vectors], prec, info["max_tile"], info["global_vectors"])
        check(name, "apply 32 rhs", _cols(z), pre.apply(b), tol)
        check(name, "apply_transpose 32 rhs", _cols(zt), pre.apply_transpose(b), tol)
        if prec == 2 and info["v_bf16"]:
            # 32 right-hand sides take the matrix-core low-rank products; tiles
            # of 8 the vector ones: the same operator up to FP32 summation
            # order, amplified like any FP32 difference by kappa = 2.6e3 (the
            # case's FP32 bound)
            z8 = torch.zeros_like(z)
            zt8 = torch.zeros_like(z)
            for c in range(0, 32, 8):
                P.pslr_apply(h, _tens(b[:, c:c + 8]), z8[c:c + 8])
                P.pslr_apply_transpose(h, _tens(b[:, c:c + 8]), zt8[c:c + 8])
            torch.cuda.synchronize()
            assert info["mfma_min_rhs"] == 16
            check(name, "matrix-core vs vector low-rank products", _cols(z), _cols(z8), tol)
            check(name, "matrix-core vs vector low-rank products (transposed)", _cols(zt),
                  _cols(zt8), tol)


def test_c2_full_size_apply_parity():
    """64^3 shifted Laplacian, 4x4x4 split, m=4, k=64: the bench configuration."""
    w = wl.c2()
    A = w.A
    lab = opart.geometric_labels((64, 64, 64), (4, 4, 4))
    blk = opslr.make_blocks(A.to_scipy(), lab)
    # an orthonormal V and a small H stand in for the Arnoldi output (the apply
    # does not depend on where they come from)
    rng = np.random.default_rng(11)
    V, _ = np.linalg.qr(rng.standard_normal((blk.q, 64)))
    H = 0.3 * np.triu(rng.standard_normal((64, 64)), -1) / 8.0
    pre = opslr.PSLR(A.to_scipy(), lab, 4, 0, V=V, H=H)
    b = w.b
    ref = pre.apply(b)
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 64, m=4, rank=0, precision=prec)
        P.pslr_set_lowrank(h, V, H)
        z = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
        P.pslr_apply(h, _tens(b), z)
        torch.cuda.synchronize()
        check("c2", "precision %d apply" % prec, _cols(z), ref, tol)


@pytest.mark.timeout(900)
def test_c2_fgmres_iterations_match_oracle():
    """64^3 workload: FGMRES(200) to 1e-8 with the oracle's own 64-step
    Arnoldi basis imported into the library; the oracle's FGMRES with its
    own preconditioner needs the same number of iterations (within one)."""
    w = wl.c2()
    A = w.A
    lab = opart.geometric_labels((64, 64, 64), (4, 4, 4))
    blk = opslr.make_blocks(A.to_scipy(), lab)
    pre = opslr.PSLR(A.to_scipy(), lab, 4, 64, v0=wl.start_vector(blk.q, 2))
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 64, m=4, rank=0)
    P.pslr_set_lowrank(h, pre.V, pre.H)
    x = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
    st, its, rel = P.fgmres_solve(h, _tens(w.b), x, restart=200, maxit=500, tol=1e-8)
    print("c2 library FGMRES(200): its", its, "relres", rel, flush=True)
    xo, ito, relo, oko = okry.fgmres(A.to_scipy(), w.b[:, 0], pre.apply, restart=200, tol=1e-8)
    print("c2 oracle FGMRES(200): its", ito, "relres", relo, flush=True)
    assert st == P.PSLR_OK and rel[0] <= 1e-8 and oko
    assert abs(int(its[0]) - ito) <= 1


@pytest.mark.parametrize("precision", [0, 1])
def test_tile_paths_agree(precision):
    """Right-hand sides applied one at a time (single-rhs path: entry form on
    narrow levels in FP64, chunked products) and together in tiles of 2, 4 and
    8, including ragged counts that leave a tile partly empty (3, 5, 11), give
    the same preconditioned vectors."""
    A = wl.laplacian3d(14, 0.3)
    lab = opart.geometric_labels((14, 14, 14), (2, 2, 2))
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 8, m=3, rank=8, precision=precision,
                     want_transpose=True, seed=11)
    b = wl.normal_rhs(A.n, 11, 21)
    tol = 1e-13 if precision == 0 else 1e-5
    for apply in (P.pslr_apply, P.pslr_apply_transpose):
        single = np.empty_like(b)
        for j in range(b.shape[1]):
            z1 = torch.zeros((1, A.n), dtype=torch.float64, device=_dev())
            apply(h, _tens(b[:, j:j + 1]), z1)
            torch.cuda.synchronize()
            single[:, j] = _cols(z1)[:, 0]
        for nr in (2, 3, 4, 5, 8, 11):
            z = torch.zeros((nr, A.n), dtype=torch.float64, device=_dev())
            apply(h, _tens(b[:, :nr]), z)
            torch.cuda.synchronize()
            zc = _cols(z)
            err = np.linalg.norm(zc - single[:, :nr], axis=0) / np.linalg.norm(single[:, :nr], axis=0)
            print(apply.__name__, "precision", precision, "tile", nr, "max rel diff", err.max())
            assert np.all(err <= tol)


def test_matrix_core_lowrank_well_conditioned():
    """The matrix-core low-rank products on a well-conditioned case (2D 37 x 23,
    15 parts, kappa(B_i, C_i) = 19), rank 40 (two 32-column blocks, the second
    ragged) and 40 right-hand sides (two tiles of 32, the second ragged):
    against the oracle with the same BF16-rounded V at the plain FP32 bound."""
    A = wl.laplacian2d(37, 0.05, Ny=23)
    lab = opart.geometric_labels((37, 23), (3, 5))
    h, pre = _pair(A, lab, 2, 40, precision=2, want_T=True)
    info = P.pslr_info(h)
    print("well-conditioned: rank", info["rank"], "v_bf16", info["v_bf16"], "bf16_probe %.2e"
          % info["bf16_probe"], "mfma_min_rhs", info["mfma_min_rhs"], flush=True)
    assert info["rank"] == 40 and info["v_bf16"] == 1 and info["mfma_min_rhs"] == 16
    pre.set_lowrank(bf16_round(pre.V), pre.H)
    b = wl.normal_rhs(A.n, 40, 41)
    z = torch.zeros((40, A.n), dtype=torch.float64, device=_dev())
    zt = torch.zeros_like(z)
    P.pslr_apply(h, _tens(b), z)
    P.pslr_apply_transpose(h, _tens(b), zt)
    torch.cuda.synchronize()
    check("lap2d_37x23 rank 40, 40 rhs", "matrix-core low-rank apply", _cols(z), pre.apply(b), 1e-5)
    check("lap2d_37x23 rank 40, 40 rhs", "matrix-core low-rank apply_transpose", _cols(zt),
          pre.apply_transpose(b), 1e-5)
