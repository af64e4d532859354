"""Differentiation through PSLR-FGMRES (transposed apply + SDDMM), on the GPU.

Workload: -div(kappa grad u) - sigma u on a 256 x 256 grid, log kappa a unit
Gaussian random field (correlation length 0.1, seed 5), 4 x 4 subdomains,
m = 3, r_k = 16; loss L = ||z - z*||^2 with z* the exact solution for a
reference kappa (seed 6).  The gradient with respect to A's nonzeros is checked
against the oracle's exact-solve adjoint gradient and against central finite
differences (step 1e-6, exact sparse solves) on 20 seeded nonzeros.
"""
import numpy as np
import pytest

from paper_2002_00917_amd import workloads as wl
from paper_2002_00917_amd import pslr as P
from oracle import adjoint as oadj
from oracle import partition as opart

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_gradcheck_tiny():
    from paper_2002_00917_amd.autograd import pslr_solve
    dev = _dev()
    kappa = np.exp(wl.gaussian_random_field(10, 0.3, 5))
    A = wl.variable_coeff2d(kappa, 0.5)
    lab = opart.geometric_labels((10, 10), (2, 2))
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 4, m=2, rank=4, want_transpose=True)
    vals = torch.tensor(A.vals, dtype=torch.float64, device=dev, requires_grad=True)
    b = torch.tensor(np.linspace(0.5, 1.5, A.n), dtype=torch.float64, device=dev, requires_grad=True)
    zstar = torch.tensor(np.cos(np.arange(A.n)), dtype=torch.float64, device=dev)
    z = pslr_solve(vals, b, h, 1e-13, 40, 500)
    loss = ((z - zstar) ** 2).sum()
    loss.backward()
    L, zo, lam, go = oadj.loss_and_grad(A.to_scipy(), np.linspace(0.5, 1.5, A.n), np.cos(np.arange(A.n)))
    gv = vals.grad.cpu().numpy()
    assert np.linalg.norm(gv - go) <= 1e-9 * np.linalg.norm(go)
    assert np.linalg.norm(b.grad.cpu().numpy() - lam) <= 1e-9 * np.linalg.norm(lam)
    assert abs(float(loss) - L) <= 1e-10 * abs(L)


def test_c5_gradient_vs_oracle_and_finite_differences():
    from paper_2002_00917_amd.autograd import pslr_solve
    dev = _dev()
    w, kappa, kref, sigma = wl.c5(256)
    A = w.A
    Aref = wl.variable_coeff2d(kref, sigma)
    b = w.b[:, 0]
    zstar = oadj.solve(Aref.to_scipy(), b)
    lab = opart.geometric_labels((256, 256), (4, 4))
    h = P.pslr_setup(A.rowptr, A.colind, A.vals, lab, 16, m=3, rank=16, want_transpose=True)
    vals = torch.tensor(A.vals, dtype=torch.float64, device=dev, requires_grad=True)
    bt = torch.tensor(b, dtype=torch.float64, device=dev)
    zs = torch.tensor(zstar, dtype=torch.float64, device=dev)
    # FP64 residual floors of this system: ~1.7e-12 for the forward solve
    # (eps |A| |z| / |b| with b = h^2 * 1) and ~2e-11 for the adjoint one
    z = pslr_solve(vals, bt, h, 1e-11, 200, 3000, 1e-10)
    loss = ((z - zs) ** 2).sum()
    loss.backward()
    g = vals.grad.cpu().numpy()
    As = A.to_scipy()
    L, zo, lam, go = oadj.loss_and_grad(As, b, zstar)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print("c5 gradient: loss %.6e (oracle %.6e), normwise rel. error vs exact adjoint %.3e"
          % (float(loss), L, rel))
    assert rel <= 1e-6
    rng = np.random.default_rng(7)
    ks = rng.choice(A.nnz, size=20, replace=False)
    fd = np.empty(20)
    d = 1e-6
    for t, k in enumerate(ks):
        Ap = As.copy(); Ap.data[k] += d
        Am = As.copy(); Am.data[k] -= d
        fd[t] = (oadj.loss_and_grad(Ap, b, zstar)[0] - oadj.loss_and_grad(Am, b, zstar)[0]) / (2 * d)
    err = np.linalg.norm(g[ks] - fd) / np.linalg.norm(fd)
    print("c5 gradient vs central differences on 20 nonzeros: normwise rel. error %.3e" % err)
    assert err <= 1e-5
