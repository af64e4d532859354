"""Seeded synthetic inputs for PSLR solves.

This module only *generates inputs*: sparse matrices from finite-difference
stencils, shifts chosen from closed-form spectra, right-hand sides and start
vectors.  It holds none of the preconditioner's arithmetic, so both the HIP
library path and the CPU oracle may use it.

Matrix conventions (paper, Sec. 4.1 Test 1): the stencils are *unscaled*
(diagonal 4 in 2D, 6 in 3D, off-diagonals -1) and the shift is subtracted
from the unscaled operator, which is the paper's "shift the discretized
Laplacian by h^2 beta".  Grid index v = ix + Nx*(iy + Ny*iz) (x fastest),
Dirichlet boundaries (neighbours outside the grid are dropped).

Every generator returns CSR arrays (rowptr int64, colind int32, vals float64)
with sorted column indices and no duplicates.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# CSR container
# --------------------------------------------------------------------------


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64[n+1]
    colind: np.ndarray  # int32[nnz]
    vals: np.ndarray    # float64[nnz]
    grid: tuple = ()    # grid dimensions (x fastest) when the matrix is a stencil

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(a, grid=()) -> "CSR":
        a = sp.csr_matrix(a)
        a.sum_duplicates()
        a.sort_indices()
        return CSR(a.shape[0], a.indptr.astype(np.int64), a.indices.astype(np.int32),
                   a.data.astype(np.float64), tuple(grid))


def _stencil(dims, diag, lower, upper):
    """Constant-coefficient nearest-neighbour stencil on a box grid.

    diag: scalar diagonal; lower[d] / upper[d]: coefficient of the neighbour
    at v - e_d / v + e_d.
    """
    dims = tuple(int(x) for x in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for N in dims:
        coords.append(rem % N)
        rem //= N
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, float(diag))]
    stride = 1
    for d, N in enumerate(dims):
        c = coords[d]
        m = c > 0
        rows.append(idx[m]); cols.append(idx[m] - stride); vals.append(np.full(m.sum(), float(lower[d])))
        m = c < N - 1
        rows.append(idx[m]); cols.append(idx[m] + stride); vals.append(np.full(m.sum(), float(upper[d])))
        stride *= N
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return CSR.from_scipy(a.tocsr(), grid=dims)


def laplacian2d(N: int, sigma: float = 0.0, Ny: int | None = None) -> CSR:
    """5-point -Laplacian (unscaled) minus sigma*I on an N x Ny grid."""
    Ny = N if Ny is None else Ny
    return _stencil((N, Ny), 4.0 - sigma, (-1.0, -1.0), (-1.0, -1.0))


def laplacian3d(N: int, sigma: float = 0.0) -> CSR:
    """7-point -Laplacian (unscaled) minus sigma*I on an N^3 grid."""
    return _stencil((N, N, N), 6.0 - sigma, (-1.0,) * 3, (-1.0,) * 3)


def convdiff3d(N: int, beta: float, sigma: float) -> CSR:
    """First-order upwind -Lap u + beta*(1,1,1).grad u - sigma*u on N^3, scaled by h^2.

    h = 1/(N+1); backward differences for the convection term give diagonal
    6 + 3*beta*h - sigma, -(1+beta*h) at v - e_d and -1 at v + e_d.
    """
    bh = beta / (N + 1)
    return _stencil((N, N, N), 6.0 + 3.0 * bh - sigma, (-(1.0 + bh),) * 3, (-1.0,) * 3)


def convdiff3d_central(N: int, gamma: float, shift: float) -> CSR:
    """The paper's Test 2 operator: -Lap u - gamma (1,1,1).grad u - shift*u on N^3
    by the standard 7-point stencil (central differences), scaled by h^2,
    h = 1/(N+1): diagonal 6 - shift, -1 - gamma*h/2 at v + e_d and
    -1 + gamma*h/2 at v - e_d."""
    gh = 0.5 * gamma / (N + 1)
    return _stencil((N, N, N), 6.0 - shift, (-1.0 + gh,) * 3, (-1.0 - gh,) * 3)


def variable_coeff2d(kappa: np.ndarray, sigma: float) -> CSR:
    """-div(kappa grad u) - sigma*u on an N x N grid (cell-centred kappa, unscaled).

    Face coefficient kappa_f = (kappa_v + kappa_w)/2 between grid neighbours,
    A[v,w] = -kappa_f and A[v,v] = sum of the four face coefficients - sigma;
    a Dirichlet boundary face takes kappa_f = kappa_v.
    """
    N = kappa.shape[0]
    assert kappa.shape == (N, N)
    k = kappa.T.reshape(-1)  # v = ix + N*iy, kappa indexed [ix, iy]
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    ix = idx % N
    iy = idx // N
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for d, (c, stride) in enumerate(((ix, 1), (iy, N))):
        for sgn in (-1, 1):
            inside = (c > 0) if sgn < 0 else (c < N - 1)
            w = idx + sgn * stride
            kf = np.where(inside, 0.5 * (k + k[np.where(inside, w, idx)]), k)
            diag += kf
            rows.append(idx[inside]); cols.append(w[inside]); vals.append(-kf[inside])
    rows.append(idx); cols.append(idx); vals.append(diag - sigma)
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return CSR.from_scipy(a.tocsr(), grid=(N, N))


# --------------------------------------------------------------------------
# Closed-form spectra used to place the shift
# --------------------------------------------------------------------------


def _lap1d_eigs(N):
    k = np.arange(1, N + 1)
    return 4.0 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2


def laplacian_eigs(dims) -> np.ndarray:
    """Sorted eigenvalues of the unscaled, unshifted Dirichlet -Laplacian on a box."""
    e = np.zeros(1)
    for N in dims:
        e = (e[:, None] + _lap1d_eigs(N)[None, :]).ravel()
    return np.sort(e)


def convdiff_eigs(N: int, beta: float) -> np.ndarray:
    """Sorted eigenvalues of the unshifted upwind operator of convdiff3d.

    In 1D the operator is tridiagonal with constant sub/super diagonals
    -(1+beta*h) and -1, hence diagonally similar to a symmetric one with
    off-diagonals -sqrt(1+beta*h).
    """
    bh = beta / (N + 1)
    k = np.arange(1, N + 1)
    e1 = (2.0 + bh) - 2.0 * np.sqrt(1.0 + bh) * np.cos(k * np.pi / (N + 1))
    e = (e1[:, None, None] + e1[None, :, None] + e1[None, None, :]).ravel()
    return np.sort(e)


def sigma_for_negatives(eigs: np.ndarray, count: int) -> float:
    """Shift placed midway between the count-th and (count+1)-th eigenvalue."""
    if not eigs[count] > eigs[count - 1]:
        raise ValueError("eigenvalues %d and %d coincide: no shift gives exactly %d negatives"
                         % (count, count + 1, count))
    return float(0.5 * (eigs[count - 1] + eigs[count]))


def sigma20_2d(N: int) -> float:
    return sigma_for_negatives(laplacian_eigs((N, N)), 20)


# --------------------------------------------------------------------------
# Vectors
# --------------------------------------------------------------------------


def normal_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """n x nrhs standard-normal matrix (column-major, i.e. Fortran order), PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


def start_vector(q: int, seed: int) -> np.ndarray:
    """Arnoldi start vector of length q (standard normal, PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(q)


def gaussian_random_field(N: int, corr_len: float, seed: int) -> np.ndarray:
    """Zero-mean unit-variance field on an N x N cell grid of [0,1]^2.

    Squared-exponential covariance exp(-r^2 / (2 l^2)), synthesised by FFT on a
    2x-padded periodic grid and cropped.  Indexed [ix, iy].
    """
    M = 2 * N
    h = 1.0 / N
    f = np.fft.fftfreq(M, d=h)
    kx, ky = np.meshgrid(f, f, indexing="ij")
    # spectral density of the SE kernel in 2D (up to a constant)
    psd = np.exp(-2.0 * (np.pi * corr_len) ** 2 * (kx ** 2 + ky ** 2))
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    field = np.real(np.fft.ifft2(np.sqrt(psd) * w))[:N, :N]
    field -= field.mean()
    field /= field.std()
    return field


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

SIGMA_C1 = 0.0768115308440700   # 2D 64^2: exactly 20 negative eigenvalues
SIGMA_C2 = 0.0989012132740537   # 3D 64^3: exactly 102 negative eigenvalues
SIGMA_C4 = 0.0353793815078993   # 3D 128^3 upwind, beta = 10: 133 negative eigenvalues


@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    grid_parts: tuple | None      # geometric split (P_x, P_y[, P_z]) or None
    region_parts: int | None      # region-growing part count or None
    region_seed: int | None
    m: int
    rank: int
    restart: int
    b: np.ndarray                 # n x nrhs, Fortran order
    tol: float = 1e-8


def c1(N: int = 64) -> Workload:
    """2D 5-point shifted Laplacian, 2x2 split, m=3, k=16, FGMRES(40), b = A*1."""
    sigma = SIGMA_C1 if N == 64 else sigma20_2d(N)
    A = laplacian2d(N, sigma)
    b = np.asfortranarray((A.to_scipy() @ np.ones(A.n)).reshape(-1, 1))
    return Workload("c1_lap2d_%d" % N, A, (2, 2), None, None, 3, 16, 40, b)


def c2(N: int = 64, nrhs: int = 1) -> Workload:
    """3D 7-point shifted Laplacian, 4x4x4 split, m=4, k=64, FGMRES(60), N(0,1) rhs seed 2."""
    sigma = SIGMA_C2 if N == 64 else sigma_for_negatives(laplacian_eigs((N, N, N)), 102)
    A = laplacian3d(N, sigma)
    return Workload("c2_lap3d_%d" % N, A, (4, 4, 4), None, None, 4, 64, 60, normal_rhs(A.n, nrhs, 2))


def c4(N: int = 128, nrhs: int = 32, parts: int = 256) -> Workload:
    """3D upwind convection-diffusion, beta=10, region growing, m=4, k=64, 32 rhs seed 40."""
    sigma = SIGMA_C4 if N == 128 else sigma_for_negatives(convdiff_eigs(N, 10.0), 133)
    A = convdiff3d(N, 10.0, sigma)
    return Workload("c4_convdiff3d_%d" % N, A, None, parts, 4, 4, 64, 60, normal_rhs(A.n, nrhs, 40))


def c3_systems(count: int = 48, side_lo: int = 32, side_hi: int = 512, seed: int = 3, nrhs: int = 8):
    """Batched uneven 2D shifted Laplacians (all draws from one PCG64 stream, seed 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    scales = rng.uniform(0.5, 1.5, size=count)
    parts = rng.integers(4, 33, size=count)
    out = []
    for i in range(count):
        N = int(sides[i])
        sigma = float(scales[i]) * sigma20_2d(N)
        A = laplacian2d(N, sigma)
        b = np.asfortranarray(rng.standard_normal((A.n, nrhs)))
        out.append(Workload("c3_sys%02d_lap2d_%d" % (i, N), A, None, int(parts[i]), seed * 1000 + i,
                            3, 32, 40, b))
    return out


def union(systems):
    """Block-diagonal union of several workloads' matrices.

    Returns (CSR, sys_ptr) with system s on rows sys_ptr[s] .. sys_ptr[s+1]-1.
    """
    mats = [w.A.to_scipy() for w in systems]
    U = CSR.from_scipy(sp.block_diag(mats, format="csr"))
    sys_ptr = np.concatenate([[0], np.cumsum([m.shape[0] for m in mats])]).astype(np.int64)
    return U, sys_ptr


def c5(N: int = 256, kappa_seed: int = 5, ref_seed: int = 6):
    """2D variable-coefficient Helmholtz-type problem for the gradient check.

    log kappa is a unit-variance Gaussian random field with correlation length
    0.1; sigma = sigma_20neg(N) * exp(mean log kappa); b = h^2 * 1; 4x4 split;
    m=3, k=16, FGMRES(40).  Returns (workload, kappa, kappa_ref).
    """
    logk = gaussian_random_field(N, 0.1, kappa_seed)
    logk_ref = gaussian_random_field(N, 0.1, ref_seed)
    kappa = np.exp(logk)
    kappa_ref = np.exp(logk_ref)
    sigma = sigma20_2d(N) * float(np.exp(logk.mean()))
    A = variable_coeff2d(kappa, sigma)
    h = 1.0 / (N + 1)
    b = np.asfortranarray(np.full((A.n, 1), h * h))
    return Workload("c5_helmholtz2d_%d" % N, A, (4, 4), None, None, 3, 16, 40, b), kappa, kappa_ref, sigma
