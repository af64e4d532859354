"""Python binding of the PSLR C ABI (include/pslr.h): argument marshalling only.

Every computation runs in libpslr.so (HIP kernels on the GPU, C++ host setup);
this module converts numpy arrays / torch device tensors into the pointers
and sizes the C functions take.  Names match the C entry points.

Device vectors are torch float64 tensors on a HIP device, either 1-D (n,) or
2-D (nrhs, n) row-major, i.e. column-major n x nrhs with leading dimension
equal to the row stride.  The library is required: nothing here has a CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpslr.so")
_lib = None

PSLR_OK, PSLR_EINVAL, PSLR_ESINGULAR, PSLR_ENOCONV, PSLR_EBREAKDOWN, PSLR_ENOMEM, PSLR_EHIP, \
    PSLR_ENOTSUP = range(8)


class PslrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


class pslr_options(C.Structure):
    _fields_ = [("m", C.c_int32), ("rank", C.c_int32), ("precision", C.c_int32),
                ("want_transpose", C.c_int32), ("v0", C.POINTER(C.c_double)),
                ("seed", C.c_uint64), ("pivot_threshold", C.c_double), ("nthreads", C.c_int32),
                ("working_vectors", C.c_int32), ("autotune", C.c_int32), ("threads", C.c_int32),
                ("factor", C.c_int32), ("drop_tol", C.c_double), ("lowrank", C.c_int32),
                ("team", C.c_int32), ("team_top", C.c_int32), ("team_rhs", C.c_int32)]


class pslr_host_stats_t(C.Structure):
    _fields_ = [("nnz_LU_B", C.c_int64), ("nnz_LU_C0", C.c_int64), ("max_levels_B", C.c_int32),
                ("max_levels_C0", C.c_int32), ("levels_valid", C.c_int32),
                ("factor_residual", C.c_double), ("solve_residual", C.c_double),
                ("team", C.c_int32), ("team_valid", C.c_int32), ("team_residual", C.c_double),
                ("team_lds_slots_B", C.c_int64), ("team_lds_slots_C", C.c_int64),
                ("team_groups_max_B", C.c_int32), ("team_items_B", C.c_int32)]


class pslr_info_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("p", C.c_int64), ("q", C.c_int64), ("nparts", C.c_int32),
                ("m", C.c_int32), ("rank", C.c_int32), ("precision", C.c_int32),
                ("nnz_A", C.c_int64), ("nnz_E", C.c_int64), ("nnz_F", C.c_int64),
                ("nnz_Cg", C.c_int64), ("nnz_LU_B", C.c_int64), ("nnz_LU_C0", C.c_int64),
                ("supernodes_B", C.c_int32), ("supernodes_C0", C.c_int32),
                ("max_levels_B", C.c_int32), ("max_levels_C0", C.c_int32),
                ("fill_lu", C.c_double), ("fill_lowrank", C.c_double), ("fill_total", C.c_double),
                ("apply_bytes", C.c_int64), ("apply_bytes_rhs", C.c_int64),
                ("series_bytes", C.c_int64), ("seconds_reorder", C.c_double),
                ("seconds_factor", C.c_double), ("seconds_arnoldi", C.c_double),
                ("nsys", C.c_int32), ("global_vectors", C.c_int32), ("threads", C.c_int32),
                ("lane_shift", C.c_int32), ("max_tile", C.c_int32), ("v_bf16", C.c_int32),
                ("bf16_probe", C.c_double), ("lowrank", C.c_int32), ("ks_restarts", C.c_int32),
                ("ks_applies", C.c_int64), ("ks_residual", C.c_double),
                ("ritz_above_one", C.c_int32), ("mfma_min_rhs", C.c_int32), ("team", C.c_int32),
                ("team_top", C.c_int32), ("team_c", C.c_int32), ("team_top_c", C.c_int32),
                ("team_apply", C.c_int32)]


class pslr_trace_t(C.Structure):
    _fields_ = [("applies", C.c_int64), ("series_launches", C.c_int64), ("ms_head", C.c_double),
                ("ms_lowrank", C.c_double), ("ms_series", C.c_double), ("ms_tail", C.c_double)]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_F64P = C.POINTER(C.c_double)

_SIGS = {
    "pslr_default_options": (None, [C.POINTER(pslr_options)]),
    "pslr_setup": (C.c_int, [C.c_int64, _I64P, _I32P, _F64P, _I32P, C.c_int32,
                             C.POINTER(pslr_options), _P, C.POINTER(_P)]),
    "pslr_setup_batched": (C.c_int, [C.c_int64, _I64P, _I32P, _F64P, _I32P, C.c_int32, C.c_int32,
                                     _I64P, C.POINTER(pslr_options), _P, C.POINTER(_P)]),
    "pslr_refactor": (C.c_int, [_P, _F64P, _P]),
    "pslr_apply": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "pslr_apply_noalloc": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "pslr_apply_transpose": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "fgmres_solve": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64, C.c_int32, C.c_int32,
                               C.c_double, C.c_int32, _I32P, _F64P, _P]),
    "pslr_sddmm_grad": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P, _P]),
    "pslr_info": (C.c_int, [_P, C.POINTER(pslr_info_t)]),
    "pslr_trace_enable": (C.c_int, [_P, C.c_int32]),
    "pslr_trace_read": (C.c_int, [_P, C.POINTER(pslr_trace_t), C.c_int32]),
    "pslr_set_lowrank": (C.c_int, [_P, C.c_int32, _F64P, C.c_int64, _F64P, C.c_int64]),
    "pslr_get_lowrank": (C.c_int, [_P, _I32P, _F64P, C.c_int64, _F64P, C.c_int64]),
    "pslr_delta": (C.c_int, [_P, C.c_int32, C.c_uint64, _F64P, _F64P, _F64P, _P]),
    "pslr_partition_geometric": (C.c_int, [C.c_int32, _I32P, _I32P, _I32P]),
    "pslr_partition_region_growing": (C.c_int, [C.c_int64, _I64P, _I32P, C.c_int32, C.c_uint64,
                                                _I32P, _I32P]),
    "pslr_reorder": (C.c_int, [C.c_int64, _I64P, _I32P, _I32P, C.c_int32, _I64P, _I64P, _I64P]),
    "pslr_host_selfcheck": (C.c_int, [C.c_int64, _I64P, _I32P, _F64P, _I32P, C.c_int32,
                                      C.POINTER(pslr_options), _F64P, _F64P]),
    "pslr_host_stats": (C.c_int, [C.c_int64, _I64P, _I32P, _F64P, _I32P, C.c_int32,
                                  C.POINTER(pslr_options), C.POINTER(pslr_host_stats_t)]),
    "pslr_host_schur_select": (C.c_int, [C.c_int32, _F64P, C.c_int64, C.c_int32, _F64P, C.c_int64,
                                         _F64P, C.c_int64, _F64P, _F64P, _I32P]),
    "pslr_destroy": (C.c_int, [_P]),
    "pslr_status_string": (C.c_char_p, [C.c_int]),
    "pslr_last_error": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libpslr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpslr.so is not built: run `python -m paper_2002_00917_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_name(s):
    try:
        return lib().pslr_status_string(s).decode()
    except Exception:
        return "status %d" % s


def _check(status, allowed=(PSLR_OK,)):
    if status not in allowed:
        raise PslrError(status, lib().pslr_last_error().decode())
    return status


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _vec(t, n):
    """(pointer, nrhs, ld) of a float64 device tensor shaped (n,) or (nrhs, n)."""
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError("device float64 tensor required")
    if t.dim() == 1:
        if t.shape[0] != n or t.stride(0) != 1:
            raise ValueError("bad vector shape")
        return C.c_void_p(t.data_ptr()), 1, n
    if t.dim() != 2 or t.shape[1] != n or (n > 1 and t.stride(1) != 1):
        raise ValueError("expected shape (nrhs, n) with unit stride along n")
    # the stride of a size-1 dimension carries no layout information
    ld = t.stride(0) if t.shape[0] > 1 else n
    return C.c_void_p(t.data_ptr()), t.shape[0], ld


# ----------------------------------------------------------------- handle


class Handle:
    """An opaque library handle plus what the binding checks arguments against:
    n, nnz(A), and a fingerprint of A's values (count, sum, sum of squares)."""

    def __init__(self, ptr, n, status, nsys=1, vals=None):
        self.ptr = ptr
        self.n = n
        self.status = status
        self.nsys = nsys
        v = np.zeros(0) if vals is None else np.asarray(vals, dtype=np.float64)
        self.nnz = int(v.size)
        self.vals_fingerprint = (int(v.size), float(np.sum(v)), float(np.sum(v * v)))

    def __del__(self):
        if getattr(self, "ptr", None) is not None and _lib is not None:
            _lib.pslr_destroy(self.ptr)
            self.ptr = None


def pslr_default_options():
    o = pslr_options()
    lib().pslr_default_options(C.byref(o))
    return o


FACTORS = {"lu": 0, "ilut": 1}


LOWRANK = {"arnoldi": 0, "krylov_schur": 1, "deflate_unit": 2}


def _options(m, rank, precision, want_transpose, v0, seed, pivot_threshold, nthreads,
             working_vectors, autotune=False, threads=0, factor="lu", drop_tol=1e-2,
             lowrank="arnoldi", team=0, team_top=0, team_rhs=0):
    o = pslr_default_options()
    o.lowrank = LOWRANK[lowrank]
    o.team = int(team)
    o.team_top = int(team_top)
    o.team_rhs = int(team_rhs)
    o.threads = int(threads)
    o.factor = FACTORS[factor]
    o.drop_tol = float(drop_tol)
    o.m, o.rank, o.precision = int(m), int(rank), int(precision)
    o.want_transpose = 1 if want_transpose else 0
    o.seed, o.pivot_threshold, o.nthreads = int(seed), float(pivot_threshold), int(nthreads)
    o.working_vectors = int(working_vectors)
    o.autotune = 1 if autotune else 0
    keep = None
    if v0 is not None:
        keep, o.v0 = _arr(v0, np.float64)
    return o, keep


def pslr_setup(rowptr, colind, vals, part, nparts, m=3, rank=16, precision=0,
               want_transpose=False, v0=None, seed=1, pivot_threshold=0.1, nthreads=0,
               working_vectors=0, autotune=False, threads=0, factor="lu", drop_tol=1e-2,
               lowrank="arnoldi", team=0, team_top=0, team_rhs=0, stream=None) -> Handle:
    L = lib()
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    va, vap = _arr(vals, np.float64)
    pa, pap = _arr(part, np.int32)
    o, keep = _options(m, rank, precision, want_transpose, v0, seed, pivot_threshold, nthreads,
                       working_vectors, autotune, threads, factor, drop_tol, lowrank, team,
                       team_top, team_rhs)
    out = C.c_void_p()
    n = len(rp) - 1
    st = L.pslr_setup(n, rpp, cip, vap, pap, int(nparts), C.byref(o), _stream_ptr(stream),
                      C.byref(out))
    _check(st, (PSLR_OK, PSLR_EBREAKDOWN))
    del keep
    return Handle(out, n, st, vals=va)


def pslr_setup_batched(rowptr, colind, vals, part, nparts, sys_ptr, m=3, rank=16, precision=0,
                       want_transpose=False, v0=None, seed=1, pivot_threshold=0.1, nthreads=0,
                       working_vectors=0, autotune=False, threads=0, factor="lu", drop_tol=1e-2,
                       lowrank="arnoldi", team=0, team_top=0, team_rhs=0, stream=None) -> Handle:
    L = lib()
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    va, vap = _arr(vals, np.float64)
    pa, pap = _arr(part, np.int32)
    sp, spp = _arr(sys_ptr, np.int64)
    o, keep = _options(m, rank, precision, want_transpose, v0, seed, pivot_threshold, nthreads,
                       working_vectors, autotune, threads, factor, drop_tol, lowrank, team,
                       team_top, team_rhs)
    out = C.c_void_p()
    n = len(rp) - 1
    st = L.pslr_setup_batched(n, rpp, cip, vap, pap, int(nparts), len(sp) - 1, spp, C.byref(o),
                              _stream_ptr(stream), C.byref(out))
    _check(st, (PSLR_OK, PSLR_EBREAKDOWN))
    del keep
    return Handle(out, n, st, nsys=len(sp) - 1, vals=va)


def pslr_refactor(h: Handle, vals, stream=None):
    """New values on the handle's sparsity pattern (original CSR order)."""
    va, vap = _arr(vals, np.float64)
    if va.size != h.nnz:
        raise ValueError("vals must have nnz(A) = %d entries" % h.nnz)
    st = lib().pslr_refactor(h.ptr, vap, _stream_ptr(stream))
    _check(st, (PSLR_OK, PSLR_EBREAKDOWN))
    h.vals_fingerprint = (int(va.size), float(np.sum(va)), float(np.sum(va * va)))
    return st


def pslr_apply(h: Handle, b, z, stream=None):
    bp, nrhs, ldb = _vec(b, h.n)
    zp, nrz, ldz = _vec(z, h.n)
    if nrz != nrhs:
        raise ValueError("b and z have different column counts")
    _check(lib().pslr_apply(h.ptr, nrhs, bp, ldb, zp, ldz, _stream_ptr(stream)))


def pslr_apply_noalloc(h: Handle, b, z, stream=None):
    bp, nrhs, ldb = _vec(b, h.n)
    zp, nrz, ldz = _vec(z, h.n)
    if nrz != nrhs:
        raise ValueError("b and z have different column counts")
    _check(lib().pslr_apply_noalloc(h.ptr, nrhs, bp, ldb, zp, ldz, _stream_ptr(stream)))


def pslr_apply_transpose(h: Handle, b, z, stream=None):
    bp, nrhs, ldb = _vec(b, h.n)
    zp, nrz, ldz = _vec(z, h.n)
    if nrz != nrhs:
        raise ValueError("b and z have different column counts")
    _check(lib().pslr_apply_transpose(h.ptr, nrhs, bp, ldb, zp, ldz, _stream_ptr(stream)))


def fgmres_solve(h: Handle, b, x, restart=40, maxit=500, tol=1e-8, transpose=False, stream=None):
    """Returns (status, iters, relres); x holds the initial guess and the result.

    iters/relres have nrhs entries, or nrhs * nsys (index r * nsys + s) on a
    batched handle."""
    bp, nrhs, ldb = _vec(b, h.n)
    xp, nrx, ldx = _vec(x, h.n)
    if nrx != nrhs:
        raise ValueError("b and x have different column counts")
    its = np.zeros(nrhs * h.nsys, dtype=np.int32)
    rel = np.zeros(nrhs * h.nsys, dtype=np.float64)
    st = lib().fgmres_solve(h.ptr, nrhs, bp, ldb, xp, ldx, int(restart), int(maxit), float(tol),
                            1 if transpose else 0, its.ctypes.data_as(_I32P),
                            rel.ctypes.data_as(_F64P), _stream_ptr(stream))
    _check(st, (PSLR_OK, PSLR_ENOCONV))
    return st, its, rel


def pslr_sddmm_grad(h: Handle, lam, z, grad, stream=None):
    """grad: float64 device tensor with nnz(A) contiguous entries (original CSR order)."""
    import torch
    lp, nrhs, ldl = _vec(lam, h.n)
    zp, nrz, ldz = _vec(z, h.n)
    if nrz != nrhs:
        raise ValueError("lambda and z have different column counts")
    if grad.dtype != torch.float64 or not grad.is_cuda or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float64 device tensor")
    if grad.numel() != h.nnz:
        raise ValueError("grad has %d entries, A has %d stored entries" % (grad.numel(), h.nnz))
    _check(lib().pslr_sddmm_grad(h.ptr, nrhs, lp, ldl, zp, ldz, C.c_void_p(grad.data_ptr()),
                                 _stream_ptr(stream)))


def pslr_info(h: Handle) -> dict:
    info = pslr_info_t()
    _check(lib().pslr_info(h.ptr, C.byref(info)))
    return {k: getattr(info, k) for k, _ in pslr_info_t._fields_}


def pslr_trace_enable(h: Handle, enable=True):
    _check(lib().pslr_trace_enable(h.ptr, 1 if enable else 0))


def pslr_trace_read(h: Handle, reset=False) -> dict:
    t = pslr_trace_t()
    _check(lib().pslr_trace_read(h.ptr, C.byref(t), 1 if reset else 0))
    return {k: getattr(t, k) for k, _ in pslr_trace_t._fields_}


def pslr_set_lowrank(h: Handle, V, H):
    V = np.asfortranarray(V, dtype=np.float64)
    H = np.asfortranarray(H, dtype=np.float64)
    k = V.shape[1] if V.ndim == 2 else 0
    q = V.shape[0]
    _check(lib().pslr_set_lowrank(h.ptr, k, V.ctypes.data_as(_F64P), max(q, 1),
                                  H.ctypes.data_as(_F64P), max(k, 1)))


def pslr_delta(h: Handle, nprobe=0, seed=1, stream=None):
    """(Delta(m, r_k), ||X||_F, ||Z^{-1}||_F) of Prop. l3; nprobe = 0: exact."""
    d, nx, nz = C.c_double(), C.c_double(), C.c_double()
    _check(lib().pslr_delta(h.ptr, int(nprobe), int(seed), C.byref(d), C.byref(nx), C.byref(nz),
                            _stream_ptr(stream)))
    return d.value, nx.value, nz.value


def pslr_get_lowrank(h: Handle):
    info = pslr_info(h)
    q, k = info["q"], info["rank"]
    V = np.zeros((q, k), order="F")
    H = np.zeros((k, k), order="F")
    kk = C.c_int32()
    _check(lib().pslr_get_lowrank(h.ptr, C.byref(kk), V.ctypes.data_as(_F64P), max(q, 1),
                                  H.ctypes.data_as(_F64P), max(k, 1)))
    return V[:, :kk.value], H[:kk.value, :kk.value]


def pslr_partition_geometric(dims, parts) -> np.ndarray:
    d, dp = _arr(dims, np.int32)
    p, pp = _arr(parts, np.int32)
    out = np.zeros(int(np.prod(d)), dtype=np.int32)
    _check(lib().pslr_partition_geometric(len(d), dp, pp, out.ctypes.data_as(_I32P)))
    return out


def pslr_partition_region_growing(rowptr, colind, nparts, seed):
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    n = len(rp) - 1
    out = np.zeros(n, dtype=np.int32)
    nl = C.c_int32()
    _check(lib().pslr_partition_region_growing(n, rpp, cip, int(nparts), C.c_uint64(seed),
                                               out.ctypes.data_as(_I32P), C.byref(nl)))
    return out, nl.value


def pslr_reorder(rowptr, colind, part, nparts):
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    pa, pap = _arr(part, np.int32)
    n = len(rp) - 1
    perm = np.zeros(n, dtype=np.int64)
    p = C.c_int64()
    q = C.c_int64()
    _check(lib().pslr_reorder(n, rpp, cip, pap, int(nparts), perm.ctypes.data_as(_I64P),
                              C.byref(p), C.byref(q)))
    return perm, p.value, q.value


def pslr_host_stats(rowptr, colind, vals, part, nparts, want_transpose=True, pivot_threshold=0.1,
                    nthreads=0, factor="lu", drop_tol=1e-2, team=0) -> dict:
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    va, vap = _arr(vals, np.float64)
    pa, pap = _arr(part, np.int32)
    o = pslr_default_options()
    o.want_transpose = 1 if want_transpose else 0
    o.pivot_threshold = float(pivot_threshold)
    o.nthreads = int(nthreads)
    o.factor = FACTORS[factor]
    o.drop_tol = float(drop_tol)
    o.team = int(team)
    out = pslr_host_stats_t()
    _check(lib().pslr_host_stats(len(rp) - 1, rpp, cip, vap, pap, int(nparts), C.byref(o),
                                 C.byref(out)))
    return {k: getattr(out, k) for k, _ in pslr_host_stats_t._fields_}


def pslr_host_selfcheck(rowptr, colind, vals, part, nparts, want_transpose=True,
                        pivot_threshold=0.1, nthreads=0, factor="lu", drop_tol=1e-2):
    rp, rpp = _arr(rowptr, np.int64)
    ci, cip = _arr(colind, np.int32)
    va, vap = _arr(vals, np.float64)
    pa, pap = _arr(part, np.int32)
    o = pslr_default_options()
    o.want_transpose = 1 if want_transpose else 0
    o.pivot_threshold = float(pivot_threshold)
    o.nthreads = int(nthreads)
    o.factor = FACTORS[factor]
    o.drop_tol = float(drop_tol)
    fr = C.c_double()
    sr = C.c_double()
    _check(lib().pslr_host_selfcheck(len(rp) - 1, rpp, cip, vap, pap, int(nparts), C.byref(o),
                                     C.byref(fr), C.byref(sr)))
    return fr.value, sr.value


def pslr_host_schur_select(Hm, k):
    """(W, Hk, ritz) of the host-only Krylov-Schur truncation step (no GPU)."""
    Hm = np.asfortranarray(Hm, dtype=np.float64)
    n = Hm.shape[0]
    kk = max(n, 1)
    W = np.zeros((kk, kk), dtype=np.float64, order="F")
    Hk = np.zeros((kk, kk), dtype=np.float64, order="F")
    rr = np.zeros(max(n, 1))
    ri = np.zeros(max(n, 1))
    kept = C.c_int32()
    dp = lambda a: a.ctypes.data_as(_F64P)  # noqa: E731
    _check(lib().pslr_host_schur_select(n, dp(Hm), max(n, 1), int(k), dp(W), kk, dp(Hk), kk,
                                        dp(rr), dp(ri), C.byref(kept)))
    kp = kept.value
    return W[:n, :kp].copy(), Hk[:kp, :kp].copy(), rr[:n] + 1j * ri[:n]

