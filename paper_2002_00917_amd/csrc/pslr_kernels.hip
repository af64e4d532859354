// HIP kernels of the PSLR preconditioner apply (paper Algorithm 3) and of the
// FP64 vector work of Arnoldi (Algorithm 4) and flexible GMRES, for gfx950.
//
// Design: one workgroup owns one subdomain (and one right-hand side) and keeps
// that subdomain's working vectors in LDS.  The B_i and C_i solves are
// level-scheduled over the supernodal elimination tree of an exact LU
// factorisation: each level is (1) a sweep of independent dot products that
// pulls the already-solved unknowns (CSR rows for lower factors, dense panels
// over a shared column list for upper factors) and (2) a sweep of dense
// products with the level's inverted diagonal triangles.  Both sweeps stream
// the factor entries from HBM exactly once, coalesced, with lane groups sized
// per level to the average row length; gathers hit LDS only.  The coupling
// SpMVs with E, F and C_g are fused into the kernels that produce or consume
// their operands, so one power-series step of eq. approx1 is one launch.
#include "pslr_dev.h"

namespace pslr {

namespace {

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

__device__ __forceinline__ float tv_to_float(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float tv_to_float(float v) { return v; }
__device__ __forceinline__ double tv_to_float(double v) { return v; }

// sum_j v[j] * X[idx[j]] over this lane's share (j = lane, lane+G, ...), with
// eight independent loads in flight per lane.
template <typename T>
__device__ __forceinline__ T dot_gather(const T* __restrict__ v, const int32_t* __restrict__ idx,
                                        int len, const T* X, int lane, int G) {
  T a0 = 0, a1 = 0;
  int j = lane;
  for (; j + 7 * G < len; j += 8 * G) {
    T v0 = v[j], v1 = v[j + G], v2 = v[j + 2 * G], v3 = v[j + 3 * G];
    T v4 = v[j + 4 * G], v5 = v[j + 5 * G], v6 = v[j + 6 * G], v7 = v[j + 7 * G];
    int c0 = idx[j], c1 = idx[j + G], c2 = idx[j + 2 * G], c3 = idx[j + 3 * G];
    int c4 = idx[j + 4 * G], c5 = idx[j + 5 * G], c6 = idx[j + 6 * G], c7 = idx[j + 7 * G];
    a0 += v0 * X[c0];
    a1 += v1 * X[c1];
    a0 += v2 * X[c2];
    a1 += v3 * X[c3];
    a0 += v4 * X[c4];
    a1 += v5 * X[c5];
    a0 += v6 * X[c6];
    a1 += v7 * X[c7];
  }
  for (; j < len; j += G) a0 += v[j] * X[idx[j]];
  return a0 + a1;
}

// sum_j v[j] * R[j] over this lane's share, eight loads in flight per lane.
template <typename T>
__device__ __forceinline__ T dot_dense(const T* __restrict__ v, int len, const T* R, int lane, int G) {
  T a0 = 0, a1 = 0;
  int j = lane;
  for (; j + 7 * G < len; j += 8 * G) {
    T v0 = v[j], v1 = v[j + G], v2 = v[j + 2 * G], v3 = v[j + 3 * G];
    T v4 = v[j + 4 * G], v5 = v[j + 5 * G], v6 = v[j + 6 * G], v7 = v[j + 7 * G];
    a0 += v0 * R[j];
    a1 += v1 * R[j + G];
    a0 += v2 * R[j + 2 * G];
    a1 += v3 * R[j + 3 * G];
    a0 += v4 * R[j + 4 * G];
    a1 += v5 * R[j + 5 * G];
    a0 += v6 * R[j + 6 * G];
    a1 += v7 * R[j + 7 * G];
  }
  for (; j < len; j += G) a0 += v[j] * R[j];
  return a0 + a1;
}

// Solve one packed triangular factor of block `bi` in place on the LDS vector X
// (positions 0..n-1); Rb is LDS scratch of max_lrows entries.  All threads of
// the workgroup must call it.  Ends with a barrier.
template <typename T>
__device__ void tri_solve(const TriArrays<T>& A, int bi, T* X, T* Rb, int gshift) {
  const DevTriBlock B = A.blk[bi];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int4* rec = A.rec + 2 * B.rec_base;
  const T* val = A.val + B.val_base;
  const int32_t* col = A.col + B.val_base;
  const int32_t* ridx = A.ridx + B.ridx_base;
  const T* tri = A.tri + B.tri_base;
  const int32_t* lev_ptr = A.lev_ptr + B.lev_base;
  const int32_t* lev_g = A.lev_g + B.lev_base;
  for (int li = 0; li < B.nlev; ++li) {
    const int l = B.lower ? li : B.nlev - 1 - li;
    const int b = lev_ptr[l];
    const int cnt = lev_ptr[l + 1] - b;
    const int g = lev_g[l];
    int G1 = g & 0xff, G2 = (g >> 8) & 0xff;
    if (gshift > 0) {
      G1 = min(64, G1 << gshift);
      G2 = min(64, G2 << gshift);
    } else if (gshift < 0) {
      G1 = max(1, G1 >> -gshift);
      G2 = max(1, G2 >> -gshift);
    }
    // sweep 1: r_k = x_p - (off-diagonal part of row p) . x
    {
      const int grp = tid / G1, lane = tid - grp * G1, ngrp = nthr / G1;
      for (int k = grp; k < cnt; k += ngrp) {
        const int4 r = rec[2 * (b + k)];
        T acc = dot_gather(val + r.y, B.lower ? col + r.y : ridx + r.w, r.z, X, lane, G1);
        acc = group_sum(acc, G1);
        if (lane == 0) Rb[k] = X[r.x] - acc;
      }
    }
    __syncthreads();
    // sweep 2: x_s = inv(T_ss) r_s for every supernode of the level
    {
      const int grp = tid / G2, lane = tid - grp * G2, ngrp = nthr / G2;
      for (int k = grp; k < cnt; k += ngrp) {
        const int p = rec[2 * (b + k)].x;
        const int4 r = rec[2 * (b + k) + 1];
        T acc = dot_dense(tri + r.x, r.y, Rb + r.z, lane, G2);
        acc = group_sum(acc, G2);
        if (lane == 0) X[p] = acc;
      }
    }
    __syncthreads();
  }
}

template <typename T>
struct Lds {
  T *XB, *Rb, *XC, *U, *W;
};

// Working vectors of block blockIdx.x for right-hand side blockIdx.y: in LDS,
// or (GX) in the handle's global workspace when a subdomain is too large for
// LDS.  The global layout per right-hand side is [X_B: p][X_C: q][U: q]
// [scratch: sum of per-block level sizes][W: 2k per block].
template <typename T, bool GX>
__device__ Lds<T> carve(const ApplyArrays<T>& A) {
  Lds<T> L;
  if (GX) {
    const int i = blockIdx.x, r = blockIdx.y;
    T* base = reinterpret_cast<T*>(A.gws) + (int64_t)r * A.gws_stride;
    L.XB = base + A.int_ptr[i];
    L.XC = base + A.p + A.if_ptr[i];
    L.U = base + A.p + A.q + A.if_ptr[i];
    L.Rb = base + A.p + 2 * A.q + A.rb_off[i];
    L.W = base + A.p + 2 * A.q + A.rb_off[A.nparts] + (int64_t)i * 2 * A.kmax;
  } else {
    extern __shared__ __align__(16) unsigned char smem[];
    L.XB = reinterpret_cast<T*>(smem);
    L.Rb = L.XB + A.maxPB;
    L.XC = L.Rb + A.maxLR;
    L.U = L.XC + A.maxQB;
    L.W = L.U + A.maxQB;
  }
  return L;
}

// t = B^{-1} f;  y = g - F t   (Algorithm 3, line 2)
template <typename T, bool GX>
__global__ void __launch_bounds__(1024) k_head(ApplyArrays<T> A, const double* __restrict__ b, int64_t ldb, T* y,
                       int64_t ldy) {
  Lds<T> L = carve<T, GX>(A);
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const double* br = b + r * ldb;
  for (int64_t p = tid; p < pi; p += nt) L.XB[p] = (T)br[A.gB_in[i0 + p]];
  __syncthreads();
  tri_solve(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve(A.UB, i, L.XB, L.Rb, A.gshift);
  T* yr = y + r * ldy;
  for (int64_t k = tid; k < qi; k += nt) {
    const int64_t row = f0 + k;
    T acc = (T)br[A.if_orig[row]];
    for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q) acc -= A.Fout.val[q] * L.XB[A.Fout.col[q]];
    yr[row] = acc;
  }
}

// partial[chunk][r][j] = sum_{rows in chunk} V[row][j] y_r[row]   (V^T y, line 3)
template <typename T, typename TV>
__global__ void k_lr_partial(const LrChunk* __restrict__ chunks, int k, const TV* __restrict__ V,
                             const T* __restrict__ y, int64_t ldy, T* partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* red = reinterpret_cast<T*>(smem);
  const int chunk = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const LrChunk C = chunks[chunk];
  const int ng = nt / k;
  const int g = tid / k, j = tid - g * k;
  T acc = 0;
  if (g < ng) {
    const T* yr = y + r * ldy;
    for (int64_t row = C.r0 + g; row < C.r1; row += ng) acc += (T)tv_to_float(V[row * k + j]) * yr[row];
    red[g * k + j] = acc;
  }
  __syncthreads();
  if (tid < k) {
    T s = 0;
    for (int gg = 0; gg < ng; ++gg) s += red[gg * k + tid];
    partial[((int64_t)chunk * gridDim.y + r) * k + tid] = s;
  }
}

// y += V (G (V^T y)) on the rows of block i; optionally u = C0^{-1} y (line 3, line 4 start)
template <typename T, typename TV, bool GX>
__global__ void __launch_bounds__(1024) k_lr_expand(ApplyArrays<T> A, int k, const TV* __restrict__ V,
                            const T* __restrict__ Gall, int gtrans, const T* __restrict__ partial,
                            const int32_t* __restrict__ sys_chunk, T* y, int64_t ldy, int do_c0,
                            T* u, int64_t ldu) {
  Lds<T> L = carve<T, GX>(A);
  T* Wv = L.W;
  T* Zv = L.W + k;
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int nrhs = gridDim.y;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const int sys = A.part_sys[i];
  const T* G = Gall + (int64_t)sys * k * k;
  const int c0 = sys_chunk[sys], c1 = sys_chunk[sys + 1];
  for (int j = tid; j < k; j += nt) {
    T s = 0;
    for (int c = c0; c < c1; ++c) s += partial[((int64_t)c * nrhs + r) * k + j];
    Wv[j] = s;
  }
  __syncthreads();
  for (int j = tid; j < k; j += nt) {
    T s = 0;
    for (int l = 0; l < k; ++l) s += (gtrans ? G[(int64_t)l * k + j] : G[(int64_t)j * k + l]) * Wv[l];
    Zv[j] = s;
  }
  __syncthreads();
  T* yr = y + r * ldy;
  const int GL = k >= 64 ? 64 : (k >= 32 ? 32 : (k >= 16 ? 16 : (k >= 8 ? 8 : (k >= 4 ? 4 : (k >= 2 ? 2 : 1)))));
  const int grp = tid / GL, lane = tid - grp * GL, ngrp = nt / GL;
  for (int64_t kr = grp; kr < qi; kr += ngrp) {
    const int64_t row = f0 + kr;
    T acc = 0;
    for (int j = lane; j < k; j += GL) acc += (T)tv_to_float(V[row * k + j]) * Zv[j];
    acc = group_sum(acc, GL);
    if (lane == 0) {
      const T v = yr[row] + acc;
      yr[row] = v;
      if (do_c0) L.XC[A.gC_inv[row]] = v;
    }
  }
  if (!do_c0) return;
  __syncthreads();
  tri_solve(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve(A.UC, i, L.XC, L.Rb, A.gshift);
  T* ur = u + r * ldu;
  for (int64_t c = tid; c < qi; c += nt) ur[f0 + A.gC_out[f0 + c]] = L.XC[c];
}

// dst = C0^{-1} src
template <typename T, bool GX>
__global__ void __launch_bounds__(1024) k_c0solve(ApplyArrays<T> A, const T* __restrict__ src, int64_t lds_, T* dst,
                          int64_t ldd) {
  Lds<T> L = carve<T, GX>(A);
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const T* sr = src + r * lds_;
  for (int64_t p = tid; p < qi; p += nt) L.XC[p] = sr[f0 + A.gC_in[f0 + p]];
  __syncthreads();
  tri_solve(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve(A.UC, i, L.XC, L.Rb, A.gshift);
  T* dr = dst + r * ldd;
  for (int64_t c = tid; c < qi; c += nt) dr[f0 + A.gC_out[f0 + c]] = L.XC[c];
}

// One power-series step (eq. approx1 by its recurrence):
//   w = E_s u = -C_g u + F B^{-1} E u;  r = [y +] w;  u_next = [C0^{-1}] r
template <typename T, bool GX>
__global__ void __launch_bounds__(1024) k_series(ApplyArrays<T> A, const T* __restrict__ y, int64_t ldy,
                         const T* __restrict__ uprev, T* unext, int64_t ldu, int add_y, int do_c0) {
  Lds<T> L = carve<T, GX>(A);
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const T* ur = uprev + r * ldu;
  for (int64_t k = tid; k < qi; k += nt) L.U[k] = ur[f0 + k];
  __syncthreads();
  for (int64_t p = tid; p < pi; p += nt) {
    const int64_t row = i0 + p;
    T acc = 0;
    for (int64_t q = A.Ein.ptr[row]; q < A.Ein.ptr[row + 1]; ++q) acc += A.Ein.val[q] * L.U[A.Ein.col[q]];
    L.XB[p] = acc;
  }
  __syncthreads();
  tri_solve(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve(A.UB, i, L.XB, L.Rb, A.gshift);
  const T* yr = y + r * ldy;
  T* vr = unext + r * ldu;
  for (int64_t k = tid; k < qi; k += nt) {
    const int64_t row = f0 + k;
    T acc = add_y ? yr[row] : (T)0;
    for (int64_t q = A.Cg.ptr[row]; q < A.Cg.ptr[row + 1]; ++q) acc -= A.Cg.val[q] * ur[A.Cg.col[q]];
    for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q) acc += A.Fout.val[q] * L.XB[A.Fout.col[q]];
    if (do_c0) L.XC[A.gC_inv[row]] = acc;
    else vr[row] = acc;
  }
  if (!do_c0) return;
  __syncthreads();
  tri_solve(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve(A.UC, i, L.XC, L.Rb, A.gshift);
  for (int64_t c = tid; c < qi; c += nt) vr[f0 + A.gC_out[f0 + c]] = L.XC[c];
}

// x = B^{-1}(f - E u);  z = P^T (x; u)   (Algorithm 3, lines 5-6)
template <typename T, bool GX>
__global__ void __launch_bounds__(1024) k_tail(ApplyArrays<T> A, const double* __restrict__ b, int64_t ldb,
                       const T* __restrict__ u, int64_t ldu, double* z, int64_t ldz) {
  Lds<T> L = carve<T, GX>(A);
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const T* ur = u + r * ldu;
  const double* br = b + r * ldb;
  double* zr = z + r * ldz;
  for (int64_t k = tid; k < qi; k += nt) {
    const T v = ur[f0 + k];
    L.U[k] = v;
    zr[A.if_orig[f0 + k]] = (double)v;
  }
  __syncthreads();
  for (int64_t p = tid; p < pi; p += nt) {
    const int64_t row = i0 + p;
    T acc = (T)br[A.gB_in[row]];
    for (int64_t q = A.Ein.ptr[row]; q < A.Ein.ptr[row + 1]; ++q) acc -= A.Ein.val[q] * L.U[A.Ein.col[q]];
    L.XB[p] = acc;
  }
  __syncthreads();
  tri_solve(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve(A.UB, i, L.XB, L.Rb, A.gshift);
  for (int64_t c = tid; c < pi; c += nt) zr[A.gB_out[i0 + c]] = (double)L.XB[c];
}

// ---------------------------------------------------------------- FP64 vector kernels

__global__ void k_spmv(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, const double* __restrict__ x, int64_t ldx,
                       double* y, int64_t ldy, const double* __restrict__ bsub, int64_t ldb) {
  const int r = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const double* xr = x + r * ldx;
  double acc = 0.0;
  for (int64_t q = ptr[row]; q < ptr[row + 1]; ++q) acc += val[q] * xr[col[q]];
  y[r * ldy + row] = bsub ? bsub[r * ldb + row] - acc : acc;
}

__global__ void k_mdot(int64_t n, int nv, const double* __restrict__ V, int64_t ldv, int64_t ldvr,
                       const double* __restrict__ w, int64_t ldw, int nchunk, double* partial) {
  __shared__ double red[8];
  const int chunk = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int64_t rows = (n + nchunk - 1) / nchunk;
  const int64_t r0 = chunk * rows, r1 = min(n, r0 + rows);
  const double* wr = w + r * ldw;
  for (int i = 0; i < nv; ++i) {
    const double* vi = V + r * ldvr + i * ldv;
    double acc = 0.0;
    for (int64_t row = r0 + tid; row < r1; row += blockDim.x) acc += vi[row] * wr[row];
    acc = group_sum(acc, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
      partial[((int64_t)chunk * gridDim.y + r) * nv + i] = s;
    }
    __syncthreads();
  }
}

// out[r][i] = sum over chunks of partial[c][r][i]: one workgroup per (i, r)
__global__ void k_reduce(int nchunk, int nrhs, int nv, const double* __restrict__ partial, double* out) {
  __shared__ double red[4];
  const int i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  double s = 0.0;
  for (int c = tid; c < nchunk; c += blockDim.x) s += partial[((int64_t)c * nrhs + r) * nv + i];
  s = group_sum(s, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[(int64_t)r * nv + i] = t;
  }
}

__global__ void k_maxpy(int64_t n, int nv, const double* __restrict__ V, int64_t ldv, int64_t ldvr,
                        const double* __restrict__ h, int hld, double* w, int64_t ldw, double sign) {
  const int r = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const double* hr = h + (int64_t)r * hld;
  double acc = 0.0;
  for (int i = 0; i < nv; ++i) acc += hr[i] * V[r * ldvr + i * ldv + row];
  w[r * ldw + row] -= sign * acc;
}

__global__ void k_scale(int64_t n, const double* __restrict__ w, int64_t ldw,
                        const double* __restrict__ scale, double* v, int64_t ldv) {
  const int r = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  v[r * ldv + row] = w[r * ldw + row] * scale[r];
}

__global__ void k_mdot_seg(const Seg* __restrict__ vcols, const Seg* __restrict__ wcols, int nv,
                           const double* __restrict__ V, int64_t ldv, const double* __restrict__ W,
                           int nchunk, double* partial) {
  __shared__ double red[8];
  const int chunk = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const Seg sv = vcols[c], sw = wcols[c];
  const int64_t rows = (sw.len + nchunk - 1) / nchunk;
  const int64_t r0 = chunk * rows, r1 = min(sw.len, r0 + rows);
  const double* wr = W + sw.base;
  for (int i = 0; i < nv; ++i) {
    const double* vi = V + sv.base + i * ldv;
    double acc = 0.0;
    for (int64_t row = r0 + tid; row < r1; row += blockDim.x) acc += vi[row] * wr[row];
    acc = group_sum(acc, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
      partial[((int64_t)chunk * gridDim.y + c) * nv + i] = s;
    }
    __syncthreads();
  }
}

__global__ void k_maxpy_seg(const Seg* __restrict__ vcols, const Seg* __restrict__ wcols, int nv,
                            const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                            int hld, double* W, double sign) {
  const int c = blockIdx.y;
  const Seg sv = vcols[c], sw = wcols[c];
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= sw.len) return;
  const double* hr = h + (int64_t)c * hld;
  double acc = 0.0;
  for (int i = 0; i < nv; ++i) acc += hr[i] * V[sv.base + i * ldv + row];
  W[sw.base + row] -= sign * acc;
}

__global__ void k_scale_seg(const Seg* __restrict__ scols, const Seg* __restrict__ dcols,
                            const double* __restrict__ S, const double* __restrict__ scale, double* D) {
  const int c = blockIdx.y;
  const Seg ss = scols[c], sd = dcols[c];
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= sd.len) return;
  D[sd.base + row] = S[ss.base + row] * scale[c];
}

__global__ void k_cast(int64_t count, const double* __restrict__ s, float* d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) d[i] = (float)s[i];
}

__global__ void k_sddmm(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                        int nrhs, const double* __restrict__ lam, int64_t ldl,
                        const double* __restrict__ z, int64_t ldz, double* grad) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  for (int64_t q = ptr[row]; q < ptr[row + 1]; ++q) {
    double s = 0.0;
    for (int r = 0; r < nrhs; ++r) s += lam[r * ldl + row] * z[r * ldz + col[q]];
    grad[q] = -s;
  }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t set_lds_limit(size_t bytes) {
  hipError_t e;
  const int b = (int)bytes;
  if ((e = hipFuncSetAttribute((const void*)k_head<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_c0solve<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_series<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_tail<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_lr_expand<T, T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_lr_expand<T, __hip_bfloat16, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  return hipSuccess;
}

template <typename T>
hipError_t launch_head(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, T* y, int64_t ldy) {
  if (A.gws) hipLaunchKernelGGL((k_head<T, true>), dim3(A.nparts, nrhs), dim3(c.threads), 0, c.stream, A, b, ldb, y, ldy);
  else hipLaunchKernelGGL((k_head<T, false>), dim3(A.nparts, nrhs), dim3(c.threads), c.lds, c.stream, A, b, ldb, y, ldy);
  return hipGetLastError();
}

template <typename T, typename TV>
hipError_t launch_lr_partial(int nchunk, const LrChunk* chunks, int k, const TV* V, const T* y,
                             int64_t ldy, int nrhs, T* partial, hipStream_t s) {
  const int threads = 256;
  size_t lds = sizeof(T) * threads;
  hipLaunchKernelGGL((k_lr_partial<T, TV>), dim3(nchunk, nrhs), dim3(threads), lds, s, chunks, k, V,
                     y, ldy, partial);
  return hipGetLastError();
}

template <typename T, typename TV>
hipError_t launch_lr_expand(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, int k,
                            const TV* V, const T* G, int gtrans, const T* partial, int nchunk,
                            const int32_t* sys_chunk, T* y, int64_t ldy, int do_c0, T* u,
                            int64_t ldu) {
  (void)nchunk;
  if (A.gws)
    hipLaunchKernelGGL((k_lr_expand<T, TV, true>), dim3(A.nparts, nrhs), dim3(c.threads), 0, c.stream,
                       A, k, V, G, gtrans, partial, sys_chunk, y, ldy, do_c0, u, ldu);
  else
    hipLaunchKernelGGL((k_lr_expand<T, TV, false>), dim3(A.nparts, nrhs), dim3(c.threads), c.lds,
                       c.stream, A, k, V, G, gtrans, partial, sys_chunk, y, ldy, do_c0, u, ldu);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c0solve(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* src,
                          int64_t lds_, T* dst, int64_t ldd) {
  if (A.gws)
    hipLaunchKernelGGL((k_c0solve<T, true>), dim3(A.nparts, nrhs), dim3(c.threads), 0, c.stream, A,
                       src, lds_, dst, ldd);
  else
    hipLaunchKernelGGL((k_c0solve<T, false>), dim3(A.nparts, nrhs), dim3(c.threads), c.lds, c.stream,
                       A, src, lds_, dst, ldd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_series(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* y,
                         int64_t ldy, const T* uprev, T* unext, int64_t ldu, int add_y, int do_c0) {
  if (A.gws)
    hipLaunchKernelGGL((k_series<T, true>), dim3(A.nparts, nrhs), dim3(c.threads), 0, c.stream, A, y,
                       ldy, uprev, unext, ldu, add_y, do_c0);
  else
    hipLaunchKernelGGL((k_series<T, false>), dim3(A.nparts, nrhs), dim3(c.threads), c.lds, c.stream,
                       A, y, ldy, uprev, unext, ldu, add_y, do_c0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, const T* u, int64_t ldu, double* z, int64_t ldz) {
  if (A.gws)
    hipLaunchKernelGGL((k_tail<T, true>), dim3(A.nparts, nrhs), dim3(c.threads), 0, c.stream, A, b,
                       ldb, u, ldu, z, ldz);
  else
    hipLaunchKernelGGL((k_tail<T, false>), dim3(A.nparts, nrhs), dim3(c.threads), c.lds, c.stream, A,
                       b, ldb, u, ldu, z, ldz);
  return hipGetLastError();
}

hipError_t launch_spmv(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                       int nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                       const double* bsub, int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, n, ptr, col, val, x, ldx, y,
                     ldy, bsub, ldb);
  return hipGetLastError();
}

hipError_t launch_mdot(int64_t n, int nv, const double* V, int64_t ldv, int64_t ldvr,
                       const double* w, int64_t ldw, int nrhs, int nchunk, double* partial,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(nchunk, nrhs), dim3(512), 0, s, n, nv, V, ldv, ldvr, w, ldw,
                     nchunk, partial);
  return hipGetLastError();
}

hipError_t launch_reduce(int nchunk, int nrhs, int nv, const double* partial, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nv, nrhs), dim3(256), 0, s, nchunk, nrhs, nv, partial, out);
  return hipGetLastError();
}

hipError_t launch_maxpy(int64_t n, int nv, const double* V, int64_t ldv, int64_t ldvr,
                        const double* h, int hld, double* w, int64_t ldw, int nrhs, double sign,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_maxpy, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, n, nv, V, ldv, ldvr, h,
                     hld, w, ldw, sign);
  return hipGetLastError();
}

hipError_t launch_scale(int64_t n, const double* w, int64_t ldw, const double* scale, double* v,
                        int64_t ldv, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, n, w, ldw, scale, v, ldv);
  return hipGetLastError();
}

hipError_t launch_mdot_seg(int ncol, const Seg* vcols, const Seg* wcols, int nv, const double* V,
                           int64_t ldv, const double* W, int nchunk, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot_seg, dim3(nchunk, ncol), dim3(512), 0, s, vcols, wcols, nv, V, ldv, W,
                     nchunk, partial);
  return hipGetLastError();
}

hipError_t launch_maxpy_seg(int ncol, const Seg* vcols, const Seg* wcols, int64_t maxlen, int nv,
                            const double* V, int64_t ldv, const double* h, int hld, double* W,
                            double sign, hipStream_t s) {
  if (maxlen <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maxpy_seg, dim3(nblk(maxlen, 256), ncol), dim3(256), 0, s, vcols, wcols, nv,
                     V, ldv, h, hld, W, sign);
  return hipGetLastError();
}

hipError_t launch_scale_seg(int ncol, const Seg* scols, const Seg* dcols, int64_t maxlen,
                            const double* S, const double* scale, double* D, hipStream_t s) {
  if (maxlen <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_seg, dim3(nblk(maxlen, 256), ncol), dim3(256), 0, s, scols, dcols, S,
                     scale, D);
  return hipGetLastError();
}

hipError_t launch_copy_cast_to_f32(int64_t count, const double* src, float* dst, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast, dim3(nblk(count, 256)), dim3(256), 0, s, count, src, dst);
  return hipGetLastError();
}

hipError_t launch_sddmm(int64_t n, const int64_t* ptr, const int32_t* col, int nrhs,
                        const double* lam, int64_t ldl, const double* z, int64_t ldz,
                        double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_sddmm, dim3(nblk(n, 256)), dim3(256), 0, s, n, ptr, col, nrhs, lam, ldl, z,
                     ldz, grad);
  return hipGetLastError();
}

#define PSLR_INST(T)                                                                             \
  template hipError_t set_lds_limit<T>(size_t);                                                  \
  template hipError_t launch_head<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const double*, \
                                     int64_t, T*, int64_t);                                      \
  template hipError_t launch_c0solve<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const T*,   \
                                        int64_t, T*, int64_t);                                   \
  template hipError_t launch_series<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const T*,    \
                                       int64_t, const T*, T*, int64_t, int, int);                \
  template hipError_t launch_tail<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const double*, \
                                     int64_t, const T*, int64_t, double*, int64_t);

PSLR_INST(double)
PSLR_INST(float)

template hipError_t launch_lr_partial<double, double>(int, const LrChunk*, int, const double*,
                                                      const double*, int64_t, int, double*,
                                                      hipStream_t);
template hipError_t launch_lr_partial<float, float>(int, const LrChunk*, int, const float*,
                                                    const float*, int64_t, int, float*, hipStream_t);
template hipError_t launch_lr_partial<float, __hip_bfloat16>(int, const LrChunk*, int,
                                                             const __hip_bfloat16*, const float*,
                                                             int64_t, int, float*, hipStream_t);
template hipError_t launch_lr_expand<double, double>(const ApplyArrays<double>&, const LaunchCfg&,
                                                     int, int, const double*, const double*, int,
                                                     const double*, int, const int32_t*, double*,
                                                     int64_t, int, double*, int64_t);
template hipError_t launch_lr_expand<float, float>(const ApplyArrays<float>&, const LaunchCfg&, int,
                                                   int, const float*, const float*, int,
                                                   const float*, int, const int32_t*, float*,
                                                   int64_t, int, float*, int64_t);
template hipError_t launch_lr_expand<float, __hip_bfloat16>(
    const ApplyArrays<float>&, const LaunchCfg&, int, int, const __hip_bfloat16*, const float*, int,
    const float*, int, const int32_t*, float*, int64_t, int, float*, int64_t);

}  // namespace pslr
