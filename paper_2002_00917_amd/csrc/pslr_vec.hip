// FP64 vector kernels of the Krylov and Arnoldi processes (flexible GMRES and
// the r_k-step Arnoldi of Algorithm 4), and the gradient SDDMM, for gfx950.
#include "pslr_dev.h"

namespace pslr {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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

// Chunked vector kernels: 256 threads per chunk, each thread owns rows
// r0 + tid + t*256 (t < kRows) of its chunk; vectors go in groups of kUnroll so
// that kUnroll * kRows independent loads are in flight per thread.
#ifndef PSLR_VEC_UNROLL
#define PSLR_VEC_UNROLL 4
#endif
constexpr int kChunkThreads = 256, kRows = (int)((kChunkRows + 255) / 256), kUnroll = PSLR_VEC_UNROLL,
              kDotGroup = 64;
static_assert(kRows * kChunkThreads >= kChunkRows, "chunk longer than one workgroup covers");

// partial[i * nchunk + c] = sum over chunk c's rows of V_i[vbase + row] * W[wbase + row]
__global__ void __launch_bounds__(kChunkThreads)
k_mdot_chunk(const Chunk* __restrict__ ch, const Seg* __restrict__ vcols,
             const Seg* __restrict__ wcols, int nv, const double* __restrict__ V, int64_t ldv,
             const double* __restrict__ W, double* partial) {
  __shared__ double red[kChunkThreads / 64][kDotGroup];
  const Chunk C = ch[blockIdx.x];
  const Seg sv = vcols[C.col], sw = wcols[C.col];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int64_t nrow = C.r1 - C.r0;
  double wreg[kRows];
#pragma unroll
  for (int t = 0; t < kRows; ++t) {
    const int64_t row = tid + (int64_t)t * kChunkThreads;
    wreg[t] = row < nrow ? W[sw.base + C.r0 + row] : 0.0;
  }
  const double* vb = V + sv.base + C.r0;
  for (int i0 = 0; i0 < nv; i0 += kDotGroup) {
    const int ni = min(kDotGroup, nv - i0);
    for (int ii = 0; ii < ni; ii += kUnroll) {
      double acc[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        acc[u] = 0.0;
        if (ii + u < ni) {
          const double* vi = vb + (int64_t)(i0 + ii + u) * ldv;
#pragma unroll
          for (int t = 0; t < kRows; ++t) {
            const int64_t row = tid + (int64_t)t * kChunkThreads;
            if (row < nrow) acc[u] += vi[row] * wreg[t];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const double v = wave_sum(acc[u]);
        if ((tid & 63) == 0 && ii + u < ni) red[wave][ii + u] = v;
      }
    }
    __syncthreads();
    if (tid < ni) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kChunkThreads / 64; ++w) s += red[w][tid];
      partial[(int64_t)(i0 + tid) * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[c * nv + i] = sum of partial[i * nchunk + k] over column c's chunks k
__global__ void k_reduce_chunk(const int32_t* __restrict__ cptr, int nv, int nchunk,
                               const double* __restrict__ partial, double* out) {
  const int i = blockIdx.x, c = blockIdx.y;
  const double* p = partial + (int64_t)i * nchunk;
  double s = 0.0;
  for (int k = cptr[c] + (int)threadIdx.x; k < cptr[c + 1]; k += blockDim.x) s += p[k];
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[(int64_t)c * nv + i] = t;
  }
}

// W[wbase + row] -= sign * sum_i h[col * hld + i] * V_i[vbase + row]; terms with
// h == 0 are skipped (vectors never written may hold stale values)
__global__ void __launch_bounds__(kChunkThreads)
k_maxpy_chunk(const Chunk* __restrict__ ch, const Seg* __restrict__ vcols,
              const Seg* __restrict__ wcols, int nv, const double* __restrict__ V, int64_t ldv,
              const double* __restrict__ h, int hld, double* W, double sign) {
  __shared__ double hs[kDotGroup];
  const Chunk C = ch[blockIdx.x];
  const Seg sv = vcols[C.col], sw = wcols[C.col];
  const int tid = threadIdx.x;
  const int64_t nrow = C.r1 - C.r0;
  const double* hc = h + (int64_t)C.col * hld;
  const double* vb = V + sv.base + C.r0;
  double acc[kRows];
#pragma unroll
  for (int t = 0; t < kRows; ++t) acc[t] = 0.0;
  for (int i0 = 0; i0 < nv; i0 += kDotGroup) {
    const int ni = min(kDotGroup, nv - i0);
    __syncthreads();
    if (tid < ni) hs[tid] = hc[i0 + tid];
    __syncthreads();
    for (int ii = 0; ii < ni; ii += kUnroll) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const double hi = ii + u < ni ? hs[ii + u] : 0.0;
        if (hi != 0.0) {
          const double* vi = vb + (int64_t)(i0 + ii + u) * ldv;
#pragma unroll
          for (int t = 0; t < kRows; ++t) {
            const int64_t row = tid + (int64_t)t * kChunkThreads;
            if (row < nrow) acc[t] += hi * vi[row];
          }
        }
      }
    }
  }
  double* wb = W + sw.base + C.r0;
#pragma unroll
  for (int t = 0; t < kRows; ++t) {
    const int64_t row = tid + (int64_t)t * kChunkThreads;
    if (row < nrow) wb[row] -= sign * acc[t];
  }
}

__global__ void k_scale_chunk(const Chunk* __restrict__ ch, const Seg* __restrict__ scols,
                              const Seg* __restrict__ dcols, const double* __restrict__ S,
                              const double* __restrict__ scale, double* D) {
  const Chunk C = ch[blockIdx.x];
  const Seg ss = scols[C.col], sd = dcols[C.col];
  const double f = scale[C.col];
  for (int64_t row = C.r0 + threadIdx.x; row < C.r1; row += blockDim.x) D[sd.base + row] = S[ss.base + row] * f;
}

// scl[c] = 1 / sqrt(nn[c]) for active columns with nn[c] > 0, else 0
__global__ void k_inv_sqrt(int ncol, const double* __restrict__ nn, const uint8_t* __restrict__ active,
                           double* scl) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double v = nn[c];
  scl[c] = (active[c] && v > 0.0) ? 1.0 / sqrt(v) : 0.0;
}

// Vn[:, c] = sum_j V[:, j] W_s[j, c] (c < ncols) on the rows of the listed
// chunks, whose column index is the system s; W holds one mcols x ncols
// column-major matrix per system.  The basis change of a Krylov-Schur restart.
constexpr int kRotTile = 8;
__global__ void k_basis_rotate(const Chunk* __restrict__ ch, const Seg* __restrict__ cols, int mcols,
                               int ncols, const double* __restrict__ V, int64_t ldv,
                               const double* __restrict__ W, double* Vn, int64_t ldn) {
  const Chunk C = ch[blockIdx.x];
  const Seg sg = cols[C.col];
  const double* Ws = W + (int64_t)C.col * mcols * ncols;
  for (int64_t r = C.r0 + threadIdx.x; r < C.r1; r += blockDim.x) {
    const int64_t row = sg.base + r;
    for (int c0 = 0; c0 < ncols; c0 += kRotTile) {
      double acc[kRotTile];
#pragma unroll
      for (int t = 0; t < kRotTile; ++t) acc[t] = 0.0;
      for (int j = 0; j < mcols; ++j) {
        const double v = V[(int64_t)j * ldv + row];
#pragma unroll
        for (int t = 0; t < kRotTile; ++t)
          if (c0 + t < ncols) acc[t] += v * Ws[(int64_t)(c0 + t) * mcols + j];
      }
#pragma unroll
      for (int t = 0; t < kRotTile; ++t)
        if (c0 + t < ncols) Vn[(int64_t)(c0 + t) * ldn + row] = acc[t];
    }
  }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_mdot_chunk(int nchunk, const Chunk* ch, const Seg* vcols, const Seg* wcols, int nv,
                             const double* V, int64_t ldv, const double* W, double* partial,
                             hipStream_t s) {
  if (nchunk <= 0 || nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mdot_chunk, dim3(nchunk), dim3(kChunkThreads), 0, s, ch, vcols, wcols, nv, V,
                     ldv, W, partial);
  return hipGetLastError();
}

hipError_t launch_reduce_chunk(int ncol, const int32_t* cptr, int nv, int nchunk,
                               const double* partial, double* out, hipStream_t s) {
  if (ncol <= 0 || nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_chunk, dim3(nv, ncol), dim3(256), 0, s, cptr, nv, nchunk, partial, out);
  return hipGetLastError();
}

hipError_t launch_maxpy_chunk(int nchunk, const Chunk* ch, const Seg* vcols, const Seg* wcols,
                              int nv, const double* V, int64_t ldv, const double* h, int hld,
                              double* W, double sign, hipStream_t s) {
  if (nchunk <= 0 || nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maxpy_chunk, dim3(nchunk), dim3(kChunkThreads), 0, s, ch, vcols, wcols, nv, V,
                     ldv, h, hld, W, sign);
  return hipGetLastError();
}

hipError_t launch_inv_sqrt(int ncol, const double* nn, const uint8_t* active, double* scl,
                           hipStream_t s) {
  if (ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inv_sqrt, dim3(nblk(ncol, 256)), dim3(256), 0, s, ncol, nn, active, scl);
  return hipGetLastError();
}

hipError_t launch_scale_chunk(int nchunk, const Chunk* ch, const Seg* scols, const Seg* dcols,
                              const double* S, const double* scale, double* D, hipStream_t s) {
  if (nchunk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_chunk, dim3(nchunk), dim3(kChunkThreads), 0, s, ch, scols, dcols, S,
                     scale, D);
  return hipGetLastError();
}

hipError_t launch_basis_rotate(int nchunk, const Chunk* ch, const Seg* cols, int mcols, int ncols,
                               const double* V, int64_t ldv, const double* W, double* Vn, int64_t ldn,
                               hipStream_t s) {
  if (nchunk <= 0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_basis_rotate, dim3(nchunk), dim3(kChunkThreads), 0, s, ch, cols, mcols, ncols, V,
                     ldv, W, Vn, ldn);
  return hipGetLastError();
}

hipError_t launch_spmv(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                       int nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                       const double* bsub, int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, n, ptr, col, val, x, ldx, y,
                     ldy, bsub, ldb);
  return hipGetLastError();
}

hipError_t launch_sddmm(int64_t n, const int64_t* ptr, const int32_t* col, int nrhs,
                        const double* lam, int64_t ldl, const double* z, int64_t ldz,
                        double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_sddmm, dim3(nblk(n, 256)), dim3(256), 0, s, n, ptr, col, nrhs, lam, ldl, z,
                     ldz, grad);
  return hipGetLastError();
}

}  // namespace pslr
