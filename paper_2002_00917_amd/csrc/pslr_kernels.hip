// HIP kernels of the PSLR preconditioner apply (paper Algorithm 3), for gfx950.
//
// Design: one workgroup owns one subdomain and one tile of right-hand sides
// and keeps that subdomain's working vectors in LDS (or, when they do not fit,
// in a global workspace).  The B_i and C_i solves are level-scheduled over the
// supernodal elimination tree of an exact LU factorisation; every level is two
// sweeps of lane-per-row dense products: L right-looking (inverted diagonal
// triangles, then column panels pushed into the ancestor rows), U left-looking
// (row panels pulled from the ancestor rows, then the inverted triangles).
// Factor data streams from HBM once, coalesced; vector operands are LDS
// broadcasts.  The coupling SpMVs with E, F and C_g are fused into the kernels
// that produce or consume their operands, so one power-series step of
// eq. approx1 is one launch.
#include "pslr_dev.h"

#include <hip/hip_ext.h>

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

// Vectors of a workgroup hold a tile of R right-hand sides interleaved:
// element (position p, rhs r) at X[p * R + r].  Each factor entry is loaded
// once and applied to all R of them.

template <typename T, int R>
__device__ __forceinline__ void group_sum_r(T (&acc)[R], int G) {
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = group_sum(acc[r], G);
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* addr, T v) {
  unsafeAtomicAdd(addr, v);
}

// Chunk counts of a level, scaled by 2^gshift (the setup autotuner's knob).
__device__ __forceinline__ void level_chunks(int c, int gshift, int& CT, int& CP) {
  CT = c & 0xff;
  CP = (c >> 8) & 0xff;
  if (gshift > 0) {
    CT = min(255, CT << gshift);
    CP = min(255, CP << gshift);
  } else if (gshift < 0) {
    CT = max(1, CT >> -gshift);
    CP = max(1, CP >> -gshift);
  }
}

// Dense factor blocks store their columns in interleaved pairs (2c, 2c + 1),
// so that one 16-byte (FP64) or 8-byte (FP32) load brings a lane two columns.
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

#ifndef PSLR_PAIR_U
#define PSLR_PAIR_U 4
#endif

// acc[r] += sum over the columns of pairs c = c0 + d * t, 0 <= t < np (d = +1
// or -1), of M(j) * S[j * R + r]: one lane's share of a dense product.  Lanes
// of a supernode start at the same pair and walk in step, so consecutive lanes
// (consecutive rows) read consecutive pairs while their counts np differ; S is
// the same for all of them.  The pair at walk index half_t (-1: none) holds one
// column only: its second stored value is a zero (across the diagonal, or
// padding), and S is read at its first column instead of the second, which
// the lane does not own.
// The walk uses 32-bit pair indices from a block-uniform base (so that every
// load is a uniform base plus a 32-bit lane offset): pair t of
// the walk is Mb[o_t] with o_{t+1} = o_t + delta_t and delta_{t+1} = delta_t +
// dd (a triangle's column pairs are a quadratic sequence, a panel's an
// arithmetic one); its columns are S[t * ds] and S[t * ds + R] (S[t * ds]
// twice at t = half_t).
// base[idx] with a 32-bit byte offset, so that the load can take the form
// "uniform base + 32-bit lane offset" (a block's packed arrays stay below 4 GiB)
template <typename V>
__device__ __forceinline__ V ld32(const V* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(V)));
}

template <typename T, int R>
__device__ __forceinline__ void pair_walk(const typename Pair<T>::type* __restrict__ Mb, uint32_t o,
                                          int delta, int dd, int np, int half_t, const T* S, int ds,
                                          T (&acc)[R]) {
  constexpr int U = R == 1 ? PSLR_PAIR_U : 2;
  int t = 0;
  for (; t + U <= np; t += U) {
    typename Pair<T>::type v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ld32(Mb, o);
      o += (uint32_t)delta;
      delta += dd;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* s = S + (t + u) * ds;
      const int k2 = t + u == half_t ? 0 : R;
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += v[u].x * s[r] + v[u].y * s[k2 + r];
    }
  }
  if (t < np) {
    // last round masked: slots past np re-read pair np - 1, products dropped
    typename Pair<T>::type v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ld32(Mb, o);
      const bool adv = t + u + 1 < np;
      o += adv ? (uint32_t)delta : 0u;
      delta += adv ? dd : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tu = min(t + u, np - 1);
      const T* s = S + tu * ds;
      const int k2 = tu == half_t ? 0 : R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T a = v[u].x * s[r] + v[u].y * s[k2 + r];
        acc[r] += t + u < np ? a : (T)0;
      }
    }
  }
}

// even chunk length covering len in C chunks
__device__ __forceinline__ int pair_chunk(int len, int C) { return (((len + C - 1) / C) + 1) & ~1; }

// Entry-form off-diagonal part of a level: for e in [e0, e1),
// D[dst(e)] -= v[e] * S[src(e)] with atomic adds.  Every entry is one 16-byte
// record (value, target/source position, level-local row), loaded with one
// instruction; each thread keeps U of them in flight.
#ifndef PSLR_ENT_U
#define PSLR_ENT_U 4
#endif

template <typename T, int R>
__device__ __forceinline__ void entry_sweep(const double2* __restrict__ er, int e0, int e1, T* D,
                                            const T* S, bool lower) {
  constexpr int U = PSLR_ENT_U;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int e = e0 + tid; e < e1; e += U * nthr) {
    // unconditional loads and adds, so that the compiler keeps all U loads in
    // flight together instead of sinking each into a branch of its own: a
    // slot past e1 re-reads the thread's own entry e and adds zero (to the
    // target of that entry, so that such slots do not all meet on one address)
    double2 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = er[e + u * nthr < e1 ? e + u * nthr : e];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T v = e + u * nthr < e1 ? (T)q[u].x : (T)0;
      // second half: lower: (target position, level-local source row);
      // upper: (source position, level-local target row)
      const int a = __double2loint(q[u].y), c = __double2hiint(q[u].y);
      const int d = lower ? a : c, s = lower ? c : a;
#pragma unroll
      for (int r = 0; r < R; ++r) atomic_add(&D[d * R + r], -v * S[s * R + r]);
    }
  }
}

// Solve one packed triangular factor of block `bi` in place on the vector tile
// X (positions 0..n-1, R right-hand sides).  Rb is scratch of 2 * max_lrows * R
// entries (halves alternating over the levels).  All threads of the workgroup
// must call it; it ends with a barrier.
//
// The panels are folded with the inverted triangles (see TriPacked), so each
// level is one step between two barriers over values from before the level.
// Lower factors run right-looking: every row item forms s_k = sum_j Tinv(i, j)
// x[f + j] into the level's half of Rb while every push item subtracts
// Pf(a, :) x[f ..] from x[ridx[a]] (atomic adds: supernodes of a level may
// update the same rows); the level's s goes into x during the next level,
// which reads none of its rows.  Upper factors run left-looking: x[p] =
// sum_j Tinv(i, j) r_j - sum_a Pf(i, a) x[ridx[a]] with r the level's rows
// before the level, copied into Rb one level ahead; where a level's products
// are chunked or in entry form, x[p] starts at zero and every part adds
// atomically.  Inner loops are split into CT / CP chunks whose partial sums
// meet through atomic adds; levels of narrow supernodes use the entry form
// instead of panels.
//
// Records do not depend on x, so each thread's first record of a level is
// loaded before the barrier that precedes the level, and the record of its
// next task while it works on the current one.
template <typename T, int R, bool GX>
__device__ void tri_solve(const TriArrays<T>& A, int bi, T* X, T* Rb, int gshift) {
  const DevTriBlock B = A.blk[bi];
  if (B.nlev <= 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int4* rec = A.rec + 2 * B.rec_base;
  const int4* prec = A.prec + B.prec_base;
  const T* pan = A.val + B.val_base;
  const int32_t* ridx = A.ridx + B.ridx_base;
  const T* tri = A.tri + B.tri_base;
  const int32_t* lev_ptr = A.lev_ptr + B.lev_base;
  const int32_t* push_ptr = A.push_ptr + B.lev_base;
  const int32_t* ent_ptr = A.ent_ptr + B.lev_base;
  const double2* ent_rec = A.ent + B.ent_base;
  const int32_t* lev_c = A.lev_c + B.lev_base;
  const int64_t RS = (int64_t)R * B.max_lrows;
  // entry form for FP64 single right-hand sides in LDS (one atomic add per
  // entry; in FP32 the two indices per value cost more than they save)
  auto use_ent = [&](int l) __attribute__((always_inline)) { return sizeof(T) == 8 && R == 1 && !GX && ((lev_c[l] >> 16) & 1); };
  // first row record of this thread in the coming level: row tid % cnt
  // (records past the end of a level keep the previous values, never used)
  int4 f0 = make_int4(0, 0, 0, 0), f1 = f0;
  {
    const int l0 = B.lower ? 0 : B.nlev - 1;
    const int b0 = lev_ptr[l0], c0 = lev_ptr[l0 + 1] - b0;
    if (c0 > 0) {
      f0 = rec[2 * (b0 + tid % c0)];
      f1 = rec[2 * (b0 + tid % c0) + 1];
    }
  }
  if (B.lower) {
    // two halves of the scratch alternate over the levels: level l's results
    // go to half l & 1 while the other half (level l - 1's results) is copied
    // into x and, when level l + 1 accumulates chunks, cleared for it
    int bp = 0, cntp = 0, pfx = 0;  // the previous level's rows and this thread's first position
    T* Rp = Rb + RS;
    for (int l = 0; l < B.nlev; ++l) {
      const int b = lev_ptr[l];
      const int cnt = lev_ptr[l + 1] - b;
      int CT, CP;
      level_chunks(lev_c[l], gshift, CT, CP);
      const bool ent = use_ent(l);
      T* Rc = Rb + (l & 1) * RS;
      int bn = 0, cntn = 0, CTn = 1, CPn = 1;
      if (l + 1 < B.nlev) {
        bn = lev_ptr[l + 1];
        cntn = lev_ptr[l + 2] - bn;
        level_chunks(lev_c[l + 1], gshift, CTn, CPn);
      }
      if (l == 0 && CT > 1) {
        for (int e = tid; e < cnt * R; e += nthr) Rc[e] = (T)0;
        __syncthreads();
      }
      const int pb = push_ptr[l], np = ent ? 0 : push_ptr[l + 1] - pb;
      int4 fq = f0;
      if (np > 0) fq = prec[pb + tid % np];
      // the previous level's results into x, then (by the same thread, after
      // its read) that half cleared for the next level when its triangle items
      // are chunked
      {
        const int kz = CTn > 1 ? cntn : 0;
        for (int k = tid; k < max(cntp, kz); k += nthr) {
          if (k < cntp) {
            const int p = k == tid ? pfx : rec[2 * (bp + k)].x;
#pragma unroll
            for (int r = 0; r < R; ++r) X[p * R + r] = Rp[k * R + r];
          }
          if (k < kz)
#pragma unroll
            for (int r = 0; r < R; ++r) Rp[k * R + r] = (T)0;
        }
      }
      // s_k = Tinv(i, 0..i) x[f .. f+i]
      {
        int4 r0 = f0, r1 = f1;
        for (int t = tid; t < cnt * CT; t += nthr) {
          const int tn = t + nthr;
          int4 n0 = r0, n1 = r1;
          if (tn < cnt * CT) {
            n0 = rec[2 * (b + tn % cnt)];
            n1 = rec[2 * (b + tn % cnt) + 1];
          }
          const int c = t / cnt, k = t - c * cnt;
          const int i = r0.y, w = r0.z;
          const int Lc = pair_chunk(w, CT);
          const int j0 = c * Lc, j1 = min(w, j0 + Lc);
          T acc[R];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = 0;
          // columns j0 .. min(j1, i + 1) - 1; pair c of a lower triangle holds
          // rows 2c .. w-1 at pair index c (w - c + 1) + (i - 2c)
          const int ncol = min(j1, i + 1) - j0;
          if (ncol > 0) {
            const int c0 = j0 >> 1;
            const uint32_t o = (uint32_t)(r1.x >> 1) + (uint32_t)(c0 * (w - c0 + 1) + (i - 2 * c0));
            const T* S = X + (int64_t)(r0.x - i + 2 * c0) * R;
            const int npr = (ncol + 1) >> 1;
            pair_walk<T, R>(reinterpret_cast<const typename Pair<T>::type*>(tri), o, w - 2 * c0 - 2, -2, npr,
                            (ncol & 1) ? npr - 1 : -1, S, 2 * R, acc);
          }
          if (CT == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) Rc[k * R + r] = acc[r];
          } else if (j0 <= i) {
#pragma unroll
            for (int r = 0; r < R; ++r) atomic_add(&Rc[k * R + r], acc[r]);
          }
          r0 = n0;
          r1 = n1;
        }
      }
      // x[ridx[a]] -= Pf(a, :) x[f ..]
      if (ent) entry_sweep<T, R>(ent_rec, ent_ptr[l], ent_ptr[l + 1], X, X, true);
      {
        int4 q = fq;
        for (int t = tid; t < np * CP; t += nthr) {
          const int tn = t + nthr;
          const int4 qn = tn < np * CP ? prec[pb + tn % np] : q;
          const int c = t / np;
          const int w = q.z & 0xffff, h = q.z >> 16;
          const int Lc = pair_chunk(w, CP);
          const int j0 = c * Lc, j1 = min(w, j0 + Lc);
          if (j0 < j1) {
            T acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = 0;
            // panel row a: pair c at pair index q.y + c h
            const int c0 = j0 >> 1;
            const T* S = X + (int64_t)(q.w + 2 * c0) * R;
            const int ncol = j1 - j0;
            const int npr = (ncol + 1) >> 1;
            pair_walk<T, R>(reinterpret_cast<const typename Pair<T>::type*>(pan), (uint32_t)(q.y + c0 * h), h, 0,
                            npr, (ncol & 1) ? npr - 1 : -1, S, 2 * R, acc);
#pragma unroll
            for (int r = 0; r < R; ++r) atomic_add(&X[q.x * R + r], -acc[r]);
          }
          q = qn;
        }
      }
      bp = b;
      cntp = cnt;
      pfx = f0.x;
      Rp = Rc;
      if (cntn > 0) {
        f0 = rec[2 * (bn + tid % cntn)];
        f1 = rec[2 * (bn + tid % cntn) + 1];
      }
      __syncthreads();
    }
    for (int k = tid; k < cntp; k += nthr) {
      const int p = k == tid ? pfx : rec[2 * (bp + k)].x;
#pragma unroll
      for (int r = 0; r < R; ++r) X[p * R + r] = Rp[k * R + r];
    }
    __syncthreads();
    return;
  }
  // upper: levels from the top; Rc holds the level's rows before the level
  auto joint = [&](int l) __attribute__((always_inline)) {
    int ct, cp;
    level_chunks(lev_c[l], gshift, ct, cp);
    return ct == 1 && cp == 1 && !use_ent(l);
  };
  {
    const int l = B.nlev - 1;
    const int b = lev_ptr[l], cnt = lev_ptr[l + 1] - b;
    const bool jn = joint(l);
    for (int k = tid; k < cnt; k += nthr) {
      const int p = k == tid ? f0.x : rec[2 * (b + k)].x;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Rb[k * R + r] = X[p * R + r];
        if (!jn) X[p * R + r] = (T)0;
      }
    }
    __syncthreads();
  }
  for (int li = 0; li < B.nlev; ++li) {
    const int l = B.nlev - 1 - li;
    const int b = lev_ptr[l];
    const int cnt = lev_ptr[l + 1] - b;
    int CT, CP;
    level_chunks(lev_c[l], gshift, CT, CP);
    const bool ent = use_ent(l);
    const bool jn = CT == 1 && CP == 1 && !ent;
    T* Rc = Rb + (li & 1) * RS;
    T* Rn = Rb + ((li + 1) & 1) * RS;
    int bn = 0, cntn = 0;
    if (l > 0) {
      bn = lev_ptr[l - 1];
      cntn = lev_ptr[l] - bn;
    }
    // the triangle part of row item t of chunk c over columns [j0, j1)
    auto tri_part = [&](int4 r0, int4 r1, int c, int CTc, T (&acc)[R]) __attribute__((always_inline)) {
      const int i = r0.y, w = r0.z;
      const int Lc = pair_chunk(w, CTc);
      const int j0 = c * Lc, j1 = min(w, j0 + Lc);
      // columns j1-1 down to jlo = max(j0, i), a common start for the lanes;
      // pair c of an upper triangle holds rows 0 .. 2c+1 at pair index
      // c (c + 1) + i (entries left of the diagonal are zeros).  An odd j1
      // (= w) leaves the top pair with one column.
      const int jlo = max(j0, i);
      const int top = (j1 & 1) ? (j1 >> 1) : (j1 >> 1) - 1;
      const int npr = jlo < j1 ? top - (jlo >> 1) + 1 : 0;
      const T* S = Rc + (int64_t)(r1.w + 2 * top) * R;
      const uint32_t o = (uint32_t)(r1.x >> 1) + (uint32_t)(top * (top + 1) + i);
      if (npr > 0)
        pair_walk<T, R>(reinterpret_cast<const typename Pair<T>::type*>(tri), o, -2 * top, 2, npr,
                        (j1 & 1) ? 0 : -1, S, -2 * R, acc);
      return j1 > i;
    };
    // the panel part: acc += Pf(i, a0 .. a1-1) x[ridx[a0 .. a1-1]]
    auto pan_part = [&](int4 r0, int4 r1, int c, int CPc, T (&acc)[R]) __attribute__((always_inline)) {
      const int i = r0.y, w = r0.z, h = r0.w;
      const int Lc = pair_chunk(h, CPc);
      const int a0 = c * Lc, a1 = min(h, a0 + Lc);
      // row i: pair g (columns 2g, 2g + 1) at pair index g w + i, positions
      // ridx[2g], ridx[2g + 1] (an odd last column pairs with a zero value
      // and a repeated position)
      // (32-bit pair indices from the block-uniform bases pan and ridx)
      const auto* pc = reinterpret_cast<const typename Pair<T>::type*>(pan);
      const int2* rc = reinterpret_cast<const int2*>(ridx);
      const uint32_t pbase = (uint32_t)((r1.y >> 1) + i), rbase = (uint32_t)(r1.z >> 1);
      constexpr int U = R == 1 ? PSLR_PAIR_U : 2;
      int g = a0 >> 1;
      const int g1 = (a1 + 1) >> 1;
      for (; g + U <= g1; g += U) {
        typename Pair<T>::type v[U];
        int2 cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          v[u] = ld32(pc, pbase + (uint32_t)((g + u) * w));
          cc[u] = ld32(rc, rbase + (uint32_t)(g + u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] += v[u].x * X[cc[u].x * R + r] + v[u].y * X[cc[u].y * R + r];
      }
      if (g < g1) {
        // last round masked (slots past g1 re-read pair g1 - 1, products dropped)
        typename Pair<T>::type v[U];
        int2 cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          v[u] = ld32(pc, pbase + (uint32_t)(min(g + u, g1 - 1) * w));
          cc[u] = ld32(rc, rbase + (uint32_t)min(g + u, g1 - 1));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const T a = v[u].x * X[cc[u].x * R + r] + v[u].y * X[cc[u].y * R + r];
            acc[r] += g + u < g1 ? a : (T)0;
          }
      }
      return a0 < a1;
    };
    if (jn) {
      // one item per row: x[p] = Tinv(i, :) r - Pf(i, :) x[ridx]
      int4 r0 = f0, r1 = f1;
      for (int t = tid; t < cnt; t += nthr) {
        const int tn = t + nthr;
        int4 n0 = r0, n1 = r1;
        if (tn < cnt) {
          n0 = rec[2 * (b + tn)];
          n1 = rec[2 * (b + tn) + 1];
        }
        T at[R], ap[R];
#pragma unroll
        for (int r = 0; r < R; ++r) at[r] = ap[r] = 0;
        tri_part(r0, r1, 0, 1, at);
        pan_part(r0, r1, 0, 1, ap);
#pragma unroll
        for (int r = 0; r < R; ++r) X[r0.x * R + r] = at[r] - ap[r];
        r0 = n0;
        r1 = n1;
      }
    } else {
      {
        int4 r0 = f0, r1 = f1;
        for (int t = tid; t < cnt * CT; t += nthr) {
          const int tn = t + nthr;
          int4 n0 = r0, n1 = r1;
          if (tn < cnt * CT) {
            n0 = rec[2 * (b + tn % cnt)];
            n1 = rec[2 * (b + tn % cnt) + 1];
          }
          T acc[R];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = 0;
          if (tri_part(r0, r1, t / cnt, CT, acc))
#pragma unroll
            for (int r = 0; r < R; ++r) atomic_add(&X[r0.x * R + r], acc[r]);
          r0 = n0;
          r1 = n1;
        }
      }
      if (ent) {
        entry_sweep<T, R>(ent_rec, ent_ptr[l], ent_ptr[l + 1], X, X, false);
      } else {
        int4 r0 = f0, r1 = f1;
        for (int t = tid; t < cnt * CP; t += nthr) {
          const int tn = t + nthr;
          int4 n0 = r0, n1 = r1;
          if (tn < cnt * CP) {
            n0 = rec[2 * (b + tn % cnt)];
            n1 = rec[2 * (b + tn % cnt) + 1];
          }
          T acc[R];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = 0;
          if (pan_part(r0, r1, t / cnt, CP, acc))
#pragma unroll
            for (int r = 0; r < R; ++r) atomic_add(&X[r0.x * R + r], -acc[r]);
          r0 = n0;
          r1 = n1;
        }
      }
    }
    // the next level's rows before it into Rn (cleared in x where its parts
    // add atomically); its first records
    if (cntn > 0) {
      f0 = rec[2 * (bn + tid % cntn)];
      f1 = rec[2 * (bn + tid % cntn) + 1];
      const bool jnn = joint(l - 1);
      for (int k = tid; k < cntn; k += nthr) {
        const int p = k == tid ? f0.x : rec[2 * (bn + k)].x;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Rn[k * R + r] = X[p * R + r];
          if (!jnn) X[p * R + r] = (T)0;
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
struct Lds {
  T *XB, *Rb, *XC, *U, *W;
};

// Working vectors of block blockIdx.x for the right-hand-side tile blockIdx.y:
// in LDS, or (GX) in the handle's global workspace when a subdomain does not
// fit.  Global layout of one tile: [X_B: p][X_C: q][U: q][scratch: sum of
// per-block level sizes][W: 2k per block], every element an R-vector.
template <typename T, int R, bool GX>
__device__ Lds<T> carve(const ApplyArrays<T>& A) {
  Lds<T> L;
  if (GX) {
    const int i = blockIdx.x, t = blockIdx.y;
    T* base = reinterpret_cast<T*>(A.gws) + (int64_t)t * R * A.gws_stride;
    L.XB = base + R * A.int_ptr[i];
    L.XC = base + R * (A.p + A.if_ptr[i]);
    L.U = base + R * (A.p + A.q + A.if_ptr[i]);
    L.Rb = base + R * (A.p + 2 * A.q + A.rb_off[i]);
    L.W = base + R * (A.p + 2 * A.q + A.rb_off[A.nparts] + (int64_t)i * 2 * A.kmax);
  } else {
    extern __shared__ __align__(16) unsigned char smem[];
    L.XB = reinterpret_cast<T*>(smem);
    L.Rb = L.XB + R * A.maxPB;
    L.XC = L.Rb + 2 * R * A.maxLR;
    L.U = L.XC + R * A.maxQB;
    L.W = L.U + R * A.maxQB;
  }
  return L;
}

// right-hand sides r0 .. r0 + nr - 1 of this workgroup's tile; false when the
// whole tile is masked out (converged FGMRES columns)
template <typename T, int R>
__device__ __forceinline__ bool tile_rhs(const ApplyArrays<T>& A, int nrhs, int i, int& r0, int& nr) {
  r0 = blockIdx.y * R;
  nr = min(R, nrhs - r0);
  if (!A.active) return true;
  const int s = A.part_sys[i];
  for (int r = 0; r < nr; ++r)
    if (A.active[(r0 + r) * A.nsys + s]) return true;
  return false;
}

// t = B^{-1} f;  y = g - F t   (Algorithm 3, line 2)
template <typename T, int R, bool GX>
__global__ void __launch_bounds__(1024) k_head(ApplyArrays<T> A, int nrhs, const double* __restrict__ b,
                                               int64_t ldb, T* y, int64_t ldy) {
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, R>(A, nrhs, i, r0, nr)) return;
  Lds<T> L = carve<T, R, GX>(A);
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  for (int64_t e = tid; e < pi * R; e += nt) {
    const int64_t p = e / R;
    const int r = (int)(e - p * R);
    L.XB[e] = r < nr ? (T)b[(r0 + r) * ldb + A.gB_in[i0 + p]] : (T)0;
  }
  __syncthreads();
  tri_solve<T, R, GX>(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UB, i, L.XB, L.Rb, A.gshift);
  for (int64_t k = tid; k < qi; k += nt) {
    const int64_t row = f0 + k;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = r < nr ? (T)b[(r0 + r) * ldb + A.if_orig[row]] : (T)0;
    for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q) {
      const T v = A.Fout.val[q];
      const int c = A.Fout.col[q];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] -= v * L.XB[c * R + r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nr) y[(r0 + r) * ldy + row] = acc[r];
  }
}

// partial[(chunk * nrhs + r) * k + j] = sum over the chunk's rows of V[j][row] y_r[row]
// (V^T y, Algorithm 3 line 3).  V is column-major.  Tiles of 64 rows x 64
// columns are staged through LDS (loads coalesced along the rows, rows padded
// to 65 entries so that column reads are conflict free); thread (g, j) then
// sums 16 rows of column j, and the four row groups meet in LDS at the end.
constexpr int kLrThreads = 256, kLrTile = 64;

template <typename T, typename TV>
__global__ void __launch_bounds__(kLrThreads)
k_lr_partial(const LrChunk* __restrict__ chunks, int k, const TV* __restrict__ V, int64_t ldv,
             const T* __restrict__ y, int64_t ldy, T* partial, const uint8_t* __restrict__ active,
             int nsys) {
  __shared__ T tile[kLrTile * (kLrTile + 1)];
  __shared__ T ys[kLrTile];
  const int chunk = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const LrChunk C = chunks[chunk];
  if (active && !active[r * nsys + C.sys]) return;
  const int jl = tid & (kLrTile - 1), g = tid >> 6;  // column in block, row group (0..3)
  for (int jb = 0; jb < k; jb += kLrTile) {
    const int nj = min(kLrTile, k - jb);
    T acc = 0;
    for (int64_t t0 = C.r0; t0 < C.r1; t0 += kLrTile) {
      const int nr = (int)min<int64_t>(kLrTile, C.r1 - t0);
      // load: lane = row of the tile, 16 columns per thread
#pragma unroll
      for (int m = 0; m < kLrTile / 4; ++m) {
        const int j = g + 4 * m;
        tile[j * (kLrTile + 1) + jl] =
            (j < nj && jl < nr) ? (T)tv_to_float(V[(int64_t)(jb + j) * ldv + t0 + jl]) : (T)0;
      }
      if (tid < kLrTile) ys[tid] = tid < nr ? y[r * ldy + t0 + tid] : (T)0;
      __syncthreads();
      const T* tj = tile + jl * (kLrTile + 1) + g * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) acc += tj[q] * ys[g * 16 + q];
      __syncthreads();
    }
    tile[g * kLrTile + jl] = acc;
    __syncthreads();
    if (tid < nj) {
      const T s = tile[tid] + tile[kLrTile + tid] + tile[2 * kLrTile + tid] + tile[3 * kLrTile + tid];
      partial[((int64_t)chunk * gridDim.y + r) * k + jb + tid] = s;
    }
    __syncthreads();
  }
}

// ---- the low-rank term for one right-hand side (Algorithm 3, line 3):
// y += V (G (V^T y)) in three launches that spread V over the whole chip.
// V column-major (ldv); a column's rows are contiguous, so lanes run along
// the rows in both products.
//  1. partial[c * k + j] = sum over chunk c's rows of V[row][j] y[row]:
//     workgroup (c, block of 16 columns), wave w the columns 4w .. 4w + 3 of
//     the block; every lane keeps all its loads of the chunk in flight.
//  2. z_s = G_s W_s (or G_s^T W_s), W_s the sum of system s's chunk
//     partials, in column slices that meet in LDS.
//  3. y[row] += V[row, :] z_s: workgroup (c, block of 64 rows), wave w the
//     w-th quarter of the columns, lanes along the rows; the waves meet in LDS.
constexpr int kLr1Cols = 16;
constexpr int kLr1Rows = 64;

template <typename T, typename TV>
__global__ void __launch_bounds__(256) k_lr1_partial(const LrChunk* __restrict__ chunks, int k,
                                                     const TV* __restrict__ V, int64_t ldv,
                                                     const T* __restrict__ y, T* partial,
                                                     const uint8_t* __restrict__ active) {
  __shared__ T ys[kLrChunkRows];
  const LrChunk C = chunks[blockIdx.x];
  if (active && !active[C.sys]) return;
  const int nr = (int)(C.r1 - C.r0);
  for (int t = threadIdx.x; t < nr; t += blockDim.x) ys[t] = y[C.r0 + t];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int jb = blockIdx.y * kLr1Cols + 4 * w;
  if (jb >= k) return;
  const TV* Vc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) Vc[u] = V + (int64_t)min(jb + u, k - 1) * ldv + C.r0;
  T acc[4] = {(T)0, (T)0, (T)0, (T)0};
  constexpr int S = 4;  // rows per lane per round: 16 loads in flight
  for (int t = lane; t < nr; t += 64 * S) {
    TV v[S][4];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int ts = min(t + 64 * s, nr - 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) v[s][u] = Vc[u][ts];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const T yv = t + 64 * s < nr ? ys[t + 64 * s] : (T)0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += (T)tv_to_float(v[s][u]) * yv;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = group_sum(acc[u], 64);
  if (lane == 0)
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (jb + u < k) partial[(int64_t)blockIdx.x * k + jb + u] = acc[u];
}

template <typename T>
__global__ void __launch_bounds__(1024) k_lr1_gz(int k, const T* __restrict__ Gall, int gtrans,
                                                 const T* __restrict__ partial,
                                                 const int32_t* __restrict__ sys_chunk, T* zout,
                                                 const uint8_t* __restrict__ active) {
  __shared__ T W[256];
  __shared__ T red[1024];
  const int s = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  if (active && !active[s]) return;
  const int c0 = sys_chunk[s], c1 = sys_chunk[s + 1];
  const int S = max(1, min(nt / max(k, 1), 32));  // slices of the summation range
  const int j = tid % k, sl = tid / k;
  // eight independent partial sums per thread keep eight loads in flight
  constexpr int UG = 8;
  {
    T a[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) a[u] = (T)0;
    if (sl < S) {
      int c = c0 + sl;
      for (; c + (UG - 1) * S < c1; c += UG * S)
#pragma unroll
        for (int u = 0; u < UG; ++u) a[u] += partial[(int64_t)(c + u * S) * k + j];
      for (; c < c1; c += S) a[0] += partial[(int64_t)c * k + j];
    }
    T t = (T)0;
#pragma unroll
    for (int u = 0; u < UG; ++u) t += a[u];
    red[tid] = t;
  }
  __syncthreads();
  if (tid < k) {
    T a = (T)0;
    for (int t = 0; t < S; ++t) a += red[t * k + tid];
    W[tid] = a;
  }
  __syncthreads();
  const T* G = Gall + (int64_t)s * k * k;
  {
    T a[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) a[u] = (T)0;
    if (sl < S) {
      int l = sl;
      for (; l + (UG - 1) * S < k; l += UG * S)
#pragma unroll
        for (int u = 0; u < UG; ++u) {
          const int lu = l + u * S;
          a[u] += (gtrans ? G[(int64_t)lu * k + j] : G[(int64_t)j * k + lu]) * W[lu];
        }
      for (; l < k; l += S) a[0] += (gtrans ? G[(int64_t)l * k + j] : G[(int64_t)j * k + l]) * W[l];
    }
    T t = (T)0;
#pragma unroll
    for (int u = 0; u < UG; ++u) t += a[u];
    red[tid] = t;
  }
  __syncthreads();
  if (tid < k) {
    T a = (T)0;
    for (int t = 0; t < S; ++t) a += red[t * k + tid];
    zout[(int64_t)s * k + tid] = a;
  }
}

template <typename T, typename TV>
__global__ void __launch_bounds__(256) k_lr1_expand(const LrChunk* __restrict__ chunks, int k,
                                                    const TV* __restrict__ V, int64_t ldv,
                                                    const T* __restrict__ zall, T* y,
                                                    const uint8_t* __restrict__ active) {
  __shared__ T zs[256];
  __shared__ T red[3 * kLr1Rows];
  const LrChunk C = chunks[blockIdx.x];
  if (active && !active[C.sys]) return;
  const int64_t r0 = C.r0 + (int64_t)blockIdx.y * kLr1Rows;
  if (r0 >= C.r1) return;  // uniform over the workgroup
  for (int j = threadIdx.x; j < k; j += blockDim.x) zs[j] = zall[(int64_t)C.sys * k + j];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = min(r0 + lane, C.r1 - 1);
  const int kq = (k + 3) / 4, ja = w * kq, je = min(k, ja + kq);
  T acc = (T)0;
  constexpr int U = 8;
  for (int j = ja; j < je; j += U) {
    TV v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = V[(int64_t)min(j + u, je - 1) * ldv + row];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += j + u < je ? (T)tv_to_float(v[u]) * zs[j + u] : (T)0;
  }
  if (w > 0) red[(w - 1) * kLr1Rows + lane] = acc;
  __syncthreads();
  if (w == 0 && r0 + lane < C.r1)
    y[row] += acc + red[lane] + red[kLr1Rows + lane] + red[2 * kLr1Rows + lane];
}

// ---- the low-rank products on the matrix cores (many right-hand sides, V in BF16)
//
// With V stored in BF16 the two tall-skinny products of the low-rank term,
// V^T Y (k x nrhs) and V Z (q x nrhs), are dense contractions over q and k.
// They run on v_mfma_f32_32x32x16_bf16 (32 x 32 output block, 16-deep
// contraction, FP32 accumulation).  The FP32 operand (Y, or Z = G V^T Y) is
// split into three BF16 parts hi + mid + lo that carry its 24 significant
// bits, so the three products summed equal the FP32 product with the
// BF16-rounded V.  Operand fragments: lane l holds A[l % 32][8 (l / 32) .. +7]
// and B[8 (l / 32) .. +7][l % 32]; accumulator element i of lane l is
// C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int kMfmaThreads = 256;

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r = x - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

// partial[(chunk * nrhs + r) * k + j] = sum over the chunk's rows of V[row][j] y_r[row]
// (V^T y, Algorithm 3 line 3).  V: BF16 column-major (ldv), y: FP32 column-major.
// Workgroup (chunk, tile of 32 right-hand sides); wave w owns the 32-column
// blocks w, w + 4, ... of V and walks the chunk's rows 16 at a time.
__global__ void __launch_bounds__(kMfmaThreads)
k_lr_partial_mfma(const LrChunk* __restrict__ chunks, int k, const __hip_bfloat16* __restrict__ V,
                  int64_t ldv, const float* __restrict__ y, int64_t ldy, int nrhs, float* partial,
                  const uint8_t* __restrict__ active, int nsys) {
  const LrChunk C = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int r = blockIdx.y * 32 + col;
  const bool rok = r < nrhs && (!active || active[r * nsys + C.sys]);
  const float* yr = y + (int64_t)(rok ? r : 0) * ldy;
  const int njb = (k + 31) / 32;
  for (int jb = wave; jb < njb; jb += kMfmaThreads / 64) {
    const int j = jb * 32 + col;
    const bool jok = j < k;
    const __hip_bfloat16* vj = V + (int64_t)(jok ? j : 0) * ldv;
    f32x16_t acc = {};
    for (int64_t r0 = C.r0; r0 < C.r1; r0 += 16) {
      const int64_t row = r0 + 8 * half;
      bf16x8_t a, bh, bm, bl;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const bool ok = row + t < C.r1;
        a[t] = (jok && ok) ? __builtin_bit_cast(__bf16, vj[row + t]) : (__bf16)0.0f;
        __bf16 h = (__bf16)0.0f, m = (__bf16)0.0f, l = (__bf16)0.0f;
        if (rok && ok) split3(yr[row + t], h, m, l);
        bh[t] = h;
        bm[t] = m;
        bl[t] = l;
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
    }
    if (r < nrhs) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int jj = jb * 32 + 8 * (i / 4) + 4 * half + (i % 4);
        if (jj < k) partial[((int64_t)blockIdx.x * nrhs + r) * k + jj] = acc[i];
      }
    }
  }
}

// Z_s = G_s W (gtrans: G_s^T W) with W = V^T y summed over the system's chunk
// partials, written as three BF16 parts: Zp[((s * 3 + part) * nrhs + r) * kp + j]
// (kp = k rounded up to 16, zero beyond k).  Workgroup (system, right-hand side).
__global__ void __launch_bounds__(kMfmaThreads)
k_lr_gz(int k, int kp, const float* __restrict__ Gall, int gtrans, const float* __restrict__ partial,
        const int32_t* __restrict__ sys_chunk, int nrhs, __hip_bfloat16* Zp) {
  __shared__ float W[256];
  const int s = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const float* G = Gall + (int64_t)s * k * k;
  const int c0 = sys_chunk[s], c1 = sys_chunk[s + 1];
  for (int j = tid; j < k; j += blockDim.x) {
    float w = 0.0f;
    for (int c = c0; c < c1; ++c) w += partial[((int64_t)c * nrhs + r) * k + j];
    W[j] = w;
  }
  __syncthreads();
  __hip_bfloat16* zh = Zp + ((int64_t)(s * 3 + 0) * nrhs + r) * kp;
  __hip_bfloat16* zm = Zp + ((int64_t)(s * 3 + 1) * nrhs + r) * kp;
  __hip_bfloat16* zl = Zp + ((int64_t)(s * 3 + 2) * nrhs + r) * kp;
  for (int j = tid; j < kp; j += blockDim.x) {
    float z = 0.0f;
    if (j < k)
      for (int l = 0; l < k; ++l) z += (gtrans ? G[(int64_t)l * k + j] : G[(int64_t)j * k + l]) * W[l];
    __bf16 h, m, lo;
    split3(z, h, m, lo);
    zh[j] = __builtin_bit_cast(__hip_bfloat16, h);
    zm[j] = __builtin_bit_cast(__hip_bfloat16, m);
    zl[j] = __builtin_bit_cast(__hip_bfloat16, lo);
  }
}

// y[row][r] += sum_j V[row][j] Z_s[j][r] (V G V^T y, Algorithm 3 line 3) for
// the rows of a chunk (system s) and a tile of 32 right-hand sides.  Vr: BF16
// row-major q x kp (zero beyond k); one wave per 32-row block.
__global__ void __launch_bounds__(kMfmaThreads)
k_lr_expand_mfma(const LrChunk* __restrict__ chunks, int kp, const __hip_bfloat16* __restrict__ Vr,
                 const __hip_bfloat16* __restrict__ Zp, int nrhs, float* y, int64_t ldy,
                 const uint8_t* __restrict__ active, int nsys) {
  const LrChunk C = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int r = blockIdx.y * 32 + col;
  const bool rok = r < nrhs && (!active || active[r * nsys + C.sys]);
  const int64_t len = C.r1 - C.r0;
  const bf16x8_t* zp[3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
    zp[p] = reinterpret_cast<const bf16x8_t*>(Zp + ((int64_t)(C.sys * 3 + p) * nrhs + (rok ? r : 0)) * kp);
  const bf16x8_t z8 = {};
  for (int64_t rb = wave; rb * 32 < len; rb += kMfmaThreads / 64) {
    const int64_t row = C.r0 + rb * 32 + col;
    const bool ok = row < C.r1;
    const bf16x8_t* vr = reinterpret_cast<const bf16x8_t*>(Vr + (ok ? row : C.r0) * kp);
    f32x16_t acc = {};
    for (int kk = 0; kk < kp; kk += 16) {
      const int q8 = (kk >> 3) + half;
      const bf16x8_t a = ok ? vr[q8] : z8;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const bf16x8_t b = rok ? zp[p][q8] : z8;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
    if (rok) {
      float* yr = y + (int64_t)r * ldy;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t rr = C.r0 + rb * 32 + 8 * (i / 4) + 4 * half + (i % 4);
        if (rr < C.r1) yr[rr] += acc[i];
      }
    }
  }
}

// LDS slots k_lr_expand uses for its slice sums (static, on top of the dynamic
// working vectors; the launch configuration leaves room for them)
constexpr int kLrSlots = kLrExpandSlots;

// y += V (G (V^T y)) on the rows of block i; optionally u = C0^{-1} y (line 3, line 4 start)
template <typename T, typename TV, int R, bool GX>
__global__ void __launch_bounds__(1024) k_lr_expand(ApplyArrays<T> A, int nrhs, int k,
                            const TV* __restrict__ V, const T* __restrict__ Gall, int gtrans,
                            const T* __restrict__ partial, const int32_t* __restrict__ sys_chunk,
                            T* y, int64_t ldy, int do_c0, T* u, int64_t ldu, int nslice) {
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, R>(A, nrhs, i, r0, nr)) return;
  Lds<T> L = carve<T, R, GX>(A);
  T* Wv = L.W;
  T* Zv = L.W + k * R;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  const int sys = A.part_sys[i];
  const T* G = Gall + (int64_t)sys * k * k;
  const int c0 = sys_chunk[sys], c1 = sys_chunk[sys + 1];
  // W = V^T y (sum of the system's chunk partials), then Z = G W; both spread
  // over the workgroup in S slices of the summation range, joined through LDS
  // (S = lr_slices(k, R, blockDim.x) >= 1, chosen by the launcher)
  __shared__ T red[kLrSlots];
  const int KR = k * R;
  const int S = nslice;
  for (int t = tid; t < (S > 1 ? S * KR : KR); t += nt) {
    const int sl = S > 1 ? t / KR : 0, e = t - sl * KR;
    const int j = e / R, r = e - j * R;
    T s = 0;
    if (r < nr)
      for (int c = c0 + sl; c < c1; c += S) s += partial[((int64_t)c * nrhs + r0 + r) * k + j];
    if (S > 1) red[t] = s;
    else Wv[e] = s;
  }
  __syncthreads();
  if (S > 1) {
    for (int e = tid; e < KR; e += nt) {
      T s = 0;
      for (int sl = 0; sl < S; ++sl) s += red[sl * KR + e];
      Wv[e] = s;
    }
    __syncthreads();
  }
  for (int t = tid; t < (S > 1 ? S * KR : KR); t += nt) {
    const int sl = S > 1 ? t / KR : 0, e = t - sl * KR;
    const int j = e / R, r = e - j * R;
    T s = 0;
    for (int l = sl; l < k; l += S) s += (gtrans ? G[(int64_t)l * k + j] : G[(int64_t)j * k + l]) * Wv[l * R + r];
    if (S > 1) red[t] = s;
    else Zv[e] = s;
  }
  __syncthreads();
  if (S > 1) {
    for (int e = tid; e < KR; e += nt) {
      T s = 0;
      for (int sl = 0; sl < S; ++sl) s += red[sl * KR + e];
      Zv[e] = s;
    }
    __syncthreads();
  }
  // lane per interface row: acc = V[row, :] . Z with V column-major, Z broadcast from LDS
  const int64_t ldv = A.q;
  for (int64_t kr = tid; kr < qi; kr += nt) {
    const int64_t row = f0 + kr;
    const TV* vr = V + row;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    constexpr int U = 8;
    int j = 0;
    for (; j + U <= k; j += U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = (T)tv_to_float(vr[(int64_t)(j + u) * ldv]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += v[u] * Zv[(j + u) * R + r];
    }
    for (; j < k; ++j) {
      const T v = (T)tv_to_float(vr[(int64_t)j * ldv]);
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += v * Zv[j * R + r];
    }
    const int64_t pos = A.gC_inv[row];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T v = r < nr ? y[(r0 + r) * ldy + row] + acc[r] : (T)0;
      if (r < nr) y[(r0 + r) * ldy + row] = v;
      if (do_c0) L.XC[pos * R + r] = v;
    }
  }
  if (!do_c0) return;
  __syncthreads();
  tri_solve<T, R, GX>(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UC, i, L.XC, L.Rb, A.gshift);
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t c = e / R;
    const int r = (int)(e - c * R);
    if (r < nr) u[(r0 + r) * ldu + f0 + A.gC_out[f0 + c]] = L.XC[e];
  }
}

// dst = C0^{-1} src
template <typename T, int R, bool GX>
__global__ void __launch_bounds__(1024) k_c0solve(ApplyArrays<T> A, int nrhs, const T* __restrict__ src,
                                                  int64_t lds_, T* dst, int64_t ldd) {
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, R>(A, nrhs, i, r0, nr)) return;
  Lds<T> L = carve<T, R, GX>(A);
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t p = e / R;
    const int r = (int)(e - p * R);
    L.XC[e] = r < nr ? src[(r0 + r) * lds_ + f0 + A.gC_in[f0 + p]] : (T)0;
  }
  __syncthreads();
  tri_solve<T, R, GX>(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UC, i, L.XC, L.Rb, A.gshift);
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t c = e / R;
    const int r = (int)(e - c * R);
    if (r < nr) dst[(r0 + r) * ldd + f0 + A.gC_out[f0 + c]] = L.XC[e];
  }
}

// One power-series step (eq. approx1 by its recurrence):
//   w = E_s u = -C_g u + F B^{-1} E u;  r = [y +] w;  u_next = [C0^{-1}] r
// C0 = true: the full step of the apply (k_series); false: the bare product
// w = E_s u (k_es, used by the Arnoldi process on (E_s C0^{-1})^{m+1}).
template <typename T, int R, bool GX, bool C0>
__device__ __forceinline__ void series_body(const ApplyArrays<T>& A, int nrhs, const T* __restrict__ y,
                                            int64_t ldy, const T* __restrict__ uprev, T* unext,
                                            int64_t ldu, int add_y) {
  constexpr bool do_c0 = C0;
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, R>(A, nrhs, i, r0, nr)) return;
  Lds<T> L = carve<T, R, GX>(A);
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t kk = e / R;
    const int r = (int)(e - kk * R);
    L.U[e] = r < nr ? uprev[(r0 + r) * ldu + f0 + kk] : (T)0;
  }
  __syncthreads();
  for (int64_t p = tid; p < pi; p += nt) {
    const int64_t row = i0 + p;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    for (int64_t q = A.Ein.ptr[row]; q < A.Ein.ptr[row + 1]; ++q) {
      const T v = A.Ein.val[q];
      const int c = A.Ein.col[q];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += v * L.U[c * R + r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) L.XB[p * R + r] = acc[r];
  }
  __syncthreads();
  tri_solve<T, R, GX>(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UB, i, L.XB, L.Rb, A.gshift);
  for (int64_t kk = tid; kk < qi; kk += nt) {
    const int64_t row = f0 + kk;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = (add_y && r < nr) ? y[(r0 + r) * ldy + row] : (T)0;
    for (int64_t q = A.Cg.ptr[row]; q < A.Cg.ptr[row + 1]; ++q) {
      const T v = A.Cg.val[q];
      const int64_t c = A.Cg.col[q];
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < nr) acc[r] -= v * uprev[(r0 + r) * ldu + c];
    }
    for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q) {
      const T v = A.Fout.val[q];
      const int c = A.Fout.col[q];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += v * L.XB[c * R + r];
    }
    if (do_c0) {
      const int64_t pos = A.gC_inv[row];
#pragma unroll
      for (int r = 0; r < R; ++r) L.XC[pos * R + r] = acc[r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < nr) unext[(r0 + r) * ldu + row] = acc[r];
    }
  }
  if (!do_c0) return;
  __syncthreads();
  tri_solve<T, R, GX>(A.LC, i, L.XC, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UC, i, L.XC, L.Rb, A.gshift);
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t c = e / R;
    const int r = (int)(e - c * R);
    if (r < nr) unext[(r0 + r) * ldu + f0 + A.gC_out[f0 + c]] = L.XC[e];
  }
}

template <typename T, int R, bool GX>
__global__ void __launch_bounds__(1024) k_series(ApplyArrays<T> A, int nrhs, const T* __restrict__ y,
                                                 int64_t ldy, const T* __restrict__ uprev, T* unext,
                                                 int64_t ldu, int add_y) {
  series_body<T, R, GX, true>(A, nrhs, y, ldy, uprev, unext, ldu, add_y);
}

template <typename T, int R, bool GX>
__global__ void __launch_bounds__(1024) k_es(ApplyArrays<T> A, int nrhs, const T* __restrict__ uprev,
                                             T* unext, int64_t ldu) {
  series_body<T, R, GX, false>(A, nrhs, nullptr, 0, uprev, unext, ldu, 0);
}

// x = B^{-1}(f - E u);  z = P^T (x; u)   (Algorithm 3, lines 5-6)
template <typename T, int R, bool GX>
__global__ void __launch_bounds__(1024) k_tail(ApplyArrays<T> A, int nrhs, const double* __restrict__ b,
                                               int64_t ldb, const T* __restrict__ u, int64_t ldu,
                                               double* z, int64_t ldz) {
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, R>(A, nrhs, i, r0, nr)) return;
  Lds<T> L = carve<T, R, GX>(A);
  const int64_t i0 = A.int_ptr[i], pi = A.int_ptr[i + 1] - i0;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  for (int64_t e = tid; e < qi * R; e += nt) {
    const int64_t kk = e / R;
    const int r = (int)(e - kk * R);
    const T v = r < nr ? u[(r0 + r) * ldu + f0 + kk] : (T)0;
    L.U[e] = v;
    if (r < nr) z[(r0 + r) * ldz + A.if_orig[f0 + kk]] = (double)v;
  }
  __syncthreads();
  for (int64_t p = tid; p < pi; p += nt) {
    const int64_t row = i0 + p;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = r < nr ? (T)b[(r0 + r) * ldb + A.gB_in[row]] : (T)0;
    for (int64_t q = A.Ein.ptr[row]; q < A.Ein.ptr[row + 1]; ++q) {
      const T v = A.Ein.val[q];
      const int c = A.Ein.col[q];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] -= v * L.U[c * R + r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) L.XB[p * R + r] = acc[r];
  }
  __syncthreads();
  tri_solve<T, R, GX>(A.LB, i, L.XB, L.Rb, A.gshift);
  tri_solve<T, R, GX>(A.UB, i, L.XB, L.Rb, A.gshift);
  for (int64_t e = tid; e < pi * R; e += nt) {
    const int64_t c = e / R;
    const int r = (int)(e - c * R);
    if (r < nr) z[(r0 + r) * ldz + A.gB_out[i0 + c]] = (double)L.XB[e];
  }
}

// ---- Team solves (a group's working vector in LDS, one right-hand side per
// workgroup: column blockIdx.y).  The supernodal tree of every B_i (family 0)
// and C_i (family 1) is cut into t_i groups of whole subtrees and a top group
// (BlockFactor::loS/upS), all blocks' subtree groups forming one work list.
// Launch 1, work item (i, g): group g's rows from the right-hand side and its
// lower solve on an LDS copy whose top rows start at their right-hand side
// (g = 0) or zero; the group's rows go to the family vector xw, its top rows
// (right-hand side minus its pushes) to dtop.  Launch 2: the top group from
// the sum of the groups' top rows, by its packed lower and upper solves (one
// workgroup per block) or by its dense inverse (one workgroup per 64 top
// rows).  Launch 3, work item (i, g): group g's upper solve, pulling the top
// rows.
//
// Right-hand sides and results by family and MODE:
//   B, 0 (power-series step): E u                  x to xb
//   B, 1 (head):              f gathered from b    x to xb
//   B, 2 (tail):              f - E u              x to z (top rows also to xb)
//   C, 0 (power-series step): [y] - C_g u + F xb   x to out (top rows also to xc)
//   C, 1 (C0 solve):          y                    x to out (top rows also to xc)
template <typename T>
struct TeamIO {
  const double* b;  // B modes 1, 2
  const T* u;       // B modes 0, 2: interface vector; C mode 0: u of the previous step
  const T* y;       // C: [y] of mode 0, the vector solved in mode 1
  const T* xb;      // C mode 0: B^{-1} E u
  T* xw;            // the family's vector between the launches
  T* dtop;          // nitems x ntopmax pushes into the top rows (one slice per item)
  double* z;        // B mode 2
  T* out;           // C: the result
  int add_y;
  // distances between the columns of a multi-right-hand-side launch (column
  // blockIdx.y), in elements of each array
  int64_t ldb, ldu, ldy, ldxb, ldxw, lddt, ldz, ldo;
};

// io moved to column blockIdx.y of a multi-right-hand-side team launch
template <typename T>
__device__ __forceinline__ void team_col(TeamIO<T>& io) {
  const int64_t r = blockIdx.y;
  if (r == 0) return;
  if (io.b) io.b += r * io.ldb;
  if (io.u) io.u += r * io.ldu;
  if (io.y) io.y += r * io.ldy;
  if (io.xb) io.xb += r * io.ldxb;
  if (io.xw) io.xw += r * io.ldxw;
  if (io.dtop) io.dtop += r * io.lddt;
  if (io.z) io.z += r * io.ldz;
  if (io.out) io.out += r * io.ldo;
}

template <typename T, int FAM>
__device__ __forceinline__ const TeamArrays<T>& team_fam(const ApplyArrays<T>& A) {
  return FAM == 0 ? A.TB : A.TC;
}

// first position of block i in the family's vectors
template <typename T, int FAM>
__device__ __forceinline__ int64_t team_base(const ApplyArrays<T>& A, int i) {
  return FAM == 0 ? A.int_ptr[i] : A.if_ptr[i];
}

// right-hand side of position p of block i (base: team_base); U: block i's
// interface values (B modes 0 and 2)
template <typename T, int FAM, int MODE>
__device__ __forceinline__ T team_rhs(const ApplyArrays<T>& A, const TeamIO<T>& io, int i, int64_t base,
                                      int p, const T* U) {
  if (FAM == 0) {
    const int64_t row = base + p;
    T acc = MODE == 0 ? (T)0 : (T)io.b[A.gB_in[row]];
    if (MODE != 1)
      for (int64_t q = A.Ein.ptr[row]; q < A.Ein.ptr[row + 1]; ++q) {
        const T v = A.Ein.val[q] * U[A.Ein.col[q]];
        acc = MODE == 0 ? acc + v : acc - v;
      }
    return acc;
  } else {
    const int64_t row = base + A.gC_in[base + p];
    if (MODE == 1) return io.y[row];
    T acc = io.add_y ? io.y[row] : (T)0;
    for (int64_t q = A.Cg.ptr[row]; q < A.Cg.ptr[row + 1]; ++q) acc -= A.Cg.val[q] * io.u[A.Cg.col[q]];
    const int64_t i0 = A.int_ptr[i];
    for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q)
      acc += A.Fout.val[q] * io.xb[i0 + A.Fout.col[q]];
    return acc;
  }
}

// the solved value x of position p (top: a top-group row, which the upper
// solves read back from xw)
template <typename T, int FAM, int MODE>
__device__ __forceinline__ void team_out(const ApplyArrays<T>& A, const TeamIO<T>& io, int64_t base, int p,
                                         T x, bool top) {
  if (FAM == 0) {
    if (MODE == 2) io.z[A.gB_out[base + p]] = (double)x;
    if (MODE != 2 || top) io.xw[base + p] = x;
  } else {
    io.out[base + A.gC_out[base + p]] = x;
    if (top) io.xw[base + p] = x;
  }
}

// group g of block i of a team family: its local positions (own rows first,
// then for a subtree group the top rows) and its own-row count
template <typename T>
struct TeamGroup {
  const int32_t* P;  // local position -> block position
  int nloc, nown;
};
template <typename T>
__device__ __forceinline__ TeamGroup<T> team_group(const TeamArrays<T>& TA, int bi) {
  TeamGroup<T> G;
  const int64_t o = TA.pos_off[bi];
  G.P = TA.pos + o;
  G.nloc = (int)(TA.pos_off[bi + 1] - o);
  const DevTriBlock B = TA.L.blk[bi];
  G.nown = B.nlev > 0 ? TA.L.lev_ptr[B.lev_base + B.nlev] : 0;
  return G;
}

// LDS of a team launch (team_lds_bytes): the local vector, level scratch and
// the block's interface values
template <typename T>
struct TeamLds {
  T *X, *Rb, *U;
};
template <typename T>
__device__ __forceinline__ TeamLds<T> team_lds(const TeamArrays<T>& TA) {
  extern __shared__ __align__(16) unsigned char smem[];
  TeamLds<T> L;
  L.X = reinterpret_cast<T*>(smem);
  L.Rb = L.X + ((TA.maxloc + 1) & ~1);
  L.U = L.Rb + 2 * TA.maxlr;
  return L;
}

// block i's interface values into LDS (B modes 0, 2); the tail's group 0 also
// writes them to z
template <typename T, int FAM, int MODE>
__device__ __forceinline__ void team_load_u(const ApplyArrays<T>& A, const TeamIO<T>& io, int i, T* U,
                                            bool write_z) {
  if (FAM != 0 || MODE == 1) return;
  const int64_t f0 = A.if_ptr[i], qi = A.if_ptr[i + 1] - f0;
  for (int64_t kk = threadIdx.x; kk < qi; kk += blockDim.x) {
    const T v = io.u[f0 + kk];
    U[kk] = v;
    if (MODE == 2 && write_z) io.z[A.if_orig[f0 + kk]] = (double)v;
  }
  __syncthreads();
}

template <typename T, int FAM, int MODE>
__global__ void __launch_bounds__(1024) k_team_lower(ApplyArrays<T> A, TeamIO<T> io) {
  const TeamArrays<T>& TA = team_fam<T, FAM>(A);
  // work item w: subtree group g of block i, group index gi in TA.L / TA.U
  const int w = blockIdx.x;
  const int4 it = TA.item[w];
  const int i = it.x, gi = it.y, g = it.z;
  const int tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, 1>(A, gridDim.y, i, r0, nr)) return;
  team_col(io);
  TeamLds<T> L = team_lds<T>(TA);
  T* X = L.X;
  const int64_t base = team_base<T, FAM>(A, i);
  team_load_u<T, FAM, MODE>(A, io, i, L.U, g == 0);
  const TeamGroup<T> G = team_group<T>(TA, gi);
  for (int k = tid; k < G.nown; k += nt) X[k] = team_rhs<T, FAM, MODE>(A, io, i, base, G.P[k], L.U);
  // the top rows start from their right-hand side in group 0 and from zero in
  // the others, so that the sum of the groups' top rows is the right-hand side
  // minus every push, each term formed once
  for (int k = G.nown + tid; k < G.nloc; k += nt)
    X[k] = g == 0 ? team_rhs<T, FAM, MODE>(A, io, i, base, G.P[k], L.U) : (T)0;
  __syncthreads();
  tri_solve<T, 1, false>(TA.L, gi, X, L.Rb, A.gshift);
  __syncthreads();
  for (int k = tid; k < G.nown; k += nt) io.xw[base + G.P[k]] = X[k];
  T* d = io.dtop + (int64_t)w * TA.ntopmax;
  for (int k = G.nown + tid; k < G.nloc; k += nt) d[k - G.nown] = X[k];
}

// the top group by its packed factors, one workgroup per block
template <typename T, int FAM, int MODE>
__global__ void __launch_bounds__(1024) k_team_top(ApplyArrays<T> A, TeamIO<T> io) {
  const TeamArrays<T>& TA = team_fam<T, FAM>(A);
  const int i = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, 1>(A, gridDim.y, i, r0, nr)) return;
  team_col(io);
  TeamLds<T> L = team_lds<T>(TA);
  T* X = L.X;
  const int64_t base = team_base<T, FAM>(A, i);
  const int bs = TA.gptr[i], team = TA.gptr[i + 1] - bs - 1;
  const TeamGroup<T> G = team_group<T>(TA, bs + team);
  const T* d = io.dtop + (int64_t)(bs - i) * TA.ntopmax;
  for (int k = tid; k < G.nloc; k += nt) {
    T acc = (T)0;  // the right-hand side came with group 0's top rows
    for (int t = 0; t < team; ++t) acc += d[(int64_t)t * TA.ntopmax + k];
    X[k] = acc;
  }
  __syncthreads();
  tri_solve<T, 1, false>(TA.L, bs + team, X, L.Rb, A.gshift);
  tri_solve<T, 1, false>(TA.U, bs + team, X, L.Rb, A.gshift);
  __syncthreads();
  for (int k = tid; k < G.nloc; k += nt) team_out<T, FAM, MODE>(A, io, base, G.P[k], X[k], true);
}

// The top group through its dense inverse: workgroup (i, rb) sums the
// groups' top rows into d (the right-hand side minus every push) and forms
// the 64 rows rb * 64 .. of x_T = M_i d, the waves splitting the
// column pairs and meeting in LDS.  Lane l of a wave reads row rb * 64 + l of
// a column pair: 64 consecutive pairs, one coalesced load per pair.
constexpr int kTopRows = 64;

template <typename T, int FAM, int MODE>
__global__ void __launch_bounds__(1024) k_team_topinv(ApplyArrays<T> A, TeamIO<T> io) {
  using P2 = typename Pair<T>::type;
  const TeamArrays<T>& TA = team_fam<T, FAM>(A);
  const int nrb = TA.nrb;
  const int i = blockIdx.x / nrb, rb = blockIdx.x - i * nrb, tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, 1>(A, gridDim.y, i, r0, nr)) return;
  team_col(io);
  const int bs = TA.gptr[i], team = TA.gptr[i + 1] - bs - 1;
  const TeamGroup<T> G = team_group<T>(TA, bs + team);
  const int ntop = G.nloc;
  if (rb * kTopRows >= ntop) return;  // uniform over the workgroup
  extern __shared__ __align__(16) unsigned char smem[];
  T* D = reinterpret_cast<T*>(smem);          // ntopmax + 2
  T* Ps = D + ((TA.ntopmax + 2 + 1) & ~1);    // (nt / 64) x 64 partial sums
  const int64_t base = team_base<T, FAM>(A, i);
  const int wv = tid >> 6, lane = tid & 63, nw = nt >> 6;
  const int row = rb * kTopRows + lane;
  const int npair = (ntop + 1) >> 1, ld = (ntop + 15) & ~15;  // the host's top_ld
  const P2* M = reinterpret_cast<const P2*>(TA.TI + TA.ti_off[i]);
  // the first round of this lane's pairs does not depend on d: loaded before
  // d is formed (slots past the end re-read pair wv, products dropped)
  constexpr int UN = 4;
  P2 v0[UN];
  if (row < ntop)
#pragma unroll
    for (int s = 0; s < UN; ++s) {
      const int cs = wv + s * nw < npair ? wv + s * nw : wv;
      v0[s] = M[(int64_t)cs * ld + row];
    }
  const T* d = io.dtop + (int64_t)(bs - i) * TA.ntopmax;
  for (int k = tid; k < ntop; k += nt) {
    T acc = (T)0;  // the right-hand side came with group 0's top rows
    for (int t = 0; t < team; ++t) acc += d[(int64_t)t * TA.ntopmax + k];
    D[k] = acc;
  }
  if (tid == 0) D[ntop] = (T)0;  // partner of an odd last column
  __syncthreads();
  T acc = (T)0;
  if (row < ntop) {
#pragma unroll
    for (int s = 0; s < UN; ++s) {
      const int cs = wv + s * nw < npair ? wv + s * nw : wv;
      const T a = v0[s].x * D[2 * cs] + v0[s].y * D[2 * cs + 1];
      acc += wv + s * nw < npair ? a : (T)0;
    }
    for (int c = wv + UN * nw; c < npair; c += UN * nw) {
      // every slot loads (a slot past the end re-reads pair c); the extra
      // products are dropped
      P2 v[UN];
#pragma unroll
      for (int s = 0; s < UN; ++s) {
        const int cs = c + s * nw < npair ? c + s * nw : c;
        v[s] = M[(int64_t)cs * ld + row];
      }
#pragma unroll
      for (int s = 0; s < UN; ++s) {
        const int cs = c + s * nw < npair ? c + s * nw : c;
        const T a = v[s].x * D[2 * cs] + v[s].y * D[2 * cs + 1];
        acc += c + s * nw < npair ? a : (T)0;
      }
    }
  }
  Ps[wv * kTopRows + lane] = acc;
  __syncthreads();
  if (wv == 0 && row < ntop) {
    T x = (T)0;
    for (int w = 0; w < nw; ++w) x += Ps[w * kTopRows + lane];
    team_out<T, FAM, MODE>(A, io, base, G.P[row], x, true);
  }
}

template <typename T, int FAM, int MODE>
__global__ void __launch_bounds__(1024) k_team_upper(ApplyArrays<T> A, TeamIO<T> io) {
  const TeamArrays<T>& TA = team_fam<T, FAM>(A);
  const int4 it = TA.item[blockIdx.x];
  const int i = it.x, gi = it.y;
  const int tid = threadIdx.x, nt = blockDim.x;
  int r0, nr;
  if (!tile_rhs<T, 1>(A, gridDim.y, i, r0, nr)) return;
  team_col(io);
  TeamLds<T> L = team_lds<T>(TA);
  T* X = L.X;
  const int64_t base = team_base<T, FAM>(A, i);
  const TeamGroup<T> G = team_group<T>(TA, gi);
  // own rows (the lower solve's results) and the top rows
  for (int k = tid; k < G.nloc; k += nt) X[k] = io.xw[base + G.P[k]];
  __syncthreads();
  tri_solve<T, 1, false>(TA.U, gi, X, L.Rb, A.gshift);
  __syncthreads();
  for (int k = tid; k < G.nown; k += nt) team_out<T, FAM, MODE>(A, io, base, G.P[k], X[k], false);
}

// y = g - F t of the head with t = B^{-1} f read from xb (one thread per interface row)
template <typename T>
__global__ void __launch_bounds__(256) k_team_headF(ApplyArrays<T> A, const double* __restrict__ b,
                                                    const T* __restrict__ xb, T* y, int64_t ldb,
                                                    int64_t ldxb, int64_t ldy) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= A.q) return;
  // column blockIdx.y
  const int64_t r = blockIdx.y;
  b += r * ldb;
  xb += r * ldxb;
  y += r * ldy;
  // subdomain of the row: the last i with if_ptr[i] <= row (binary search)
  int lo = 0, hi = A.nparts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.if_ptr[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  if (A.active && !A.active[r * A.nsys + A.part_sys[lo]]) return;
  const int64_t i0 = A.int_ptr[lo];
  T acc = (T)b[A.if_orig[row]];
  for (int64_t q = A.Fout.ptr[row]; q < A.Fout.ptr[row + 1]; ++q)
    acc -= A.Fout.val[q] * xb[i0 + A.Fout.col[q]];
  y[row] = acc;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------- launchers

// dispatch a block kernel over the rhs-tile width R (1, 2, 4, 8) and the
// working-vector placement (LDS or global)
#define PSLR_DISPATCH(c, BODY)                        \
  do {                                                \
    switch ((c).R) {                                  \
      case 1: { constexpr int RR = 1; BODY; } break;  \
      case 2: { constexpr int RR = 2; BODY; } break;  \
      case 4: { constexpr int RR = 4; BODY; } break;  \
      case 8: { constexpr int RR = 8; BODY; } break;  \
      default: return hipErrorInvalidValue;           \
    }                                                 \
  } while (0)

inline unsigned ntiles(int nrhs, int R) { return (unsigned)((nrhs + R - 1) / R); }

template <typename T>
hipError_t set_lds_limit(size_t bytes) {
  hipError_t e;
  const int b = (int)bytes;
#define PSLR_SETATTR(RR)                                                                              \
  if ((e = hipFuncSetAttribute((const void*)k_head<T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_c0solve<T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_series<T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_es<T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_tail<T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_lr_expand<T, T, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b - (int)(kLrSlots * sizeof(T))))) return e; \
  if ((e = hipFuncSetAttribute((const void*)k_lr_expand<T, __hip_bfloat16, RR, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b - (int)(kLrSlots * sizeof(T))))) return e;
  PSLR_SETATTR(1)
  PSLR_SETATTR(2)
  PSLR_SETATTR(4)
  PSLR_SETATTR(8)
#undef PSLR_SETATTR
#define PSLR_SETATTR_TEAM(K)                                                                         \
  if ((e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, b))) return e;
  PSLR_SETATTR_TEAM((k_team_lower<T, 0, 0>))
  PSLR_SETATTR_TEAM((k_team_lower<T, 0, 1>))
  PSLR_SETATTR_TEAM((k_team_lower<T, 0, 2>))
  PSLR_SETATTR_TEAM((k_team_lower<T, 1, 0>))
  PSLR_SETATTR_TEAM((k_team_lower<T, 1, 1>))
  PSLR_SETATTR_TEAM((k_team_top<T, 0, 0>))
  PSLR_SETATTR_TEAM((k_team_top<T, 0, 1>))
  PSLR_SETATTR_TEAM((k_team_top<T, 0, 2>))
  PSLR_SETATTR_TEAM((k_team_top<T, 1, 0>))
  PSLR_SETATTR_TEAM((k_team_top<T, 1, 1>))
  PSLR_SETATTR_TEAM((k_team_upper<T, 0, 0>))
  PSLR_SETATTR_TEAM((k_team_upper<T, 0, 1>))
  PSLR_SETATTR_TEAM((k_team_upper<T, 0, 2>))
  PSLR_SETATTR_TEAM((k_team_upper<T, 1, 0>))
  PSLR_SETATTR_TEAM((k_team_upper<T, 1, 1>))
#undef PSLR_SETATTR_TEAM
  return hipSuccess;
}

template <typename T>
hipError_t launch_head(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, T* y, int64_t ldy) {
  PSLR_DISPATCH(c, {
    const dim3 grid(A.nparts, ntiles(nrhs, RR));
    if (c.gx) hipLaunchKernelGGL((k_head<T, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs, b, ldb, y, ldy);
    else hipLaunchKernelGGL((k_head<T, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A, nrhs, b, ldb, y, ldy);
  });
  return hipGetLastError();
}

template <typename T, typename TV>
hipError_t launch_lr_partial(int nchunk, const LrChunk* chunks, int k, const TV* V, int64_t ldv,
                             const T* y, int64_t ldy, int nrhs, T* partial, const uint8_t* active,
                             int nsys, hipStream_t s) {
  if (nchunk <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_lr_partial<T, TV>), dim3(nchunk, nrhs), dim3(kLrThreads), 0, s, chunks, k, V,
                     ldv, y, ldy, partial, active, nsys);
  return hipGetLastError();
}

template <typename T, typename TV>
hipError_t launch_lr1(int nchunk, const LrChunk* chunks, int maxrows, int nsys, const int32_t* sys_chunk,
                      int k, const TV* V, int64_t ldv, const T* G, int gtrans, T* y, T* partial, T* z,
                      const uint8_t* active, hipStream_t s) {
  if (nchunk <= 0 || k <= 0) return hipSuccess;
  if (k > 256 || maxrows > kLrChunkRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_lr1_partial<T, TV>), dim3(nchunk, (k + kLr1Cols - 1) / kLr1Cols), dim3(256), 0, s,
                     chunks, k, V, ldv, y, partial, active);
  hipLaunchKernelGGL((k_lr1_gz<T>), dim3(nsys), dim3(1024), 0, s, k, G, gtrans, partial, sys_chunk, z,
                     active);
  hipLaunchKernelGGL((k_lr1_expand<T, TV>), dim3(nchunk, (maxrows + kLr1Rows - 1) / kLr1Rows), dim3(256), 0,
                     s, chunks, k, V, ldv, z, y, active);
  return hipGetLastError();
}

hipError_t launch_lr_mfma(int nchunk, const LrChunk* chunks, int nsys, const int32_t* sys_chunk,
                          int k, const __hip_bfloat16* V, int64_t ldv, const __hip_bfloat16* Vr,
                          const float* G, int gtrans, float* y, int64_t ldy, int nrhs,
                          float* partial, __hip_bfloat16* Zp, const uint8_t* active,
                          hipStream_t s) {
  if (nchunk <= 0 || k <= 0 || nrhs <= 0) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;  // k_lr_gz holds W for up to 256 columns
  const int kp = (k + 15) / 16 * 16;
  const unsigned tiles = (unsigned)((nrhs + 31) / 32);
  hipLaunchKernelGGL(k_lr_partial_mfma, dim3(nchunk, tiles), dim3(kMfmaThreads), 0, s, chunks, k, V,
                     ldv, y, ldy, nrhs, partial, active, nsys);
  hipLaunchKernelGGL(k_lr_gz, dim3(nsys, nrhs), dim3(kMfmaThreads), 0, s, k, kp, G, gtrans, partial,
                     sys_chunk, nrhs, Zp);
  hipLaunchKernelGGL(k_lr_expand_mfma, dim3(nchunk, tiles), dim3(kMfmaThreads), 0, s, chunks, kp, Vr,
                     Zp, nrhs, y, ldy, active, nsys);
  return hipGetLastError();
}

template <typename T, typename TV>
hipError_t launch_lr_expand(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, int k,
                            const TV* V, const T* G, int gtrans, const T* partial, int nchunk,
                            const int32_t* sys_chunk, T* y, int64_t ldy, int do_c0, T* u,
                            int64_t ldu) {
  (void)nchunk;
  PSLR_DISPATCH(c, {
    const dim3 grid(A.nparts, ntiles(nrhs, RR));
    const int S = lr_slices(k, RR, c.threads);
    // every slice loop must advance, and the slice sums must fit the static LDS slots
    if (S < 1 || (S > 1 && S * k * RR > kLrSlots)) return hipErrorInvalidValue;
    if (c.gx)
      hipLaunchKernelGGL((k_lr_expand<T, TV, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs,
                         k, V, G, gtrans, partial, sys_chunk, y, ldy, do_c0, u, ldu, S);
    else
      hipLaunchKernelGGL((k_lr_expand<T, TV, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A,
                         nrhs, k, V, G, gtrans, partial, sys_chunk, y, ldy, do_c0, u, ldu, S);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c0solve(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* src,
                          int64_t lds_, T* dst, int64_t ldd) {
  PSLR_DISPATCH(c, {
    const dim3 grid(A.nparts, ntiles(nrhs, RR));
    if (c.gx) hipLaunchKernelGGL((k_c0solve<T, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs, src, lds_, dst, ldd);
    else hipLaunchKernelGGL((k_c0solve<T, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A, nrhs, src, lds_, dst, ldd);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_series(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* y,
                         int64_t ldy, const T* uprev, T* unext, int64_t ldu, int add_y, int do_c0) {
  PSLR_DISPATCH(c, {
    const dim3 grid(A.nparts, ntiles(nrhs, RR));
    if (!do_c0) {
      // the bare product w = E_s u (no y term, no C0 solve)
      if (add_y) return hipErrorInvalidValue;
      if (c.gx) hipLaunchKernelGGL((k_es<T, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs, uprev, unext, ldu);
      else hipLaunchKernelGGL((k_es<T, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A, nrhs, uprev, unext, ldu);
    } else if (c.ev_start || c.ev_stop) {
      if (c.gx)
        hipExtLaunchKernelGGL((k_series<T, RR, true>), grid, dim3(c.threads), 0, c.stream, c.ev_start,
                              c.ev_stop, 0, A, nrhs, y, ldy, uprev, unext, ldu, add_y);
      else
        hipExtLaunchKernelGGL((k_series<T, RR, false>), grid, dim3(c.threads), (uint32_t)c.lds, c.stream,
                              c.ev_start, c.ev_stop, 0, A, nrhs, y, ldy, uprev, unext, ldu, add_y);
    } else if (c.gx) {
      hipLaunchKernelGGL((k_series<T, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs, y, ldy,
                         uprev, unext, ldu, add_y);
    } else {
      hipLaunchKernelGGL((k_series<T, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A, nrhs, y,
                         ldy, uprev, unext, ldu, add_y);
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, const T* u, int64_t ldu, double* z, int64_t ldz) {
  PSLR_DISPATCH(c, {
    const dim3 grid(A.nparts, ntiles(nrhs, RR));
    if (c.gx)
      hipLaunchKernelGGL((k_tail<T, RR, true>), grid, dim3(c.threads), 0, c.stream, A, nrhs, b, ldb, u,
                         ldu, z, ldz);
    else
      hipLaunchKernelGGL((k_tail<T, RR, false>), grid, dim3(c.threads), c.lds, c.stream, A, nrhs, b,
                         ldb, u, ldu, z, ldz);
  });
  return hipGetLastError();
}

// the three launches of a team solve of family FAM; ev0 / ev1 (may be null)
// are recorded at the start of the first and the end of the last launch
template <typename T, int FAM, int MODE>
void launch_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const TeamIO<T>& io, hipEvent_t ev0,
                 hipEvent_t ev1) {
  const TeamArrays<T>& TA = FAM == 0 ? A.TB : A.TC;
  const unsigned ny = (unsigned)nrhs;
  const dim3 gt((unsigned)TA.nitems, ny), bt(c.threads);
  const size_t lds = team_lds_bytes(TA, A.maxQB);
  if (ev0)
    hipExtLaunchKernelGGL((k_team_lower<T, FAM, MODE>), gt, bt, (uint32_t)lds, c.stream, ev0, nullptr, 0, A,
                          io);
  else
    hipLaunchKernelGGL((k_team_lower<T, FAM, MODE>), gt, bt, lds, c.stream, A, io);
  if (TA.TI && TA.nrb > 0) {
    const size_t lds = sizeof(T) * ((size_t)((TA.ntopmax + 3) & ~1) + (size_t)(c.threads / 64) * kTopRows);
    hipLaunchKernelGGL((k_team_topinv<T, FAM, MODE>), dim3((unsigned)(A.nparts * TA.nrb), ny), bt, lds,
                       c.stream, A, io);
  } else {
    hipLaunchKernelGGL((k_team_top<T, FAM, MODE>), dim3((unsigned)A.nparts, ny), bt, lds, c.stream, A, io);
  }
  if (ev1)
    hipExtLaunchKernelGGL((k_team_upper<T, FAM, MODE>), gt, bt, (uint32_t)lds, c.stream, nullptr, ev1, 0, A,
                          io);
  else
    hipLaunchKernelGGL((k_team_upper<T, FAM, MODE>), gt, bt, lds, c.stream, A, io);
}

template <typename T>
TeamIO<T> team_io(const TeamWs& W) {
  TeamIO<T> io;
  io.b = nullptr;
  io.u = io.y = io.xb = nullptr;
  io.xw = io.dtop = io.out = nullptr;
  io.z = nullptr;
  io.add_y = 0;
  io.ldb = io.ldu = io.ldy = io.ldz = io.ldo = 0;
  io.ldxb = W.ldxb;
  io.ldxw = W.ldxb;
  io.lddt = W.lddb;
  return io;
}

template <typename T>
hipError_t launch_series_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* y,
                              const T* uprev, T* unext, int64_t ldv, int add_y, const TeamWs& W) {
  if (A.TB.team < 2 || A.TC.team < 2 || nrhs < 1) return hipErrorInvalidValue;
  TeamIO<T> io = team_io<T>(W);
  io.u = uprev;
  io.ldu = ldv;
  io.xw = (T*)W.xb;
  io.dtop = (T*)W.dtopb;
  launch_team<T, 0, 0>(A, c, nrhs, io, c.ev_start, nullptr);
  {
    TeamIO<T> ic = team_io<T>(W);
    ic.u = uprev;
    ic.y = y;
    ic.ldu = ic.ldy = ic.ldo = ldv;
    ic.xb = (const T*)W.xb;
    ic.xw = (T*)W.xc;
    ic.ldxw = W.ldxc;
    ic.dtop = (T*)W.dtopc;
    ic.lddt = W.lddc;
    ic.out = unext;
    ic.add_y = add_y;
    launch_team<T, 1, 0>(A, c, nrhs, ic, nullptr, c.ev_stop);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_head_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                            int64_t ldb, T* y, int64_t ldy, const TeamWs& W) {
  if (A.TB.team < 2 || nrhs < 1) return hipErrorInvalidValue;
  TeamIO<T> io = team_io<T>(W);
  io.b = b;
  io.ldb = ldb;
  io.xw = (T*)W.xb;
  io.dtop = (T*)W.dtopb;
  launch_team<T, 0, 1>(A, c, nrhs, io, nullptr, nullptr);
  if (A.q > 0)
    hipLaunchKernelGGL((k_team_headF<T>), dim3(nblk(A.q, 256), (unsigned)nrhs), dim3(256), 0, c.stream, A, b,
                       (const T*)W.xb, y, ldb, W.ldxb, ldy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                            int64_t ldb, const T* u, int64_t ldu, double* z, int64_t ldz, const TeamWs& W) {
  if (A.TB.team < 2 || nrhs < 1) return hipErrorInvalidValue;
  TeamIO<T> io = team_io<T>(W);
  io.b = b;
  io.ldb = ldb;
  io.u = u;
  io.ldu = ldu;
  io.z = z;
  io.ldz = ldz;
  io.xw = (T*)W.xb;
  io.dtop = (T*)W.dtopb;
  launch_team<T, 0, 2>(A, c, nrhs, io, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c0_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* src, T* dst,
                          int64_t ldv, const TeamWs& W) {
  if (A.TC.team < 2 || nrhs < 1) return hipErrorInvalidValue;
  TeamIO<T> io = team_io<T>(W);
  io.y = src;
  io.ldy = io.ldo = ldv;
  io.xw = (T*)W.xc;
  io.ldxw = W.ldxc;
  io.dtop = (T*)W.dtopc;
  io.lddt = W.lddc;
  io.out = dst;
  launch_team<T, 1, 1>(A, c, nrhs, io, nullptr, nullptr);
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
                                     int64_t, const T*, int64_t, double*, int64_t);              \
  template hipError_t launch_series_team<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const T*, \
                                            const T*, T*, int64_t, int, const TeamWs&);           \
  template hipError_t launch_head_team<T>(const ApplyArrays<T>&, const LaunchCfg&, int,            \
                                          const double*, int64_t, T*, int64_t, const TeamWs&);     \
  template hipError_t launch_tail_team<T>(const ApplyArrays<T>&, const LaunchCfg&, int,            \
                                          const double*, int64_t, const T*, int64_t, double*,      \
                                          int64_t, const TeamWs&);                                 \
  template hipError_t launch_c0_team<T>(const ApplyArrays<T>&, const LaunchCfg&, int, const T*, T*, \
                                        int64_t, const TeamWs&);

PSLR_INST(double)
PSLR_INST(float)

template hipError_t launch_lr1<double, double>(int, const LrChunk*, int, int, const int32_t*, int,
                                               const double*, int64_t, const double*, int, double*,
                                               double*, double*, const uint8_t*, hipStream_t);
template hipError_t launch_lr1<float, float>(int, const LrChunk*, int, int, const int32_t*, int,
                                             const float*, int64_t, const float*, int, float*, float*,
                                             float*, const uint8_t*, hipStream_t);
template hipError_t launch_lr1<float, __hip_bfloat16>(int, const LrChunk*, int, int, const int32_t*, int,
                                                      const __hip_bfloat16*, int64_t, const float*, int,
                                                      float*, float*, float*, const uint8_t*,
                                                      hipStream_t);
template hipError_t launch_lr_partial<double, double>(int, const LrChunk*, int, const double*,
                                                      int64_t, const double*, int64_t, int, double*,
                                                      const uint8_t*, int, hipStream_t);
template hipError_t launch_lr_partial<float, float>(int, const LrChunk*, int, const float*, int64_t,
                                                    const float*, int64_t, int, float*,
                                                    const uint8_t*, int, hipStream_t);
template hipError_t launch_lr_partial<float, __hip_bfloat16>(int, const LrChunk*, int,
                                                             const __hip_bfloat16*, int64_t,
                                                             const float*, int64_t, int, float*,
                                                             const uint8_t*, int, hipStream_t);
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
