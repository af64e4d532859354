// Device layouts of the PSLR preconditioner and the launchers of its HIP
// kernels (gfx950).  All offsets stored in these arrays are absolute indices
// into the concatenated per-family arrays.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>

namespace pslr {

// Per-block descriptor of one packed triangular factor (see TriPacked): rows
// and factor data are stored level by level; a row record is 8 int32 =
// {p, row in supernode, w, h, triangle start, panel start, ridx start,
// level-local index of the supernode's first row}.
struct DevTriBlock {
  int32_t n, nlev, max_lrows, lower;
  int64_t lev_base;   // lev_ptr/push_ptr/ent_ptr[lev_base .. +nlev], lev_c[lev_base .. +nlev)
  int64_t rec_base;   // row records, in rows
  int64_t prec_base;  // push records, in items
  int64_t ent_base;   // entry-form values and indices
  int64_t val_base;   // panels
  int64_t ridx_base;  // panel position lists
  int64_t tri_base;   // inverted diagonal triangles
};

// One family of packed triangular factors (e.g. "L of every B_i").
template <typename T>
struct TriArrays {
  const DevTriBlock* blk;
  const int32_t* lev_ptr;
  const int32_t* push_ptr;
  const int32_t* ent_ptr;
  const int32_t* lev_c;
  const int4* rec;
  const int4* prec;
  const T* val;
  const int32_t* ridx;
  const T* tri;
  // entry form, one 16-byte record per entry: x = value, y = the bits of
  // {eidx (low word), eloc (high word)}; FP64 factors only
  const double2* ent;
};

// Block-diagonal CSR over all subdomains with 64-bit row offsets.
template <typename T>
struct DevCsr {
  const int64_t* ptr;
  const int32_t* col;
  const T* val;
};

// Team split of one family of diagonal blocks (B_i or C_i): the supernodal
// tree of block i cut into t_i groups of whole subtrees and a top group (see
// BlockFactor::loS/upS), t_i sized to the block.  L / U hold group g of block
// i at index gptr[i] + g, the top group at gptr[i + 1] - 1 (so t_i =
// gptr[i + 1] - gptr[i] - 1).  The subtree groups of all blocks form one work
// list of nitems items: item[w] = {i, gptr[i] + g, g, 0} for group g of block
// i (one load gives a workgroup its block and group).
// dtop holds ntopmax values (the most top rows of any block) per item.  TI:
// the dense inverses of the top groups (null: the top group runs its packed
// factors), block i's at TI + ti_off[i] in the column-pair layout of
// BlockFactor::topinv, nrb workgroups of 64 top rows per block.  team: the
// largest t_i (0: no split).
template <typename T>
struct TeamArrays {
  TriArrays<T> L, U;
  int32_t team, ntopmax, nrb, nitems;
  const int32_t* gptr;
  const int4* item;
  const T* TI;
  const int64_t* ti_off;
  // the groups' local positions (TriPacked::pos): group g of block i at
  // pos[pos_off[gptr[i] + g] ..), its own rows first, then (subtree groups)
  // the top group's rows; maxloc, maxlr: the most local positions and level
  // rows of any group (the team kernels' LDS)
  const int32_t* pos;
  const int64_t* pos_off;
  int32_t maxloc, maxlr;
};

// LDS of a team launch: the group's local vector, two halves of level
// scratch, and the block's interface values (interior family)
template <typename T>
inline size_t team_lds_bytes(const TeamArrays<T>& TA, int32_t maxQB) {
  return sizeof(T) * ((size_t)((TA.maxloc + 1) & ~1) + 2 * (size_t)TA.maxlr + (size_t)maxQB);
}

// Everything one direction (forward or transposed) of the apply needs.
template <typename T>
struct ApplyArrays {
  int32_t nparts;
  int64_t n, p, q;
  const int64_t* int_ptr;     // nparts + 1
  const int64_t* if_ptr;      // nparts + 1
  TriArrays<T> LB, UB, LC, UC;
  const int32_t* gB_in;       // p: original index feeding B-solve input position
  const int32_t* gB_out;      // p: original index receiving B-solve output position
  const int32_t* gC_in;       // q: local interface index feeding C0-solve input position
  const int32_t* gC_out;      // q: local interface index receiving C0-solve output position
  const int32_t* gC_inv;      // q: inverse of gC_in (local)
  const int32_t* if_orig;     // q: original index of interface unknown k
  DevCsr<T> Ein;              // rows = B-solve input positions, cols = local interface
  DevCsr<T> Fout;             // rows = global interface, cols = B-solve output positions
  DevCsr<T> Cg;               // rows/cols = global interface
  const int32_t* part_sys;    // nparts: system (batched handles) owning each subdomain
  int32_t maxPB, maxQB, maxLR;
  int32_t gshift;             // per-level chunk counts are scaled by 2^gshift (autotuned)
  // global working vectors (used instead of LDS when a subdomain does not fit)
  void* gws;                  // null: working vectors in LDS
  int64_t gws_stride;         // elements per right-hand side
  const int64_t* rb_off;      // nparts + 1: per-block level-scratch offsets
  int32_t kmax;
  int32_t nsys;
  // optional (system, rhs) mask, index r * nsys + s: a block skips its work for
  // right-hand side r when its system's entry is 0 (converged FGMRES columns)
  const uint8_t* active;
  // team splits of the single-right-hand-side B_i and C_i solves
  TeamArrays<T> TB, TC;
};

// A row chunk of the interface vectors for the V^T y partial sums; chunks never
// straddle two systems.
struct LrChunk {
  int64_t r0, r1;
  int32_t sys, pad;
};
// longest row chunk of the V^T y partial sums (keeps several chunks per system)
constexpr int64_t kLrChunkRows = 2048;

// One column of a segmented vector operation: elements [base, base + len).
struct Seg {
  int64_t base, len;
};

// A row range of one column of a segmented vector operation.
struct Chunk {
  int32_t col, pad;
  int64_t r0, r1;
};
// longest row chunk of the chunked vector kernels (16 rows per thread at 256 threads)
#ifndef PSLR_CHUNK_ROWS
#define PSLR_CHUNK_ROWS 1024
#endif
constexpr int64_t kChunkRows = PSLR_CHUNK_ROWS;

// LDS slots of k_lr_expand's slice sums, and its slice count: the k x R
// sums of V^T y and G W are each split into S slices of the summation range
// joined through those slots.  S >= 1 always (S = 1: no slices, direct sums).
constexpr int kLrExpandSlots = 1024;
inline int lr_slices(int k, int R, int threads) {
  const int KR = k * R;
  if (KR <= 0 || KR > kLrExpandSlots) return 1;
  const int S = (threads < kLrExpandSlots ? threads : kLrExpandSlots) / KR;
  return S < 1 ? 1 : S;
}

struct LaunchCfg {
  int threads;
  size_t lds;          // dynamic LDS bytes (LDS working vectors)
  hipStream_t stream;
  int R;               // right-hand sides per workgroup tile: 1, 2, 4 or 8
  bool gx;             // working vectors in the global workspace
  // optional events stamped at the start and end of the kernel itself
  // (launch_series only; used by the phase tracer)
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

// ---- preconditioner kernels (T = double or float; TV = V's storage type)
template <typename T>
hipError_t launch_head(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, T* y, int64_t ldy);
template <typename T, typename TV>
// V is column-major (column j at V + j*ldv); chunks hold at most kLrChunkRows rows
hipError_t launch_lr_partial(int nchunk, const LrChunk* chunks, int k, const TV* V, int64_t ldv,
                             const T* y, int64_t ldy, int nrhs, T* partial, const uint8_t* active,
                             int nsys, hipStream_t s);
// G holds one k x k row-major matrix per system; block i uses system part_sys[i]
// and the partial sums of chunks sys_chunk[s] .. sys_chunk[s+1].
template <typename T, typename TV>
hipError_t launch_lr_expand(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, int k,
                            const TV* V, const T* G, int gtrans, const T* partial, int nchunk,
                            const int32_t* sys_chunk, T* y, int64_t ldy, int do_c0, T* u,
                            int64_t ldu);
// y += V G V^T y (gtrans: V G^T V^T y) for one right-hand side: V^T y per row
// chunk into partial (nchunk * k), z_s = G_s W_s into z (nsys * k), then the
// expansion; maxrows: the most rows of any chunk; k <= 256
template <typename T, typename TV>
hipError_t launch_lr1(int nchunk, const LrChunk* chunks, int maxrows, int nsys, const int32_t* sys_chunk,
                      int k, const TV* V, int64_t ldv, const T* G, int gtrans, T* y, T* partial, T* z,
                      const uint8_t* active, hipStream_t s);
// y += V G V^T y (gtrans: V G^T V^T y) on the matrix cores for FP32 applies with
// V in BF16: V column-major (ldv) and row-major Vr (q x kp, kp = k rounded up to
// 16, zero padded); partial: nchunk * nrhs * k floats; Zp: nsys * 3 * nrhs * kp
// BF16 values; k <= 256
hipError_t launch_lr_mfma(int nchunk, const LrChunk* chunks, int nsys, const int32_t* sys_chunk,
                          int k, const __hip_bfloat16* V, int64_t ldv, const __hip_bfloat16* Vr,
                          const float* G, int gtrans, float* y, int64_t ldy, int nrhs,
                          float* partial, __hip_bfloat16* Zp, const uint8_t* active,
                          hipStream_t s);
// right-hand-side count from which FP32 applies with V in BF16 use launch_lr_mfma
constexpr int kMfmaMinRhs = 16;
template <typename T>
hipError_t launch_c0solve(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* src,
                          int64_t lds_, T* dst, int64_t ldd);
template <typename T>
hipError_t launch_series(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* y,
                         int64_t ldy, const T* uprev, T* unext, int64_t ldu, int add_y, int do_c0);
template <typename T>
hipError_t launch_tail(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                       int64_t ldb, const T* u, int64_t ldu, double* z, int64_t ldz);
template <typename T>
hipError_t set_lds_limit(size_t bytes);
// Solves spread over the team of workgroups of each block, one right-hand
// side per workgroup (column blockIdx.y, working vectors in LDS), three
// launches per family: the subtree groups' lower solves, the top group, the
// groups' upper solves.  Between the launches the family's vector and the top
// rows' pushed updates live in the workspace TeamWs, one slice per column.
struct TeamWs {
  void* xb;     // per column p values: the B-solve vector
  void* dtopb;  // per column TB.nitems * TB.ntopmax values
  void* xc;     // per column q values: the C0-solve vector
  void* dtopc;  // per column TC.nitems * TC.ntopmax values
  int64_t ldxb, lddb, ldxc, lddc;  // the slices' lengths (column strides)
};
// Vectors of nrhs columns with the given leading dimensions (y, u, src, dst:
// ldv; b: ldb; z: ldz):
//   series step: unext = C0^{-1}(y [add_y] - C_g u + F B^{-1} E u)
//   head:        y = g - F B^{-1} f                                (+ a launch for F)
//   tail:        z = P^T (B^{-1}(f - E u); u)
//   c0:          dst = C0^{-1} src
// (both families split: A.TB.team > 1 and A.TC.team > 1)
template <typename T>
hipError_t launch_series_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* y,
                              const T* uprev, T* unext, int64_t ldv, int add_y, const TeamWs& W);
template <typename T>
hipError_t launch_head_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                            int64_t ldb, T* y, int64_t ldy, const TeamWs& W);
template <typename T>
hipError_t launch_tail_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const double* b,
                            int64_t ldb, const T* u, int64_t ldu, double* z, int64_t ldz, const TeamWs& W);
template <typename T>
hipError_t launch_c0_team(const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs, const T* src, T* dst,
                          int64_t ldv, const TeamWs& W);

// ---- FP64 vector kernels for Arnoldi and FGMRES
hipError_t launch_spmv(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                       int nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                       const double* bsub, int64_t ldb, hipStream_t s);
// Chunked forms: chunk c covers rows r0..r1 (at most kChunkRows) of column
// ch[c].col; the chunks of column j are cptr[j] .. cptr[j+1].  Dot products:
// partial[i * nchunk + c] per chunk, then out[j * nv + i] per column.
hipError_t launch_mdot_chunk(int nchunk, const Chunk* ch, const Seg* vcols, const Seg* wcols, int nv,
                             const double* V, int64_t ldv, const double* W, double* partial,
                             hipStream_t s);
hipError_t launch_reduce_chunk(int ncol, const int32_t* cptr, int nv, int nchunk,
                               const double* partial, double* out, hipStream_t s);
hipError_t launch_maxpy_chunk(int nchunk, const Chunk* ch, const Seg* vcols, const Seg* wcols,
                              int nv, const double* V, int64_t ldv, const double* h, int hld,
                              double* W, double sign, hipStream_t s);
// scl[c] = 1 / sqrt(nn[c]) where active[c] and nn[c] > 0, else 0
hipError_t launch_inv_sqrt(int ncol, const double* nn, const uint8_t* active, double* scl,
                           hipStream_t s);
hipError_t launch_scale_chunk(int nchunk, const Chunk* ch, const Seg* scols, const Seg* dcols,
                              const double* S, const double* scale, double* D, hipStream_t s);
// Vn[:, c] = sum_{j < mcols} V[:, j] W_s[j, c] for c < ncols on the rows of the
// chunks (chunk column = system s; W: per system mcols x ncols column-major)
hipError_t launch_basis_rotate(int nchunk, const Chunk* ch, const Seg* cols, int mcols, int ncols,
                               const double* V, int64_t ldv, const double* W, double* Vn, int64_t ldn,
                               hipStream_t s);
hipError_t launch_sddmm(int64_t n, const int64_t* ptr, const int32_t* col, int nrhs,
                        const double* lam, int64_t ldl, const double* z, int64_t ldz,
                        double* grad, hipStream_t s);

}  // namespace pslr
