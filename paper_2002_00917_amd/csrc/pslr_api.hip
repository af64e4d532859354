// C ABI of the PSLR preconditioner (include/pslr.h): setup (Algorithm 4),
// apply (Algorithm 3) and its transpose, FP64 flexible GMRES, the gradient
// SDDMM, and the host-only partition / reordering helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pslr.h"
#include "pslr_host.h"
#include "pslr_dev.h"

using namespace pslr;

namespace {

thread_local std::string g_last_error;

pslr_status fail(pslr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(PSLR_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_));        \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device allocation list owned by a handle.
struct DevPool {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  ~DevPool() { release(); }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
  template <typename X>
  hipError_t upload(const std::vector<X>& h, const X** out) {
    X* d = nullptr;
    size_t nb = std::max<size_t>(h.size(), 1) * sizeof(X);
    hipError_t e = hipMalloc((void**)&d, nb);
    if (e != hipSuccess) return e;
    ptrs.push_back(d);
    bytes += nb;
    if (!h.empty()) e = hipMemcpy(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice);
    *out = d;
    return e;
  }
  template <typename X>
  hipError_t alloc(size_t count, X** out) {
    X* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, std::max<size_t>(count, 1) * sizeof(X));
    if (e != hipSuccess) return e;
    ptrs.push_back(d);
    bytes += std::max<size_t>(count, 1) * sizeof(X);
    *out = d;
    return hipSuccess;
  }
};

// Concatenate one factor family over all blocks.  `bytes` receives the
// algorithmic bytes of one single-right-hand-side solve of every block (LDS
// working vectors): each value it reads once (triangles, panels or entries),
// the indices and records it reads once, the level tables.
template <typename T>
hipError_t upload_tri_list(DevPool& pool, const std::vector<const TriPacked*>& F, TriArrays<T>& out,
                           int& max_lrows, int64_t& bytes) {
  std::vector<DevTriBlock> blk(F.size());
  std::vector<int32_t> lev_ptr, push_ptr, ent_ptr, lev_c, rec, prec, ridx, ent;
  std::vector<T> val, tri;
  // the entry form is read by FP64 solves only
  const bool want_ent = sizeof(T) == 8;
  int64_t nent = 0;
  bytes = 0;
  for (size_t i = 0; i < F.size(); ++i) {
    const TriPacked& H = *F[i];
    DevTriBlock& B = blk[i];
    B.n = H.n;
    B.nlev = H.nlev;
    B.max_lrows = H.max_lrows;
    B.lower = H.lower ? 1 : 0;
    B.lev_base = (int64_t)lev_ptr.size();
    B.rec_base = (int64_t)rec.size() / 8;
    B.prec_base = (int64_t)prec.size() / 4;
    B.ent_base = nent;
    B.val_base = (int64_t)val.size();
    B.ridx_base = (int64_t)ridx.size();
    B.tri_base = (int64_t)tri.size();
    max_lrows = std::max(max_lrows, H.max_lrows);
    lev_ptr.insert(lev_ptr.end(), H.lev_ptr.begin(), H.lev_ptr.end());
    push_ptr.insert(push_ptr.end(), H.push_ptr.begin(), H.push_ptr.end());
    if (H.push_ptr.size() < H.lev_ptr.size()) push_ptr.resize(lev_ptr.size(), 0);
    ent_ptr.insert(ent_ptr.end(), H.ent_ptr.begin(), H.ent_ptr.end());
    if (H.ent_ptr.size() < H.lev_ptr.size()) ent_ptr.resize(lev_ptr.size(), 0);
    lev_c.insert(lev_c.end(), H.lev_c.begin(), H.lev_c.end());
    lev_c.resize(lev_ptr.size(), 0);
    rec.insert(rec.end(), H.rec.begin(), H.rec.end());
    prec.insert(prec.end(), H.prec.begin(), H.prec.end());
    for (double v : H.val) val.push_back((T)v);
    ridx.insert(ridx.end(), H.ridx.begin(), H.ridx.end());
    for (double v : H.tri) tri.push_back((T)v);
    if (want_ent)
      for (size_t q = 0; q < H.eval.size(); ++q) {
        int32_t bits[2];
        std::memcpy(bits, &H.eval[q], sizeof(double));
        ent.insert(ent.end(), {bits[0], bits[1], H.eidx[q], H.eloc[q]});
      }
    nent += want_ent ? (int64_t)H.eval.size() : 0;
    const int path = sizeof(T) == 8 ? 0 : 1;  // entry form only in FP64
    bytes += H.read_vals[path] * (int64_t)sizeof(T) + 4 * H.read_ints[path];
  }
  hipError_t e;
  if ((e = pool.upload(blk, &out.blk))) return e;
  if ((e = pool.upload(lev_ptr, &out.lev_ptr))) return e;
  if ((e = pool.upload(push_ptr, &out.push_ptr))) return e;
  if ((e = pool.upload(ent_ptr, &out.ent_ptr))) return e;
  if ((e = pool.upload(lev_c, &out.lev_c))) return e;
  const int32_t* p = nullptr;
  if ((e = pool.upload(rec, &p))) return e;
  out.rec = reinterpret_cast<const int4*>(p);
  if ((e = pool.upload(prec, &p))) return e;
  out.prec = reinterpret_cast<const int4*>(p);
  if ((e = pool.upload(val, &out.val))) return e;
  if ((e = pool.upload(ridx, &out.ridx))) return e;
  if ((e = pool.upload(tri, &out.tri))) return e;
  if ((e = pool.upload(ent, &p))) return e;
  out.ent = reinterpret_cast<const double2*>(p);
  return hipSuccess;
}

template <typename T>
hipError_t upload_tri(DevPool& pool, const std::vector<BlockFactor>& F, TriPacked BlockFactor::*mem,
                      TriArrays<T>& out, int& max_lrows, int64_t& bytes) {
  std::vector<const TriPacked*> list(F.size());
  for (size_t i = 0; i < F.size(); ++i) list[i] = &(F[i].*mem);
  return upload_tri_list(pool, list, out, max_lrows, bytes);
}

// Host CSR of the coupling blocks in the layouts the kernels read.
struct CouplingHost {
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

template <typename T>
hipError_t upload_csr(DevPool& pool, const CouplingHost& C, DevCsr<T>& out) {
  std::vector<T> v(C.val.begin(), C.val.end());
  hipError_t e;
  if ((e = pool.upload(C.ptr, &out.ptr))) return e;
  if ((e = pool.upload(C.col, &out.col))) return e;
  return pool.upload(v, &out.val);
}

// Apply workspace of pslr_apply_noalloc: one file-scope device array per GPU
// (each device that loads the library holds its own copy until the process
// ends).  Host code never uses the array's name as an address: its device
// address is looked up once per device at setup (scratch_attach) and kept in
// g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Resolve the scratch array's address on `device` (which must be current).
pslr_status scratch_attach(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(PSLR_ENOTSUP, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PSLR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(PSLR_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return PSLR_OK;
}

// Element counts (in doubles) of an apply workspace: y, u0, u1 (q x nrhs
// each), the V^T y partial sums and the global working vectors.
struct WsSizes {
  size_t vec = 0, partial = 0, gws = 0, zp = 0, team = 0;
};

// Everything one direction of the apply needs, host side.
struct DirHost {
  std::vector<int32_t> gB_in, gB_out, gC_in, gC_out, gC_inv;
  CouplingHost Ein, Fout, Cg;
};

}  // namespace

struct pslr_ctx {
  int device = 0;
  Reordering R;
  int32_t m = 3, rank = 0, precision = 0, want_T = 0;
  int64_t nnzA = 0;
  std::vector<int64_t> hA_ptr;   // host pattern of A (original order), kept for pslr_refactor
  std::vector<int32_t> hA_col;
  pslr_options opt{};            // the setup's options (v0 copied to hv0)
  std::vector<double> hv0;
  DevPool facpool;               // data that depends on A's values: factors, couplings, A's values
  const int64_t* d_int_ptr = nullptr;
  const int64_t* d_if_ptr = nullptr;
  const int32_t* d_if_orig = nullptr;
  DevPool pool;      // factor and matrix data
  DevPool ws;        // workspaces (grown on demand)
  DevPool vpool;     // low-rank data
  DevPool vretired;  // low-rank data replaced by pslr_set_lowrank (freed at destroy)
  // device copies of A (original order) and optionally A^T
  const int64_t* A_ptr = nullptr;
  const int32_t* A_col = nullptr;
  const double* A_val = nullptr;
  const int64_t* AT_ptr = nullptr;
  const int32_t* AT_col = nullptr;
  const double* AT_val = nullptr;
  ApplyArrays<double> fw64{}, tr64{};
  ApplyArrays<float> fw32{}, tr32{};
  bool have64 = false, have32 = false, haveT = false;
  int threads = kSolveThreads;
  bool threads_fixed = false;  // set by the caller: the autotuner keeps it
  // low rank: Vcm (FP64 q x k column-major, host), H, G; device V row-major and G
  int32_t k = 0;
  std::vector<double> hV, hH, hG;
  const double* V64 = nullptr;
  const double* G64 = nullptr;
  const __hip_bfloat16* Vbf = nullptr;
  const __hip_bfloat16* Vbr = nullptr;  // BF16 V row-major q x kp (matrix-core products)
  const float* V32 = nullptr;
  // precision 2: V is read in BF16 only while the setup probe allows it
  bool v_bf16 = false;
  double bf16_probe = 0.0;
  const float* G32 = nullptr;
  int nchunk = 256;
  // systems of a batched handle (one system otherwise): row ranges in the
  // original ordering, interface ranges, achieved ranks
  int32_t nsys = 1;
  std::vector<int64_t> sys_n, sys_q;
  std::vector<int32_t> sys_k;
  const int32_t* d_part_sys = nullptr;
  const LrChunk* d_chunks = nullptr;
  const int32_t* d_sys_chunk = nullptr;
  int nchunk_lr = 1;
  int lr_maxrows = 0;           // the most rows of a V^T y chunk
  const Seg* d_qcols = nullptr;
  // global working vectors when a subdomain does not fit in LDS
  bool gx = false;          // working vectors forced to global memory
  size_t lds_max = 65536;   // LDS bytes a workgroup may use
  int64_t gws_stride = 0;
  int tuned_threads = 0, tuned_gshift = 0;
  int rmax = 8;      // widest right-hand-side tile of a launch (autotuned)
  int team_rhs = 0;  // pslr_options.team_rhs (0: automatic, see run_apply)
  const int64_t* d_rb_off = nullptr;
  // apply workspaces (grow-only, see ensure_ws)
  int ws_nrhs = 0;
  WsSizes ws_cap;
  void* y = nullptr;
  void* u0 = nullptr;
  void* u1 = nullptr;
  void* partial = nullptr;
  void* gws = nullptr;
  void* zp = nullptr;
  void* tws = nullptr;  // team solves: interior vector, then the top-row updates
  // FGMRES workspace (kept between calls)
  DevPool fpool;
  int f_nrhs = 0, f_restart = 0;
  double *fVb = nullptr, *fZb = nullptr, *fW = nullptr, *fdbuf = nullptr, *fh = nullptr,
         *fscl = nullptr, *fy = nullptr;
  Seg *fcolsV = nullptr, *fcolsB = nullptr, *fcolsX = nullptr, *fcolsM = nullptr;
  Chunk *fchF = nullptr, *fchM = nullptr;
  int32_t *fcpF = nullptr, *fcpM = nullptr;
  int64_t f_maxch = 0;
  uint8_t* factive = nullptr;
  double* fpin = nullptr;  // pinned host staging of the Hessenberg columns (two slots)
  size_t fpin_n = 0;
  const uint8_t* cur_active = nullptr;  // mask of (system, rhs) columns the apply works on
  // info
  pslr_info_t info{};
  // phase tracing: each traced apply leaves a list of (phase, event) marks
  bool trace = false;
  std::vector<hipEvent_t> ev_free, ev_all;
  std::deque<std::vector<std::pair<int, hipEvent_t>>> ev_pending;
  pslr_trace_t tr{};
  ~pslr_ctx() {
    for (hipEvent_t e : ev_all) (void)hipEventDestroy(e);
    if (fpin) (void)hipHostFree(fpin);
  }
};

namespace {

#ifndef PSLR_TEAM_ROWS
#define PSLR_TEAM_ROWS 2048
#endif
constexpr int64_t kTeamRows = PSLR_TEAM_ROWS;
constexpr int kTeamRhsAuto = 8;

// Team size of the B_i solves: exact LU only; automatic = 4 workgroups per
// subdomain when the subdomains alone would leave most of the 256 CUs idle,
// else 2 when a subdomain has more than kTeamRows rows (the split then
// mainly cuts large blocks to what one workgroup's LDS holds).
int resolve_team(const pslr_options& o, int64_t n, const int32_t* part, int32_t nparts) {
  if (o.factor != 0 || o.team == 1) return 0;
  if (o.team >= 2) return std::min(o.team, 8);
  if (nparts <= 128) return 4;
  std::vector<int64_t> cnt(nparts, 0);
  for (int64_t i = 0; i < n; ++i) cnt[part[i]]++;
  return *std::max_element(cnt.begin(), cnt.end()) > kTeamRows ? 2 : 0;
}

// Groups of every block of a split family (B_i then C_i, 2 * nparts entries;
// all 0 when team < 2): the team size scaled by the block's share of its
// family's largest block, so that the groups of one launch hold about the
// same number of rows whatever the spread of block sizes, and at least one
// group per kTeamRows rows, so that a group's rows and level scratch fit one
// workgroup's LDS; between 1 and kTeamMax.  2048 rows was the fastest of
// 1024, 2048 and 4096 on 48 uneven 2D systems (blocks of up to 53k rows):
// smaller groups need less LDS, so more workgroups share a CU, until the
// top groups' extra work outweighs that.
constexpr int kTeamMax = 32;
std::vector<int> block_teams(const Blocks& Bk, int team) {
  const int np = (int)Bk.B.size();
  std::vector<int> t(2 * (size_t)np, 0);
  if (team < 2) return t;
  for (int fam = 0; fam < 2; ++fam) {
    const std::vector<CsrL>& M = fam == 0 ? Bk.B : Bk.C0;
    int64_t nmax = 1;
    for (int i = 0; i < np; ++i) nmax = std::max<int64_t>(nmax, M[i].nrows);
    for (int i = 0; i < np; ++i) {
      const int64_t n = M[i].nrows;
      const int64_t share = std::lround(team * (double)n / nmax), fit = (n + kTeamRows - 1) / kTeamRows;
      t[(size_t)fam * np + i] = (int)std::clamp<int64_t>(std::max(share, fit), 1, kTeamMax);
    }
  }
  return t;
}

pslr_status validate_csr(int64_t n, const int64_t* rowptr, const int32_t* colind) {
  if (n < 0 || (n > 0 && (!rowptr || !colind))) return fail(PSLR_EINVAL, "null CSR arrays");
  if (n > 0x7fffffff) return fail(PSLR_EINVAL, "n must fit in int32");
  if (rowptr[0] != 0) return fail(PSLR_EINVAL, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return fail(PSLR_EINVAL, "rowptr not non-decreasing");
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (colind[k] < 0 || colind[k] >= n) return fail(PSLR_EINVAL, "column index out of range");
  }
  return PSLR_OK;
}

pslr_status validate_part(int64_t n, const int32_t* part, int32_t nparts) {
  if (nparts <= 0 || (n > 0 && !part)) return fail(PSLR_EINVAL, "bad part/nparts");
  for (int64_t i = 0; i < n; ++i)
    if (part[i] < 0 || part[i] >= nparts) return fail(PSLR_EINVAL, "label outside [0, nparts)");
  return PSLR_OK;
}

// Build the per-direction host index maps and coupling matrices.
DirHost build_dir(const Reordering& R, const Blocks& Bk, const std::vector<BlockFactor>& fB,
                  const std::vector<BlockFactor>& fC, bool transpose) {
  DirHost D;
  const int np = R.nparts;
  D.gB_in.resize(R.p);
  D.gB_out.resize(R.p);
  D.gC_in.resize(R.q);
  D.gC_out.resize(R.q);
  D.gC_inv.resize(R.q);
  D.Ein.ptr.assign(R.p + 1, 0);
  D.Fout.ptr.assign(R.q + 1, 0);
  for (int i = 0; i < np; ++i) {
    const int64_t i0 = R.int_ptr[i], f0 = R.if_ptr[i];
    const BlockFactor& B = fB[i];
    const BlockFactor& C = fC[i];
    const std::vector<int32_t>& bin = transpose ? B.gout : B.gin;
    const std::vector<int32_t>& bout = transpose ? B.gin : B.gout;
    const std::vector<int32_t>& cin = transpose ? C.gout : C.gin;
    const std::vector<int32_t>& cout = transpose ? C.gin : C.gout;
    for (int p = 0; p < B.n; ++p) {
      D.gB_in[i0 + p] = (int32_t)R.perm[i0 + bin[p]];
      D.gB_out[i0 + p] = (int32_t)R.perm[i0 + bout[p]];
    }
    for (int p = 0; p < C.n; ++p) {
      D.gC_in[f0 + p] = cin[p];
      D.gC_out[f0 + p] = cout[p];
      D.gC_inv[f0 + cin[p]] = p;
    }
  }
  // Ein: row = B-solve input position (global i0 + p); forward: E_i row bin[p];
  // transposed: F_i^T row bin[p] = column bin[p] of F_i.
  // Fout: row = global interface; forward: F_i with columns mapped to B output
  // positions; transposed: E_i^T with columns mapped likewise.
  for (int i = 0; i < np; ++i) {
    const int64_t i0 = R.int_ptr[i], f0 = R.if_ptr[i];
    const BlockFactor& B = fB[i];
    const std::vector<int32_t>& bin = transpose ? B.gout : B.gin;
    const std::vector<int32_t>& bout = transpose ? B.gin : B.gout;
    std::vector<int32_t> boutinv(B.n);
    for (int c = 0; c < B.n; ++c) boutinv[bout[c]] = c;
    const CsrL& E = Bk.E[i];   // p_i x q_i
    const CsrL& F = Bk.F[i];   // q_i x p_i
    // column lists of the matrix feeding Ein (rows = local interior)
    std::vector<std::vector<std::pair<int32_t, double>>> inrows(B.n), outrows(F.nrows);
    if (!transpose) {
      for (int r = 0; r < E.nrows; ++r)
        for (int k = E.ptr[r]; k < E.ptr[r + 1]; ++k) inrows[r].push_back({E.col[k], E.val[k]});
      for (int r = 0; r < F.nrows; ++r)
        for (int k = F.ptr[r]; k < F.ptr[r + 1]; ++k) outrows[r].push_back({boutinv[F.col[k]], F.val[k]});
    } else {
      for (int r = 0; r < F.nrows; ++r)  // F^T: row = local interior F.col, col = r
        for (int k = F.ptr[r]; k < F.ptr[r + 1]; ++k) inrows[F.col[k]].push_back({r, F.val[k]});
      for (int r = 0; r < E.nrows; ++r)  // E^T: row = local interface E.col, col = interior r
        for (int k = E.ptr[r]; k < E.ptr[r + 1]; ++k) outrows[E.col[k]].push_back({boutinv[r], E.val[k]});
    }
    for (int p = 0; p < B.n; ++p) {
      auto& rw = inrows[bin[p]];
      std::sort(rw.begin(), rw.end());
      for (auto& e : rw) {
        D.Ein.col.push_back(e.first);
        D.Ein.val.push_back(e.second);
      }
      D.Ein.ptr[i0 + p + 1] = (int64_t)D.Ein.col.size();
    }
    for (int r = 0; r < F.nrows; ++r) {
      auto& rw = outrows[r];
      std::sort(rw.begin(), rw.end());
      for (auto& e : rw) {
        D.Fout.col.push_back(e.first);
        D.Fout.val.push_back(e.second);
      }
      D.Fout.ptr[f0 + r + 1] = (int64_t)D.Fout.col.size();
    }
  }
  const CsrG& G = Bk.Cg;
  if (!transpose) {
    D.Cg.ptr = G.ptr;
    D.Cg.col = G.col;
    D.Cg.val = G.val;
  } else {
    D.Cg.ptr.assign(R.q + 1, 0);
    for (int32_t c : G.col) D.Cg.ptr[c + 1]++;
    for (int64_t r = 0; r < R.q; ++r) D.Cg.ptr[r + 1] += D.Cg.ptr[r];
    D.Cg.col.resize(G.col.size());
    D.Cg.val.resize(G.col.size());
    std::vector<int64_t> pos(D.Cg.ptr.begin(), D.Cg.ptr.end() - 1);
    for (int64_t r = 0; r < R.q; ++r)
      for (int64_t k = G.ptr[r]; k < G.ptr[r + 1]; ++k) {
        int64_t d = pos[G.col[k]]++;
        D.Cg.col[d] = (int32_t)r;
        D.Cg.val[d] = G.val[k];
      }
  }
  return D;
}

// Team split of one family of blocks (block i in F[i].team subtree groups and
// a top group; no split when no block is divided).  team_top as
// pslr_options.team_top.
// bytes: set to what the team solves read (the groups' packed factors, the
// top groups' packed factors or dense inverses and their row records).
template <typename T>
hipError_t upload_team(DevPool& pool, const std::vector<BlockFactor>& F, int team_top, TeamArrays<T>& out,
                       int& mlr, int64_t& bytes) {
  out = TeamArrays<T>{};
  int team = 0;
  for (const BlockFactor& f : F) team = std::max<int>(team, f.team);
  if (team <= 1) return hipSuccess;  // no block divided: no split
  const int w = (int)sizeof(T);
  const int path = w == 8 ? 0 : 1;
  auto rd = [&](const TriPacked& P) { return P.read_vals[path] * (int64_t)w + 4 * P.read_ints[path]; };
  std::vector<const TriPacked*> ls, us;
  std::vector<int32_t> gptr(1, 0);
  std::vector<int4> item;
  int64_t groups = 0, top_packed = 0, all_vals = 0, dense_vals = 0;
  bool dense_ok = true;
  for (size_t i = 0; i < F.size(); ++i) {
    const BlockFactor& f = F[i];
    const int t = f.team;
    if (t < 1 || (int)f.loS.size() != t + 1 || (int)f.upS.size() != t + 1) return hipErrorInvalidValue;
    for (int g = 0; g <= t; ++g) {
      ls.push_back(&f.loS[g]);
      us.push_back(&f.upS[g]);
      (g < t ? groups : top_packed) += rd(f.loS[g]) + rd(f.upS[g]);
      all_vals += f.loS[g].read_vals[path] + f.upS[g].read_vals[path];
    }
    for (int g = 0; g < t; ++g) item.push_back(make_int4((int)i, gptr.back() + g, g, 0));
    gptr.push_back(gptr.back() + t + 1);
    dense_vals += (int64_t)f.ntop * f.ntop;
    if (f.ntop > 0 && f.topinv.empty()) dense_ok = false;
    out.ntopmax = std::max(out.ntopmax, f.loS[t].n);
  }
  hipError_t e;
  int64_t tb;
  int tmlr = 0;
  if ((e = upload_tri_list(pool, ls, out.L, tmlr, tb))) return e;
  if ((e = upload_tri_list(pool, us, out.U, tmlr, tb))) return e;
  if ((e = pool.upload(gptr, &out.gptr))) return e;
  if ((e = pool.upload(item, &out.item))) return e;
  out.team = team;
  out.nitems = (int32_t)item.size();
  out.maxlr = std::max(tmlr, 1);
  {
    std::vector<int32_t> pos;
    std::vector<int64_t> off(1, 0);
    int maxloc = 1;
    for (const TriPacked* P : ls) {
      if (P->pos.empty() && P->n > 0) return hipErrorInvalidValue;  // groups are packed locally
      pos.insert(pos.end(), P->pos.begin(), P->pos.end());
      off.push_back((int64_t)pos.size());
      maxloc = std::max<int>(maxloc, (int)P->pos.size());
    }
    if (pos.empty()) pos.push_back(0);
    if ((e = pool.upload(pos, &out.pos))) return e;
    if ((e = pool.upload(off, &out.pos_off))) return e;
    out.maxloc = maxloc;
  }
  if (team_top == 2 && !dense_ok) return hipErrorInvalidValue;
  // (blocks without top rows keep the packed path: nothing to multiply)
  const bool dense =
      dense_ok && dense_vals > 0 && (team_top == 2 || (team_top == 0 && dense_vals <= 2 * all_vals));
  bytes = groups + top_packed;
  if (dense) {
    std::vector<T> ti;
    std::vector<int64_t> off(1, 0);
    int64_t rec_bytes = 0;
    for (const BlockFactor& f : F) {
      for (double v : f.topinv) ti.push_back((T)v);
      off.push_back((int64_t)ti.size());
      rec_bytes += 16 * (int64_t)f.ntop;
    }
    if ((e = pool.upload(ti, &out.TI))) return e;
    if ((e = pool.upload(off, &out.ti_off))) return e;
    out.nrb = (out.ntopmax + 63) / 64;
    bytes = groups + dense_vals * w + rec_bytes;
  }
  return hipSuccess;
}

template <typename T>
hipError_t upload_dir(DevPool& pool, const Reordering& R, const std::vector<BlockFactor>& fB,
                      const std::vector<BlockFactor>& fC, const DirHost& D, bool transpose,
                      int team_top, const int64_t* d_int_ptr, const int64_t* d_if_ptr, const int32_t* d_if_orig,
                      ApplyArrays<T>& A, int64_t bytes_out[4]) {
  hipError_t e;
  A.nparts = R.nparts;
  A.n = R.n;
  A.p = R.p;
  A.q = R.q;
  A.int_ptr = d_int_ptr;
  A.if_ptr = d_if_ptr;
  A.if_orig = d_if_orig;
  int mlr = 0;
  int64_t by;
  TriPacked BlockFactor::*lo = transpose ? &BlockFactor::loT : &BlockFactor::lo;
  TriPacked BlockFactor::*up = transpose ? &BlockFactor::upT : &BlockFactor::up;
  const int w = (int)sizeof(T);
  if ((e = upload_tri(pool, fB, lo, A.LB, mlr, by))) return e;
  bytes_out[0] = by;
  if ((e = upload_tri(pool, fB, up, A.UB, mlr, by))) return e;
  bytes_out[0] += by;
  if ((e = upload_tri(pool, fC, lo, A.LC, mlr, by))) return e;
  bytes_out[1] = by;
  if ((e = upload_tri(pool, fC, up, A.UC, mlr, by))) return e;
  bytes_out[1] += by;
  A.TB = TeamArrays<T>{};
  A.TC = TeamArrays<T>{};
  if (!transpose) {
    if ((e = upload_team(pool, fB, team_top, A.TB, mlr, bytes_out[0]))) return e;
    if ((e = upload_team(pool, fC, team_top, A.TC, mlr, bytes_out[1]))) return e;
  }
  A.maxLR = std::max(mlr, 1);
  A.maxPB = A.maxQB = 1;
  for (int i = 0; i < R.nparts; ++i) {
    A.maxPB = std::max<int>(A.maxPB, (int)(R.int_ptr[i + 1] - R.int_ptr[i]));
    A.maxQB = std::max<int>(A.maxQB, (int)(R.if_ptr[i + 1] - R.if_ptr[i]));
  }
  if ((e = pool.upload(D.gB_in, &A.gB_in))) return e;
  if ((e = pool.upload(D.gB_out, &A.gB_out))) return e;
  if ((e = pool.upload(D.gC_in, &A.gC_in))) return e;
  if ((e = pool.upload(D.gC_out, &A.gC_out))) return e;
  if ((e = pool.upload(D.gC_inv, &A.gC_inv))) return e;
  if ((e = upload_csr(pool, D.Ein, A.Ein))) return e;
  if ((e = upload_csr(pool, D.Fout, A.Fout))) return e;
  if ((e = upload_csr(pool, D.Cg, A.Cg))) return e;
  bytes_out[2] = (int64_t)(D.Ein.val.size() + D.Fout.val.size()) * (w + 4) + 8 * (R.p + R.q + 2);
  bytes_out[3] = (int64_t)D.Cg.val.size() * (w + 4) + 8 * (R.q + 1);
  return hipSuccess;
}

template <typename T>
size_t lds_bytes(const ApplyArrays<T>& A, int kmax, int R = 1) {
  return sizeof(T) * (size_t)R *
         ((size_t)A.maxPB + 2 * (size_t)A.maxLR + 2 * (size_t)A.maxQB + 2 * (size_t)std::max(kmax, 1));
}

WsSizes ws_sizes(const pslr_ctx* h, int nrhs) {
  WsSizes z;
  z.vec = (size_t)std::max<int64_t>(h->R.q, 1) * nrhs;
  // V^T y chunk partials, then G W per system (one right-hand side)
  z.partial = (size_t)h->nchunk_lr * nrhs * std::max(h->k, 1) + (size_t)h->nsys * std::max(h->k, 1);
  z.gws = h->gws_stride > 0 ? (size_t)h->gws_stride * ((nrhs + 7) / 8 * 8) : 0;
  // the family vectors and top-row updates of the team solves, each with one
  // slice per right-hand side: [xb: p][dtopb: nitems x ntopmax of B]
  // [xc: q][dtopc: the same of C]
  if (h->fw64.TB.team > 1) {
    const TeamArrays<double>&TB = h->fw64.TB, &TC = h->fw64.TC;
    z.team = (size_t)std::max<int64_t>(h->R.p, 1) + (size_t)TB.nitems * TB.ntopmax;
    if (TC.team > 1) z.team += (size_t)std::max<int64_t>(h->R.q, 1) + (size_t)TC.nitems * TC.ntopmax;
    z.team *= (size_t)std::min(nrhs, h->team_rhs > 0 ? h->team_rhs : kTeamRhsAuto);
  }
  // split G V^T y of the matrix-core low-rank products (BF16 V only)
  if (h->Vbr && nrhs >= kMfmaMinRhs)
    z.zp = ((size_t)h->nsys * 3 * nrhs * ((h->k + 15) / 16 * 16) * 2 + 7) / 8;
  return z;
}

// The handle's apply workspace, grown on demand and never freed while the
// handle lives: a workspace that is outgrown stays allocated (until
// pslr_destroy), so that a HIP graph captured with it still replays on valid
// memory.  Growth rounds the right-hand-side count up to a power of two.
pslr_status ensure_ws(pslr_ctx* h, int nrhs) {
  const WsSizes need = ws_sizes(h, nrhs);
  if (nrhs <= h->ws_nrhs && need.partial <= h->ws_cap.partial && need.gws <= h->ws_cap.gws &&
      need.zp <= h->ws_cap.zp && need.team <= h->ws_cap.team)
    return PSLR_OK;
  int grow = 1;
  while (grow < std::max(nrhs, h->ws_nrhs)) grow *= 2;
  const WsSizes z = ws_sizes(h, grow);
  HIP_TRY(h->ws.alloc<double>(z.vec, (double**)&h->y));
  HIP_TRY(h->ws.alloc<double>(z.vec, (double**)&h->u0));
  HIP_TRY(h->ws.alloc<double>(z.vec, (double**)&h->u1));
  HIP_TRY(h->ws.alloc<double>(z.partial, (double**)&h->partial));
  h->gws = nullptr;
  if (z.gws > 0) HIP_TRY(h->ws.alloc<double>(z.gws, (double**)&h->gws));
  h->zp = nullptr;
  if (z.zp > 0) HIP_TRY(h->ws.alloc<double>(z.zp, (double**)&h->zp));
  h->tws = nullptr;
  if (z.team > 0) HIP_TRY(h->ws.alloc<double>(z.team, (double**)&h->tws));
  h->ws_nrhs = grow;
  h->ws_cap = z;
  return PSLR_OK;
}

// V^T y partial sums and the expansion y += V G V^T y in the handle's V storage type.
template <typename T>
hipError_t lowrank_partial(pslr_ctx* h, const T* y, int64_t ldy, int nrhs, T* part, hipStream_t s);
template <>
hipError_t lowrank_partial<double>(pslr_ctx* h, const double* y, int64_t ldy, int nrhs, double* part,
                                   hipStream_t s) {
  return launch_lr_partial<double, double>(h->nchunk_lr, h->d_chunks, h->k, h->V64, h->R.q, y, ldy, nrhs,
                                           part, h->cur_active, h->nsys, s);
}
template <>
hipError_t lowrank_partial<float>(pslr_ctx* h, const float* y, int64_t ldy, int nrhs, float* part,
                                  hipStream_t s) {
  if (h->Vbf && h->v_bf16)
    return launch_lr_partial<float, __hip_bfloat16>(h->nchunk_lr, h->d_chunks, h->k, h->Vbf, h->R.q, y, ldy,
                                                    nrhs, part, h->cur_active, h->nsys, s);
  return launch_lr_partial<float, float>(h->nchunk_lr, h->d_chunks, h->k, h->V32, h->R.q, y, ldy, nrhs, part,
                                         h->cur_active, h->nsys, s);
}
// y += V G V^T y (gtrans: G^T) for one right-hand side over the whole chip;
// part: nchunk_lr * k values, then nsys * k for G W
template <typename T>
hipError_t lowrank1(pslr_ctx* h, T* y, T* part, int gtrans, hipStream_t s);
template <>
hipError_t lowrank1<double>(pslr_ctx* h, double* y, double* part, int gtrans, hipStream_t s) {
  return launch_lr1<double, double>(h->nchunk_lr, h->d_chunks, h->lr_maxrows, h->nsys, h->d_sys_chunk, h->k,
                                    h->V64, h->R.q, h->G64, gtrans, y, part,
                                    part + (int64_t)h->nchunk_lr * h->k, h->cur_active, s);
}
template <>
hipError_t lowrank1<float>(pslr_ctx* h, float* y, float* part, int gtrans, hipStream_t s) {
  float* z = part + (int64_t)h->nchunk_lr * h->k;
  if (h->Vbf && h->v_bf16)
    return launch_lr1<float, __hip_bfloat16>(h->nchunk_lr, h->d_chunks, h->lr_maxrows, h->nsys, h->d_sys_chunk,
                                             h->k, h->Vbf, h->R.q, h->G32, gtrans, y, part, z, h->cur_active,
                                             s);
  return launch_lr1<float, float>(h->nchunk_lr, h->d_chunks, h->lr_maxrows, h->nsys, h->d_sys_chunk, h->k,
                                  h->V32, h->R.q, h->G32, gtrans, y, part, z, h->cur_active, s);
}
template <typename T>
hipError_t lowrank_expand(pslr_ctx* h, const ApplyArrays<T>& A, const LaunchCfg& c, int nrhs,
                          int gtrans, const T* part, T* y, int64_t ldy, int do_c0, T* u, int64_t ldu);
template <>
hipError_t lowrank_expand<double>(pslr_ctx* h, const ApplyArrays<double>& A, const LaunchCfg& c,
                                  int nrhs, int gtrans, const double* part, double* y, int64_t ldy,
                                  int do_c0, double* u, int64_t ldu) {
  return launch_lr_expand<double, double>(A, c, nrhs, h->k, h->V64, h->G64, gtrans, part,
                                          h->nchunk_lr, h->d_sys_chunk, y, ldy, do_c0, u, ldu);
}
template <>
hipError_t lowrank_expand<float>(pslr_ctx* h, const ApplyArrays<float>& A, const LaunchCfg& c,
                                 int nrhs, int gtrans, const float* part, float* y, int64_t ldy,
                                 int do_c0, float* u, int64_t ldu) {
  if (h->Vbf && h->v_bf16)
    return launch_lr_expand<float, __hip_bfloat16>(A, c, nrhs, h->k, h->Vbf, h->G32, gtrans, part,
                                                   h->nchunk_lr, h->d_sys_chunk, y, ldy, do_c0, u,
                                                   ldu);
  return launch_lr_expand<float, float>(A, c, nrhs, h->k, h->V32, h->G32, gtrans, part, h->nchunk_lr,
                                        h->d_sys_chunk, y, ldy, do_c0, u, ldu);
}

// PH_GAP ends the interval before a kernel-stamped span (not attributed)
enum { PH_START = -1, PH_HEAD = 0, PH_LOWRANK = 1, PH_SERIES = 2, PH_TAIL = 3, PH_GAP = 4 };

// Sum the elapsed times of completed traced applies (all of them if wait).
hipError_t trace_collect(pslr_ctx* h, bool wait) {
  while (!h->ev_pending.empty()) {
    auto& marks = h->ev_pending.front();
    hipEvent_t last = marks.back().second;
    if (wait) {
      hipError_t e = hipEventSynchronize(last);
      if (e != hipSuccess) return e;
    } else if (hipEventQuery(last) != hipSuccess) {
      break;
    }
    for (size_t i = 1; i < marks.size(); ++i) {
      float ms = 0.f;
      hipError_t e = hipEventElapsedTime(&ms, marks[i - 1].second, marks[i].second);
      if (e != hipSuccess) return e;
      switch (marks[i].first) {
        case PH_HEAD: h->tr.ms_head += ms; break;
        case PH_LOWRANK: h->tr.ms_lowrank += ms; break;
        case PH_SERIES: h->tr.ms_series += ms; h->tr.series_launches++; break;
        case PH_TAIL: h->tr.ms_tail += ms; break;
      }
    }
    h->tr.applies++;
    for (auto& mk : marks) h->ev_free.push_back(mk.second);
    h->ev_pending.pop_front();
  }
  return hipSuccess;
}

struct Tracer {
  pslr_ctx* h;
  hipStream_t s;
  std::vector<std::pair<int, hipEvent_t>> marks;
  hipError_t mark(int phase) {
    if (!h->trace) return hipSuccess;
    hipEvent_t e;
    if (!h->ev_free.empty()) {
      e = h->ev_free.back();
      h->ev_free.pop_back();
    } else {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      h->ev_all.push_back(e);
    }
    marks.push_back({phase, e});
    return hipEventRecord(e, s);
  }
  // Events for a launch that stamps its own start and end: the interval up to
  // the start is not attributed, the kernel's duration goes to `phase`.
  hipError_t span(int phase, LaunchCfg& c) {
    if (!h->trace) return hipSuccess;
    hipEvent_t e[2];
    for (hipEvent_t& x : e) {
      if (!h->ev_free.empty()) {
        x = h->ev_free.back();
        h->ev_free.pop_back();
      } else {
        hipError_t r = hipEventCreate(&x);
        if (r != hipSuccess) return r;
        h->ev_all.push_back(x);
      }
    }
    marks.push_back({PH_GAP, e[0]});
    marks.push_back({phase, e[1]});
    c.ev_start = e[0];
    c.ev_stop = e[1];
    return hipSuccess;
  }
  hipError_t finish() {
    if (!h->trace) return hipSuccess;
    h->ev_pending.push_back(std::move(marks));
    return trace_collect(h, h->ev_pending.size() > 512);
  }
};

// Rows per chunk for columns cols: at least ~1024 chunks over all columns so
// that every CU holds several, between 256 and kChunkRows rows each (1024:
// per FGMRES iteration on the 64^3 workload the vector work took 154.5 us
// against 163.3 us with chunks of up to 4096 rows).
int64_t chunk_rows(const std::vector<Seg>& cols) {
  int64_t tot = 0;
  for (const Seg& s : cols) tot += s.len;
  const int64_t r = ((tot + 1023) / 1024 + 255) / 256 * 256;
  return std::min<int64_t>(kChunkRows, std::max<int64_t>(256, r));
}

// Split columns into row chunks of at most rows rows; columns with
// active[c] == 0 get no chunks.  cptr[c] .. cptr[c+1] are column c's chunks.
int make_chunks(const std::vector<Seg>& cols, int64_t rows, const std::vector<uint8_t>* active,
                std::vector<Chunk>& ch, std::vector<int32_t>& cptr) {
  ch.clear();
  cptr.assign(cols.size() + 1, 0);
  for (size_t c = 0; c < cols.size(); ++c) {
    if (!active || (*active)[c])
      for (int64_t r0 = 0; r0 < cols[c].len; r0 += rows)
        ch.push_back(Chunk{(int32_t)c, 0, r0, std::min(cols[c].len, r0 + rows)});
    cptr[c + 1] = (int32_t)ch.size();
  }
  return (int)ch.size();
}

int64_t count_chunks(const std::vector<Seg>& cols, int64_t rows) {
  int64_t t = 0;
  for (const Seg& s : cols) t += (s.len + rows - 1) / rows;
  return std::max<int64_t>(t, 1);
}

constexpr size_t kLrStaticLds = 8192;

// Right-hand-side tile width and working-vector placement of an apply: LDS with
// the widest tile that fits, unless several right-hand sides would then be
// solved one or two at a time (each tile re-reads every factor entry), in
// which case the global workspace with tiles of up to 8.
template <typename T>
LaunchCfg choose_launch(pslr_ctx* h, const ApplyArrays<T>& A, int nrhs, hipStream_t s) {
  LaunchCfg c{h->threads, 0, s, 1, false};
  int want = 1;
  while (want < h->rmax && want < nrhs) want *= 2;
  int Rl = 0;
  if (!h->gx)
    for (int R = want; R >= 1; R /= 2)
      // 8 KB stay free for k_lr_expand's static slice sums
      if (lds_bytes(A, A.kmax, R) + kLrStaticLds <= h->lds_max) {
        Rl = R;
        break;
      }
  if (Rl == 0 || (nrhs >= 4 && Rl < 4)) {
    c.gx = true;
    c.R = want;
  } else {
    c.R = Rl;
    c.lds = lds_bytes(A, A.kmax, Rl);
  }
  return c;
}

// Whether a forward apply (of at most team_rhs right-hand sides) takes the
// team solves: every B_i and C_i solve split over a team of workgroups, each
// holding its group's rows in LDS, so that subdomains too large for one
// workgroup's LDS are served too, as long as each group fits.
template <typename T>
bool team_path(const pslr_ctx* h, const ApplyArrays<T>& A) {
  return A.TB.team > 1 && A.TC.team > 1 && team_lds_bytes(A.TB, A.maxQB) <= h->lds_max &&
         team_lds_bytes(A.TC, A.maxQB) <= h->lds_max;
}

// Device workspace of one apply (see WsSizes).
struct ApplyWs {
  void *y, *u0, *u1, *partial, *gws, *zp, *team;
};

// z = M^{-1} b (or M^{-T} b) with apply arrays A and workspace W (large
// enough for nrhs right-hand sides); trace: record the phase events.
template <typename T>
pslr_status run_apply(pslr_ctx* h, const ApplyArrays<T>& Ah, const ApplyWs& W, bool transpose,
                      int nrhs, const double* b, int64_t ldb, double* z, int64_t ldz, hipStream_t s,
                      bool trace = true) {
  ApplyArrays<T> A = Ah;
  A.active = h->cur_active;
  A.gws = W.gws;
  const int64_t q = std::max<int64_t>(h->R.q, 1);
  LaunchCfg cfg = choose_launch(h, A, nrhs, s);
  T* y = (T*)W.y;
  T* ua = (T*)W.u0;
  T* ub = (T*)W.u1;
  T* part = (T*)W.partial;
  const int k = h->k;
  const bool tr_on = h->trace;
  if (!trace) h->trace = false;
  struct Restore {
    pslr_ctx* h;
    bool v;
    ~Restore() { h->trace = v; }
  } restore{h, tr_on};
  Tracer tr{h, s, {}};
  // the team solves (workspace layout as in ws_sizes) for up to team_rhs
  // right-hand sides; automatic: one, or up to kTeamRhsAuto when the tiled
  // path would keep its working vectors in global memory (each right-hand
  // side then costs a read of the factors, but in LDS)
  const int trhs = h->team_rhs > 0 ? h->team_rhs : (cfg.gx ? kTeamRhsAuto : 1);
  const bool team = W.team && nrhs <= trhs && !transpose && team_path<T>(h, A);
  TeamWs tw{};
  if (team) {
    T* t = (T*)W.team;
    tw.ldxb = std::max<int64_t>(h->R.p, 1);
    tw.lddb = (int64_t)A.TB.nitems * A.TB.ntopmax;
    tw.ldxc = std::max<int64_t>(h->R.q, 1);
    tw.lddc = (int64_t)A.TC.nitems * A.TC.ntopmax;
    tw.xb = t;
    t += tw.ldxb * nrhs;
    tw.dtopb = t;
    t += tw.lddb * nrhs;
    tw.xc = t;
    t += tw.ldxc * nrhs;
    tw.dtopc = t;
  }
  HIP_TRY(tr.mark(PH_START));
  if (team) HIP_TRY(launch_head_team<T>(A, cfg, nrhs, b, ldb, y, q, tw));
  else HIP_TRY(launch_head<T>(A, cfg, nrhs, b, ldb, y, q));
  HIP_TRY(tr.mark(PH_HEAD));
  // FP32 applies with V in BF16 and many right-hand sides: the low-rank
  // products on the matrix cores, then the C0 solve on its own
  const bool mfma = sizeof(T) == 4 && k > 0 && h->Vbf && h->v_bf16 && h->Vbr && W.zp &&
                    nrhs >= kMfmaMinRhs;
  if (!transpose) {
    if (mfma) {
      HIP_TRY(launch_lr_mfma(h->nchunk_lr, h->d_chunks, h->nsys, h->d_sys_chunk, k, h->Vbf, h->R.q,
                             h->Vbr, h->G32, 0, (float*)y, q, nrhs, (float*)part,
                             (__hip_bfloat16*)W.zp, h->cur_active, s));
      if (team) HIP_TRY(launch_c0_team<T>(A, cfg, nrhs, y, ua, q, tw));
      else HIP_TRY(launch_c0solve<T>(A, cfg, nrhs, y, q, ua, q));
    } else if (k > 0 && nrhs == 1) {
      HIP_TRY(lowrank1<T>(h, y, part, 0, s));
      if (team) HIP_TRY(launch_c0_team<T>(A, cfg, nrhs, y, ua, q, tw));
      else HIP_TRY(launch_c0solve<T>(A, cfg, nrhs, y, q, ua, q));
    } else if (k > 0) {
      HIP_TRY(lowrank_partial<T>(h, y, q, nrhs, part, s));
      // the expansion fused with the C0 solve, or the C_i team solves after it
      HIP_TRY(lowrank_expand<T>(h, A, cfg, nrhs, 0, part, y, q, team ? 0 : 1, ua, q));
      if (team) HIP_TRY(launch_c0_team<T>(A, cfg, nrhs, y, ua, q, tw));
    } else if (team) {
      HIP_TRY(launch_c0_team<T>(A, cfg, nrhs, y, ua, q, tw));
    } else {
      HIP_TRY(launch_c0solve<T>(A, cfg, nrhs, y, q, ua, q));
    }
    HIP_TRY(tr.mark(PH_LOWRANK));
    for (int i = 0; i < h->m; ++i) {
      LaunchCfg c1 = cfg;
      HIP_TRY(tr.span(PH_SERIES, c1));
      if (team) HIP_TRY(launch_series_team<T>(A, c1, nrhs, y, ua, ub, q, 1, tw));
      else HIP_TRY(launch_series<T>(A, c1, nrhs, y, q, ua, ub, q, 1, 1));
      std::swap(ua, ub);
    }
  } else {
    HIP_TRY(launch_c0solve<T>(A, cfg, nrhs, y, q, ua, q));
    HIP_TRY(tr.mark(PH_LOWRANK));
    for (int i = 0; i < h->m; ++i) {
      LaunchCfg c1 = cfg;
      HIP_TRY(tr.span(PH_SERIES, c1));
      HIP_TRY(launch_series<T>(A, c1, nrhs, y, q, ua, ub, q, 1, 1));
      std::swap(ua, ub);
    }
    if (mfma) {
      HIP_TRY(launch_lr_mfma(h->nchunk_lr, h->d_chunks, h->nsys, h->d_sys_chunk, k, h->Vbf, h->R.q,
                             h->Vbr, h->G32, 1, (float*)ua, q, nrhs, (float*)part,
                             (__hip_bfloat16*)W.zp, h->cur_active, s));
      HIP_TRY(tr.mark(PH_LOWRANK));
    } else if (k > 0 && nrhs == 1) {
      HIP_TRY(lowrank1<T>(h, ua, part, 1, s));
      HIP_TRY(tr.mark(PH_LOWRANK));
    } else if (k > 0) {
      HIP_TRY(lowrank_partial<T>(h, ua, q, nrhs, part, s));
      HIP_TRY(lowrank_expand<T>(h, A, cfg, nrhs, 1, part, ua, q, 0, ub, q));
      HIP_TRY(tr.mark(PH_LOWRANK));
    }
  }
  if (team) HIP_TRY(launch_tail_team<T>(A, cfg, nrhs, b, ldb, ua, q, z, ldz, tw));
  else HIP_TRY(launch_tail<T>(A, cfg, nrhs, b, ldb, ua, q, z, ldz));
  HIP_TRY(tr.mark(PH_TAIL));
  HIP_TRY(tr.finish());
  return PSLR_OK;
}

pslr_status apply_dir(pslr_ctx* h, bool transpose, int nrhs, const double* b, int64_t ldb, double* z,
                      int64_t ldz, hipStream_t s, bool force64 = false) {
  if (h->R.n == 0) return PSLR_OK;
  pslr_status st = ensure_ws(h, nrhs);
  if (st != PSLR_OK) return st;
  const ApplyWs W{h->y, h->u0, h->u1, h->partial, h->gws, h->zp, h->tws};
  if (h->precision >= 1 && !force64 && h->have32)
    return run_apply<float>(h, transpose ? h->tr32 : h->fw32, W, transpose, nrhs, b, ldb, z, ldz, s);
  if (!h->have64) return fail(PSLR_EINVAL, "FP64 apply arrays not available");
  return run_apply<double>(h, transpose ? h->tr64 : h->fw64, W, transpose, nrhs, b, ldb, z, ldz, s);
}

// ---- small dense helpers (host)

// G = (I - H)^{-1} - I with LU and partial pivoting; false if I - H is singular.
bool compute_G(int k, const std::vector<double>& H, std::vector<double>& G) {
  std::vector<double> M((size_t)k * k), X((size_t)k * k, 0.0);
  double nrm = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      M[(size_t)i * k + j] = (i == j ? 1.0 : 0.0) - H[(size_t)j * k + i];  // H column-major
      nrm = std::max(nrm, std::fabs(M[(size_t)i * k + j]));
    }
  for (int i = 0; i < k; ++i) X[(size_t)i * k + i] = 1.0;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(M[(size_t)r * k + c]) > std::fabs(M[(size_t)piv * k + c])) piv = r;
    if (!(std::fabs(M[(size_t)piv * k + c]) > 1e-14 * nrm)) return false;
    if (piv != c)
      for (int j = 0; j < k; ++j) {
        std::swap(M[(size_t)c * k + j], M[(size_t)piv * k + j]);
        std::swap(X[(size_t)c * k + j], X[(size_t)piv * k + j]);
      }
    for (int r = 0; r < k; ++r) {
      if (r == c) continue;
      const double f = M[(size_t)r * k + c] / M[(size_t)c * k + c];
      if (f == 0.0) continue;
      for (int j = 0; j < k; ++j) {
        M[(size_t)r * k + j] -= f * M[(size_t)c * k + j];
        X[(size_t)r * k + j] -= f * X[(size_t)c * k + j];
      }
    }
  }
  G.assign((size_t)k * k, 0.0);  // row-major
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      G[(size_t)i * k + j] = X[(size_t)i * k + j] / M[(size_t)i * k + i] - (i == j ? 1.0 : 0.0);
  return true;
}

// Upload V (union q x k row-major, apply precision) and one G per system for
// the current hV (q x k column-major) and hH (nsys blocks of k x k column-major).
pslr_status upload_lowrank(pslr_ctx* h) {
  // the replaced V and G stay allocated until the handle is destroyed (a
  // captured apply may still read them)
  for (void* p : h->vpool.ptrs) h->vretired.ptrs.push_back(p);
  h->vretired.bytes += h->vpool.bytes;
  h->vpool.ptrs.clear();
  h->vpool.bytes = 0;
  h->V64 = h->G64 = nullptr;
  h->Vbf = nullptr;
  h->Vbr = nullptr;
  h->V32 = nullptr;
  h->G32 = nullptr;
  const int k = h->k;
  const int64_t q = h->R.q;
  if (k == 0) return PSLR_OK;
  h->hG.assign((size_t)h->nsys * k * k, 0.0);
  for (int s = 0; s < h->nsys; ++s) {
    const int ks = h->sys_k[s];
    if (ks == 0) continue;
    std::vector<double> Hs((size_t)ks * ks), Gs;
    for (int j = 0; j < ks; ++j)
      for (int i = 0; i < ks; ++i) Hs[(size_t)j * ks + i] = h->hH[(size_t)s * k * k + (size_t)j * k + i];
    if (!compute_G(ks, Hs, Gs)) return fail(PSLR_ESINGULAR, "I - H is singular");
    for (int i = 0; i < ks; ++i)
      for (int j = 0; j < ks; ++j) h->hG[(size_t)s * k * k + (size_t)i * k + j] = Gs[(size_t)i * ks + j];
  }
  // V is kept column-major (column j at V + j*q), as the Arnoldi process builds it
  if (h->precision == 0) {
    HIP_TRY(h->vpool.upload(h->hV, &h->V64));
    HIP_TRY(h->vpool.upload(h->hG, &h->G64));
  } else {
    std::vector<float> G32(h->hG.begin(), h->hG.end());
    HIP_TRY(h->vpool.upload(G32, &h->G32));
    // FP32 V always (the BF16 form falls back to it, see probe_bf16)
    std::vector<float> Vr(h->hV.begin(), h->hV.end());
    HIP_TRY(h->vpool.upload(Vr, &h->V32));
    if (h->precision == 2) {
      std::vector<__hip_bfloat16> Vb((size_t)q * k);
      for (size_t e = 0; e < Vb.size(); ++e) Vb[e] = __float2bfloat16((float)h->hV[e]);
      HIP_TRY(h->vpool.upload(Vb, &h->Vbf));
      // the same values row-major with k padded to a multiple of 16 (matrix-core expansion)
      if (k <= 256) {
        const int kp = (k + 15) / 16 * 16;
        std::vector<__hip_bfloat16> Vr((size_t)q * kp, __float2bfloat16(0.0f));
        for (int j = 0; j < k; ++j)
          for (int64_t r = 0; r < q; ++r) Vr[(size_t)r * kp + j] = Vb[(size_t)j * q + r];
        HIP_TRY(h->vpool.upload(Vr, &h->Vbr));
      }
    }
  }
  return PSLR_OK;
}

// Precision 2 keeps V in BF16 only where that rounding (8 significant bits)
// leaves the apply within kBf16ProbeTol of the FP32-V apply, measured on one
// fixed vector: BF16 rounding breaks the orthonormality of V, and the
// resulting change of the low-rank term is amplified by the conditioning of
// the rest of the preconditioner, up to O(1) on ill-conditioned blocks.  Else
// V stays in FP32 (pslr_info.v_bf16 = 0).  bf16_probe keeps the measured
// relative difference.
constexpr double kBf16ProbeTol = 2.5e-2;
pslr_status probe_bf16(pslr_ctx* h, hipStream_t s) {
  h->v_bf16 = false;
  h->bf16_probe = 0.0;
  if (h->precision != 2 || h->k == 0 || !h->Vbf || !h->have32 || h->R.n == 0) return PSLR_OK;
  const int64_t n = h->R.n;
  DevPool tmp;
  double *b, *z;
  HIP_TRY(tmp.alloc<double>(n, &b));
  HIP_TRY(tmp.alloc<double>(2 * n, &z));
  std::vector<double> hb(n), hz(2 * n);
  uint64_t st = 0x5eed;
  for (int64_t i = 0; i < n; ++i) hb[i] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 - 0.5;
  HIP_TRY(hipMemcpy(b, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  const bool tr = h->trace;
  h->trace = false;
  for (int pass = 0; pass < 2; ++pass) {
    h->v_bf16 = pass == 0;
    pslr_status r = apply_dir(h, false, 1, b, n, z + pass * n, n, s, false);
    if (r) {
      h->trace = tr;
      return r;
    }
  }
  h->trace = tr;
  HIP_TRY(hipMemcpyAsync(hz.data(), z, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double d2 = 0.0, r2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    d2 += (hz[i] - hz[n + i]) * (hz[i] - hz[n + i]);
    r2 += hz[n + i] * hz[n + i];
  }
  h->bf16_probe = r2 > 0 ? std::sqrt(d2 / r2) : 0.0;
  h->v_bf16 = std::isfinite(h->bf16_probe) && h->bf16_probe <= kBf16ProbeTol;
  return PSLR_OK;
}

// r_k-step Arnoldi on E_rr(m) = (E_s C0^{-1})^{m+1} (Theorem t2), classical
// Gram-Schmidt with one full re-orthogonalisation, FP64 on the device.  The
// systems of a batched handle run their Arnoldi processes together: E_rr is
// block diagonal by system, and the Gram-Schmidt sums are taken per system.
pslr_status arnoldi(pslr_ctx* h, const double* v0host, uint64_t seed, hipStream_t s, bool& breakdown) {
  const int64_t q = h->R.q;
  const int ns = h->nsys;
  int64_t qmax = 0;
  for (int c = 0; c < ns; ++c) qmax = std::max(qmax, h->sys_q[c + 1] - h->sys_q[c]);
  int kreq = (int)std::min<int64_t>(h->rank, qmax);
  breakdown = false;
  h->k = 0;
  h->sys_k.assign(ns, 0);
  h->hV.clear();
  h->hH.clear();
  if (kreq <= 0) return upload_lowrank(h);
  DevPool tmp;
  double *Vd, *w, *ua, *ub, *dbuf, *dhh, *scl;
  HIP_TRY(tmp.alloc<double>((size_t)q * (kreq + 1), &Vd));
  HIP_TRY(tmp.alloc<double>(q, &w));
  HIP_TRY(tmp.alloc<double>(q, &ua));
  HIP_TRY(tmp.alloc<double>(q, &ub));
  std::vector<Seg> qcols(ns);
  for (int c = 0; c < ns; ++c) qcols[c] = Seg{h->sys_q[c], h->sys_q[c + 1] - h->sys_q[c]};
  std::vector<Chunk> chv;
  std::vector<int32_t> cpv;
  const int nch = make_chunks(qcols, chunk_rows(qcols), nullptr, chv, cpv);
  Chunk* dch;
  int32_t* dcp;
  HIP_TRY(tmp.alloc<Chunk>(std::max(nch, 1), &dch));
  HIP_TRY(tmp.alloc<int32_t>(ns + 1, &dcp));
  if (nch > 0) HIP_TRY(hipMemcpy(dch, chv.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dcp, cpv.data(), sizeof(int32_t) * (ns + 1), hipMemcpyHostToDevice));
  HIP_TRY(tmp.alloc<double>((size_t)std::max(nch, 1) * (kreq + 1), &dbuf));
  HIP_TRY(tmp.alloc<double>((size_t)ns * (2 * (kreq + 1) + 2), &dhh));
  HIP_TRY(tmp.alloc<double>(ns, &scl));
  double* dh1 = dhh;
  double* dh2 = dhh + (size_t)ns * (kreq + 1);
  double* dnn = dh2 + (size_t)ns * (kreq + 1);
  double* dwn = dnn + ns;
  std::vector<double> v(q);
  if (v0host) {
    std::copy(v0host, v0host + q, v.begin());
  } else {
    uint64_t st = seed;
    for (int64_t i = 0; i < q; ++i) v[i] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 - 0.5;
  }
  std::vector<int> active(ns, 0);
  for (int c = 0; c < ns; ++c) {
    double nv = 0.0;
    for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    const int64_t qc = h->sys_q[c + 1] - h->sys_q[c];
    if (nv > 0.0 && qc > 0) {
      active[c] = 1;
      for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) v[i] /= nv;
    } else {
      for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) v[i] = 0.0;
    }
  }
  HIP_TRY(hipMemcpy(Vd, v.data(), sizeof(double) * q, hipMemcpyHostToDevice));
  ApplyArrays<double> A = h->fw64;
  A.gws = h->gws;  // the workspace for one right-hand side exists (ensure_ws at setup)
  LaunchCfg cfg = choose_launch(h, A, 1, s);
  std::vector<double> Hb((size_t)ns * (kreq + 1) * kreq, 0.0), hb((size_t)ns * (2 * (kreq + 1) + 2)),
      sc(ns);
  std::vector<int> kdone(ns, 0);
  const Seg* cols = h->d_qcols;
  for (int j = 0; j < kreq; ++j) {
    const double* cur = Vd + (size_t)j * q;
    for (int r = 0; r <= h->m; ++r) {
      HIP_TRY(launch_c0solve<double>(A, cfg, 1, cur, q, ua, q));
      HIP_TRY(launch_series<double>(A, cfg, 1, ua, q, ua, ub, q, 0, 0));
      cur = ub;
    }
    HIP_TRY(hipMemcpyAsync(w, ub, sizeof(double) * q, hipMemcpyDeviceToDevice, s));
    const int nv = j + 1;
    HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, 1, w, 0, w, dbuf, s));
    HIP_TRY(launch_reduce_chunk(ns, dcp, 1, nch, dbuf, dwn, s));
    HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, nv, Vd, q, w, dbuf, s));
    HIP_TRY(launch_reduce_chunk(ns, dcp, nv, nch, dbuf, dh1, s));
    HIP_TRY(launch_maxpy_chunk(nch, dch, cols, cols, nv, Vd, q, dh1, nv, w, 1.0, s));
    HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, nv, Vd, q, w, dbuf, s));
    HIP_TRY(launch_reduce_chunk(ns, dcp, nv, nch, dbuf, dh2, s));
    HIP_TRY(launch_maxpy_chunk(nch, dch, cols, cols, nv, Vd, q, dh2, nv, w, 1.0, s));
    HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, 1, w, 0, w, dbuf, s));
    HIP_TRY(launch_reduce_chunk(ns, dcp, 1, nch, dbuf, dnn, s));
    HIP_TRY(hipMemcpyAsync(hb.data(), dhh, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* h1 = hb.data();
    const double* h2 = h1 + (size_t)ns * (kreq + 1);
    const double* nn = h2 + (size_t)ns * (kreq + 1);
    const double* wn = nn + ns;
    bool any = false;
    for (int c = 0; c < ns; ++c) {
      sc[c] = 0.0;
      if (!active[c]) continue;
      double* Hc = &Hb[((size_t)c * kreq + j) * (kreq + 1)];
      for (int i = 0; i <= j; ++i) Hc[i] = h1[(size_t)c * nv + i] + h2[(size_t)c * nv + i];
      const double hn = std::sqrt(nn[c]);
      Hc[j + 1] = hn;
      const int64_t qc = h->sys_q[c + 1] - h->sys_q[c];
      if (hn <= 1e-14 * std::sqrt(wn[c]) || j + 1 >= qc) {
        kdone[c] = j + 1;
        active[c] = 0;
        if (j + 1 < kreq && j + 1 < qc) breakdown = true;
        continue;
      }
      kdone[c] = j + 1;
      sc[c] = 1.0 / hn;
      any = true;
    }
    if (!any) break;
    HIP_TRY(hipMemcpyAsync(scl, sc.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_scale_chunk(nch, dch, cols, cols, w, scl, Vd + (size_t)(j + 1) * q, s));
  }
  int kmax = 0;
  for (int c = 0; c < ns; ++c) kmax = std::max(kmax, kdone[c]);
  h->k = kmax;
  h->sys_k = kdone;
  h->hV.assign((size_t)q * kmax, 0.0);
  if (kmax > 0) HIP_TRY(hipMemcpy(h->hV.data(), Vd, sizeof(double) * q * kmax, hipMemcpyDeviceToHost));
  for (int c = 0; c < ns; ++c)  // columns beyond a system's rank are zero on its rows
    for (int j = kdone[c]; j < kmax; ++j)
      for (int64_t r = h->sys_q[c]; r < h->sys_q[c + 1]; ++r) h->hV[(size_t)j * q + r] = 0.0;
  h->hH.assign((size_t)ns * kmax * kmax, 0.0);
  for (int c = 0; c < ns; ++c)
    for (int j = 0; j < kdone[c]; ++j)
      for (int i = 0; i < kdone[c]; ++i)
        h->hH[(size_t)c * kmax * kmax + (size_t)j * kmax + i] = Hb[((size_t)c * kreq + j) * (kreq + 1) + i];
  return upload_lowrank(h);
}

// Widen the apply layouts for a low-rank term of k columns: the global
// workspace holds 2k scratch values per block, the LDS working set 2k.
void grow_kmax(pslr_ctx* h, int k) {
  if (k <= h->fw64.kmax) return;
  h->gws_stride += (int64_t)h->R.nparts * 2 * (k - h->fw64.kmax);
  for (ApplyArrays<double>* A : {&h->fw64, &h->tr64}) {
    A->kmax = k;
    A->gws_stride = h->gws_stride;
  }
  for (ApplyArrays<float>* A : {&h->fw32, &h->tr32}) {
    A->kmax = k;
    A->gws_stride = h->gws_stride;
  }
  if (k > h->rank) h->rank = k;
}

// Deflated low-rank correction (lowrank = 1, 2): Krylov-Schur restarting
// (Stewart, SIAM J. Matrix Anal. Appl. 23, 2001) of the Arnoldi process on
// E_rr(m) = (E_s C0^{-1})^{m+1} (Thm. t2).  The paper motivates the low-rank
// term as a deflation of the eigenvalues of modulus above 1 (Sec. 3.2.2); a
// raw r_k-step Arnoldi basis only approximates that invariant subspace, this
// converges it.  Each cycle expands the basis to k + p vectors (FP64 CGS2 on
// the device, as in arnoldi()), then on the host keeps the invariant subspace
// of the projected matrix for its k Ritz values of largest modulus
// (schur_select), rotates the basis on the device and continues from the
// coupling vector, until the coupling is below kKsTol times the smallest kept
// modulus.  lowrank = 2 also raises k (up to 256) while every kept Ritz value
// lies outside the unit circle, so that all of modulus above 1 are kept.
// The result keeps the paper's form: V orthonormal, H = V^T E_rr V, G from H.
//
// Systems of a batched handle run together: every apply acts on one global
// basis column for all systems.  Each system's basis occupies positions
// 0..k_s-1 after a restart (zero columns up to the common continuation
// position K, the largest k_s) and its own rows of V.
constexpr double kKsTol = 1e-9;
constexpr int kKsMaxRestarts = 60;
constexpr int kKsMaxRank = 256;

pslr_status krylov_schur(pslr_ctx* h, const double* v0host, uint64_t seed, int mode, hipStream_t s,
                         bool& breakdown) {
  const int64_t q = h->R.q;
  const int ns = h->nsys;
  std::vector<int64_t> qs(ns);
  int64_t qmax = 0;
  for (int c = 0; c < ns; ++c) {
    qs[c] = h->sys_q[c + 1] - h->sys_q[c];
    qmax = std::max(qmax, qs[c]);
  }
  const int kreq = (int)std::min<int64_t>(h->rank, qmax);
  breakdown = false;
  h->k = 0;
  h->sys_k.assign(ns, 0);
  h->hV.clear();
  h->hH.clear();
  h->info.ks_restarts = 0;
  h->info.ks_applies = 0;
  h->info.ks_residual = 0.0;
  h->info.ritz_above_one = 0;
  if (kreq <= 0) return upload_lowrank(h);
  const int kcap = mode == 2 ? (int)std::min<int64_t>(kKsMaxRank, qmax) : kreq;
  // global basis positions: at most kcap kept + p expansion vectors + 1
  const int Mc = (int)std::min<int64_t>(qmax + 1, (int64_t)kcap + std::max(kcap, 16) + 1);
  DevPool tmp;
  double *Vd, *Vn, *w, *ua, *ub, *dbuf, *dhh, *scl, *dW;
  HIP_TRY(tmp.alloc<double>((size_t)q * (Mc + 1), &Vd));
  HIP_TRY(tmp.alloc<double>((size_t)q * (Mc + 1), &Vn));
  HIP_TRY(tmp.alloc<double>(q, &w));
  HIP_TRY(tmp.alloc<double>(q, &ua));
  HIP_TRY(tmp.alloc<double>(q, &ub));
  std::vector<Seg> qcols(ns);
  for (int c = 0; c < ns; ++c) qcols[c] = Seg{h->sys_q[c], qs[c]};
  std::vector<Chunk> chv;
  std::vector<int32_t> cpv;
  const int nch = make_chunks(qcols, chunk_rows(qcols), nullptr, chv, cpv);
  Chunk *dch, *dchr;
  int32_t* dcp;
  HIP_TRY(tmp.alloc<Chunk>(std::max(nch, 1), &dch));
  HIP_TRY(tmp.alloc<Chunk>(std::max(nch, 1), &dchr));
  HIP_TRY(tmp.alloc<int32_t>(ns + 1, &dcp));
  if (nch > 0) HIP_TRY(hipMemcpy(dch, chv.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dcp, cpv.data(), sizeof(int32_t) * (ns + 1), hipMemcpyHostToDevice));
  HIP_TRY(tmp.alloc<double>((size_t)std::max(nch, 1) * (Mc + 1), &dbuf));
  HIP_TRY(tmp.alloc<double>((size_t)ns * (2 * (Mc + 1) + 2), &dhh));
  HIP_TRY(tmp.alloc<double>(ns, &scl));
  HIP_TRY(tmp.alloc<double>((size_t)ns * (Mc + 1) * (Mc + 1), &dW));
  double* dh1 = dhh;
  double* dh2 = dhh + (size_t)ns * (Mc + 1);
  double* dnn = dh2 + (size_t)ns * (Mc + 1);
  double* dwn = dnn + ns;
  // start vector (the same rule as arnoldi())
  std::vector<double> v(q);
  if (v0host) {
    std::copy(v0host, v0host + q, v.begin());
  } else {
    uint64_t st = seed;
    for (int64_t i = 0; i < q; ++i) v[i] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 - 0.5;
  }
  struct Sys {
    bool active = false;  // still expanding in this cycle
    bool done = false;    // final basis at positions 0..kept-1
    bool broke = false;   // invariant subspace found in this cycle
    int ktarget = 0, kept = 0;
    std::vector<int> pos;  // basis positions (the continuation vector last, when present)
    std::vector<double> Hk;
    double res = 0.0;
    int restarts = 0;
  };
  std::vector<Sys> S(ns);
  for (int c = 0; c < ns; ++c) {
    double nv = 0.0;
    for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    S[c].ktarget = (int)std::min<int64_t>(kreq, qs[c]);
    if (nv > 0.0 && qs[c] > 0 && S[c].ktarget > 0) {
      S[c].active = true;
      S[c].pos = {0};
      for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) v[i] /= nv;
    } else {
      S[c].done = true;
      for (int64_t i = h->sys_q[c]; i < h->sys_q[c + 1]; ++i) v[i] = 0.0;
    }
  }
  HIP_TRY(hipMemcpy(Vd, v.data(), sizeof(double) * q, hipMemcpyHostToDevice));
  // per-system projected matrix in global positions, (Mc + 1) x Mc column-major
  const size_t ldH = (size_t)Mc + 1;
  std::vector<double> Hs((size_t)ns * ldH * Mc, 0.0);
  auto Hat = [&](int c, int i, int j) -> double& { return Hs[((size_t)c * Mc + j) * ldH + i]; };
  ApplyArrays<double> A = h->fw64;
  A.gws = h->gws;
  LaunchCfg cfg = choose_launch(h, A, 1, s);
  std::vector<double> hb((size_t)ns * (2 * (Mc + 1) + 2)), sc(ns);
  const Seg* cols = h->d_qcols;
  int K = 0;  // continuation position of this cycle
  int64_t applies = 0;
  for (int cycle = 0;; ++cycle) {
    // basis of k + p vectors (p = max(k, 16)): the kept ones (positions below
    // K) and the new ones from the continuation position K on
    int kt = 0;
    for (int c = 0; c < ns; ++c)
      if (!S[c].done) kt = std::max(kt, S[c].ktarget);
    const int mend = std::min(std::max(K, kt) + std::max(kt, 16), Mc - 1);
    for (int c = 0; c < ns; ++c) S[c].broke = false;
    // ---- expansion: columns K .. mend-1 produce positions K+1 .. mend
    for (int j = K; j < mend; ++j) {
      bool any = false;
      for (int c = 0; c < ns; ++c) any = any || S[c].active;
      if (!any) break;
      const double* cur = Vd + (size_t)j * q;
      for (int r = 0; r <= h->m; ++r) {
        HIP_TRY(launch_c0solve<double>(A, cfg, 1, cur, q, ua, q));
        HIP_TRY(launch_series<double>(A, cfg, 1, ua, q, ua, ub, q, 0, 0));
        cur = ub;
      }
      ++applies;
      HIP_TRY(hipMemcpyAsync(w, ub, sizeof(double) * q, hipMemcpyDeviceToDevice, s));
      const int nv = j + 1;
      HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, 1, w, 0, w, dbuf, s));
      HIP_TRY(launch_reduce_chunk(ns, dcp, 1, nch, dbuf, dwn, s));
      HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, nv, Vd, q, w, dbuf, s));
      HIP_TRY(launch_reduce_chunk(ns, dcp, nv, nch, dbuf, dh1, s));
      HIP_TRY(launch_maxpy_chunk(nch, dch, cols, cols, nv, Vd, q, dh1, nv, w, 1.0, s));
      HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, nv, Vd, q, w, dbuf, s));
      HIP_TRY(launch_reduce_chunk(ns, dcp, nv, nch, dbuf, dh2, s));
      HIP_TRY(launch_maxpy_chunk(nch, dch, cols, cols, nv, Vd, q, dh2, nv, w, 1.0, s));
      HIP_TRY(launch_mdot_chunk(nch, dch, cols, cols, 1, w, 0, w, dbuf, s));
      HIP_TRY(launch_reduce_chunk(ns, dcp, 1, nch, dbuf, dnn, s));
      HIP_TRY(hipMemcpyAsync(hb.data(), dhh, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double* h1 = hb.data();
      const double* h2 = h1 + (size_t)ns * (Mc + 1);
      const double* nn = h2 + (size_t)ns * (Mc + 1);
      const double* wn = nn + ns;
      for (int c = 0; c < ns; ++c) {
        sc[c] = 0.0;
        if (!S[c].active) continue;
        for (int i = 0; i <= j; ++i) Hat(c, i, j) = h1[(size_t)c * nv + i] + h2[(size_t)c * nv + i];
        const double hn = std::sqrt(nn[c]);
        Hat(c, j + 1, j) = hn;
        if (hn <= 1e-14 * std::sqrt(wn[c]) || (int64_t)S[c].pos.size() >= qs[c]) {
          // invariant subspace, or the whole space of this system
          S[c].active = false;
          S[c].broke = true;
          Hat(c, j + 1, j) = 0.0;
          continue;
        }
        S[c].pos.push_back(j + 1);
        sc[c] = 1.0 / hn;
      }
      HIP_TRY(hipMemcpyAsync(scl, sc.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
      HIP_TRY(launch_scale_chunk(nch, dch, cols, cols, w, scl, Vd + (size_t)(j + 1) * q, s));
    }
    // ---- host: sorted Schur truncation per system
    std::vector<char> rot(ns, 0);
    for (int c = 0; c < ns; ++c) rot[c] = !S[c].done;
    std::vector<std::vector<double>> Wsel(ns);
    std::vector<std::vector<double>> bcoup(ns);
    int Knext = 0, ncols = 0;
    bool cont_any = false;
    for (int c = 0; c < ns; ++c) {
      Sys& y = S[c];
      if (y.done) continue;
      const bool has_cont = !y.broke;  // the last position is the continuation vector
      const int mb = (int)y.pos.size() - (has_cont ? 1 : 0);
      std::vector<double> Hm((size_t)mb * mb);
      for (int b = 0; b < mb; ++b)
        for (int a = 0; a < mb; ++a) Hm[(size_t)b * mb + a] = Hat(c, y.pos[a], y.pos[b]);
      const double hlast = has_cont ? Hat(c, y.pos[mb], y.pos[mb - 1]) : 0.0;
      std::vector<double> W, Hk, rr, ri;
      std::string err;
      const int kept = schur_select(mb, Hm.data(), mb, std::min(y.ktarget, mb), W, Hk, rr, ri, err);
      if (kept < 0) return fail(PSLR_ESINGULAR, "Krylov-Schur: " + err);
      if (kept > kKsMaxRank)
        return fail(PSLR_ENOTSUP, "Krylov-Schur: eigenvalues tied in modulus at the cut take the "
                                  "kept count above 256");
      std::vector<double> b(kept);
      double bn = 0.0;
      for (int t = 0; t < kept; ++t) {
        b[t] = hlast * W[(size_t)t * mb + (mb - 1)];
        bn += b[t] * b[t];
      }
      bn = std::sqrt(bn);
      const double minmod = kept > 0 ? std::hypot(rr[kept - 1], ri[kept - 1]) : 1.0;
      y.res = kept > 0 ? bn / std::max(minmod, 1e-300) : 0.0;
      y.restarts = cycle;
      const bool full = !has_cont || (int64_t)mb >= qs[c];
      bool conv = full || bn <= kKsTol * std::max(minmod, 1e-300) || cycle >= kKsMaxRestarts;
      if (conv && mode == 2 && !full && kept > 0 && minmod > 1.0 && y.ktarget < kcap &&
          cycle < kKsMaxRestarts) {
        // every kept Ritz value lies outside the unit circle: keep more
        int above = 0;
        for (int t = 0; t < mb; ++t) above += std::hypot(rr[t], ri[t]) > 1.0;
        y.ktarget = std::min(kcap, std::max(y.ktarget + 16, above + 16));
        conv = false;
      }
      if (kept == 0) conv = true;
      y.kept = kept;
      y.Hk = Hk;
      bcoup[c] = b;
      if (conv) {
        y.done = true;
        y.active = false;
      } else {
        cont_any = true;
        Knext = std::max(Knext, kept);
      }
      Wsel[c] = std::move(W);
      ncols = std::max(ncols, kept);
    }
    // ---- device: rotate the basis of every system that restarted or finished
    // in this cycle; continuing systems get their continuation vector at Knext
    if (cont_any) ncols = std::max(ncols, Knext + 1);
    if (ncols > 0) {
      const int mcols = mend + 1;
      std::vector<double> Wall((size_t)ns * mcols * ncols, 0.0);
      std::vector<Chunk> chr;
      for (int c = 0; c < ns; ++c) {
        if (!rot[c]) continue;
        const Sys& y = S[c];
        const int mb = (int)y.pos.size() - (y.broke ? 0 : 1);
        double* Wc = &Wall[(size_t)c * mcols * ncols];
        for (int t = 0; t < y.kept; ++t)
          for (int a = 0; a < mb; ++a) Wc[(size_t)t * mcols + y.pos[a]] = Wsel[c][(size_t)t * mb + a];
        if (!y.done) Wc[(size_t)Knext * mcols + y.pos.back()] = 1.0;  // continuation vector
        for (int e = cpv[c]; e < cpv[c + 1]; ++e) chr.push_back(chv[e]);
      }
      if (!chr.empty()) {
        HIP_TRY(hipMemcpyAsync(dW, Wall.data(), sizeof(double) * Wall.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(dchr, chr.data(), sizeof(Chunk) * chr.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_basis_rotate((int)chr.size(), dchr, cols, mcols, ncols, Vd, q, dW, Vn, q, s));
        // copy the rotated columns back (rows of the rotated systems only)
        for (int c = 0; c < ns; ++c) sc[c] = 1.0;
        HIP_TRY(hipMemcpyAsync(scl, sc.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
        for (int t = 0; t < ncols; ++t)
          HIP_TRY(launch_scale_chunk((int)chr.size(), dchr, cols, cols, Vn + (size_t)t * q, scl,
                                     Vd + (size_t)t * q, s));
        HIP_TRY(hipStreamSynchronize(s));
      }
    }
    // ---- projected matrices of the continuing systems
    for (int c = 0; c < ns; ++c) {
      Sys& y = S[c];
      if (y.done) continue;
      std::fill(&Hat(c, 0, 0), &Hat(c, 0, 0) + ldH * Mc, 0.0);
      for (int jj = 0; jj < y.kept; ++jj)
        for (int i = 0; i < y.kept; ++i) Hat(c, i, jj) = y.Hk[(size_t)jj * y.kept + i];
      for (int t = 0; t < y.kept; ++t) Hat(c, Knext, t) = bcoup[c][t];
      y.pos.clear();
      for (int t = 0; t < y.kept; ++t) y.pos.push_back(t);
      y.pos.push_back(Knext);
      y.active = true;
    }
    if (!cont_any) break;
    K = Knext;
  }
  // ---- results: V (union q x kmax, zero beyond each system's rank) and H per system
  int kmax = 0;
  for (int c = 0; c < ns; ++c) kmax = std::max(kmax, S[c].kept);
  h->k = kmax;
  for (int c = 0; c < ns; ++c) h->sys_k[c] = S[c].kept;
  h->hV.assign((size_t)q * kmax, 0.0);
  if (kmax > 0) HIP_TRY(hipMemcpy(h->hV.data(), Vd, sizeof(double) * q * kmax, hipMemcpyDeviceToHost));
  for (int c = 0; c < ns; ++c)
    for (int j = S[c].kept; j < kmax; ++j)
      for (int64_t r = h->sys_q[c]; r < h->sys_q[c + 1]; ++r) h->hV[(size_t)j * q + r] = 0.0;
  h->hH.assign((size_t)ns * kmax * kmax, 0.0);
  int above = 0, rmax = 0;
  double resmax = 0.0;
  for (int c = 0; c < ns; ++c) {
    const int kc = S[c].kept;
    for (int j = 0; j < kc; ++j)
      for (int i = 0; i < kc; ++i) h->hH[(size_t)c * kmax * kmax + (size_t)j * kmax + i] = S[c].Hk[(size_t)j * kc + i];
    if (kc > 0) {
      std::vector<double> W, Hk, rr, ri;
      std::string err;
      if (schur_select(kc, S[c].Hk.data(), kc, kc, W, Hk, rr, ri, err) >= 0)
        for (int t = 0; t < kc; ++t) above += std::hypot(rr[t], ri[t]) > 1.0;
    }
    resmax = std::max(resmax, S[c].res);
    rmax = std::max(rmax, S[c].restarts);
    if (S[c].kept < std::min<int64_t>(kreq, qs[c])) breakdown = true;
  }
  h->info.ks_restarts = rmax;
  h->info.ks_applies = applies;
  h->info.ks_residual = resmax;
  h->info.ritz_above_one = above;
  if (kmax > h->fw64.kmax) grow_kmax(h, kmax);
  return upload_lowrank(h);
}

// Pick the workgroup size and the chunk-count scaling of the triangular solves by
// timing applies (one right-hand side, HIP events) over a small grid of choices,
// then the widest right-hand-side tile (applies of 8 right-hand sides).
pslr_status autotune(pslr_ctx* h, hipStream_t s) {
  const int64_t n = h->R.n;
  if (n == 0) return PSLR_OK;
  DevPool tmp;
  double *b, *z;
  HIP_TRY(tmp.alloc<double>(n, &b));
  HIP_TRY(tmp.alloc<double>(n, &z));
  {
    std::vector<double> hb(n);
    uint64_t st = 12345;
    for (int64_t i = 0; i < n; ++i) hb[i] = (double)(splitmix64_next(st) >> 11) * 0x1.0p-53 - 0.5;
    HIP_TRY(hipMemcpy(b, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const bool tr = h->trace;
  h->trace = false;
  float best = 1e30f;
  int bt = h->threads, bg = 0;
  const int fixed = h->threads_fixed ? h->threads : 0;
  for (int threads : {512, 1024})
    for (int gs : {-1, 0, 1}) {
      if (fixed && threads != fixed) continue;
      h->threads = threads;
      for (auto* A : {&h->fw64, &h->tr64}) A->gshift = gs;
      for (auto* A : {&h->fw32, &h->tr32}) A->gshift = gs;
      float tmin = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(hipEventRecord(e0, s));
        pslr_status st = apply_dir(h, false, 1, b, n, z, n, s);
        if (st) return st;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        bt = threads;
        bg = gs;
      }
    }
  h->threads = bt;
  for (auto* A : {&h->fw64, &h->tr64}) A->gshift = bg;
  for (auto* A : {&h->fw32, &h->tr32}) A->gshift = bg;
  // widest right-hand-side tile: applies of 8 right-hand sides with tiles of at
  // most 8, 4, 2 and 1.  Narrower tiles read each factor more often but spread
  // the largest subdomains over more workgroups.
  {
    const int nr = 8;
    double *b8, *z8;
    HIP_TRY(tmp.alloc<double>(n * nr, &b8));
    HIP_TRY(tmp.alloc<double>(n * nr, &z8));
    for (int r = 0; r < nr; ++r)
      HIP_TRY(hipMemcpyAsync(b8 + (int64_t)r * n, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    // the narrowest cap within 5% of the fastest: inside FGMRES, tiles whose
    // columns have all converged are skipped, which favours narrow tiles
    float tr_ms[4];
    const int caps[4] = {8, 4, 2, 1};
    for (int ci = 0; ci < 4; ++ci) {
      const int rm = caps[ci];
      h->rmax = rm;
      float tmin = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(hipEventRecord(e0, s));
        pslr_status st = apply_dir(h, false, nr, b8, n, z8, n, s);
        if (st) return st;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tmin = std::min(tmin, ms);
      }
      tr_ms[ci] = tmin;
    }
    const float bestr = *std::min_element(tr_ms, tr_ms + 4);
    int br = 8;
    for (int ci = 0; ci < 4; ++ci)
      if (tr_ms[ci] <= 1.05f * bestr) br = caps[ci];
    h->rmax = br;
  }
  h->trace = tr;
  h->tuned_threads = bt;
  h->tuned_gshift = bg;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PSLR_OK;
}

void fill_info(pslr_ctx* h, const std::vector<BlockFactor>& fB, const std::vector<BlockFactor>& fC,
               const Blocks& Bk, const int64_t bytes[4]) {
  pslr_info_t& I = h->info;
  I.n = h->R.n;
  I.p = h->R.p;
  I.q = h->R.q;
  I.nparts = h->R.nparts;
  I.m = h->m;
  I.rank = h->k;
  I.precision = h->precision;
  I.nnz_A = h->nnzA;
  I.nnz_E = I.nnz_F = 0;
  for (auto& E : Bk.E) I.nnz_E += E.nnz();
  for (auto& F : Bk.F) I.nnz_F += F.nnz();
  I.nnz_Cg = (int64_t)Bk.Cg.col.size();
  I.nnz_LU_B = I.nnz_LU_C0 = 0;
  I.supernodes_B = I.supernodes_C0 = 0;
  I.max_levels_B = I.max_levels_C0 = 0;
  for (auto& f : fB) {
    I.nnz_LU_B += f.nnz_L + f.nnz_U;
    I.supernodes_B += f.nsuper;
    I.max_levels_B = std::max(I.max_levels_B, f.lo.nlev);
  }
  for (auto& f : fC) {
    I.nnz_LU_C0 += f.nnz_L + f.nnz_U;
    I.supernodes_C0 += f.nsuper;
    I.max_levels_C0 = std::max(I.max_levels_C0, f.lo.nlev);
  }
  const double nA = std::max<int64_t>(h->nnzA, 1);
  I.fill_lu = (double)(I.nnz_LU_B + I.nnz_LU_C0) / nA;
  I.fill_lowrank = ((double)h->R.q * h->k + (double)h->k * h->k) / nA;
  I.fill_total = I.fill_lu + I.fill_lowrank;
  // algorithmic bytes: factor/matrix data once per use, vectors once per read/write
  const int w = h->precision >= 1 ? 4 : 8;
  const int wv = h->precision == 2 && h->v_bf16 ? 2 : w;
  const int m = h->m;
  const int64_t p = h->R.p, q = h->R.q, n = h->R.n, k = h->k;
  const int64_t bB = bytes[0], bC = bytes[1], bEF = bytes[2], bCg = bytes[3];
  const int64_t vecB = (int64_t)w * 2 * p, vecC = (int64_t)w * 2 * q;  // one gather in, one scatter out
  const int64_t series = bB + bC + bEF + bCg + vecB + vecC + (int64_t)w * 3 * q + 8 * 2 * q;
  I.series_bytes = series;
  I.team = h->fw64.TB.team > 1 ? h->fw64.TB.team : 0;
  I.team_top = I.team ? (h->fw64.TB.TI ? 2 : 1) : 0;
  I.team_c = h->fw64.TC.team > 1 ? h->fw64.TC.team : 0;
  I.team_top_c = I.team_c ? (h->fw64.TC.TI ? 2 : 1) : 0;
  const bool tp = h->precision >= 1 ? team_path<float>(h, h->fw32) : team_path<double>(h, h->fw64);
  I.team_apply = tp ? 2 : 0;
  const int64_t matrix = (m + 2) * bB + (m + 1) * bC + (m + 1) * bEF + m * bCg + 2 * q * k * wv +
                         k * k * w;
  const int64_t vectors = (int64_t)(m + 2) * vecB + (m + 1) * vecC + (int64_t)w * (2 * m + 3) * q +
                          (int64_t)(8 + w) * n * 2;
  I.apply_bytes = matrix + vectors;
  I.apply_bytes_rhs = vectors;
  I.nsys = h->nsys;
  I.global_vectors = h->gx ? 1 : 0;
  I.threads = h->threads;
  I.lane_shift = h->fw64.gshift;
  I.max_tile = h->rmax;
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================

extern "C" {

void pslr_default_options(pslr_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m = 3;
  o->rank = 16;
  o->precision = 0;
  o->want_transpose = 0;
  o->v0 = nullptr;
  o->seed = 1;
  o->pivot_threshold = 0.1;
  o->nthreads = 0;
  o->working_vectors = 0;
  o->autotune = 0;
  o->threads = 0;
  o->factor = 0;
  o->drop_tol = 1e-2;
  o->lowrank = 0;
  o->team = 0;
  o->team_top = 0;
  o->team_rhs = 0;
}

const char* pslr_status_string(pslr_status s) {
  switch (s) {
    case PSLR_OK: return "PSLR_OK";
    case PSLR_EINVAL: return "PSLR_EINVAL";
    case PSLR_ESINGULAR: return "PSLR_ESINGULAR";
    case PSLR_ENOCONV: return "PSLR_ENOCONV";
    case PSLR_EBREAKDOWN: return "PSLR_EBREAKDOWN";
    case PSLR_ENOMEM: return "PSLR_ENOMEM";
    case PSLR_EHIP: return "PSLR_EHIP";
    case PSLR_ENOTSUP: return "PSLR_ENOTSUP";
  }
  return "PSLR_UNKNOWN";
}

const char* pslr_last_error(void) { return g_last_error.c_str(); }

pslr_status pslr_partition_geometric(int32_t ndim, const int32_t* dims, const int32_t* parts,
                                     int32_t* label) {
  if (ndim < 1 || ndim > 3 || !dims || !parts || !label) return fail(PSLR_EINVAL, "bad arguments");
  int64_t n = 1;
  for (int d = 0; d < ndim; ++d) {
    if (dims[d] <= 0 || parts[d] <= 0 || parts[d] > dims[d]) return fail(PSLR_EINVAL, "bad dims/parts");
    n *= dims[d];
  }
  for (int64_t v = 0; v < n; ++v) {
    int64_t rem = v, mult = 1, lab = 0;
    for (int d = 0; d < ndim; ++d) {
      const int64_t i = rem % dims[d];
      rem /= dims[d];
      lab += mult * ((i * parts[d]) / dims[d]);
      mult *= parts[d];
    }
    label[v] = (int32_t)lab;
  }
  return PSLR_OK;
}

pslr_status pslr_partition_region_growing(int64_t n, const int64_t* rowptr, const int32_t* colind,
                                          int32_t nparts, uint64_t seed, int32_t* label,
                                          int32_t* nlabels) {
  pslr_status st = validate_csr(n, rowptr, colind);
  if (st) return st;
  if (nparts <= 0 || !label) return fail(PSLR_EINVAL, "bad nparts/label");
  std::vector<int64_t> sp;
  std::vector<int32_t> si;
  symmetric_pattern(n, rowptr, colind, sp, si);
  std::fill(label, label + n, -1);
  std::vector<int64_t> queue;
  queue.reserve(n);
  uint64_t state = seed;
  int32_t next = 0;
  const int32_t want = (int32_t)std::min<int64_t>(nparts, n);
  while (next < want) {
    const int64_t v = (int64_t)(splitmix64_next(state) % (uint64_t)n);
    if (label[v] >= 0) continue;
    label[v] = next++;
    queue.push_back(v);
  }
  auto grow = [&](size_t head) {
    while (head < queue.size()) {
      const int64_t v = queue[head++];
      for (int64_t k = sp[v]; k < sp[v + 1]; ++k) {
        const int32_t w = si[k];
        if (label[w] < 0) {
          label[w] = label[v];
          queue.push_back(w);
        }
      }
    }
  };
  grow(0);
  for (int64_t v = 0; v < n; ++v)
    if (label[v] < 0) {
      label[v] = next++;
      const size_t h0 = queue.size();
      queue.push_back(v);
      grow(h0);
    }
  if (nlabels) *nlabels = next;
  return PSLR_OK;
}

pslr_status pslr_reorder(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const int32_t* part, int32_t nparts, int64_t* perm, int64_t* p, int64_t* q) {
  pslr_status st = validate_csr(n, rowptr, colind);
  if (st) return st;
  if ((st = validate_part(n, part, nparts))) return st;
  Reordering R = reorder(n, rowptr, colind, part, nparts);
  if (perm) std::copy(R.perm.begin(), R.perm.end(), perm);
  if (p) *p = R.p;
  if (q) *q = R.q;
  return PSLR_OK;
}

pslr_status pslr_host_stats(int64_t n, const int64_t* rowptr, const int32_t* colind,
                            const double* vals, const int32_t* part, int32_t nparts,
                            const pslr_options* opt, pslr_host_stats_t* out) {
  pslr_status st = validate_csr(n, rowptr, colind);
  if (st) return st;
  if ((st = validate_part(n, part, nparts))) return st;
  if (!out) return fail(PSLR_EINVAL, "out is NULL");
  pslr_options o;
  pslr_default_options(&o);
  if (opt) o = *opt;
  if (o.factor != 0 && o.factor != 1) return fail(PSLR_EINVAL, "factor must be 0 or 1");
  if (o.lowrank < 0 || o.lowrank > 2) return fail(PSLR_EINVAL, "lowrank must be 0, 1 or 2");
  if (o.team < 0 || o.team > 8) return fail(PSLR_EINVAL, "team must be 0 .. 8");
  const int team = resolve_team(o, n, part, nparts);
  const double tau = o.pivot_threshold > 0 ? o.pivot_threshold : 0.1;
  const double drop = o.drop_tol > 0 ? o.drop_tol : 1e-2;
  Reordering R = reorder(n, rowptr, colind, part, nparts);
  Blocks Bk = extract_blocks(n, rowptr, colind, vals, R);
  std::vector<const CsrL*> mats;
  for (auto& b : Bk.B) mats.push_back(&b);
  for (auto& c : Bk.C0) mats.push_back(&c);
  const int nB = (int)Bk.B.size();
  const std::vector<int> bteam = block_teams(Bk, o.factor == 0 ? team : 0);
  std::vector<double> fres(mats.size(), 0.0), sres(mats.size(), 0.0);
  std::vector<std::string> errs(mats.size());
  std::vector<int> codes(mats.size(), 0), lvl(mats.size(), 0), valid(mats.size(), 1),
      tvalid(mats.size(), 1);
  std::vector<double> tres(mats.size(), 0.0);
  std::vector<int64_t> tslots(mats.size(), 0);
  std::vector<int64_t> nnz(mats.size(), 0);
  parallel_for((int)mats.size(), o.nthreads, [&](int t) {
    const CsrL& M = *mats[t];
    const int narrow = t < nB ? kNarrowWidthB : kNarrowWidthC;
    BlockFactor f;
    IlutFactors I;
    if (o.factor == 1) {
      codes[t] = ilut_block(M, drop, o.want_transpose != 0, narrow, f, errs[t]);
      if (!codes[t]) codes[t] = ilut_factor(M, drop, I, errs[t]);
    } else {
      codes[t] = factor_block(M, tau, o.want_transpose != 0, narrow, f, errs[t], bteam[t],
                              t < nB ? kTopRowsB : kTopRowsC);
    }
    if (codes[t] || M.nrows == 0) return;
    if (f.team >= 1) {
      // team split: structure, and the groups applied in turn (subtrees, then
      // the top group's lower and upper solves, then the subtrees' upper
      // solves) against the plain packed solve
      std::string terr;
      if (!check_team(f, terr)) tvalid[t] = 0;
      // LDS slots of one team workgroup: the group's local vector and two
      // halves of level scratch (as the device layout)
      int maxloc = 1, maxlr = 1;
      for (int g = 0; g <= f.team; ++g) {
        maxloc = std::max<int>(maxloc, (int)f.loS[g].pos.size());
        maxlr = std::max({maxlr, f.loS[g].max_lrows, f.upS[g].max_lrows});
      }
      tslots[t] = ((maxloc + 1) & ~1) + 2 * (int64_t)maxlr;
      const int nb = M.nrows;
      std::vector<double> X0(nb), X1(nb);
      for (int i = 0; i < nb; ++i) X0[i] = X1[i] = std::cos(0.3 + 0.71 * i);
      host_tri_solve(f.lo, X0, true);
      host_tri_solve(f.up, X0, true);
      std::vector<double> X2(X1);
      for (int g = 0; g <= f.team; ++g) host_tri_solve_pos(f.loS[g], X1, true);
      host_tri_solve_pos(f.upS[f.team], X1, true);
      for (int g = 0; g < f.team; ++g) host_tri_solve_pos(f.upS[g], X1, true);
      // the top group through its dense inverse
      if (!f.topinv.empty()) {
        for (int g = 0; g < f.team; ++g) host_tri_solve_pos(f.loS[g], X2, true);
        const int nt = f.ntop;
        const std::vector<int32_t>& tp = f.loS[f.team].pos;
        std::vector<double> d(nt + 1, 0.0);
        for (int k = 0; k < nt; ++k) d[k] = X2[tp[k]];
        for (int r = 0; r < nt; ++r) {
          double acc = 0.0;
          const size_t ld = (size_t)top_ld(nt);
          for (int c = 0; c < (nt + 1) / 2; ++c)
            acc += f.topinv[2 * (c * ld + r)] * d[2 * c] + f.topinv[2 * (c * ld + r) + 1] * d[2 * c + 1];
          X2[tp[r]] = acc;
        }
        for (int g = 0; g < f.team; ++g) host_tri_solve_pos(f.upS[g], X2, true);
      }
      double d2 = 0.0, e2 = 0.0, n2 = 0.0;
      for (int i = 0; i < nb; ++i) {
        d2 += (X0[i] - X1[i]) * (X0[i] - X1[i]);
        if (!f.topinv.empty()) e2 += (X0[i] - X2[i]) * (X0[i] - X2[i]);
        n2 += X0[i] * X0[i];
      }
      tres[t] = n2 > 0 ? std::sqrt(std::max(d2, e2) / n2) : 0.0;
    }
    nnz[t] = f.nnz_L + f.nnz_U;
    lvl[t] = f.lo.nlev;
    std::string lerr;
    for (const TriPacked* T : {&f.lo, &f.up, &f.loT, &f.upT})
      if ((T == &f.loT || T == &f.upT) && !o.want_transpose) continue;
      else if (!check_levels(*T, lerr)) valid[t] = 0;
    const int nb = M.nrows;
    // residual of the solve layouts: x = F^{-1} b through the packed layouts
    // (narrow levels once through their entry form, once through their panels)
    // against the reference solve with the same factors: M x = b for the exact
    // LU (b = M xe), the plain sparse triangular solves for the ILU
    for (int pass = 0; pass < 2 * (o.want_transpose ? 2 : 1); ++pass) {
      const int tr = pass >> 1;
      const bool entries = (pass & 1) == 0;
      std::vector<double> xe(nb), bb(nb, 0.0), X(nb), x(nb);
      for (int i = 0; i < nb; ++i) xe[i] = std::sin(1.0 + i);
      if (o.factor == 1) {
        // reference x = (L U)^{-1} b or (L U)^{-T} b for b = sin(1 + i)
        bb = xe;
        std::vector<double> y = bb;
        if (!tr) {
          for (int i = 0; i < nb; ++i)
            for (const auto& e : I.L[i]) y[i] -= e.second * y[e.first];
          for (int i = nb - 1; i >= 0; --i) {
            for (const auto& e : I.U[i]) y[i] -= e.second * y[e.first];
            y[i] /= I.d[i];
          }
        } else {
          for (int i = 0; i < nb; ++i) {
            y[i] /= I.d[i];
            for (const auto& e : I.U[i]) y[e.first] -= e.second * y[i];
          }
          for (int i = nb - 1; i >= 0; --i)
            for (const auto& e : I.L[i]) y[e.first] -= e.second * y[i];
        }
        xe = y;
      } else {
        for (int i = 0; i < nb; ++i)
          for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
            if (!tr) bb[i] += M.val[k] * xe[M.col[k]];
            else bb[M.col[k]] += M.val[k] * xe[i];
          }
      }
      const std::vector<int32_t>& gi = tr ? f.gout : f.gin;
      const std::vector<int32_t>& go = tr ? f.gin : f.gout;
      for (int pp = 0; pp < nb; ++pp) X[pp] = bb[gi[pp]];
      host_tri_solve(tr ? f.loT : f.lo, X, entries);
      host_tri_solve(tr ? f.upT : f.up, X, entries);
      for (int c = 0; c < nb; ++c) x[go[c]] = X[c];
      double e2 = 0.0, n2 = 0.0;
      for (int i = 0; i < nb; ++i) {
        e2 += (x[i] - xe[i]) * (x[i] - xe[i]);
        n2 += xe[i] * xe[i];
      }
      sres[t] = std::max(sres[t], std::sqrt(e2 / n2));
    }
    if (o.factor == 1) {
      // (M - L U)_ij on the kept pattern of L + U, relative to ||M[i, :]||_2
      std::vector<double> urow(nb, 0.0), mrow(nb, 0.0), lu(nb, 0.0);
      for (int i = 0; i < nb; ++i) {
        double nr = 0.0;
        for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
          mrow[M.col[k]] = M.val[k];
          nr += M.val[k] * M.val[k];
        }
        nr = std::sqrt(nr);
        // row i of L U = sum_k L_ik U[k, :] + U[i, :]
        auto addrow = [&](int k, double s) {
          lu[k] += s * I.d[k];
          for (const auto& e : I.U[k]) lu[e.first] += s * e.second;
        };
        for (const auto& e : I.L[i]) addrow(e.first, e.second);
        addrow(i, 1.0);
        double worst = 0.0;
        for (const auto& e : I.L[i]) worst = std::max(worst, std::fabs(mrow[e.first] - lu[e.first]));
        worst = std::max(worst, std::fabs(mrow[i] - lu[i]));
        for (const auto& e : I.U[i]) worst = std::max(worst, std::fabs(mrow[e.first] - lu[e.first]));
        fres[t] = std::max(fres[t], worst / nr);
        for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) mrow[M.col[k]] = 0.0;
        for (const auto& e : I.L[i]) {
          lu[e.first] = 0.0;
          for (const auto& u : I.U[e.first]) lu[u.first] = 0.0;
        }
        lu[i] = 0.0;
        for (const auto& e : I.U[i]) lu[e.first] = 0.0;
      }
      return;
    }
    // exact LU: ||M x - b|| / (||M|| ||x||) for x = F^{-1} b on a second vector
    std::vector<double> bb(nb, 0.0), X(nb), x(nb), rr(nb, 0.0);
    for (int i = 0; i < nb; ++i) bb[i] = std::cos(0.5 + 0.37 * i);
    for (int pp = 0; pp < nb; ++pp) X[pp] = bb[f.gin[pp]];
    host_tri_solve(f.lo, X, true);
    host_tri_solve(f.up, X, true);
    for (int c = 0; c < nb; ++c) x[f.gout[c]] = X[c];
    double mnorm = 0.0, xn = 0.0, rn = 0.0;
    for (int i = 0; i < nb; ++i) {
      double rs = 0.0;
      for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
        rr[i] += M.val[k] * x[M.col[k]];
        rs += std::fabs(M.val[k]);
      }
      mnorm = std::max(mnorm, rs);
      xn = std::max(xn, std::fabs(x[i]));
      rn = std::max(rn, std::fabs(rr[i] - bb[i]));
    }
    fres[t] = rn / (mnorm * xn);
  });
  for (size_t t = 0; t < mats.size(); ++t)
    if (codes[t]) return fail(codes[t] == 3 ? PSLR_ENOTSUP : PSLR_ESINGULAR, errs[t]);
  *out = pslr_host_stats_t{};
  out->levels_valid = 1;
  out->team = team;
  out->team_valid = 1;
  for (size_t t = 0; t < mats.size(); ++t) {
    if (!tvalid[t]) out->team_valid = 0;
    out->team_residual = std::max(out->team_residual, tres[t]);
    int64_t& sl = (int)t < nB ? out->team_lds_slots_B : out->team_lds_slots_C;
    sl = std::max(sl, tslots[t]);
    if ((int)t < nB) {
      out->team_items_B += bteam[t];
      out->team_groups_max_B = std::max(out->team_groups_max_B, bteam[t]);
    }
  }
  for (size_t t = 0; t < mats.size(); ++t) {
    const bool b = (int)t < nB;
    (b ? out->nnz_LU_B : out->nnz_LU_C0) += nnz[t];
    int32_t& L = b ? out->max_levels_B : out->max_levels_C0;
    L = std::max(L, lvl[t]);
    out->levels_valid &= valid[t];
    out->factor_residual = std::max(out->factor_residual, fres[t]);
    out->solve_residual = std::max(out->solve_residual, sres[t]);
  }
  return PSLR_OK;
}

pslr_status pslr_host_schur_select(int32_t n, const double* Hm, int64_t ldh, int32_t k, double* W,
                                   int64_t ldw, double* Hk, int64_t ldk, double* ritz_re,
                                   double* ritz_im, int32_t* kept) {
  if (n < 0 || k < 0 || !kept || (n > 0 && (!Hm || ldh < n)) || (k > 0 && n > 0 && (!W || !Hk)) ||
      ldw < n || ldk < n)
    return fail(PSLR_EINVAL, "bad arguments");
  std::vector<double> w, hk, rr, ri;
  std::string err;
  const int kp = schur_select(n, Hm, ldh, k, w, hk, rr, ri, err);
  if (kp < 0) return fail(PSLR_ESINGULAR, err);
  for (int j = 0; j < kp; ++j) {
    for (int i = 0; i < n; ++i) W[(size_t)j * ldw + i] = w[(size_t)j * n + i];
    for (int i = 0; i < kp; ++i) Hk[(size_t)j * ldk + i] = hk[(size_t)j * kp + i];
  }
  for (int i = 0; i < n; ++i) {
    if (ritz_re) ritz_re[i] = rr[i];
    if (ritz_im) ritz_im[i] = ri[i];
  }
  *kept = kp;
  return PSLR_OK;
}

pslr_status pslr_host_selfcheck(int64_t n, const int64_t* rowptr, const int32_t* colind,
                                const double* vals, const int32_t* part, int32_t nparts,
                                const pslr_options* opt, double* factor_residual,
                                double* solve_residual) {
  pslr_host_stats_t S;
  const pslr_status st = pslr_host_stats(n, rowptr, colind, vals, part, nparts, opt, &S);
  if (st) return st;
  if (!S.levels_valid) return fail(PSLR_EINVAL, "a packed factor failed the level-schedule check");
  if (factor_residual) *factor_residual = S.factor_residual;
  if (solve_residual) *solve_residual = S.solve_residual;
  return PSLR_OK;
}

}  // extern "C"

namespace {

// Setup of a handle over nsys independent systems (rows sys_ptr[s] ..
// sys_ptr[s+1]); a plain handle is the case nsys = 1.
pslr_status setup_impl(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                       const int32_t* part, int32_t nparts, int32_t nsys, const int64_t* sys_ptr,
                       const pslr_options* opt, void* hip_stream, pslr_handle* out) {
  if (!out) return fail(PSLR_EINVAL, "out is NULL");
  *out = nullptr;
  pslr_status st = validate_csr(n, rowptr, colind);
  if (st) return st;
  if ((st = validate_part(n, part, nparts))) return st;
  if (n > 0 && !vals) return fail(PSLR_EINVAL, "vals is NULL");
  pslr_options o;
  pslr_default_options(&o);
  if (opt) o = *opt;
  if (o.m < 0) return fail(PSLR_EINVAL, "m < 0");
  if (o.rank < 0) return fail(PSLR_EINVAL, "rank < 0");
  if (o.precision < 0 || o.precision > 2) return fail(PSLR_EINVAL, "precision must be 0, 1 or 2");
  if (o.threads != 0 && o.threads != 512 && o.threads != 1024)
    return fail(PSLR_EINVAL, "threads must be 0, 512 or 1024");
  if (o.factor != 0 && o.factor != 1) return fail(PSLR_EINVAL, "factor must be 0 or 1");
  if (o.lowrank < 0 || o.lowrank > 2) return fail(PSLR_EINVAL, "lowrank must be 0, 1 or 2");
  if (o.team < 0 || o.team > 8) return fail(PSLR_EINVAL, "team must be 0 .. 8");
  if (o.team_top < 0 || o.team_top > 2) return fail(PSLR_EINVAL, "team_top must be 0, 1 or 2");
  if (o.team_rhs < 0 || o.team_rhs > 64) return fail(PSLR_EINVAL, "team_rhs must be 0 .. 64");
  o.team = resolve_team(o, n, part, nparts);
  const double tau = o.pivot_threshold > 0 ? o.pivot_threshold : 0.1;
  for (int64_t k = 0; k < (n > 0 ? rowptr[n] : 0); ++k)
    if (!std::isfinite(vals[k])) return fail(PSLR_EINVAL, "non-finite value in A");
  hipStream_t s = (hipStream_t)hip_stream;
  std::unique_ptr<pslr_ctx> h(new pslr_ctx());
  HIP_TRY(hipGetDevice(&h->device));
  {
    const pslr_status sa = scratch_attach(h->device);
    if (sa != PSLR_OK) return sa;
  }
  h->m = o.m;
  h->rank = std::min(o.rank, 256);
  h->precision = o.precision;
  h->want_T = o.want_transpose ? 1 : 0;
  h->nnzA = n > 0 ? rowptr[n] : 0;
  // systems: rows, subdomain labels and couplings must not straddle two systems,
  // and the labels of system s must precede those of system s + 1
  h->nsys = nsys;
  h->sys_n.assign(sys_ptr, sys_ptr + nsys + 1);
  if (h->sys_n[0] != 0 || h->sys_n[nsys] != n) return fail(PSLR_EINVAL, "sys_ptr must span 0..n");
  std::vector<int32_t> lab_sys(nparts, -1), row_sys(n);
  for (int s = 0; s < nsys; ++s) {
    if (h->sys_n[s + 1] < h->sys_n[s]) return fail(PSLR_EINVAL, "sys_ptr not non-decreasing");
    for (int64_t i = h->sys_n[s]; i < h->sys_n[s + 1]; ++i) {
      row_sys[i] = s;
      if (lab_sys[part[i]] >= 0 && lab_sys[part[i]] != s)
        return fail(PSLR_EINVAL, "a subdomain label is used by two systems");
      lab_sys[part[i]] = s;
    }
  }
  for (int l = 0, last = 0; l < nparts; ++l) {
    if (lab_sys[l] < 0) lab_sys[l] = last;
    if (lab_sys[l] < last) return fail(PSLR_EINVAL, "subdomain labels must be ordered by system");
    last = lab_sys[l];
  }
  if (nsys > 1)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (row_sys[colind[k]] != row_sys[i]) return fail(PSLR_EINVAL, "A couples two systems");
  const double t0 = now_s();
  h->R = reorder(n, rowptr, colind, part, nparts);
  h->sys_q.assign(nsys + 1, h->R.q);
  h->sys_q[0] = 0;
  {
    std::vector<int64_t> qs(nsys, 0);
    for (int l = 0; l < nparts; ++l) qs[lab_sys[l]] += h->R.if_ptr[l + 1] - h->R.if_ptr[l];
    for (int s = 0; s < nsys; ++s) h->sys_q[s + 1] = h->sys_q[s] + qs[s];
  }
  Blocks Bk = extract_blocks(n, rowptr, colind, vals, h->R);
  const double t1 = now_s();
  const int np = nparts;
  std::vector<BlockFactor> fB(np), fC(np);
  std::vector<std::string> errs(2 * np);
  std::vector<int> codes(2 * np, 0);
  const double drop = o.drop_tol > 0 ? o.drop_tol : 1e-2;
  const std::vector<int> bteam = block_teams(Bk, o.factor == 0 ? o.team : 0);
  parallel_for(2 * np, o.nthreads, [&](int t) {
    const CsrL& M = t < np ? Bk.B[t] : Bk.C0[t - np];
    BlockFactor& F = t < np ? fB[t] : fC[t - np];
    const int narrow = t < np ? kNarrowWidthB : kNarrowWidthC;
    codes[t] = o.factor == 1 ? ilut_block(M, drop, h->want_T != 0, narrow, F, errs[t])
                             : factor_block(M, tau, h->want_T != 0, narrow, F, errs[t],
                                            bteam[t], t < np ? kTopRowsB : kTopRowsC);
  });
  for (int t = 0; t < 2 * np; ++t)
    if (codes[t]) return fail(codes[t] == 3 ? PSLR_ENOTSUP : PSLR_ESINGULAR,
                              std::string(t < np ? "B_" : "C_") + std::to_string(t % np) + ": " + errs[t]);
  const double t2 = now_s();

  // device copies of A (and A^T)
  {
    std::vector<int64_t> ptr(rowptr, rowptr + n + 1);
    std::vector<int32_t> col(colind, colind + h->nnzA);
    std::vector<double> val(vals, vals + h->nnzA);
    HIP_TRY(h->pool.upload(ptr, &h->A_ptr));
    HIP_TRY(h->pool.upload(col, &h->A_col));
    HIP_TRY(h->facpool.upload(val, &h->A_val));
    if (h->want_T) {
      std::vector<int64_t> tp(n + 1, 0);
      for (int32_t c : col) tp[c + 1]++;
      for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
      std::vector<int32_t> tc(col.size());
      std::vector<double> tv(col.size());
      std::vector<int64_t> pos(tp.begin(), tp.end() - 1);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
          int64_t d = pos[col[k]]++;
          tc[d] = (int32_t)i;
          tv[d] = val[k];
        }
      HIP_TRY(h->pool.upload(tp, &h->AT_ptr));
      HIP_TRY(h->pool.upload(tc, &h->AT_col));
      HIP_TRY(h->facpool.upload(tv, &h->AT_val));
    }
  }
  const int64_t *d_int_ptr, *d_if_ptr;
  const int32_t* d_if_orig;
  {
    std::vector<int32_t> if_orig(h->R.q);
    for (int64_t k = 0; k < h->R.q; ++k) if_orig[k] = (int32_t)h->R.perm[h->R.p + k];
    HIP_TRY(h->pool.upload(h->R.int_ptr, &d_int_ptr));
    HIP_TRY(h->pool.upload(h->R.if_ptr, &d_if_ptr));
    HIP_TRY(h->pool.upload(if_orig, &d_if_orig));
  }
  h->d_int_ptr = d_int_ptr;
  h->d_if_ptr = d_if_ptr;
  h->d_if_orig = d_if_orig;
  h->hA_ptr.assign(rowptr, rowptr + n + 1);
  h->hA_col.assign(colind, colind + h->nnzA);
  h->opt = o;
  h->team_rhs = o.team_rhs;
  if (o.v0) h->hv0.assign(o.v0, o.v0 + h->R.q);
  h->opt.v0 = nullptr;
  // per-system tables: subdomain -> system, V^T y row chunks, interface segments
  {
    std::vector<int32_t> ps(nparts);
    for (int l = 0; l < nparts; ++l) ps[l] = lab_sys[l];
    HIP_TRY(h->pool.upload(ps, &h->d_part_sys));
    std::vector<LrChunk> ch;
    std::vector<int32_t> sc(nsys + 1, 0);
    const int64_t qtot = std::max<int64_t>(h->R.q, 1);
    for (int s = 0; s < nsys; ++s) {
      const int64_t q0 = h->sys_q[s], qs = h->sys_q[s + 1] - q0;
      if (qs > 0) {
        const int64_t c = std::max<int64_t>(1, (int64_t)std::llround((double)h->nchunk * qs / qtot));
        const int64_t rows = std::min<int64_t>((qs + c - 1) / c, kLrChunkRows);
        for (int64_t r0 = 0; r0 < qs; r0 += rows)
          ch.push_back(LrChunk{q0 + r0, q0 + std::min(qs, r0 + rows), s, 0});
      }
      sc[s + 1] = (int32_t)ch.size();
    }
    if (ch.empty()) ch.push_back(LrChunk{0, 0, 0, 0});
    h->nchunk_lr = (int)ch.size();
    h->lr_maxrows = 0;
    for (const LrChunk& c : ch) h->lr_maxrows = std::max<int>(h->lr_maxrows, (int)(c.r1 - c.r0));
    HIP_TRY(h->pool.upload(ch, &h->d_chunks));
    HIP_TRY(h->pool.upload(sc, &h->d_sys_chunk));
    std::vector<Seg> qc(nsys);
    for (int s = 0; s < nsys; ++s) qc[s] = Seg{h->sys_q[s], h->sys_q[s + 1] - h->sys_q[s]};
    const Seg* dq = nullptr;
    HIP_TRY(h->pool.upload(qc, &dq));
    h->d_qcols = dq;
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, h->device));
  h->lds_max = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
  DirHost Dfw = build_dir(h->R, Bk, fB, fC, false);
  int64_t bytes[4] = {0, 0, 0, 0};
  HIP_TRY(upload_dir<double>(h->facpool, h->R, fB, fC, Dfw, false, o.team_top, d_int_ptr, d_if_ptr, d_if_orig,
                             h->fw64, bytes));
  // global workspace layout, used by applies whose subdomains do not fit in
  // LDS or that solve wide right-hand-side tiles
  {
    std::vector<int64_t> rb(nparts + 1, 0);
    for (int i = 0; i < nparts; ++i) {
      int mx = 1;
      for (const BlockFactor* f : {&fB[i], &fC[i]})
        for (const TriPacked* T : {&f->lo, &f->up, &f->loT, &f->upT}) mx = std::max(mx, T->max_lrows);
      rb[i + 1] = rb[i] + 2 * mx;  // halves alternating over the levels
    }
    HIP_TRY(h->facpool.upload(rb, &h->d_rb_off));
    h->gws_stride = h->R.p + 2 * h->R.q + rb[nparts] + (int64_t)nparts * 2 * std::max(h->rank, 1);
  }
  h->gx = o.working_vectors == 1;
  if (o.threads) h->threads = o.threads;
  h->threads_fixed = o.threads != 0;
  auto set_gx = [&](auto& A) {
    A.part_sys = h->d_part_sys;
    A.gshift = 0;
    A.gws = nullptr;
    A.gws_stride = h->gws_stride;
    A.rb_off = h->d_rb_off;
    A.kmax = std::max(h->rank, 1);
    A.nsys = h->nsys;
    A.active = nullptr;
  };
  set_gx(h->fw64);
  HIP_TRY(set_lds_limit<double>(h->lds_max));
  HIP_TRY(set_lds_limit<float>(h->lds_max));
  h->have64 = true;

  // Arnoldi on E_rr(m) in FP64 (Algorithm 4, lines 6-8)
  bool breakdown = false;
  h->ws.release();
  h->ws_nrhs = 0;
  h->ws_cap = WsSizes{};
  st = ensure_ws(h.get(), 1);
  if (st) return st;
  h->info.lowrank = o.lowrank;
  st = o.lowrank == 0 ? arnoldi(h.get(), o.v0, o.seed, s, breakdown)
                      : krylov_schur(h.get(), o.v0, o.seed, o.lowrank, s, breakdown);
  if (st) return st;
  h->ws.release();  // the V^T y partial sums are sized by the achieved rank
  h->ws_nrhs = 0;
  h->ws_cap = WsSizes{};
  const double t3 = now_s();

  if (h->precision >= 1) {
    HIP_TRY(upload_dir<float>(h->facpool, h->R, fB, fC, Dfw, false, o.team_top, d_int_ptr, d_if_ptr, d_if_orig,
                              h->fw32, bytes));
    set_gx(h->fw32);
    h->have32 = true;
  }
  if (h->want_T) {
    DirHost Dtr = build_dir(h->R, Bk, fB, fC, true);
    int64_t tb[4];
    if (h->precision >= 1) {
      HIP_TRY(upload_dir<float>(h->facpool, h->R, fB, fC, Dtr, true, 0, d_int_ptr, d_if_ptr, d_if_orig,
                                h->tr32, tb));
      set_gx(h->tr32);
    }
    HIP_TRY(upload_dir<double>(h->facpool, h->R, fB, fC, Dtr, true, 0, d_int_ptr, d_if_ptr, d_if_orig,
                               h->tr64, tb));
    set_gx(h->tr64);
    h->haveT = true;
  }
  if ((st = probe_bf16(h.get(), s))) return st;
  if (o.autotune) {
    st = autotune(h.get(), s);
    if (st) return st;
  }
  fill_info(h.get(), fB, fC, Bk, bytes);
  h->info.seconds_reorder = t1 - t0;
  h->info.seconds_factor = t2 - t1;
  h->info.seconds_arnoldi = t3 - t2;
  HIP_TRY(hipStreamSynchronize(s));
  *out = h.release();
  return breakdown ? PSLR_EBREAKDOWN : PSLR_OK;
}

}  // namespace

extern "C" {

pslr_status pslr_refactor(pslr_handle h, const double* vals, void* hip_stream) {
  if (!h || (h->nnzA > 0 && !vals)) return fail(PSLR_EINVAL, "bad arguments");
  for (int64_t k = 0; k < h->nnzA; ++k)
    if (!std::isfinite(vals[k])) return fail(PSLR_EINVAL, "non-finite value in A");
  hipStream_t s = (hipStream_t)hip_stream;
  const pslr_options& o = h->opt;
  const int64_t n = h->R.n;
  const int np = h->R.nparts;
  const double t1 = now_s();
  // local factors of the new values (the same orderings and supernodes: they
  // depend on the pattern only; threshold ILU keeps what the new values keep)
  Blocks Bk = extract_blocks(n, h->hA_ptr.data(), h->hA_col.data(), vals, h->R);
  std::vector<BlockFactor> fB(np), fC(np);
  std::vector<std::string> errs(2 * np);
  std::vector<int> codes(2 * np, 0);
  const double tau = o.pivot_threshold > 0 ? o.pivot_threshold : 0.1;
  const double drop = o.drop_tol > 0 ? o.drop_tol : 1e-2;
  const std::vector<int> bteam = block_teams(Bk, o.factor == 0 ? o.team : 0);
  parallel_for(2 * np, o.nthreads, [&](int t) {
    const CsrL& M = t < np ? Bk.B[t] : Bk.C0[t - np];
    BlockFactor& F = t < np ? fB[t] : fC[t - np];
    const int narrow = t < np ? kNarrowWidthB : kNarrowWidthC;
    codes[t] = o.factor == 1 ? ilut_block(M, drop, h->want_T != 0, narrow, F, errs[t])
                             : factor_block(M, tau, h->want_T != 0, narrow, F, errs[t],
                                            bteam[t], t < np ? kTopRowsB : kTopRowsC);
  });
  for (int t = 0; t < 2 * np; ++t)
    if (codes[t]) return fail(codes[t] == 3 ? PSLR_ENOTSUP : PSLR_ESINGULAR,
                              std::string(t < np ? "B_" : "C_") + std::to_string(t % np) + ": " + errs[t]);
  const double t2 = now_s();
  // new device copies of everything that depends on the values
  DevPool nf;
  const double* A_val = nullptr;
  const double* AT_val = nullptr;
  {
    std::vector<double> val(vals, vals + h->nnzA);
    HIP_TRY(nf.upload(val, &A_val));
    if (h->want_T) {
      std::vector<int64_t> pos(n + 1, 0);
      for (int64_t k = 0; k < h->nnzA; ++k) pos[h->hA_col[k] + 1]++;
      for (int64_t i = 0; i < n; ++i) pos[i + 1] += pos[i];
      std::vector<double> tv(h->nnzA);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = h->hA_ptr[i]; k < h->hA_ptr[i + 1]; ++k) tv[pos[h->hA_col[k]]++] = vals[k];
      HIP_TRY(nf.upload(tv, &AT_val));
    }
  }
  ApplyArrays<double> fw64{}, tr64{};
  ApplyArrays<float> fw32{}, tr32{};
  int64_t bytes[4] = {0, 0, 0, 0}, tb[4];
  DirHost Dfw = build_dir(h->R, Bk, fB, fC, false);
  HIP_TRY(upload_dir<double>(nf, h->R, fB, fC, Dfw, false, o.team_top, h->d_int_ptr, h->d_if_ptr, h->d_if_orig,
                             fw64, bytes));
  const int64_t* d_rb_off = nullptr;
  int64_t gws_stride = 0;
  {
    std::vector<int64_t> rb(np + 1, 0);
    for (int i = 0; i < np; ++i) {
      int mx = 1;
      for (const BlockFactor* f : {&fB[i], &fC[i]})
        for (const TriPacked* T : {&f->lo, &f->up, &f->loT, &f->upT}) mx = std::max(mx, T->max_lrows);
      rb[i + 1] = rb[i] + 2 * mx;  // halves alternating over the levels
    }
    HIP_TRY(nf.upload(rb, &d_rb_off));
    gws_stride = h->R.p + 2 * h->R.q + rb[np] + (int64_t)np * 2 * std::max(h->fw64.kmax, 1);
  }
  if (h->have32) HIP_TRY(upload_dir<float>(nf, h->R, fB, fC, Dfw, false, o.team_top, h->d_int_ptr, h->d_if_ptr,
                                           h->d_if_orig, fw32, bytes));
  if (h->haveT) {
    DirHost Dtr = build_dir(h->R, Bk, fB, fC, true);
    if (h->have32) HIP_TRY(upload_dir<float>(nf, h->R, fB, fC, Dtr, true, 0, h->d_int_ptr, h->d_if_ptr,
                                             h->d_if_orig, tr32, tb));
    HIP_TRY(upload_dir<double>(nf, h->R, fB, fC, Dtr, true, 0, h->d_int_ptr, h->d_if_ptr, h->d_if_orig,
                               tr64, tb));
  }
  // the launch settings of the old arrays carry over (autotuned chunk scale)
  auto carry = [&](auto& Anew, const auto& Aold) {
    Anew.part_sys = h->d_part_sys;
    Anew.gshift = Aold.gshift;
    Anew.gws = nullptr;
    Anew.gws_stride = gws_stride;
    Anew.rb_off = d_rb_off;
    Anew.kmax = Aold.kmax;
    Anew.nsys = h->nsys;
    Anew.active = nullptr;
  };
  carry(fw64, h->fw64);
  carry(fw32, h->fw64);
  carry(tr64, h->fw64);
  carry(tr32, h->fw64);
  // nothing queued may still read the old arrays: wait, then swap and free
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipDeviceSynchronize());
  h->fw64 = fw64;
  if (h->have32) h->fw32 = fw32;
  if (h->haveT) {
    h->tr64 = tr64;
    if (h->have32) h->tr32 = tr32;
  }
  h->A_val = A_val;
  if (h->want_T) h->AT_val = AT_val;
  h->d_rb_off = d_rb_off;
  h->gws_stride = gws_stride;
  std::swap(h->facpool.ptrs, nf.ptrs);
  std::swap(h->facpool.bytes, nf.bytes);
  nf.release();
  h->ws.release();
  h->ws_nrhs = 0;
  h->ws_cap = WsSizes{};
  // the low-rank correction of the new operator, with the setup's construction;
  // Krylov-Schur starts from the sum of the previous basis vectors (warm start)
  std::vector<double> v0 = h->hv0;
  if (o.lowrank != 0 && h->k > 0) {
    v0.assign(h->R.q, 0.0);
    for (int j = 0; j < h->k; ++j)
      for (int64_t r = 0; r < h->R.q; ++r) v0[r] += h->hV[(size_t)j * h->R.q + r];
  }
  pslr_status st = ensure_ws(h, 1);
  if (st) return st;
  bool breakdown = false;
  const double* v0p = v0.empty() ? nullptr : v0.data();
  st = o.lowrank == 0 ? arnoldi(h, v0p, o.seed, s, breakdown)
                      : krylov_schur(h, v0p, o.seed, o.lowrank, s, breakdown);
  if (st) return st;
  h->ws.release();
  h->ws_nrhs = 0;
  h->ws_cap = WsSizes{};
  if ((st = probe_bf16(h, s))) return st;
  const double t3 = now_s();
  fill_info(h, fB, fC, Bk, bytes);
  h->info.seconds_factor = t2 - t1;
  h->info.seconds_arnoldi = t3 - t2;
  HIP_TRY(hipStreamSynchronize(s));
  return breakdown ? PSLR_EBREAKDOWN : PSLR_OK;
}

pslr_status pslr_setup(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                       const int32_t* part, int32_t nparts, const pslr_options* opt,
                       void* hip_stream, pslr_handle* out) {
  const int64_t sp[2] = {0, n};
  return setup_impl(n, rowptr, colind, vals, part, nparts, 1, sp, opt, hip_stream, out);
}

pslr_status pslr_setup_batched(int64_t n, const int64_t* rowptr, const int32_t* colind,
                               const double* vals, const int32_t* part, int32_t nparts,
                               int32_t nsys, const int64_t* sys_ptr, const pslr_options* opt,
                               void* hip_stream, pslr_handle* out) {
  if (nsys < 1 || !sys_ptr) return fail(PSLR_EINVAL, "bad system table");
  return setup_impl(n, rowptr, colind, vals, part, nparts, nsys, sys_ptr, opt, hip_stream, out);
}

pslr_status pslr_apply(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* z,
                       int64_t ldz, void* hip_stream) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  if (nrhs < 0 || (nrhs > 0 && (!b || !z)) || ldb < h->R.n || ldz < h->R.n)
    return fail(PSLR_EINVAL, "bad vector arguments");
  if (nrhs == 0) return PSLR_OK;
  return apply_dir(h, false, nrhs, b, ldb, z, ldz, (hipStream_t)hip_stream);
}

pslr_status pslr_apply_noalloc(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* z,
                               int64_t ldz, void* hip_stream) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  if (nrhs < 0 || (nrhs > 0 && (!b || !z)) || ldb < h->R.n || ldz < h->R.n)
    return fail(PSLR_EINVAL, "bad vector arguments");
  if (nrhs == 0 || h->R.n == 0) return PSLR_OK;
  void* base = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch_ptr[h->device] : nullptr;
  if (!base) return fail(PSLR_EINVAL, "scratch array not attached on the handle's device");
  // carve y, u0, u1, the V^T y partial sums and the global working vectors
  // out of the array, each 256-byte aligned
  const WsSizes z0 = ws_sizes(h, nrhs);
  auto up = [](size_t d) { return (d * sizeof(double) + 255) / 256 * 256; };
  const size_t need = 3 * up(z0.vec) + up(z0.partial) + up(z0.gws) + up(z0.zp) + up(z0.team);
  if (need > kScratchBytes)
    return fail(PSLR_EINVAL, "pslr_apply_noalloc needs " + std::to_string(need) +
                                 " bytes of scratch for " + std::to_string(nrhs) +
                                 " right-hand sides; the maximum is " + std::to_string(kScratchBytes));
  char* c = (char*)base;
  ApplyWs W{};
  W.y = c;
  c += up(z0.vec);
  W.u0 = c;
  c += up(z0.vec);
  W.u1 = c;
  c += up(z0.vec);
  W.partial = c;
  c += up(z0.partial);
  W.gws = z0.gws > 0 ? (void*)c : nullptr;
  c += up(z0.gws);
  W.zp = z0.zp > 0 ? (void*)c : nullptr;
  c += up(z0.zp);
  W.team = z0.team > 0 ? (void*)c : nullptr;
  hipStream_t s = (hipStream_t)hip_stream;
  // no phase tracing here: the tracer creates events on demand
  if (h->precision >= 1 && h->have32)
    return run_apply<float>(h, h->fw32, W, false, nrhs, b, ldb, z, ldz, s, false);
  if (!h->have64) return fail(PSLR_EINVAL, "FP64 apply arrays not available");
  return run_apply<double>(h, h->fw64, W, false, nrhs, b, ldb, z, ldz, s, false);
}

pslr_status pslr_apply_transpose(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb,
                                 double* z, int64_t ldz, void* hip_stream) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  if (!h->haveT) return fail(PSLR_EINVAL, "handle was built without want_transpose");
  if (nrhs < 0 || (nrhs > 0 && (!b || !z)) || ldb < h->R.n || ldz < h->R.n)
    return fail(PSLR_EINVAL, "bad vector arguments");
  if (nrhs == 0) return PSLR_OK;
  return apply_dir(h, true, nrhs, b, ldb, z, ldz, (hipStream_t)hip_stream);
}

// FGMRES enqueues iteration j + 1 before reading iteration j's results while
// every active residual estimate is above this multiple of its target.
#ifndef PSLR_SPEC_MARGIN
#define PSLR_SPEC_MARGIN 4.0
#endif
constexpr double kSpecMargin = PSLR_SPEC_MARGIN;

pslr_status fgmres_solve(pslr_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                         int64_t ldx, int32_t restart, int32_t maxit, double tol, int32_t transpose,
                         int32_t* iters, double* relres, void* hip_stream) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  if (nrhs <= 0 || !b || !x || ldb < h->R.n || ldx < h->R.n || restart <= 0 || maxit < 0 ||
      !(tol > 0))
    return fail(PSLR_EINVAL, "bad FGMRES arguments");
  if (transpose && !h->haveT) return fail(PSLR_EINVAL, "handle was built without want_transpose");
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n = h->R.n;
  const int ns = h->nsys;
  const int ncol = ns * nrhs;  // column c = r * nsys + sys: one Krylov space per (system, rhs)
  const int R1 = restart + 1;
  const int64_t* Ap = transpose ? h->AT_ptr : h->A_ptr;
  const int32_t* Ac = transpose ? h->AT_col : h->A_col;
  const double* Av = transpose ? h->AT_val : h->A_val;
  const int64_t blk = n * nrhs;  // one basis vector of every column: n x nrhs, leading dimension n
  int64_t maxlen = 0;
  for (int c = 0; c < ns; ++c) maxlen = std::max(maxlen, h->sys_n[c + 1] - h->sys_n[c]);
  std::vector<Seg> cols((size_t)3 * ncol);
  for (int r = 0; r < nrhs; ++r)
    for (int c = 0; c < ns; ++c) {
      const int64_t o = h->sys_n[c], len = h->sys_n[c + 1] - o;
      cols[r * ns + c] = Seg{r * n + o, len};
      cols[ncol + r * ns + c] = Seg{r * ldb + o, len};
      cols[2 * ncol + r * ns + c] = Seg{r * ldx + o, len};
    }
  const std::vector<Seg> vcols(cols.begin(), cols.begin() + ncol);
  const int64_t crows = chunk_rows(vcols);
  const int64_t maxch = count_chunks(vcols, crows);
  if (h->f_nrhs != nrhs || h->f_restart != restart || h->f_maxch != maxch) {
    h->fpool.release();
    HIP_TRY(h->fpool.alloc<double>((size_t)blk * R1, &h->fVb));
    HIP_TRY(h->fpool.alloc<double>((size_t)blk * restart, &h->fZb));
    HIP_TRY(h->fpool.alloc<double>((size_t)blk, &h->fW));
    HIP_TRY(h->fpool.alloc<double>((size_t)maxch * R1, &h->fdbuf));
    HIP_TRY(h->fpool.alloc<Chunk>((size_t)2 * maxch, &h->fchF));
    h->fchM = h->fchF + maxch;
    HIP_TRY(h->fpool.alloc<int32_t>((size_t)2 * (ncol + 1), &h->fcpF));
    h->fcpM = h->fcpF + ncol + 1;
    h->f_maxch = maxch;
    HIP_TRY(h->fpool.alloc<double>((size_t)ncol * (2 * R1 + 1), &h->fh));
    HIP_TRY(h->fpool.alloc<double>(ncol, &h->fscl));
    HIP_TRY(h->fpool.alloc<double>((size_t)ncol * restart, &h->fy));
    HIP_TRY(h->fpool.alloc<Seg>((size_t)4 * ncol, &h->fcolsV));
    h->fcolsB = h->fcolsV + ncol;
    h->fcolsX = h->fcolsB + ncol;
    h->fcolsM = h->fcolsX + ncol;
    HIP_TRY(h->fpool.alloc<uint8_t>(ncol, &h->factive));
    // columns a masked apply leaves unwritten must hold finite values
    HIP_TRY(hipMemsetAsync(h->fZb, 0, sizeof(double) * (size_t)blk * restart, s));
    h->f_nrhs = nrhs;
    h->f_restart = restart;
  }
  HIP_TRY(hipMemcpyAsync(h->fcolsV, cols.data(), sizeof(Seg) * cols.size(), hipMemcpyHostToDevice, s));
  std::vector<Chunk> chF, chM;
  std::vector<int32_t> cpF, cpM;
  const int nchF = make_chunks(vcols, crows, nullptr, chF, cpF);
  HIP_TRY(hipMemcpyAsync(h->fchF, chF.data(), sizeof(Chunk) * std::max(nchF, 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->fcpF, cpF.data(), sizeof(int32_t) * (ncol + 1), hipMemcpyHostToDevice, s));
  const Seg *cV = h->fcolsV, *cB = h->fcolsB, *cX = h->fcolsX;
  std::vector<uint8_t> amask(ncol, 0);
  int nchM = 0;
  double* Vb = h->fVb;
  double* Zb = h->fZb;
  double* W = h->fW;
  double* dh1 = h->fh;
  double* dh2 = dh1 + (size_t)ncol * R1;
  double* dnn = dh2 + (size_t)ncol * R1;
  std::vector<double> hbuf((size_t)ncol * (2 * R1 + 1)), sc(ncol), bn(ncol);
  const size_t hsz = (size_t)ncol * (2 * R1 + 1);
  if (h->fpin_n < 2 * hsz) {
    if (h->fpin) (void)hipHostFree(h->fpin);
    h->fpin = nullptr;
    h->fpin_n = 0;
    HIP_TRY(hipHostMalloc((void**)&h->fpin, sizeof(double) * 2 * hsz, hipHostMallocDefault));
    h->fpin_n = 2 * hsz;
  }
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } hev;
  for (hipEvent_t& x : hev.e) HIP_TRY(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  // ||b|| per column
  HIP_TRY(launch_mdot_chunk(nchF, h->fchF, cB, cB, 1, b, 0, b, h->fdbuf, s));
  HIP_TRY(launch_reduce_chunk(ncol, h->fcpF, 1, nchF, h->fdbuf, dnn, s));
  HIP_TRY(hipMemcpyAsync(bn.data(), dnn, sizeof(double) * ncol, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (double& v : bn) v = std::sqrt(v);
  std::vector<int> its(ncol, 0), done(ncol, 0), jdone(ncol, 0), act(ncol, 0);
  std::vector<double> rel(ncol, 0.0);
  for (int c = 0; c < ncol; ++c)
    if (bn[c] == 0.0) done[c] = 1;
  std::vector<double> Hh((size_t)ncol * R1 * restart), cs((size_t)ncol * restart),
      sn((size_t)ncol * restart), g((size_t)ncol * R1), yv((size_t)ncol * restart);
  for (;;) {
    // r0 = b - A x into V_0 of every column
    HIP_TRY(launch_spmv(n, Ap, Ac, Av, nrhs, x, ldx, Vb, n, b, ldb, s));
    HIP_TRY(launch_mdot_chunk(nchF, h->fchF, cV, cV, 1, Vb, 0, Vb, h->fdbuf, s));
    HIP_TRY(launch_reduce_chunk(ncol, h->fcpF, 1, nchF, h->fdbuf, dnn, s));
    HIP_TRY(hipMemcpyAsync(hbuf.data(), dnn, sizeof(double) * ncol, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (int c = 0; c < ncol; ++c) {
      const double beta = std::sqrt(hbuf[c]);
      if (!done[c]) {
        rel[c] = beta / bn[c];
        if (beta <= tol * bn[c]) done[c] = 1;
        else if (its[c] >= maxit) done[c] = 2;
      }
      act[c] = !done[c];
      any = any || act[c];
      sc[c] = act[c] ? 1.0 / beta : 0.0;
      std::fill(&g[(size_t)c * R1], &g[(size_t)c * R1] + R1, 0.0);
      g[(size_t)c * R1] = act[c] ? beta : 0.0;
      jdone[c] = 0;
    }
    if (!any) break;
    HIP_TRY(hipMemcpyAsync(h->fscl, sc.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_scale_chunk(nchF, h->fchF, cV, cV, Vb, h->fscl, Vb, s));
    // Far from convergence iteration j+1 is enqueued before the host reads
    // iteration j's Hessenberg column: V_{j+1} is normalised on the device
    // from its norm, the column travels to pinned host memory behind an
    // event, and the host's Givens update of column j overlaps the device's
    // iteration j+1 (whose results are dropped if column j converged).
    auto enqueue = [&](int j) -> pslr_status {
      double* Vj = Vb + (size_t)j * blk;
      double* Zj = Zb + (size_t)j * blk;
      // converged columns skip the apply and the vector work of this iteration
      bool changed = j == 0;
      for (int c = 0; c < ncol; ++c) changed = changed || amask[c] != (act[c] ? 1 : 0);
      if (changed) {
        HIP_TRY(hipStreamSynchronize(s));  // earlier uploads may still read these host arrays
        for (int c = 0; c < ncol; ++c) amask[c] = act[c] ? 1 : 0;
        nchM = make_chunks(vcols, crows, &amask, chM, cpM);
        HIP_TRY(hipMemcpyAsync(h->factive, amask.data(), ncol, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->fchM, chM.data(), sizeof(Chunk) * std::max(nchM, 1),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->fcpM, cpM.data(), sizeof(int32_t) * (ncol + 1), hipMemcpyHostToDevice, s));
      }
      h->cur_active = h->factive;
      pslr_status st = apply_dir(h, transpose != 0, nrhs, Vj, n, Zj, n, s);
      h->cur_active = nullptr;
      if (st) return st;
      HIP_TRY(launch_spmv(n, Ap, Ac, Av, nrhs, Zj, n, W, n, nullptr, 0, s));
      // classical Gram-Schmidt, two passes, then ||w|| and V_{j+1} = w / ||w||
      const int nv = j + 1;
      HIP_TRY(launch_mdot_chunk(nchM, h->fchM, cV, cV, nv, Vb, blk, W, h->fdbuf, s));
      HIP_TRY(launch_reduce_chunk(ncol, h->fcpM, nv, nchM, h->fdbuf, dh1, s));
      HIP_TRY(launch_maxpy_chunk(nchM, h->fchM, cV, cV, nv, Vb, blk, dh1, nv, W, 1.0, s));
      HIP_TRY(launch_mdot_chunk(nchM, h->fchM, cV, cV, nv, Vb, blk, W, h->fdbuf, s));
      HIP_TRY(launch_reduce_chunk(ncol, h->fcpM, nv, nchM, h->fdbuf, dh2, s));
      HIP_TRY(launch_maxpy_chunk(nchM, h->fchM, cV, cV, nv, Vb, blk, dh2, nv, W, 1.0, s));
      HIP_TRY(launch_mdot_chunk(nchM, h->fchM, cV, cV, 1, W, 0, W, h->fdbuf, s));
      HIP_TRY(launch_reduce_chunk(ncol, h->fcpM, 1, nchM, h->fdbuf, dnn, s));
      HIP_TRY(launch_inv_sqrt(ncol, dnn, h->factive, h->fscl, s));
      HIP_TRY(launch_scale_chunk(nchF, h->fchF, cV, cV, W, h->fscl, Vb + (size_t)(j + 1) * blk, s));
      // dh1, dh2 and dnn are one contiguous block (same offsets in the slot): one copy
      double* slot = h->fpin + (size_t)(j & 1) * hsz;
      HIP_TRY(hipMemcpyAsync(slot, dh1, sizeof(double) * hsz, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(hev.e[j & 1], s));
      return PSLR_OK;
    };
    if (pslr_status st = enqueue(0)) return st;
    for (int j = 0; j < restart; ++j) {
      // Iteration j + 1 goes ahead of the host's reading of iteration j only
      // while every active column's residual estimate |g_j| is above
      // kSpecMargin times its target: near convergence the host waits for
      // iteration j first, so that a converged solve does not pay for an
      // iteration whose results it drops (an apply and its vector work) but
      // for one host round trip per iteration instead.
      bool spec = j + 1 < restart;
      for (int c = 0; c < ncol && spec; ++c)
        if (act[c] && std::fabs(g[(size_t)c * R1 + j]) <= kSpecMargin * tol * bn[c]) spec = false;
      if (spec)
        if (pslr_status st = enqueue(j + 1)) return st;
      HIP_TRY(hipEventSynchronize(hev.e[j & 1]));
      const int nv = j + 1;
      const double* h1 = h->fpin + (size_t)(j & 1) * hsz;
      const double* h2 = h1 + (size_t)ncol * R1;
      const double* nn = h2 + (size_t)ncol * R1;
      bool cont = false;
      for (int c = 0; c < ncol; ++c) {
        if (!act[c]) continue;
        double* Hc = &Hh[((size_t)c * restart + j) * R1];
        for (int i = 0; i <= j; ++i) Hc[i] = h1[(size_t)c * nv + i] + h2[(size_t)c * nv + i];
        const double hn = std::sqrt(nn[c]);
        Hc[j + 1] = hn;
        double* c_ = &cs[(size_t)c * restart];
        double* s_ = &sn[(size_t)c * restart];
        double* g_ = &g[(size_t)c * R1];
        for (int i = 0; i < j; ++i) {
          const double t = c_[i] * Hc[i] + s_[i] * Hc[i + 1];
          Hc[i + 1] = -s_[i] * Hc[i] + c_[i] * Hc[i + 1];
          Hc[i] = t;
        }
        const double d = std::hypot(Hc[j], Hc[j + 1]);
        c_[j] = d > 0 ? Hc[j] / d : 1.0;
        s_[j] = d > 0 ? Hc[j + 1] / d : 0.0;
        Hc[j] = d;
        Hc[j + 1] = 0.0;
        g_[j + 1] = -s_[j] * g_[j];
        g_[j] = c_[j] * g_[j];
        its[c]++;
        jdone[c] = j + 1;
        if (std::fabs(g_[j + 1]) <= tol * bn[c] || its[c] >= maxit || hn == 0.0) act[c] = 0;
        else cont = true;
      }
      if (!cont) break;
      if (!spec && j + 1 < restart)
        if (pslr_status st = enqueue(j + 1)) return st;
    }
    // x += Z y
    std::fill(yv.begin(), yv.end(), 0.0);
    int jmax = 0;
    for (int c = 0; c < ncol; ++c) {
      const int jd = jdone[c];
      jmax = std::max(jmax, jd);
      double* y = &yv[(size_t)c * restart];
      for (int i = jd - 1; i >= 0; --i) {
        double acc = g[(size_t)c * R1 + i];
        for (int cc = i + 1; cc < jd; ++cc) acc -= Hh[((size_t)c * restart + cc) * R1 + i] * y[cc];
        y[i] = acc / Hh[((size_t)c * restart + i) * R1 + i];
      }
    }
    HIP_TRY(hipMemcpyAsync(h->fy, yv.data(), sizeof(double) * yv.size(), hipMemcpyHostToDevice, s));
    if (jmax > 0)
      HIP_TRY(launch_maxpy_chunk(nchF, h->fchF, cV, cX, jmax, Zb, blk, h->fy, restart, x, -1.0, s));
  }
  for (int c = 0; c < ncol; ++c) {
    if (iters) iters[c] = its[c];
    if (relres) relres[c] = rel[c];
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (int c = 0; c < ncol; ++c)
    if (done[c] != 1) return fail(PSLR_ENOCONV, "FGMRES did not converge within maxit");
  return PSLR_OK;
}

pslr_status pslr_sddmm_grad(pslr_handle h, int32_t nrhs, const double* lambda, int64_t ldl,
                            const double* z, int64_t ldz, double* grad, void* hip_stream) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  if (nrhs <= 0 || !lambda || !z || !grad || ldl < h->R.n || ldz < h->R.n)
    return fail(PSLR_EINVAL, "bad SDDMM arguments");
  HIP_TRY(launch_sddmm(h->R.n, h->A_ptr, h->A_col, nrhs, lambda, ldl, z, ldz, grad,
                       (hipStream_t)hip_stream));
  return PSLR_OK;
}

pslr_status pslr_info(pslr_handle h, pslr_info_t* out) {
  if (!h || !out) return fail(PSLR_EINVAL, "null argument");
  *out = h->info;
  out->rank = h->k;
  out->v_bf16 = h->v_bf16 ? 1 : 0;
  out->bf16_probe = h->bf16_probe;
  out->mfma_min_rhs = (h->precision >= 1 && h->v_bf16 && h->Vbr && h->k > 0) ? kMfmaMinRhs : 0;
  return PSLR_OK;
}

pslr_status pslr_trace_enable(pslr_handle h, int32_t enable) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  h->trace = enable != 0;
  return PSLR_OK;
}

pslr_status pslr_trace_read(pslr_handle h, pslr_trace_t* out, int32_t reset) {
  if (!h) return fail(PSLR_EINVAL, "null handle");
  HIP_TRY(trace_collect(h, true));
  if (out) *out = h->tr;
  if (reset) h->tr = pslr_trace_t{};
  return PSLR_OK;
}

pslr_status pslr_set_lowrank(pslr_handle h, int32_t k, const double* V, int64_t ldv,
                             const double* H, int64_t ldh) {
  if (!h || k < 0 || k > 256 || k > h->R.q || (k > 0 && (!V || !H || ldv < h->R.q || ldh < k)))
    return fail(PSLR_EINVAL, "bad low-rank arguments");
  if (h->nsys != 1) return fail(PSLR_EINVAL, "pslr_set_lowrank needs a single-system handle");
  const int64_t q = h->R.q;
  h->k = k;
  h->sys_k.assign(1, k);
  grow_kmax(h, k);
  h->hV.assign((size_t)q * k, 0.0);
  h->hH.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int64_t r = 0; r < q; ++r) h->hV[(size_t)j * q + r] = V[(size_t)j * ldv + r];
    for (int i = 0; i < k; ++i) h->hH[(size_t)j * k + i] = H[(size_t)j * ldh + i];
  }
  if (k > h->rank) h->rank = k;
  // the next apply grows the workspace if k or the global stride outgrew it
  // (ensure_ws; the old workspace stays allocated)
  pslr_status st = upload_lowrank(h);
  if (st == PSLR_OK) st = probe_bf16(h, nullptr);
  h->info.rank = h->k;
  return st;
}

pslr_status pslr_delta(pslr_handle h, int32_t nprobe, uint64_t seed, double* delta,
                       double* norm_x, double* norm_zinv, void* hip_stream) {
  if (!h || !delta || nprobe < 0) return fail(PSLR_EINVAL, "bad arguments");
  if (h->nsys != 1) return fail(PSLR_EINVAL, "pslr_delta needs a single-system handle");
  const int64_t q = h->R.q;
  const int k = h->k;
  hipStream_t s = (hipStream_t)hip_stream;
  // ||Z^{-1}||_F^2 = ||I + V G V^T||_F^2 = q + 2 tr(G) + ||G||_F^2 (V orthonormal)
  double nz2 = (double)q;
  for (int i = 0; i < k; ++i) {
    nz2 += 2.0 * h->hG[(size_t)i * k + i];
    for (int j = 0; j < k; ++j) nz2 += h->hG[(size_t)i * k + j] * h->hG[(size_t)i * k + j];
  }
  // ||X||_F^2 = sum_j ||X e_j||^2 (nprobe = 0), else the mean of ||X z||^2 over
  // nprobe Rademacher vectors z (E[z z^T] = I); X z = E_rr z - V (H (V^T z))
  const int ncols = nprobe == 0 ? (int)q : nprobe;
  const int nb = 32;
  pslr_status st = ensure_ws(h, nb);
  if (st) return st;
  DevPool tmp;
  double *zin, *ua, *ub;
  HIP_TRY(tmp.alloc<double>((size_t)q * nb, &zin));
  HIP_TRY(tmp.alloc<double>((size_t)q * nb, &ua));
  HIP_TRY(tmp.alloc<double>((size_t)q * nb, &ub));
  ApplyArrays<double> A = h->fw64;
  A.gws = h->gws;
  A.active = nullptr;
  std::vector<double> zb((size_t)q * nb), eb((size_t)q * nb), c(k), d(k);
  uint64_t state = seed;
  double nx2 = 0.0;
  for (int c0 = 0; c0 < ncols; c0 += nb) {
    const int cb = std::min(nb, ncols - c0);
    std::fill(zb.begin(), zb.end(), 0.0);
    for (int t = 0; t < cb; ++t) {
      if (nprobe == 0) {
        zb[(size_t)t * q + c0 + t] = 1.0;
      } else {
        for (int64_t i = 0; i < q; ++i)
          zb[(size_t)t * q + i] = (splitmix64_next(state) >> 63) ? 1.0 : -1.0;
      }
    }
    HIP_TRY(hipMemcpyAsync(zin, zb.data(), sizeof(double) * q * cb, hipMemcpyHostToDevice, s));
    LaunchCfg cfg = choose_launch(h, A, cb, s);
    const double* cur = zin;
    for (int r = 0; r <= h->m; ++r) {
      HIP_TRY(launch_c0solve<double>(A, cfg, cb, cur, q, ua, q));
      HIP_TRY(launch_series<double>(A, cfg, cb, ua, q, ua, ub, q, 0, 0));
      cur = ub;
    }
    HIP_TRY(hipMemcpyAsync(eb.data(), ub, sizeof(double) * q * cb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t < cb; ++t) {
      const double* z = &zb[(size_t)t * q];
      double* e = &eb[(size_t)t * q];
      for (int j = 0; j < k; ++j) {  // c = V^T z
        double a = 0.0;
        for (int64_t i = 0; i < q; ++i) a += h->hV[(size_t)j * q + i] * z[i];
        c[j] = a;
      }
      for (int i = 0; i < k; ++i) {  // d = H c
        double a = 0.0;
        for (int j = 0; j < k; ++j) a += h->hH[(size_t)j * k + i] * c[j];
        d[i] = a;
      }
      for (int j = 0; j < k; ++j)
        for (int64_t i = 0; i < q; ++i) e[i] -= h->hV[(size_t)j * q + i] * d[j];
      for (int64_t i = 0; i < q; ++i) nx2 += e[i] * e[i];
    }
  }
  if (nprobe > 0) nx2 /= nprobe;
  const double nx = std::sqrt(nx2), nz = std::sqrt(std::max(nz2, 0.0));
  *delta = nx * nz;
  if (norm_x) *norm_x = nx;
  if (norm_zinv) *norm_zinv = nz;
  return PSLR_OK;
}

pslr_status pslr_get_lowrank(pslr_handle h, int32_t* k, double* V, int64_t ldv, double* H,
                             int64_t ldh) {
  if (!h || !k) return fail(PSLR_EINVAL, "null argument");
  if (h->nsys != 1) return fail(PSLR_EINVAL, "pslr_get_lowrank needs a single-system handle");
  *k = h->k;
  const int64_t q = h->R.q;
  if (V)
    for (int j = 0; j < h->k; ++j)
      for (int64_t r = 0; r < q; ++r) V[(size_t)j * ldv + r] = h->hV[(size_t)j * q + r];
  if (H)
    for (int j = 0; j < h->k; ++j)
      for (int i = 0; i < h->k; ++i) H[(size_t)j * ldh + i] = h->hH[(size_t)j * h->k + i];
  return PSLR_OK;
}

pslr_status pslr_destroy(pslr_handle h) {
  delete h;
  return PSLR_OK;
}

}  // extern "C"
