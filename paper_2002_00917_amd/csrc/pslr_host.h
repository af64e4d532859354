// Host-side setup of the PSLR preconditioner: reordering by subdomains,
// block extraction, and exact sparse LU of every diagonal block packed into
// the level-scheduled supernodal layouts the device triangular solves read.
#pragma once
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace pslr {

// Local CSR (one subdomain block); int32 offsets suffice per block.
struct CsrL {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// Global CSR with 64-bit row offsets.
struct CsrG {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// One supernode of a packed triangular factor.  Rows f..f+w-1 (positions)
// form a dense w x w diagonal triangle stored INVERTED and packed by rows at
// tri_off; for an upper factor the off-diagonal part is a dense w x h panel
// (row-major, panel_off) over the shared column list ridx[ridx_off .. +h).
struct SnHost {
  int32_t f, w, h, pad;
  int64_t tri_off, panel_off, ridx_off;
};

// A packed triangular factor of one block, solved level by level: level l
// holds whole supernodes (rows lrows[lev_ptr[l] .. lev_ptr[l+1]), supernode
// by supernode, rows ascending).  A lower factor is solved for l = 0..nlev-1
// and pulls its off-diagonal part from CSR rows (rp/col/val) whose columns are
// all in earlier levels; an upper factor is solved for l = nlev-1..0 and pulls
// from the dense panels.
struct TriHost {
  bool lower = true;
  int32_t n = 0, nlev = 0, max_lrows = 0;
  std::vector<int32_t> lev_ptr;   // nlev + 1
  std::vector<int32_t> lev_g;     // nlev: lanes per row, phase 1 | (phase 2 << 8)
  std::vector<int32_t> lrows;     // n: positions in level order
  std::vector<int32_t> row_sn;    // n: supernode of each position
  std::vector<SnHost> sn;
  std::vector<int64_t> rp;        // lower: n + 1
  std::vector<int32_t> col;       // lower: off-diagonal columns
  std::vector<double> val;        // lower: CSR values; upper: panel values
  std::vector<int32_t> ridx;      // upper: panel column lists
  std::vector<double> tri;        // inverted diagonal triangles, packed by rows
  int64_t off_nnz() const { return (int64_t)val.size(); }
};

// Threads of the workgroup that solves one block; lane-group widths are sized for it.
constexpr int kSolveThreads = 1024;

// Device layout of one packed triangular factor of one block.  Rows are stored
// level by level (the order of TriHost::lrows) and so is all factor data, so
// every level reads one contiguous stretch of memory.  Each row has one record
// of 8 int32 (offsets relative to the block's arrays):
//   [0] position p             [1] off-diagonal start (val/col or panel val)
//   [2] off-diagonal length    [3] upper: start of the supernode's column list
//   [4] triangle-row start     [5] triangle-row length
//   [6] first scratch index of the triangle row (level-local)   [7] unused
// Solving level l: r_k = X[p] - sum_j off[j] * X[col_j] for all rows k of the
// level, then X[p] = sum_j tri[j] * r_{rec[6] + j}.
struct TriPacked {
  bool lower = true;
  int32_t n = 0, nlev = 0, max_lrows = 0;
  std::vector<int32_t> lev_ptr;   // nlev + 1
  std::vector<int32_t> lev_g;     // nlev: lanes per row, sweep 1 | (sweep 2 << 8)
  std::vector<int32_t> rec;       // 8 per row
  std::vector<double> val, tri;
  std::vector<int32_t> col, ridx;
};

// Factorisation of one block M: P (Q M Q^T) = L U with Q a nested-dissection
// ordering (postordered) and P a row permutation that only permutes rows
// inside each supernode (restricted threshold partial pivoting).
//   solve M x = b:   X[p] = b[gin[p]]; lower(lo); upper(up); x[gout[c]] = X[c]
//   solve M^T x = b: X[c] = b[gout[c]]; lower(loT); upper(upT); x[gin[p]] = X[p]
struct BlockFactor {
  int32_t n = 0;
  std::vector<int32_t> gin, gout;
  TriPacked lo, up, loT, upT;
  int64_t nnz_L = 0, nnz_U = 0;   // entries of L and U (diagonal blocks included)
  int32_t nsuper = 0;
};

// Fill `out` for block M.  Returns 0 on success, 2 on a zero pivot (message in err).
int factor_block(const CsrL& M, double tau, bool want_transpose, BlockFactor& out,
                 std::string& err);

// Reordering of Sec. 2 (interface rule and interiors-first permutation).
struct Reordering {
  int64_t n = 0, p = 0, q = 0;
  int32_t nparts = 0;
  std::vector<int64_t> perm;      // new -> old
  std::vector<int64_t> int_ptr;   // nparts + 1, positions in 0..p
  std::vector<int64_t> if_ptr;    // nparts + 1, positions in 0..q
};
void symmetric_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind,
                       std::vector<int64_t>& sptr, std::vector<int32_t>& sidx);
Reordering reorder(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* part,
                   int32_t nparts);

// Blocks of the reordered matrix.
struct Blocks {
  std::vector<CsrL> B, C0, E, F;  // per part: B_i, C_i, E_i (p_i x q_i), F_i (q_i x p_i)
  CsrG Cg;                        // q x q coupling between different parts' interfaces
};
Blocks extract_blocks(int64_t n, const int64_t* rowptr, const int32_t* colind,
                      const double* vals, const Reordering& R);

// Apply `fn(i)` for i in [0, count) on `nthreads` host threads.
void parallel_for(int count, int nthreads, const std::function<void(int)>& fn);

// Pack a TriHost into the device layout.
void pack_tri(const TriHost& T, TriPacked& P);

// Host execution of a packed factor on one vector (diagnostics only).
void host_tri_solve(const TriPacked& T, std::vector<double>& X);

uint64_t splitmix64_next(uint64_t& state);

}  // namespace pslr
