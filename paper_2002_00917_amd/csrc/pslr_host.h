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

// One supernode of a triangular factor.  Rows f..f+w-1 (positions) form a
// dense w x w diagonal triangle, stored INVERTED and packed by rows at
// tri_off (lower: row i holds columns 0..i; upper: columns i..w-1).  The
// off-diagonal part is a dense panel over the position list
// ridx[ridx_off .. +h), row-major at panel_off:
//   lower factor: h x w, entry (a, j) = L[ridx[a], f + j]  (column panel:
//                 the rows that column block f..f+w-1 updates)
//   upper factor: w x h, entry (i, a) = U[f + i, ridx[a]]  (row panel)
struct SnHost {
  int32_t f, w, h, pad;
  int64_t tri_off, panel_off, ridx_off;
};

// A triangular factor of one block, solved level by level: level l holds
// whole supernodes (rows lrows[lev_ptr[l] .. lev_ptr[l+1]), supernode by
// supernode, rows ascending).  Lower factors run l = 0..nlev-1, upper ones
// l = nlev-1..0.
struct TriHost {
  bool lower = true;
  int32_t n = 0, nlev = 0, max_lrows = 0;
  std::vector<int32_t> lev_ptr;   // nlev + 1
  std::vector<int32_t> lrows;     // n: positions in level order
  std::vector<int32_t> row_sn;    // n: supernode of each position
  std::vector<SnHost> sn;
  std::vector<double> val;        // panels
  std::vector<int32_t> ridx;      // panel position lists
  std::vector<double> tri;        // inverted diagonal triangles, packed by rows
};

// Threads of the workgroup that solves one block; chunk counts are sized for it.
constexpr int kSolveThreads = 1024;
// Levels whose supernodes average fewer rows than this store their
// off-diagonal part as entries rather than panels (measured on the 64^3
// workload: the interior blocks B_i gain from panels down to 8-row supernodes,
// the interface blocks C_i keep entries up to 24).
#ifndef PSLR_NARROW_B
#define PSLR_NARROW_B 8
#endif
#ifndef PSLR_NARROW_C
#define PSLR_NARROW_C 24
#endif
constexpr int kNarrowWidthB = PSLR_NARROW_B;
constexpr int kNarrowWidthC = PSLR_NARROW_C;

// Device layout of one packed triangular factor of one block.  All data is
// stored level by level, so every level reads one contiguous stretch of each
// array.  Per level l: row items lev_ptr[l] .. lev_ptr[l+1] (one per row);
// lev_c[l] = C_T | (C_P << 8) | (E << 16) splits the inner loop of every
// triangle item into C_T chunks and of every panel item into C_P chunks
// (chunks meet through atomic adds).  The off-diagonal part of a level is
// stored as panels and, for levels of narrow supernodes (E = 1), also as
// entries ent_ptr[l] .. ent_ptr[l+1] with one value and two positions each, so
// that every thread streams independent loads:
//   lower: x[eidx] -= eval * x0[eloc]        upper: x[eloc] -= eval * x[eidx]
// (x0: the level's rows before its solve)
// FP64 single-right-hand-side solves with working vectors in LDS use the
// entries (one atomic add per entry is cheap there); other solves use the panels.  A
// lower factor has push items push_ptr[l] .. push_ptr[l+1], one per panel row
// of each supernode.
//
// Row record, 8 int32 (offsets relative to the block's arrays):
//   [0] position p   [1] row i in its supernode   [2] w   [3] h
//   [4] triangle start (column-major packed)       [5] panel start
//   [6] ridx start   [7] level-local index of the supernode's first row
// Push record (lower panel levels), 4 int32:
//   [0] target position ridx[a]   [1] panel start + a   [2] w | (h << 16)
//   [3] position of the supernode's first row
//
// Triangles and panels store their columns in interleaved pairs (2c, 2c+1),
// so that one load brings a lane two columns, and consecutive lanes
// (consecutive rows) read consecutive pairs:
//   inverted lower triangle: pair c holds rows 2c..w-1; entry (i, 2c+t) at
//     2 (c (w - c + 1) + i - 2c) + t
//   inverted upper triangle: pair c holds rows 0..2c+1; entry (i, 2c+t) at
//     2 (c (c + 1) + i) + t
//   lower panel (a, 2c+t) at 2 (c h + a) + t; upper panel (i, 2c+t) at 2 (c w + i) + t
// Entries outside a triangle, and the partner of an odd last column, are
// stored zeros; each upper position list is padded to even length by
// repeating its last position.  Every supernode's arrays start at an even
// offset.  Entries follow the panel order within each supernode.
// The push record's panel start [1] is a pair index (panel start / 2 + a).
//
// Panels are stored folded with the inverted triangle (Pf = Lpanel Tinv for
// lower factors, Tinv Upanel for upper ones), so that each level is one step
// over values from before the level:
// Lower solve (right-looking), per level, with x0 = x[f .. f+w-1] (b minus the
// pushed updates): x[p] = sum_j Tinv(i, j) x0_j for every row item and
// x[ridx[a]] -= sum_j Pf(a, j) x0_j for every push item.
// Upper solve (left-looking), per level, with x0 the level's rows from the
// lower solve: x[p] = sum_j Tinv(i, j) x0_{first + j} - sum_a Pf(i, a) x[ridx[a]].
struct TriPacked {
  bool lower = true;
  int32_t n = 0, nlev = 0, max_lrows = 0;
  std::vector<int32_t> lev_ptr;   // nlev + 1
  std::vector<int32_t> push_ptr;  // nlev + 1
  std::vector<int32_t> ent_ptr;   // nlev + 1
  std::vector<int32_t> lev_c;     // nlev
  std::vector<int32_t> rec;       // 8 per row
  std::vector<int32_t> prec;      // 4 per push item
  std::vector<double> val, tri, eval;
  std::vector<int32_t> ridx, eidx, eloc;
  // entries a solve reads: values and int32 indices/record words, [0] on the
  // single-right-hand-side path (entry form where present), [1] on the panel path
  int64_t read_vals[2] = {0, 0}, read_ints[2] = {0, 0};
  // team groups (BlockFactor::loS/upS) store local positions: pos[k] is the
  // block position of local position k (empty: positions are block positions)
  std::vector<int32_t> pos;
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
  // Team split (team >= 1): the supernodal elimination tree cut into `team`
  // groups of whole subtrees (balanced by factor entries) and the top group
  // of the supernodes above them.  loS[g] / upS[g] hold the same supernodes
  // as lo / up restricted to group g (g = team: the top group), each with its
  // own level schedule over the block's positions: a subtree's solve needs
  // no row of another subtree, its lower solve pushes into top rows only, and
  // the top group's upper solve reads top rows only.  team = 1 (a block of a
  // split family too small to divide): one group of every supernode and an
  // empty top group.
  int32_t team = 0;
  std::vector<TriPacked> loS, upS;
  // Dense inverse of the top group's block of L U (team >= 1, top group of at
  // most kTopInvMaxRows rows; empty otherwise).  Positions of the top group in
  // the order of loS[team]'s row records, T; the top group holds every
  // ancestor of its supernodes, so L[G, T] = 0 and U[T, G] = 0 for the other
  // positions G, and the solve gives x_T = (L_TT U_TT)^{-1} (b_T - L_TG y_G)
  // with y_G the subtrees' lower solves.  Column pairs: entry (r, j) at
  // 2 ((j / 2) ld + r) + (j % 2) with ld = top_ld(ntop) (whole 256-byte FP64
  // lines per column pair), an odd last column and rows past ntop zeros.
  std::vector<double> topinv;
  int32_t ntop = 0;
  int64_t nnz_L = 0, nnz_U = 0;   // entries of L and U (diagonal blocks included)
  int32_t nsuper = 0;
};

// Fill `out` for block M.  Returns 0 on success, 2 on a zero pivot, 3 on a
// supernode too large for the device layout (message in err).
// narrow_width: the entry-form threshold of pack_tri (kNarrowWidthB for
// interior blocks, kNarrowWidthC for interface blocks).
// min_top_rows: the team split's top group is deepened (whole supernodes taken
// from the heaviest subtree downwards) until it holds at least that many rows.
int factor_block(const CsrL& M, double tau, bool want_transpose, int narrow_width, BlockFactor& out,
                 std::string& err, int team = 0, int min_top_rows = 0);

// Team groups of a supernodal elimination tree (postordered: children before
// parents, every subtree a contiguous range): grp[s] in [0, team) for the
// supernodes of the `team` groups of whole subtrees, team for the top group.
// Subtrees are taken from the roots down, moving the heaviest (by `work`) into
// the top group while the candidates are fewer than `team` or the heaviest
// exceeds 1.25 times an even share, as long as the top group stays below 45%
// of the work; the subtrees are then assigned largest first to the lightest
// group.
std::vector<int> team_groups(const std::vector<int>& spar, const std::vector<double>& work, int team,
                             const std::vector<int>* rows = nullptr, int min_top_rows = 0);

// Least top-group rows of the team splits of interior (B_i) and interface
// (C_i) blocks (see factor_block).  The interface blocks' trees are shallow
// surfaces whose subtree levels cost more than their bytes: on the 64^3
// workload top groups of at least 128, 256 and 384 rows took the FP64 series
// step from 149.0 to 144.9, 146.4 and 146.1 us (FP32: 114.8 to 110.9, 108.5,
// 106.3 us); deepening the interior blocks' tops to 600 rows cost 18 us.
#ifndef PSLR_TOP_ROWS_B
#define PSLR_TOP_ROWS_B 0
#endif
#ifndef PSLR_TOP_ROWS_C
#define PSLR_TOP_ROWS_C 256
#endif
constexpr int kTopRowsB = PSLR_TOP_ROWS_B, kTopRowsC = PSLR_TOP_ROWS_C;

// Threshold incomplete LU of block M in its given row order, no pivoting
// (the ilu() of Algorithm 4): row by row, w = M[i, :], tau_i = drop times the
// mean modulus of the stored entries of M[i, :]; for each k < i with w_k != 0,
// in increasing k: w_k /= u_kk, dropped (set to 0, no update) when
// |w_k| < tau_i, else w -= w_k U[k, :]; then the L part keeps the surviving
// w_k, the U part the diagonal and every w_j (j > i) with |w_j| >= tau_i.  drop = 0 gives the exact LU without
// pivoting.  The factors are packed as supernodes of one row each; gin and
// gout are the identity.  Returns 0, 2 on a zero pivot, 3 on a factor too
// large for the layout.
int ilut_block(const CsrL& M, double drop, bool want_T, int narrow_width, BlockFactor& out,
               std::string& err);

// The factors ilut_block packs: L[i] the strictly lower entries of row i and
// U[i] the strictly upper entries of row i, as (column, value) ascending, and
// d[i] = U(i, i) (L has a unit diagonal).
using SparseList = std::vector<std::vector<std::pair<int32_t, double>>>;
struct IlutFactors {
  SparseList L, U;
  std::vector<double> d;
};
int ilut_factor(const CsrL& M, double drop, IlutFactors& F, std::string& err);

// Structural check of a packed factor's level schedule: every position is
// scheduled once, the rows of a supernode share a level, and every
// off-diagonal dependency (panel rows, push targets, entry-form indices) is
// solved strictly before the row that needs it.
bool check_levels(const TriPacked& T, std::string& err);

// Structural check of a team split (BlockFactor::loS/upS): every position in
// one group; each subtree group's lower pushes and upper pulls reach only its
// own rows on the right side of the schedule or the top group; the top
// group's stay inside it.
bool check_team(const BlockFactor& F, std::string& err);

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

// Pack a TriHost into the device layout (levels whose supernodes average
// fewer than narrow_width rows also get the entry form); false if a supernode exceeds the
// record field widths (w or h above 32767) or a block's arrays exceed 2^31.
// map (optional): block position -> the position the packed layout stores
bool pack_tri(const TriHost& T, TriPacked& P, int narrow_width, const std::vector<int>* map = nullptr);

// Largest top group stored as a dense inverse (8 MiB of FP64 per block).
constexpr int kTopInvMaxRows = 1024;
// leading dimension (in pairs) of a dense top inverse: ntop rounded up to 16
inline int top_ld(int ntop) { return (ntop + 15) & ~15; }

// The dense inverse of BlockFactor::topinv from the top group's packed lower
// and upper factors of a block of n positions; false when a record reaches a
// position outside the top group.
bool top_inverse(const TriPacked& lo, const TriPacked& up, int n, std::vector<double>& M);

// Host execution of a packed factor on one vector (diagnostics only).
// entries: use the entry form where a level has one (else the panels).
void host_tri_solve(const TriPacked& T, std::vector<double>& X, bool entries);
// the same for a layout over local positions (TriPacked::pos): X by block position
void host_tri_solve_pos(const TriPacked& T, std::vector<double>& X, bool entries);

// Invariant subspace of a small real matrix H_m (n x n, column-major, leading
// dimension ldh) for its Ritz values of largest modulus (the Krylov-Schur
// restart of the deflated low-rank setup; pslr_schur.cpp).  Keeps the k of
// largest modulus (k - 1 when the cut would split a complex-conjugate pair),
// plus every value whose modulus ties the last kept one.
// Outputs: W (n x kept, column-major, orthonormal columns spanning the
// subspace), Hk = W^T H_m W (kept x kept, column-major), and all n Ritz values
// by decreasing modulus.  Returns kept (>= 0), or -1 with err set.
int schur_select(int n, const double* Hm, int64_t ldh, int k, std::vector<double>& W,
                 std::vector<double>& Hk, std::vector<double>& ritz_re, std::vector<double>& ritz_im,
                 std::string& err);

uint64_t splitmix64_next(uint64_t& state);

}  // namespace pslr
