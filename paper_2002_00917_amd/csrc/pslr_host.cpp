// Host-side setup of the PSLR preconditioner (paper Sec. 2 and Algorithm 4).
//
// * reorder(): interface detection and the interiors-first permutation of
//   Sec. 2 (eq. resystem).
// * extract_blocks(): B_i, E_i, F_i, C_i and the inter-subdomain coupling C_g
//   (Sec. 3.1, eq. matrixS and the proof of Lemma l2).
// * factor_block(): exact sparse LU of one diagonal block (Algorithm 4 builds
//   ILU factors; exact LU is used here).  Nested-dissection ordering by
//   recursive BFS level-set bisection, elimination tree, fundamental
//   supernodes, multifrontal numeric factorisation with threshold partial
//   pivoting restricted to each front's fully-summed rows, then packing into
//   the level-scheduled layouts read by the device triangular solves: the
//   dense diagonal triangle of every supernode is stored inverted, so each
//   level of the solve is two parallel dot-product sweeps.
#include "pslr_host.h"

#include <algorithm>
#include <functional>
#include <climits>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

namespace pslr {

uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void parallel_for(int count, int nthreads, const std::function<void(int)>& fn) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  nthreads = std::min(nthreads, std::max(count, 1));
  if (nthreads <= 1) {
    for (int i = 0; i < count; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&]() {
      for (int i = next++; i < count; i = next++) fn(i);
    });
  for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------------------
// Reordering (Sec. 2)
// ---------------------------------------------------------------------------

void symmetric_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind,
                       std::vector<int64_t>& sptr, std::vector<int32_t>& sidx) {
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      int64_t j = colind[k];
      if (j == i) continue;
      cnt[i + 1]++;
      cnt[j + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> tmp(cnt[n]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      int64_t j = colind[k];
      if (j == i) continue;
      tmp[pos[i]++] = (int32_t)j;
      tmp[pos[j]++] = (int32_t)i;
    }
  sptr.assign(n + 1, 0);
  sidx.clear();
  sidx.reserve(tmp.size());
  for (int64_t i = 0; i < n; ++i) {
    auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
    std::sort(b, e);
    auto u = std::unique(b, e);
    sidx.insert(sidx.end(), b, u);
    sptr[i + 1] = (int64_t)sidx.size();
  }
}

Reordering reorder(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* part,
                   int32_t nparts) {
  Reordering R;
  R.n = n;
  R.nparts = nparts;
  std::vector<int64_t> sptr;
  std::vector<int32_t> sidx;
  symmetric_pattern(n, rowptr, colind, sptr, sidx);
  std::vector<char> iface(n, 0);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = sptr[v]; k < sptr[v + 1]; ++k)
      if (part[sidx[k]] != part[v]) {
        iface[v] = 1;
        break;
      }
  std::vector<int64_t> nint(nparts, 0), nif(nparts, 0);
  for (int64_t v = 0; v < n; ++v) (iface[v] ? nif : nint)[part[v]]++;
  R.int_ptr.assign(nparts + 1, 0);
  R.if_ptr.assign(nparts + 1, 0);
  for (int i = 0; i < nparts; ++i) {
    R.int_ptr[i + 1] = R.int_ptr[i] + nint[i];
    R.if_ptr[i + 1] = R.if_ptr[i] + nif[i];
  }
  R.p = R.int_ptr[nparts];
  R.q = R.if_ptr[nparts];
  R.perm.assign(n, 0);
  std::vector<int64_t> ci(R.int_ptr.begin(), R.int_ptr.end() - 1);
  std::vector<int64_t> cf(R.if_ptr.begin(), R.if_ptr.end() - 1);
  for (int64_t v = 0; v < n; ++v) {
    if (iface[v]) R.perm[R.p + cf[part[v]]++] = v;
    else R.perm[ci[part[v]]++] = v;
  }
  return R;
}

static void finish_csr(CsrL& M, std::vector<std::vector<std::pair<int32_t, double>>>& rows) {
  M.ptr.assign(M.nrows + 1, 0);
  for (int32_t r = 0; r < M.nrows; ++r) M.ptr[r + 1] = M.ptr[r] + (int32_t)rows[r].size();
  M.col.resize(M.ptr[M.nrows]);
  M.val.resize(M.ptr[M.nrows]);
  for (int32_t r = 0; r < M.nrows; ++r) {
    auto& rw = rows[r];
    std::sort(rw.begin(), rw.end());
    for (size_t k = 0; k < rw.size(); ++k) {
      M.col[M.ptr[r] + k] = rw[k].first;
      M.val[M.ptr[r] + k] = rw[k].second;
    }
  }
}

Blocks extract_blocks(int64_t n, const int64_t* rowptr, const int32_t* colind,
                      const double* vals, const Reordering& R) {
  const int np = R.nparts;
  std::vector<int64_t> iperm(n);
  for (int64_t k = 0; k < n; ++k) iperm[R.perm[k]] = k;
  // owner part of each new position
  std::vector<int32_t> own(n);
  for (int i = 0; i < np; ++i) {
    for (int64_t k = R.int_ptr[i]; k < R.int_ptr[i + 1]; ++k) own[k] = i;
    for (int64_t k = R.if_ptr[i]; k < R.if_ptr[i + 1]; ++k) own[R.p + k] = i;
  }
  Blocks Bk;
  Bk.B.resize(np);
  Bk.C0.resize(np);
  Bk.E.resize(np);
  Bk.F.resize(np);
  std::vector<std::vector<std::pair<int32_t, double>>> cgrows(R.q);
  parallel_for(np, 0, [&](int i) {
    const int64_t i0 = R.int_ptr[i], pi = R.int_ptr[i + 1] - i0;
    const int64_t f0 = R.if_ptr[i], qi = R.if_ptr[i + 1] - f0;
    CsrL& B = Bk.B[i]; CsrL& E = Bk.E[i]; CsrL& F = Bk.F[i]; CsrL& C = Bk.C0[i];
    B.nrows = B.ncols = (int32_t)pi;
    E.nrows = (int32_t)pi; E.ncols = (int32_t)qi;
    F.nrows = (int32_t)qi; F.ncols = (int32_t)pi;
    C.nrows = C.ncols = (int32_t)qi;
    std::vector<std::vector<std::pair<int32_t, double>>> rb(pi), re(pi), rf(qi), rc(qi);
    for (int64_t r = 0; r < pi; ++r) {
      int64_t o = R.perm[i0 + r];
      for (int64_t k = rowptr[o]; k < rowptr[o + 1]; ++k) {
        int64_t c = iperm[colind[k]];
        if (c < R.p) rb[r].push_back({(int32_t)(c - i0), vals[k]});
        else re[r].push_back({(int32_t)(c - R.p - f0), vals[k]});
      }
    }
    for (int64_t r = 0; r < qi; ++r) {
      int64_t o = R.perm[R.p + f0 + r];
      for (int64_t k = rowptr[o]; k < rowptr[o + 1]; ++k) {
        int64_t c = iperm[colind[k]];
        if (c < R.p) rf[r].push_back({(int32_t)(c - i0), vals[k]});
        else if (own[c] == i) rc[r].push_back({(int32_t)(c - R.p - f0), vals[k]});
        else cgrows[f0 + r].push_back({(int32_t)(c - R.p), vals[k]});
      }
    }
    finish_csr(B, rb);
    finish_csr(E, re);
    finish_csr(F, rf);
    finish_csr(C, rc);
  });
  CsrG& G = Bk.Cg;
  G.nrows = G.ncols = R.q;
  G.ptr.assign(R.q + 1, 0);
  for (int64_t r = 0; r < R.q; ++r) {
    auto& rw = cgrows[r];
    std::sort(rw.begin(), rw.end());
    for (auto& e : rw) {
      G.col.push_back(e.first);
      G.val.push_back(e.second);
    }
    G.ptr[r + 1] = (int64_t)G.col.size();
  }
  return Bk;
}

// ---------------------------------------------------------------------------
// Nested dissection by recursive BFS level-set bisection
// ---------------------------------------------------------------------------

namespace {

struct Graph {
  int n = 0;
  std::vector<int> ptr, adj;
};

Graph block_graph(const CsrL& M) {
  Graph g;
  g.n = M.nrows;
  std::vector<int64_t> rp(M.nrows + 1);
  for (int i = 0; i <= M.nrows; ++i) rp[i] = M.ptr[i];
  std::vector<int64_t> sp;
  std::vector<int32_t> si;
  symmetric_pattern(M.nrows, rp.data(), M.col.data(), sp, si);
  g.ptr.assign(sp.begin(), sp.end());
  g.adj.assign(si.begin(), si.end());
  return g;
}

struct ND {
  const Graph& g;
  std::vector<int> tag, lev, order, queue;
  int ntag = 1;
  int kLeaf = 8;
  explicit ND(const Graph& gr) : g(gr), tag(gr.n, 0), lev(gr.n, -1), queue(gr.n) {}

  // BFS from r inside tag t; returns number reached, fills queue[0..cnt) in BFS order.
  int bfs(int r, int t, int& depth) {
    int head = 0, tail = 0;
    queue[tail++] = r;
    lev[r] = 0;
    depth = 0;
    while (head < tail) {
      int v = queue[head++];
      for (int k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        int w = g.adj[k];
        if (tag[w] == t && lev[w] < 0) {
          lev[w] = lev[v] + 1;
          depth = std::max(depth, lev[w]);
          queue[tail++] = w;
        }
      }
    }
    return tail;
  }
  void clear_lev(int cnt) {
    for (int i = 0; i < cnt; ++i) lev[queue[i]] = -1;
  }

  void run(std::vector<int> S, int t) {
    if ((int)S.size() <= kLeaf) {
      std::sort(S.begin(), S.end());
      order.insert(order.end(), S.begin(), S.end());
      return;
    }
    int depth;
    int cnt = bfs(S[0], t, depth);
    if (cnt < (int)S.size()) {  // several components: order them one after another
      std::vector<int> comp(queue.begin(), queue.begin() + cnt);
      clear_lev(cnt);
      int t1 = ntag++;
      for (int v : comp) tag[v] = t1;
      std::vector<int> rest;
      for (int v : S)
        if (tag[v] == t) rest.push_back(v);
      run(comp, t1);
      run(rest, t);
      return;
    }
    // pseudo-peripheral root: restart from the last vertex reached while the depth grows
    int root = queue[cnt - 1];
    clear_lev(cnt);
    for (int it = 0; it < 4; ++it) {
      int d2;
      cnt = bfs(root, t, d2);
      int far = queue[cnt - 1];
      clear_lev(cnt);
      if (d2 <= depth) {
        depth = d2;
        break;
      }
      depth = d2;
      root = far;
    }
    cnt = bfs(root, t, depth);
    if (depth < 2) {
      clear_lev(cnt);
      std::sort(S.begin(), S.end());
      order.insert(order.end(), S.begin(), S.end());
      return;
    }
    std::vector<int> lsize(depth + 1, 0);
    for (int i = 0; i < cnt; ++i) lsize[lev[queue[i]]]++;
    int k = 1, acc = lsize[0];
    while (k < depth - 1 && acc + lsize[k] < (int)S.size() / 2) acc += lsize[k++];
    std::vector<int> A, Bv, sep;
    for (int i = 0; i < cnt; ++i) {
      int v = queue[i];
      if (lev[v] < k) A.push_back(v);
      else if (lev[v] > k) Bv.push_back(v);
      else sep.push_back(v);
    }
    // shrink the separator: vertices not touching the far side join the near side
    std::vector<int> sep2;
    for (int v : sep) {
      bool touchB = false;
      for (int q = g.ptr[v]; q < g.ptr[v + 1] && !touchB; ++q) {
        int w = g.adj[q];
        touchB = (tag[w] == t && lev[w] == k + 1);
      }
      if (touchB) sep2.push_back(v);
      else A.push_back(v);
    }
    clear_lev(cnt);
    int ta = ntag++, tb = ntag++, ts = ntag++;
    for (int v : A) tag[v] = ta;
    for (int v : Bv) tag[v] = tb;
    for (int v : sep2) tag[v] = ts;
    run(std::move(A), ta);
    run(std::move(Bv), tb);
    std::sort(sep2.begin(), sep2.end());
    order.insert(order.end(), sep2.begin(), sep2.end());
  }
};

// Elimination tree of a symmetric pattern (Liu's algorithm with path compression).
std::vector<int> etree(const Graph& g) {
  std::vector<int> parent(g.n, -1), anc(g.n, -1);
  for (int k = 0; k < g.n; ++k)
    for (int q = g.ptr[k]; q < g.ptr[k + 1]; ++q) {
      int r = g.adj[q];
      if (r >= k) continue;
      while (anc[r] != -1 && anc[r] != k) {
        int t = anc[r];
        anc[r] = k;
        r = t;
      }
      if (anc[r] == -1) {
        anc[r] = k;
        parent[r] = k;
      }
    }
  return parent;
}

std::vector<int> postorder(const std::vector<int>& parent) {
  int n = (int)parent.size();
  std::vector<int> head(n, -1), next(n, -1), post;
  post.reserve(n);
  for (int v = n - 1; v >= 0; --v)
    if (parent[v] >= 0) {
      next[v] = head[parent[v]];
      head[parent[v]] = v;
    }
  std::vector<int> stack;
  for (int r = 0; r < n; ++r) {
    if (parent[r] >= 0) continue;
    stack.push_back(r);
    while (!stack.empty()) {
      int v = stack.back();
      if (head[v] >= 0) {
        int c = head[v];
        head[v] = next[c];
        stack.push_back(c);
      } else {
        stack.pop_back();
        post.push_back(v);
      }
    }
  }
  return post;
}

Graph permute_graph(const Graph& g, const std::vector<int>& perm, const std::vector<int>& iperm) {
  Graph h;
  h.n = g.n;
  h.ptr.assign(g.n + 1, 0);
  h.adj.reserve(g.adj.size());
  for (int i = 0; i < g.n; ++i) {
    int o = perm[i];
    size_t b = h.adj.size();
    for (int q = g.ptr[o]; q < g.ptr[o + 1]; ++q) h.adj.push_back(iperm[g.adj[q]]);
    std::sort(h.adj.begin() + b, h.adj.end());
    h.ptr[i + 1] = (int)h.adj.size();
  }
  return h;
}

// Inverse of a unit lower (lower = true) or upper triangular w x w matrix
// stored row-major in T; result row-major in X.
void invert_triangle(const double* T, int w, bool lower, double* X) {
  std::fill(X, X + (size_t)w * w, 0.0);
  if (lower) {
    for (int j = 0; j < w; ++j) {
      X[(size_t)j * w + j] = 1.0;
      for (int i = j + 1; i < w; ++i) {
        double s = 0.0;
        for (int k = j; k < i; ++k) s += T[(size_t)i * w + k] * X[(size_t)k * w + j];
        X[(size_t)i * w + j] = -s;
      }
    }
  } else {
    for (int j = w - 1; j >= 0; --j) {
      X[(size_t)j * w + j] = 1.0 / T[(size_t)j * w + j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += T[(size_t)i * w + k] * X[(size_t)k * w + j];
        X[(size_t)i * w + j] = -s / T[(size_t)i * w + i];
      }
    }
  }
}

// Level schedule: supernode heights in the supernodal elimination tree.
void build_levels(TriHost& T, const std::vector<int>& sfirst, const std::vector<int>& height,
                  int nlev) {
  const int ns = (int)sfirst.size() - 1;
  T.nlev = nlev;
  T.lev_ptr.assign(nlev + 1, 0);
  T.lrows.clear();
  T.lrows.reserve(T.n);
  T.row_sn.assign(T.n, 0);
  T.max_lrows = 0;
  std::vector<std::vector<int>> bylev(nlev);
  for (int s = 0; s < ns; ++s) bylev[height[s]].push_back(s);
  for (int l = 0; l < nlev; ++l) {
    for (int s : bylev[l])
      for (int r = sfirst[s]; r < sfirst[s + 1]; ++r) {
        T.lrows.push_back(r);
        T.row_sn[r] = s;
      }
    T.lev_ptr[l + 1] = (int)T.lrows.size();
    T.max_lrows = std::max(T.max_lrows, T.lev_ptr[l + 1] - T.lev_ptr[l]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Exact sparse LU of one block
// ---------------------------------------------------------------------------

std::vector<int> team_groups(const std::vector<int>& spar, const std::vector<double>& work, int team,
                             const std::vector<int>* rows, int min_top_rows) {
  const int ns = (int)spar.size();
  std::vector<int> grp(ns, team);
  if (team <= 1 || ns == 0) {
    std::fill(grp.begin(), grp.end(), 0);
    return grp;
  }
  std::vector<std::vector<int>> kids(ns);
  std::vector<double> sub(work.begin(), work.end());
  std::vector<int> lo(ns);
  for (int s = 0; s < ns; ++s) lo[s] = s;
  for (int s = 0; s < ns; ++s)
    if (spar[s] >= 0) {
      kids[spar[s]].push_back(s);
      sub[spar[s]] += sub[s];
      lo[spar[s]] = std::min(lo[spar[s]], lo[s]);
    }
  std::vector<int> cand;
  double total = 0.0, top = 0.0;
  for (int s = 0; s < ns; ++s)
    if (spar[s] < 0) {
      cand.push_back(s);
      total += sub[s];
    }
  std::vector<char> is_top(ns, 0);
  int top_rows = 0;
  for (int it = 0; it < 4 * ns; ++it) {
    std::sort(cand.begin(), cand.end(), [&](int a, int b) { return sub[a] > sub[b]; });
    double csum = 0.0;
    for (int c : cand) csum += sub[c];
    const int c0 = cand[0];
    const bool deepen = rows && top_rows < min_top_rows && top_rows + (*rows)[c0] <= kTopInvMaxRows;
    if (!deepen && (int)cand.size() >= team && sub[c0] <= 1.25 * csum / team) break;
    if (kids[c0].empty() || (!deepen && top + work[c0] > 0.45 * total)) break;
    top += work[c0];
    if (rows) top_rows += (*rows)[c0];
    is_top[c0] = 1;
    cand.erase(cand.begin());
    cand.insert(cand.end(), kids[c0].begin(), kids[c0].end());
    if (cand.empty()) break;
  }
  std::sort(cand.begin(), cand.end(), [&](int a, int b) { return sub[a] > sub[b]; });
  std::vector<double> load(team, 0.0);
  for (int c : cand) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[g] += sub[c];
    for (int j = lo[c]; j <= c; ++j) grp[j] = g;
  }
  for (int s = 0; s < ns; ++s)
    if (is_top[s]) grp[s] = team;
  return grp;
}

// Bottom-up amalgamation: merged supernodes of at most kMergeWidth rows, at
// most kMergePasses rounds (each removes one level at the bottom).  Width 32
// was the fastest of 16, 32, 64 and 128 on the 64^3 workload with team solves
// (fewer levels against more stored zeros); the build-time overrides serve
// such sweeps.
#ifndef PSLR_MERGE_W
#define PSLR_MERGE_W 32
#endif
#ifndef PSLR_MERGE_P
#define PSLR_MERGE_P 3
#endif
#ifndef PSLR_CHAIN_FILL
#define PSLR_CHAIN_FILL 0.15
#endif
constexpr int kMergeWidth = PSLR_MERGE_W, kMergePasses = PSLR_MERGE_P;

int factor_block(const CsrL& M, double tau, bool want_T, int narrow_width, BlockFactor& out,
                 std::string& err, int team, int min_top_rows) {
  const int n = M.nrows;
  out = BlockFactor();
  out.n = n;
  if (n == 0) {
    for (TriPacked* T : {&out.lo, &out.up, &out.loT, &out.upT}) {
      T->n = 0;
      T->nlev = 0;
      T->lev_ptr.assign(1, 0);
    }
    out.lo.lower = out.loT.lower = true;
    out.up.lower = out.upT.lower = false;
    if (team >= 1) {  // an empty group: every block of a split family has one
      out.team = team;
      out.loS.assign(team + 1, out.lo);
      out.upS.assign(team + 1, out.up);
    }
    return 0;
  }
  double maxabs = 0.0;
  for (double v : M.val) maxabs = std::max(maxabs, std::fabs(v));

  // --- ordering: nested dissection, then etree postorder
  Graph g = block_graph(M);
  ND nd(g);
  if (const char* e = getenv("PSLR_ND_LEAF")) nd.kLeaf = atoi(e);
  {
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    nd.run(all, 0);
  }
  std::vector<int> perm = nd.order, iperm(n);
  for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
  Graph gp = permute_graph(g, perm, iperm);
  std::vector<int> par = etree(gp);
  std::vector<int> post = postorder(par);
  {
    std::vector<int> p2(n);
    for (int i = 0; i < n; ++i) p2[i] = perm[post[i]];
    perm.swap(p2);
  }
  for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
  gp = permute_graph(g, perm, iperm);
  par = etree(gp);

  // --- symbolic: column structures of L, fundamental supernodes
  std::vector<std::vector<int>> st(n);
  std::vector<int> nchild(n, 0), mark(n, -1);
  std::vector<int> chead(n, -1), cnext(n, -1);
  for (int v = n - 1; v >= 0; --v)
    if (par[v] >= 0) {
      nchild[par[v]]++;
      cnext[v] = chead[par[v]];
      chead[par[v]] = v;
    }
  for (int j = 0; j < n; ++j) {
    std::vector<int>& s = st[j];
    mark[j] = j;
    for (int q = gp.ptr[j]; q < gp.ptr[j + 1]; ++q) {
      int i = gp.adj[q];
      if (i > j && mark[i] != j) {
        mark[i] = j;
        s.push_back(i);
      }
    }
    for (int c = chead[j]; c >= 0; c = cnext[c])
      for (int i : st[c])
        if (i > j && mark[i] != j) {
          mark[i] = j;
          s.push_back(i);
        }
    std::sort(s.begin(), s.end());
  }
  std::vector<int> sfirst;
  sfirst.push_back(0);
  for (int j = 1; j < n; ++j) {
    bool join = par[j - 1] == j && st[j - 1].size() == st[j].size() + 1 && nchild[j] == 1;
    if (!join) sfirst.push_back(j);
  }
  sfirst.push_back(n);
  // relaxed amalgamation of single-child chains: a supernode whose parent has
  // no other child is merged into it when the explicit zeros this adds stay
  // small, which shortens the level schedule of the triangular solves
  {
    const int ns0 = (int)sfirst.size() - 1;
    std::vector<int> snode0(n), par0(ns0, -1), nch(ns0, 0);
    for (int s = 0; s < ns0; ++s)
      for (int j = sfirst[s]; j < sfirst[s + 1]; ++j) snode0[j] = s;
    for (int s = 0; s < ns0; ++s) {
      const std::vector<int>& Rs = st[sfirst[s + 1] - 1];
      if (!Rs.empty()) {
        par0[s] = snode0[Rs[0]];
        nch[par0[s]]++;
      }
    }
    std::vector<int> gfirst(sfirst.begin(), sfirst.end() - 1);
    std::vector<double> truenz(ns0);
    std::vector<char> absorbed(ns0, 0);
    for (int s = 0; s < ns0; ++s) {
      const double w = sfirst[s + 1] - sfirst[s], h = (double)st[sfirst[s + 1] - 1].size();
      truenz[s] = w * (w - 1) / 2 + w * h;
    }
    for (int s = 1; s < ns0; ++s) {
      if (par0[s - 1] != s) continue;
      const int c = s - 1;
      const double mw = (double)(sfirst[s + 1] - gfirst[c]);
      const double hp = (double)st[sfirst[s + 1] - 1].size();
      const double dense = mw * (mw - 1) / 2 + mw * hp;
      const double tnz = truenz[c] + truenz[s];
      if (mw <= 512 && (mw <= 16 || dense - tnz <= PSLR_CHAIN_FILL * dense)) {
        gfirst[s] = gfirst[c];
        truenz[s] = tnz;
        absorbed[c] = 1;
      }
    }
    std::vector<int> sf2;
    for (int s = 0; s < ns0; ++s)
      if (!absorbed[s]) sf2.push_back(gfirst[s]);
    sf2.push_back(n);
    sfirst.swap(sf2);
  }
  // bottom-up amalgamation: a supernode whose children are all leaves absorbs
  // them when the merged block stays narrow (postorder keeps the subtree
  // contiguous); every pass removes one level at the bottom of the schedule
  for (int pass = 0; pass < kMergePasses; ++pass) {
    const int ns0 = (int)sfirst.size() - 1;
    std::vector<int> snode0(n), par0(ns0, -1), nch(ns0, 0), wsum(ns0, 0), lfirst(ns0);
    std::vector<char> allleaf(ns0, 1);
    for (int s = 0; s < ns0; ++s)
      for (int j = sfirst[s]; j < sfirst[s + 1]; ++j) snode0[j] = s;
    for (int s = 0; s < ns0; ++s) {
      const std::vector<int>& Rs = st[sfirst[s + 1] - 1];
      if (!Rs.empty()) par0[s] = snode0[Rs[0]];
      lfirst[s] = sfirst[s];
    }
    for (int s = 0; s < ns0; ++s)
      if (par0[s] >= 0) {
        nch[par0[s]]++;
        wsum[par0[s]] += sfirst[s + 1] - sfirst[s];
      }
    for (int s = 0; s < ns0; ++s)
      if (par0[s] >= 0) {
        if (nch[s] > 0) allleaf[par0[s]] = 0;
        lfirst[par0[s]] = std::min(lfirst[par0[s]], sfirst[s]);
      }
    std::vector<char> absorbed(ns0, 0), merge(ns0, 0);
    bool any = false;
    for (int s = 0; s < ns0; ++s)
      if (nch[s] > 0 && allleaf[s] && wsum[s] + (sfirst[s + 1] - sfirst[s]) <= kMergeWidth) {
        merge[s] = 1;
        any = true;
      }
    if (!any) break;
    for (int s = 0; s < ns0; ++s)
      if (par0[s] >= 0 && merge[par0[s]]) absorbed[s] = 1;
    std::vector<int> sf2;
    for (int s = 0; s < ns0; ++s)
      if (!absorbed[s]) sf2.push_back(merge[s] ? lfirst[s] : sfirst[s]);
    sf2.push_back(n);
    sfirst.swap(sf2);
  }
  const int ns = (int)sfirst.size() - 1;
  out.nsuper = ns;
  std::vector<int> snode(n);
  for (int s = 0; s < ns; ++s)
    for (int j = sfirst[s]; j < sfirst[s + 1]; ++j) snode[j] = s;
  std::vector<std::vector<int>> R(ns);
  std::vector<int> spar(ns, -1), height(ns, 0);
  for (int s = 0; s < ns; ++s) {
    R[s] = st[sfirst[s + 1] - 1];
    if (!R[s].empty()) spar[s] = snode[R[s][0]];
  }
  st.clear();
  st.shrink_to_fit();
  int nlev = 1;
  for (int s = 0; s < ns; ++s)
    if (spar[s] >= 0) {
      height[spar[s]] = std::max(height[spar[s]], height[s] + 1);
      nlev = std::max(nlev, height[spar[s]] + 1);
    }

  // --- permuted matrix Mp = M[perm, perm], CSR and CSC
  std::vector<int> rp(n + 1, 0), ci;
  std::vector<double> cv;
  {
    std::vector<std::pair<int, double>> row;
    for (int i = 0; i < n; ++i) {
      int o = perm[i];
      row.clear();
      for (int k = M.ptr[o]; k < M.ptr[o + 1]; ++k) row.push_back({iperm[M.col[k]], M.val[k]});
      std::sort(row.begin(), row.end());
      for (auto& e : row) {
        ci.push_back(e.first);
        cv.push_back(e.second);
      }
      rp[i + 1] = (int)ci.size();
    }
  }
  std::vector<int> cp(n + 1, 0), ri(ci.size());
  std::vector<double> rv(ci.size());
  for (int c : ci) cp[c + 1]++;
  for (int i = 0; i < n; ++i) cp[i + 1] += cp[i];
  {
    std::vector<int> pos(cp.begin(), cp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        int d = pos[ci[k]]++;
        ri[d] = i;
        rv[d] = cv[k];
      }
  }

  // --- numeric multifrontal factorisation
  struct CB {
    std::vector<int> idx;
    std::vector<double> a;
  };
  std::vector<CB> stack;
  std::vector<std::vector<double>> diagLU(ns), Lp(ns), Up(ns);
  std::vector<int> prow(n);
  std::vector<int> relpos(n, -1);
  std::vector<int> snchild(ns, 0);
  for (int s = 0; s < ns; ++s)
    if (spar[s] >= 0) snchild[spar[s]]++;
  const int NB = 32;
  for (int s = 0; s < ns; ++s) {
    const int f = sfirst[s], l = sfirst[s + 1] - 1, w = l - f + 1;
    const std::vector<int>& Rs = R[s];
    const int h = (int)Rs.size(), N = w + h;
    for (int k = 0; k < w; ++k) relpos[f + k] = k;
    for (int a = 0; a < h; ++a) relpos[Rs[a]] = w + a;
    std::vector<double> F((size_t)N * N, 0.0);
    for (int j = f; j <= l; ++j) {
      for (int k = rp[j]; k < rp[j + 1]; ++k)
        if (ci[k] >= f) F[(size_t)(j - f) * N + relpos[ci[k]]] += cv[k];
      for (int k = cp[j]; k < cp[j + 1]; ++k)
        if (ri[k] > l) F[(size_t)relpos[ri[k]] * N + (j - f)] += rv[k];
    }
    for (int c = 0; c < snchild[s]; ++c) {
      CB cb = std::move(stack.back());
      stack.pop_back();
      const int hc = (int)cb.idx.size();
      for (int a = 0; a < hc; ++a) {
        double* Fr = &F[(size_t)relpos[cb.idx[a]] * N];
        const double* Cr = &cb.a[(size_t)a * hc];
        for (int b = 0; b < hc; ++b) Fr[relpos[cb.idx[b]]] += Cr[b];
      }
    }
    std::vector<int> pr(w);
    std::iota(pr.begin(), pr.end(), f);
    for (int k0 = 0; k0 < w; k0 += NB) {
      const int kend = std::min(w, k0 + NB);
      for (int k = k0; k < kend; ++k) {
        double amax = 0.0;
        int ip = k;
        for (int i = k; i < w; ++i) {
          double a = std::fabs(F[(size_t)i * N + k]);
          if (a > amax) {
            amax = a;
            ip = i;
          }
        }
        if (!(amax > 1e-14 * maxabs)) {
          err = "zero pivot in a diagonal block (singular or numerically singular block)";
          return 2;
        }
        if (std::fabs(F[(size_t)k * N + k]) >= tau * amax) ip = k;
        if (ip != k) {
          std::swap_ranges(F.begin() + (size_t)k * N, F.begin() + (size_t)(k + 1) * N,
                           F.begin() + (size_t)ip * N);
          std::swap(pr[k], pr[ip]);
        }
        const double piv = F[(size_t)k * N + k];
        const double* Fk = &F[(size_t)k * N];
        for (int i = k + 1; i < N; ++i) {
          double* Fi = &F[(size_t)i * N];
          double lik = Fi[k] / piv;
          Fi[k] = lik;
          if (lik != 0.0)
            for (int j = k + 1; j < kend; ++j) Fi[j] -= lik * Fk[j];
        }
      }
      for (int i = k0 + 1; i < kend; ++i) {
        double* Fi = &F[(size_t)i * N];
        for (int k = k0; k < i; ++k) {
          const double lik = Fi[k];
          if (lik == 0.0) continue;
          const double* Fk = &F[(size_t)k * N];
          for (int j = kend; j < N; ++j) Fi[j] -= lik * Fk[j];
        }
      }
      for (int i = kend; i < N; ++i) {
        double* Fi = &F[(size_t)i * N];
        for (int k = k0; k < kend; ++k) {
          const double lik = Fi[k];
          if (lik == 0.0) continue;
          const double* Fk = &F[(size_t)k * N];
          for (int j = kend; j < N; ++j) Fi[j] -= lik * Fk[j];
        }
      }
    }
    for (int k = 0; k < w; ++k) prow[f + k] = pr[k];
    diagLU[s].resize((size_t)w * w);
    Lp[s].resize((size_t)h * w);
    Up[s].resize((size_t)w * h);
    for (int i = 0; i < w; ++i)
      for (int j = 0; j < w; ++j) diagLU[s][(size_t)i * w + j] = F[(size_t)i * N + j];
    for (int a = 0; a < h; ++a)
      for (int j = 0; j < w; ++j) Lp[s][(size_t)a * w + j] = F[(size_t)(w + a) * N + j];
    for (int i = 0; i < w; ++i)
      for (int a = 0; a < h; ++a) Up[s][(size_t)i * h + a] = F[(size_t)i * N + w + a];
    if (h > 0) {
      CB cb;
      cb.idx = Rs;
      cb.a.resize((size_t)h * h);
      for (int a = 0; a < h; ++a)
        std::memcpy(&cb.a[(size_t)a * h], &F[(size_t)(w + a) * N + w], sizeof(double) * h);
      stack.push_back(std::move(cb));
    }
  }

  // --- index maps
  std::vector<int> posOf(n);
  for (int p = 0; p < n; ++p) posOf[prow[p]] = p;
  out.gin.resize(n);
  out.gout.resize(n);
  for (int p = 0; p < n; ++p) {
    out.gin[p] = perm[prow[p]];
    out.gout[p] = perm[p];
  }

  // --- packed layouts
  std::vector<double> inv, tmp;
  auto init_tri = [&](TriHost& T, bool lower) {
    T = TriHost();
    T.lower = lower;
    T.n = n;
    T.sn.resize(ns);
    for (int s = 0; s < ns; ++s) {
      SnHost& S = T.sn[s];
      S.f = sfirst[s];
      S.w = sfirst[s + 1] - sfirst[s];
      S.h = lower ? 0 : (int)R[s].size();
      S.pad = 0;
      S.tri_off = S.panel_off = S.ridx_off = 0;
    }
  };
  // packed inverted triangles: lower rows hold columns 0..i, upper rows i..w-1
  auto pack_inv = [&](TriHost& T, int s, const std::vector<double>& Xinv, bool transpose) {
    const int w = T.sn[s].w;
    T.sn[s].tri_off = (int64_t)T.tri.size();
    for (int i = 0; i < w; ++i) {
      int a = T.lower ? 0 : i, b = T.lower ? i : w - 1;
      for (int k = a; k <= b; ++k)
        T.tri.push_back(transpose ? Xinv[(size_t)k * w + i] : Xinv[(size_t)i * w + k]);
    }
  };
  std::vector<std::vector<double>> invL(ns), invU(ns);
  for (int s = 0; s < ns; ++s) {
    const int w = sfirst[s + 1] - sfirst[s];
    invL[s].resize((size_t)w * w);
    invU[s].resize((size_t)w * w);
    invert_triangle(diagLU[s].data(), w, true, invL[s].data());
    invert_triangle(diagLU[s].data(), w, false, invU[s].data());
    out.nnz_L += (int64_t)w * (w + 1) / 2 + (int64_t)w * (int64_t)R[s].size();
    out.nnz_U += (int64_t)w * (w + 1) / 2 + (int64_t)w * (int64_t)R[s].size();
  }
  // lower column panels from the L panels (forward) or U panels (transposed):
  // entry (a, j) = factor[ridx[a], f + j], row-major h x w
  auto build_lower_panels = [&](TriHost& T, bool fromU) {
    for (int s = 0; s < ns; ++s) {
      SnHost& S = T.sn[s];
      const int w = S.w, h = (int)R[s].size();
      S.h = h;
      S.ridx_off = (int64_t)T.ridx.size();
      S.panel_off = (int64_t)T.val.size();
      for (int a = 0; a < h; ++a) T.ridx.push_back(fromU ? R[s][a] : posOf[R[s][a]]);
      for (int a = 0; a < h; ++a)
        for (int j = 0; j < w; ++j)
          T.val.push_back(fromU ? Up[s][(size_t)j * h + a] : Lp[s][(size_t)a * w + j]);
    }
  };
  auto build_upper_panels = [&](TriHost& T, bool fromL) {
    for (int s = 0; s < ns; ++s) {
      SnHost& S = T.sn[s];
      const int w = S.w, h = S.h;
      S.ridx_off = (int64_t)T.ridx.size();
      S.panel_off = (int64_t)T.val.size();
      for (int a = 0; a < h; ++a) T.ridx.push_back(fromL ? posOf[R[s][a]] : R[s][a]);
      for (int i = 0; i < w; ++i)
        for (int a = 0; a < h; ++a)
          T.val.push_back(fromL ? Lp[s][(size_t)a * w + i] : Up[s][(size_t)i * h + a]);
    }
  };
  // team split: the groups of the supernodes and one packed factor per group,
  // each with its own level schedule (heights counted inside the group)
  out.team = team >= 1 ? team : 0;
  std::vector<int> grp;
  if (team >= 1) {
    std::vector<double> work(ns);
    for (int s = 0; s < ns; ++s) {
      const double w = sfirst[s + 1] - sfirst[s];
      work[s] = w * (w + 1) + 2.0 * w * (double)R[s].size();
    }
    std::vector<int> srows(ns);
    for (int s = 0; s < ns; ++s) srows[s] = sfirst[s + 1] - sfirst[s];
    grp = team_groups(spar, work, team, &srows, min_top_rows);
  }
  // Every group is packed over local positions: its own rows in level order,
  // then (subtree groups) the top group's rows in the top group's level order;
  // TriPacked::pos maps them back to block positions.
  auto pack_groups = [&](TriHost& T, std::vector<TriPacked>& outS) -> bool {
    outS.assign(team + 1, TriPacked());
    std::vector<int> top_rows;
    std::vector<int> loc(n, -1);
    for (int g = team; g >= 0; --g) {
      std::vector<int> hg(ns, 0);
      int nl = 0;
      std::vector<int> sf_g(1, 0);
      for (int s = 0; s < ns; ++s)
        if (grp[s] == g) {
          nl = std::max(nl, hg[s] + 1);
          if (spar[s] >= 0 && grp[spar[s]] == g) hg[spar[s]] = std::max(hg[spar[s]], hg[s] + 1);
        }
      // level schedule of the group's supernodes only
      T.nlev = nl;
      T.lev_ptr.assign(nl + 1, 0);
      T.lrows.clear();
      T.max_lrows = 0;
      std::vector<std::vector<int>> bylev(nl);
      for (int s = 0; s < ns; ++s)
        if (grp[s] == g) bylev[hg[s]].push_back(s);
      for (int l = 0; l < nl; ++l) {
        for (int s : bylev[l])
          for (int r = sfirst[s]; r < sfirst[s + 1]; ++r) {
            T.lrows.push_back(r);
            T.row_sn[r] = s;
          }
        T.lev_ptr[l + 1] = (int)T.lrows.size();
        T.max_lrows = std::max(T.max_lrows, T.lev_ptr[l + 1] - T.lev_ptr[l]);
      }
      std::vector<int> pos(T.lrows);
      if (g == team) top_rows = pos;
      else pos.insert(pos.end(), top_rows.begin(), top_rows.end());
      for (int k = 0; k < (int)pos.size(); ++k) loc[pos[k]] = k;
      const int nfull = T.n;
      T.n = (int)T.lrows.size();
      const bool ok = pack_tri(T, outS[g], narrow_width, &loc);
      T.n = nfull;
      for (int p : pos) loc[p] = -1;
      if (!ok) return false;
      outS[g].pos = std::move(pos);
    }
    return true;
  };
  {
    TriHost T;
    init_tri(T, true);
    build_lower_panels(T, false);
    for (int s = 0; s < ns; ++s) pack_inv(T, s, invL[s], false);
    build_levels(T, sfirst, height, nlev);
    if (!pack_tri(T, out.lo, narrow_width)) {
      err = "supernode wider than 32767 rows, panel taller than 32767 rows or block factor beyond 2^31 entries";
      return 3;
    }
    if (team >= 1 && !pack_groups(T, out.loS)) {
      err = "team split: packed factor beyond 2^31 entries";
      return 3;
    }
  }
  {
    TriHost T;
    init_tri(T, false);
    build_upper_panels(T, false);
    for (int s = 0; s < ns; ++s) pack_inv(T, s, invU[s], false);
    build_levels(T, sfirst, height, nlev);
    if (!pack_tri(T, out.up, narrow_width)) {
      err = "supernode wider than 32767 rows, panel taller than 32767 rows or block factor beyond 2^31 entries";
      return 3;
    }
    if (team >= 1 && !pack_groups(T, out.upS)) {
      err = "team split: packed factor beyond 2^31 entries";
      return 3;
    }
  }
  if (team >= 1) {
    out.ntop = out.loS[team].nlev > 0 ? out.loS[team].lev_ptr[out.loS[team].nlev] : 0;
    if (out.ntop <= kTopInvMaxRows && !top_inverse(out.loS[team], out.upS[team], n, out.topinv)) {
      err = "team split: the top group reaches outside itself";
      return 3;
    }
  }
  if (want_T) {
    {
      TriHost T;
      init_tri(T, true);
      build_lower_panels(T, true);
      for (int s = 0; s < ns; ++s) pack_inv(T, s, invU[s], true);
      build_levels(T, sfirst, height, nlev);
      if (!pack_tri(T, out.loT, narrow_width)) {
      err = "supernode wider than 32767 rows, panel taller than 32767 rows or block factor beyond 2^31 entries";
      return 3;
    }
    }
    {
      TriHost T;
      init_tri(T, false);
      build_upper_panels(T, true);
      for (int s = 0; s < ns; ++s) pack_inv(T, s, invL[s], true);
      build_levels(T, sfirst, height, nlev);
      if (!pack_tri(T, out.upT, narrow_width)) {
      err = "supernode wider than 32767 rows, panel taller than 32767 rows or block factor beyond 2^31 entries";
      return 3;
    }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Device layout
// ---------------------------------------------------------------------------

namespace {
// Chunks per item: enough items x chunks to cover the workgroup, each chunk
// at least ~4 entries long (measured on the 64^3 workload against 8 and 16).
int chunks_for(int64_t items, double avg_len) {
  if (items <= 0) return 1;
  int c = (int)std::min<int64_t>(255, std::max<int64_t>(1, kSolveThreads / items));
  const int by_len = std::max(1, (int)(avg_len / 4.0));
  return std::max(1, std::min(c, by_len));
}
}  // namespace

bool pack_tri(const TriHost& T, TriPacked& P, int narrow_width, const std::vector<int>* map) {
  auto M = [&](int v) { return map ? (*map)[v] : v; };
  P = TriPacked();
  P.lower = T.lower;
  P.n = T.n;
  P.nlev = T.nlev;
  P.max_lrows = T.max_lrows;
  P.lev_ptr = T.lev_ptr;
  P.push_ptr.assign(T.nlev + 1, 0);
  P.ent_ptr.assign(T.nlev + 1, 0);
  P.lev_c.assign(T.nlev, 0);
  P.rec.assign((size_t)8 * T.n, 0);
  std::vector<double> pf;
  for (int l = 0; l < T.nlev; ++l) {
    const int b = T.lev_ptr[l], e = T.lev_ptr[l + 1];
    const int cnt = e - b;
    int nsn = 0;
    for (int k = b; k < e; k += T.sn[T.row_sn[T.lrows[k]]].w) ++nsn;
    // narrow supernodes: entry form for the off-diagonal part
    const bool ent = nsn > 0 && cnt < narrow_width * nsn;
    double tri_len = 0, panel_len = 0, push_len = 0;
    int64_t npush = 0;
    for (int k = b; k < e;) {
      const int sidx = T.row_sn[T.lrows[k]];
      const SnHost& S = T.sn[sidx];
      const int w = S.w, h = S.h;
      if (w > 32767 || h > 32767) return false;
      const int32_t toff = (int32_t)P.tri.size(), poff = (int32_t)P.val.size();
      const int32_t roff = (int32_t)P.ridx.size();
      // inverted triangle entry (i, j) of the host layout (0 outside the triangle)
      auto tinv = [&](int i, int j) -> double {
        if (i >= w || j >= w || (T.lower ? j > i : j < i)) return 0.0;
        return T.lower ? T.tri[S.tri_off + (int64_t)i * (i + 1) / 2 + j]
                       : T.tri[S.tri_off + (int64_t)i * w - (int64_t)i * (i - 1) / 2 + (j - i)];
      };
      // inverted triangle, column pairs (2c, 2c+1) interleaved: lower pair c
      // holds rows 2c..w-1, upper pair c rows 0..2c+1 (zeros outside the triangle)
      for (int c = 0; c < (w + 1) / 2; ++c) {
        const int i0 = T.lower ? 2 * c : 0, i1 = T.lower ? w - 1 : 2 * c + 1;
        for (int i = i0; i <= i1; ++i) {
          P.tri.push_back(tinv(i, 2 * c));
          P.tri.push_back(tinv(i, 2 * c + 1));
        }
      }
      // folded panels: the panel times the inverted triangle, so that a level's
      // off-diagonal products read the rows' values from before the level's
      // solve.  Lower: Pf(a, j) = sum_l Lp(a, l) Tinv(l, j) (h x w, the pushes
      // x[ridx[a]] -= Pf(a, :) x[f .. f+w-1]); upper: Pf(i, a) = sum_l
      // Tinv(i, l) Up(l, a) (w x h, x[f + i] = Tinv(i, :) x[f ..] - Pf(i, :) x[ridx]).
      pf.assign((size_t)w * h, 0.0);
      if (T.lower) {
        for (int q = 0; q < h; ++q) {
          const double* lp = &T.val[S.panel_off + (int64_t)q * w];
          for (int l = 0; l < w; ++l)
            if (lp[l] != 0.0)
              for (int j = 0; j <= l; ++j) pf[(size_t)q * w + j] += lp[l] * tinv(l, j);
        }
      } else {
        for (int i = 0; i < w; ++i)
          for (int l = i; l < w; ++l) {
            const double t = tinv(i, l);
            if (t == 0.0) continue;
            const double* up = &T.val[S.panel_off + (int64_t)l * h];
            for (int q = 0; q < h; ++q) pf[(size_t)i * h + q] += t * up[q];
          }
      }
      if (ent) {
        // entry form (kept besides the panels; the solve picks one), targets
        // and sources as positions: lower (a, j) -> x[ridx[a]] -= v x[f + j];
        // upper (i, a) -> x[f + i] -= v x[ridx[a]]
        if (T.lower) {
          for (int j = 0; j < w; ++j)
            for (int q = 0; q < h; ++q) {
              P.eval.push_back(pf[(size_t)q * w + j]);
              P.eidx.push_back(M(T.ridx[S.ridx_off + q]));
              P.eloc.push_back(M(S.f + j));
            }
        } else {
          for (int q = 0; q < h; ++q)
            for (int i = 0; i < w; ++i) {
              P.eval.push_back(pf[(size_t)i * h + q]);
              P.eidx.push_back(M(T.ridx[S.ridx_off + q]));
              P.eloc.push_back(M(S.f + i));
            }
        }
      }
      {
        // panel, column pairs interleaved: lower (a, 2c + t) at 2(c h + a) + t,
        // upper (i, 2c + t) at 2(c w + i) + t; an odd last column pairs with zeros
        if (T.lower) {
          for (int c = 0; c < (w + 1) / 2; ++c)
            for (int q = 0; q < h; ++q)
              for (int t = 0; t < 2; ++t)
                P.val.push_back(2 * c + t < w ? pf[(size_t)q * w + 2 * c + t] : 0.0);
        } else {
          for (int c = 0; c < (h + 1) / 2; ++c)
            for (int i = 0; i < w; ++i)
              for (int t = 0; t < 2; ++t)
                P.val.push_back(2 * c + t < h ? pf[(size_t)i * h + 2 * c + t] : 0.0);
        }
        // position list padded to even length with its last position (paired with zeros)
        for (int q = 0; q < h; ++q) P.ridx.push_back(M(T.ridx[S.ridx_off + q]));
        if (h & 1) P.ridx.push_back(M(T.ridx[S.ridx_off + h - 1]));
        if (T.lower) {
          for (int q = 0; q < h; ++q) {
            P.prec.push_back(M(T.ridx[S.ridx_off + q]));
            P.prec.push_back(poff / 2 + q);
            P.prec.push_back(w | (h << 16));
            P.prec.push_back(M(S.f));
          }
          npush += h;
          push_len += (double)h * w;
        }
      }
      for (int i = 0; i < w; ++i) {
        int32_t* r = &P.rec[(size_t)8 * (k + i)];
        r[0] = M(S.f + i);
        r[1] = i;
        r[2] = w;
        r[3] = h;
        r[4] = toff;
        r[5] = poff;
        r[6] = roff;
        r[7] = k - b;
        tri_len += T.lower ? i + 1 : w - i;
        panel_len += T.lower ? 0 : h;
      }
      k += w;
    }
    P.push_ptr[l + 1] = P.push_ptr[l] + (int32_t)npush;
    const int64_t nent = (int64_t)P.eval.size() - P.ent_ptr[l];
    P.ent_ptr[l + 1] = (int32_t)P.eval.size();
    {
      // what each path reads at this level besides triangles and row records
      int64_t pv = 0, pi = 0;
      for (int k = b; k < e;) {
        const SnHost& S = T.sn[T.row_sn[T.lrows[k]]];
        pv += (int64_t)S.w * S.h;
        pi += T.lower ? 4 * (int64_t)S.h : S.h;  // push records / position list
        k += S.w;
      }
      P.read_vals[1] += pv;
      P.read_ints[1] += pi;
      P.read_vals[0] += ent ? nent : pv;
      P.read_ints[0] += ent ? 2 * nent : pi;
    }
    const int ct = chunks_for(cnt, cnt ? tri_len / cnt : 0.0);
    const int cp = T.lower ? chunks_for(npush, npush ? push_len / npush : 0.0)
                           : chunks_for(cnt, cnt ? panel_len / cnt : 0.0);
    P.lev_c[l] = ct | (cp << 8) | ((ent ? 1 : 0) << 16);
  }
  // triangle entries without the pair padding, of the supernodes scheduled
  // here (a team group packs a subset of the block's supernodes)
  int64_t tri_vals = 0;
  for (int l = 0; l < T.nlev; ++l)
    for (int k = T.lev_ptr[l]; k < T.lev_ptr[l + 1];) {
      const SnHost& S = T.sn[T.row_sn[T.lrows[k]]];
      tri_vals += (int64_t)S.w * (S.w + 1) / 2;
      k += S.w;
    }
  for (int q = 0; q < 2; ++q) {
    P.read_vals[q] += tri_vals;
    P.read_ints[q] += (int64_t)P.rec.size() + 4 * (int64_t)(T.nlev + 1);
  }
  // record fields are int32 offsets into the block's arrays, and the device
  // addresses a block's values with 32-bit byte offsets (FP64: below 2^29 values)
  return P.val.size() < ((size_t)1 << 29) && P.tri.size() < ((size_t)1 << 29) &&
         P.ridx.size() < (size_t)INT32_MAX && P.eval.size() < (size_t)INT32_MAX;
}

// ---------------------------------------------------------------------------
// Host execution of a packed factor (diagnostics): the device algorithm in
// sequential order
// ---------------------------------------------------------------------------

namespace {
// pair index of triangle entry (i, j) in the column-pair layouts of pack_tri
int64_t tri_pair_lower(int i, int j, int w) {
  const int64_t c = j >> 1;
  return c * (w - c + 1) + (i - 2 * c);
}
int64_t tri_pair_upper(int i, int j) {
  const int64_t c = j >> 1;
  return c * (c + 1) + i;
}
}  // namespace

void host_tri_solve(const TriPacked& T, std::vector<double>& X, bool entries) {
  std::vector<double> Rb(std::max(T.max_lrows, 1));
  for (int li = 0; li < T.nlev; ++li) {
    const int l = T.lower ? li : T.nlev - 1 - li;
    const int b = T.lev_ptr[l], e = T.lev_ptr[l + 1];
    const bool ent = entries && ((T.lev_c[l] >> 16) & 1);
    if (T.lower) {
      // the level's new values from its rows' old ones, then the pushes (also
      // from the old ones), then the new values
      for (int k = b; k < e; ++k) {
        const int32_t* r = &T.rec[(size_t)8 * k];
        const int p = r[0], i = r[1], w = r[2];
        double acc = 0.0;
        for (int j = 0; j <= i; ++j)
          acc += T.tri[r[4] + 2 * tri_pair_lower(i, j, w) + (j & 1)] * X[p - i + j];
        Rb[k - b] = acc;
      }
      if (ent) {
        for (int q = T.ent_ptr[l]; q < T.ent_ptr[l + 1]; ++q) X[T.eidx[q]] -= T.eval[q] * X[T.eloc[q]];
      } else {
        for (int m = T.push_ptr[l]; m < T.push_ptr[l + 1]; ++m) {
          const int32_t* q = &T.prec[(size_t)4 * m];
          const int w = q[2] & 0xffff, h = q[2] >> 16;
          double acc = 0.0;
          for (int j = 0; j < w; ++j) acc += T.val[2 * (q[1] + (int64_t)(j >> 1) * h) + (j & 1)] * X[q[3] + j];
          X[q[0]] -= acc;
        }
      }
      for (int k = b; k < e; ++k) X[T.rec[(size_t)8 * k]] = Rb[k - b];
    } else {
      for (int k = b; k < e; ++k) Rb[k - b] = X[T.rec[(size_t)8 * k]];
      for (int k = b; k < e; ++k) {
        const int32_t* r = &T.rec[(size_t)8 * k];
        const int p = r[0], i = r[1], w = r[2], h = ent ? 0 : r[3];
        double acc = 0.0;
        for (int j = i; j < w; ++j) acc += T.tri[r[4] + 2 * tri_pair_upper(i, j) + (j & 1)] * Rb[r[7] + j];
        for (int a = 0; a < h; ++a)
          acc -= T.val[r[5] + 2 * ((int64_t)(a >> 1) * w + i) + (a & 1)] * X[T.ridx[r[6] + a]];
        X[p] = acc;
      }
      if (ent)
        for (int q = T.ent_ptr[l]; q < T.ent_ptr[l + 1]; ++q) X[T.eloc[q]] -= T.eval[q] * X[T.eidx[q]];
    }
  }
}

void host_tri_solve_pos(const TriPacked& T, std::vector<double>& X, bool entries) {
  if (T.pos.empty()) {
    host_tri_solve(T, X, entries);
    return;
  }
  std::vector<double> Y(T.pos.size());
  for (size_t k = 0; k < T.pos.size(); ++k) Y[k] = X[T.pos[k]];
  host_tri_solve(T, Y, entries);
  for (size_t k = 0; k < T.pos.size(); ++k) X[T.pos[k]] = Y[k];
}

// Dense inverse of the top group's diagonal block of L U (see BlockFactor::
// topinv): the packed top-group solves of host_tri_solve applied to all ntop
// unit vectors at once, every scalar operation of the sequential algorithm
// becoming an operation on a row of ntop right-hand sides.
bool top_inverse(const TriPacked& lo, const TriPacked& up, int n, std::vector<double>& M) {
  const int nt = lo.nlev > 0 ? lo.lev_ptr[lo.nlev] : 0;
  M.clear();
  if (nt == 0) return true;
  std::vector<int> loc(n, -1);
  for (int k = 0; k < nt; ++k) loc[lo.rec[(size_t)8 * k]] = k;
  std::vector<double> X((size_t)nt * nt, 0.0);
  for (int k = 0; k < nt; ++k) X[(size_t)k * nt + k] = 1.0;
  const int mr = std::max(std::max(lo.max_lrows, up.max_lrows), 1);
  std::vector<double> Rb((size_t)mr * nt);
  std::vector<double> acc(nt);
  auto row = [&](int p) -> double* {
    const int k = p >= 0 && p < n ? loc[p] : -1;
    return k < 0 ? nullptr : &X[(size_t)k * nt];
  };
  auto axpy = [&](double* y, double a, const double* x) {
    if (a != 0.0)
      for (int c = 0; c < nt; ++c) y[c] += a * x[c];
  };
  for (int li = 0; li < lo.nlev; ++li) {
    const int b = lo.lev_ptr[li], e = lo.lev_ptr[li + 1];
    for (int k = b; k < e; ++k) {
      const int32_t* r = &lo.rec[(size_t)8 * k];
      const int p = r[0], i = r[1], w = r[2];
      std::fill(acc.begin(), acc.end(), 0.0);
      for (int j = 0; j <= i; ++j) {
        const double* xj = row(p - i + j);
        if (!xj) return false;
        axpy(acc.data(), lo.tri[r[4] + 2 * tri_pair_lower(i, j, w) + (j & 1)], xj);
      }
      std::copy(acc.begin(), acc.end(), &Rb[(size_t)(k - b) * nt]);
    }
    for (int m = lo.push_ptr[li]; m < lo.push_ptr[li + 1]; ++m) {
      const int32_t* q = &lo.prec[(size_t)4 * m];
      const int w = q[2] & 0xffff, h = q[2] >> 16;
      double* xd = row(q[0]);
      if (!xd) return false;
      for (int j = 0; j < w; ++j) {
        const double* xs = row(q[3] + j);
        if (!xs) return false;
        axpy(xd, -lo.val[2 * (q[1] + (int64_t)(j >> 1) * h) + (j & 1)], xs);
      }
    }
    for (int k = b; k < e; ++k) std::copy(&Rb[(size_t)(k - b) * nt], &Rb[(size_t)(k - b + 1) * nt],
                                          row(lo.rec[(size_t)8 * k]));
  }
  for (int li = 0; li < up.nlev; ++li) {
    const int l = up.nlev - 1 - li;
    const int b = up.lev_ptr[l], e = up.lev_ptr[l + 1];
    for (int k = b; k < e; ++k) {
      const double* xp = row(up.rec[(size_t)8 * k]);
      if (!xp) return false;
      std::copy(xp, xp + nt, &Rb[(size_t)(k - b) * nt]);
    }
    for (int k = b; k < e; ++k) {
      const int32_t* r = &up.rec[(size_t)8 * k];
      const int i = r[1], w = r[2], h = r[3];
      std::fill(acc.begin(), acc.end(), 0.0);
      for (int j = i; j < w; ++j)
        axpy(acc.data(), up.tri[r[4] + 2 * tri_pair_upper(i, j) + (j & 1)], &Rb[(size_t)(r[7] + j) * nt]);
      for (int a = 0; a < h; ++a) {
        const double* xa = row(up.ridx[r[6] + a]);
        if (!xa) return false;
        axpy(acc.data(), -up.val[r[5] + 2 * ((int64_t)(a >> 1) * w + i) + (a & 1)], xa);
      }
      std::copy(acc.begin(), acc.end(), row(r[0]));
    }
  }
  // column pairs: (r, j) at 2 ((j / 2) ld + r) + (j % 2) with ld = top_ld(nt);
  // an odd last column and the rows past nt are zeros
  const int np = (nt + 1) / 2, ld = top_ld(nt);
  M.assign((size_t)2 * np * ld, 0.0);
  for (int r = 0; r < nt; ++r)
    for (int j = 0; j < nt; ++j) M[2 * ((size_t)(j >> 1) * ld + r) + (j & 1)] = X[(size_t)r * nt + j];
  return true;
}

// ---------------------------------------------------------------------------
// Threshold incomplete LU (the local factors of Algorithm 4)
// ---------------------------------------------------------------------------

namespace {

// A sparse triangular factor as supernodes of one row each: position i has
// the inverted diagonal dinv[i] and the off-diagonal entries off[i] (lower:
// column i below the diagonal as (row, value); upper: row i right of the
// diagonal as (column, value)), in the TriHost layout that pack_tri reads.
// Levels come from the dependency graph: a lower row sits one level above the
// highest column it takes an update from; an upper row is solved after every
// row it reads (levels run top down for upper factors).
TriHost sparse_tri(bool lower, int n, const std::vector<double>& dinv, const SparseList& off) {
  TriHost T;
  T.lower = lower;
  T.n = n;
  T.sn.resize(n);
  std::vector<int> height(n, 0), sfirst(n + 1);
  for (int i = 0; i <= n; ++i) sfirst[i] = i;
  int nlev = n > 0 ? 1 : 0;
  if (lower) {
    for (int k = 0; k < n; ++k)
      for (const auto& e : off[k]) height[e.first] = std::max(height[e.first], height[k] + 1);
    for (int i = 0; i < n; ++i) nlev = std::max(nlev, height[i] + 1);
  } else {
    std::vector<int> d(n, 0);
    int dmax = 0;
    for (int i = n - 1; i >= 0; --i) {
      for (const auto& e : off[i]) d[i] = std::max(d[i], d[e.first] + 1);
      dmax = std::max(dmax, d[i]);
    }
    nlev = n > 0 ? dmax + 1 : 0;
    for (int i = 0; i < n; ++i) height[i] = dmax - d[i];
  }
  for (int i = 0; i < n; ++i) {
    SnHost& S = T.sn[i];
    S.f = i;
    S.w = 1;
    S.h = (int)off[i].size();
    S.pad = 0;
    S.tri_off = (int64_t)T.tri.size();
    T.tri.push_back(dinv[i]);
    S.ridx_off = (int64_t)T.ridx.size();
    S.panel_off = (int64_t)T.val.size();
    for (const auto& e : off[i]) {
      T.ridx.push_back(e.first);
      T.val.push_back(e.second);
    }
  }
  build_levels(T, sfirst, height, nlev);
  return T;
}

}  // namespace

int ilut_factor(const CsrL& M, double drop, IlutFactors& F, std::string& err) {
  const int n = M.nrows;
  F.L.assign(n, {});
  F.U.assign(n, {});
  F.d.assign(n, 0.0);
  std::vector<double> w(n, 0.0);
  std::vector<int> seen(n, -1);
  std::vector<int> touched;
  std::vector<int> heap;  // L-part positions of the work row, smallest first
  for (int i = 0; i < n; ++i) {
    touched.clear();
    heap.clear();
    double nrm1 = 0.0;
    for (int q = M.ptr[i]; q < M.ptr[i + 1]; ++q) {
      const int j = M.col[q];
      w[j] = M.val[q];
      seen[j] = i;
      touched.push_back(j);
      if (j < i) heap.push_back(j);
      nrm1 += std::fabs(M.val[q]);
    }
    // dropping threshold of row i: drop times the mean modulus of its entries
    const int len = M.ptr[i + 1] - M.ptr[i];
    const double ti = len > 0 ? drop * (nrm1 / len) : 0.0;
    std::make_heap(heap.begin(), heap.end(), std::greater<int>());
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), std::greater<int>());
      const int k = heap.back();
      heap.pop_back();
      const double wk = w[k] / F.d[k];
      w[k] = 0.0;
      if (std::fabs(wk) < ti) continue;  // dropped: no update from row k
      F.L[i].push_back({k, wk});
      for (const auto& e : F.U[k]) {
        const int j = e.first;
        if (seen[j] != i) {
          seen[j] = i;
          w[j] = 0.0;
          touched.push_back(j);
          if (j < i) {
            heap.push_back(j);
            std::push_heap(heap.begin(), heap.end(), std::greater<int>());
          }
        }
        w[j] = w[j] - wk * e.second;
      }
    }
    if (seen[i] != i || w[i] == 0.0) {
      err = "zero pivot in the incomplete factorisation at row " + std::to_string(i);
      return 2;
    }
    F.d[i] = w[i];
    std::sort(touched.begin(), touched.end());
    for (int j : touched) {
      if (j > i && std::fabs(w[j]) >= ti) F.U[i].push_back({j, w[j]});
      w[j] = 0.0;
    }
    std::sort(F.L[i].begin(), F.L[i].end());
  }
  return 0;
}

int ilut_block(const CsrL& M, double drop, bool want_T, int narrow_width, BlockFactor& out,
               std::string& err) {
  const int n = M.nrows;
  out = BlockFactor();
  out.n = n;
  out.gin.resize(n);
  out.gout.resize(n);
  for (int i = 0; i < n; ++i) out.gin[i] = out.gout[i] = i;
  IlutFactors F;
  if (int rc = ilut_factor(M, drop, F, err)) return rc;
  const SparseList& Lrow = F.L;
  const SparseList& Urow = F.U;
  const std::vector<double>& Ud = F.d;
  // L by columns (lower solves push columns), U by rows (upper solves pull rows)
  SparseList Lcol(n);
  for (int i = 0; i < n; ++i)
    for (const auto& e : Lrow[i]) Lcol[e.first].push_back({i, e.second});
  std::vector<double> one(n, 1.0), uinv(n);
  for (int i = 0; i < n; ++i) uinv[i] = 1.0 / Ud[i];
  for (int i = 0; i < n; ++i) {
    out.nnz_L += (int64_t)Lrow[i].size();
    out.nnz_U += 1 + (int64_t)Urow[i].size();
  }
  out.nsuper = n;
  const char* wide = "block factor beyond 2^31 entries";
  if (!pack_tri(sparse_tri(true, n, one, Lcol), out.lo, narrow_width) ||
      !pack_tri(sparse_tri(false, n, uinv, Urow), out.up, narrow_width)) {
    err = wide;
    return 3;
  }
  if (want_T) {
    // M^T = U^T L^T: U^T is lower with the rows of U as its columns, L^T upper
    // with the columns of L as its rows
    if (!pack_tri(sparse_tri(true, n, uinv, Urow), out.loT, narrow_width) ||
        !pack_tri(sparse_tri(false, n, one, Lcol), out.upT, narrow_width)) {
      err = wide;
      return 3;
    }
  }
  return 0;
}

bool check_levels(const TriPacked& T, std::string& err) {
  if (T.n == 0) return true;
  // level of every position
  std::vector<int> lev(T.n, -1);
  for (int l = 0; l < T.nlev; ++l)
    for (int k = T.lev_ptr[l]; k < T.lev_ptr[l + 1]; ++k) {
      const int p = T.rec[(size_t)8 * k];
      if (p < 0 || p >= T.n || lev[p] >= 0) {
        err = "a position is missing or scheduled twice";
        return false;
      }
      lev[p] = l;
    }
  for (int p = 0; p < T.n; ++p)
    if (lev[p] < 0) {
      err = "a position is not scheduled";
      return false;
    }
  for (int l = 0; l < T.nlev; ++l) {
    // a supernode's rows share its level; every off-diagonal dependency is
    // solved strictly before: lower updates go to later levels, upper rows
    // read rows of later levels (solved first, the upper sweep runs top down)
    for (int k = T.lev_ptr[l]; k < T.lev_ptr[l + 1]; ++k) {
      const int32_t* r = &T.rec[(size_t)8 * k];
      const int first = r[0] - r[1];
      for (int j = 0; j < r[2]; ++j)
        if (lev[first + j] != l) {
          err = "a supernode spans two levels";
          return false;
        }
      if (!T.lower)
        for (int a = 0; a < r[3]; ++a)
          if (lev[T.ridx[r[6] + a]] <= l) {
            err = "an upper row reads a row that is not solved before it";
            return false;
          }
    }
    if (T.lower)
      for (int m = T.push_ptr[l]; m < T.push_ptr[l + 1]; ++m) {
        const int32_t* q = &T.prec[(size_t)4 * m];
        if (lev[q[0]] <= l) {
          err = "a lower update targets a row that is not solved after it";
          return false;
        }
        const int f = q[3], w = q[2] & 0xffff;
        if (f < 0 || f + w > T.n || lev[f] != l || lev[f + w - 1] != l) {
          err = "a lower update reads rows outside its level";
          return false;
        }
      }
    for (int q = T.ent_ptr[l]; q < T.ent_ptr[l + 1]; ++q) {
      if (lev[T.eidx[q]] <= l) {
        err = "an entry-form dependency is not across levels";
        return false;
      }
      if (T.eloc[q] < 0 || T.eloc[q] >= T.n || lev[T.eloc[q]] != l) {
        err = "an entry-form row is outside its level";
        return false;
      }
    }
  }
  return true;
}

// Team split check: the groups cover every position once; in group g the
// lower solve pushes only into its own later levels or the top group, the
// upper solve reads only its own later-solved rows or the top group (g <
// team); the top group's solves stay inside the top group.
bool check_team(const BlockFactor& F, std::string& err) {
  const int team = F.team;
  if (team < 1) return true;
  if ((int)F.loS.size() != team + 1 || (int)F.upS.size() != team + 1) {
    err = "team packing missing";
    return false;
  }
  const int n = F.n;
  for (int g = 0; g <= team; ++g)
    if (F.loS[g].pos != F.upS[g].pos) {
      err = "a team group's lower and upper packings number its rows differently";
      return false;
    }
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<TriPacked>& G = pass == 0 ? F.loS : F.upS;
    std::vector<int> grp(n, -1), lev(n, -1);
    // block position of local position p of group g (-1: out of range)
    auto bp = [&](int g, int p) {
      const TriPacked& T = G[g];
      if (T.pos.empty()) return p >= 0 && p < n ? p : -1;
      return p >= 0 && p < (int)T.pos.size() ? (int)T.pos[p] : -1;
    };
    for (int g = 0; g <= team; ++g) {
      const TriPacked& T = G[g];
      for (int l = 0; l < T.nlev; ++l)
        for (int k = T.lev_ptr[l]; k < T.lev_ptr[l + 1]; ++k) {
          const int p = bp(g, T.rec[(size_t)8 * k]);
          if (p < 0 || p >= n || grp[p] >= 0) {
            err = "a position is scheduled twice or out of range";
            return false;
          }
          grp[p] = g;
          lev[p] = l;
        }
    }
    for (int p = 0; p < n; ++p)
      if (grp[p] < 0) {
        err = "a position is in no group";
        return false;
      }
    for (int g = 0; g <= team; ++g) {
      const TriPacked& T = G[g];
      auto ok_dep = [&](int ql, int l) {
        const int q = bp(g, ql);
        if (q < 0) return false;
        if (grp[q] == g) return lev[q] > l;   // solved later (lower) / earlier in the upper sweep
        return g < team && grp[q] == team;    // a subtree may reach the top group
      };
      for (int l = 0; l < T.nlev; ++l) {
        for (int k = T.lev_ptr[l]; k < T.lev_ptr[l + 1]; ++k) {
          const int32_t* r = &T.rec[(size_t)8 * k];
          const int h = r[3], roff = r[6];
          for (int a = 0; a < h; ++a)
            if (!ok_dep(T.ridx[roff + a], l)) {
              err = "a team group depends on a row outside its reach";
              return false;
            }
        }
        for (int q = T.ent_ptr[l]; q < T.ent_ptr[l + 1]; ++q)
          if (!ok_dep(T.eidx[q], l)) {
            err = "a team group's entry form reaches outside its reach";
            return false;
          }
      }
    }
  }
  return true;
}

}  // namespace pslr
