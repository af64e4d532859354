// Small dense eigen-problems of the deflated low-rank setup (host, FP64).
//
// The Krylov-Schur restart of the low-rank correction needs, for the small
// projected matrix H_m of E_rr(m) = (E_s C0^{-1})^{m+1} (Thm. t2, eq. schur),
// an orthonormal basis of its invariant subspace for the Ritz values of
// largest modulus.  Here: Householder reduction to Hessenberg form, the
// complex single-shift QR algorithm with Wilkinson shifts (Francis; Golub and
// Van Loan, Matrix Computations, Sec. 7.5) giving H_m = Z T Z^H with T upper
// triangular, adjacent swaps of T's diagonal (each by the unitary 2 x 2
// similarity whose first column is the eigenvector of the swapped pair) to
// bring the selected eigenvalues first, and a real orthonormal basis of the
// selected subspace (closed under conjugation) from the real and imaginary
// parts of the leading Schur vectors by column-pivoted Gram-Schmidt.
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "pslr_host.h"

namespace pslr {

namespace {

using cd = std::complex<double>;

// column-major n x n accessor
struct CMat {
  int n;
  std::vector<cd> a;
  explicit CMat(int n_) : n(n_), a((size_t)n_ * n_, cd(0.0, 0.0)) {}
  cd& operator()(int i, int j) { return a[(size_t)j * n + i]; }
  const cd& operator()(int i, int j) const { return a[(size_t)j * n + i]; }
};

// rows (p, p+1) <- U^H rows, columns from c0 on
void rows_apply(CMat& T, int p, const cd U[2][2], int c0) {
  for (int j = c0; j < T.n; ++j) {
    const cd x = T(p, j), y = T(p + 1, j);
    T(p, j) = std::conj(U[0][0]) * x + std::conj(U[1][0]) * y;
    T(p + 1, j) = std::conj(U[0][1]) * x + std::conj(U[1][1]) * y;
  }
}

// columns (p, p+1) <- columns U, rows 0 .. r1-1
void cols_apply(CMat& T, int p, const cd U[2][2], int r1) {
  for (int i = 0; i < r1; ++i) {
    const cd x = T(i, p), y = T(i, p + 1);
    T(i, p) = x * U[0][0] + y * U[1][0];
    T(i, p + 1) = x * U[0][1] + y * U[1][1];
  }
}

// Unitary U with first column (x, y) / ||(x, y)||:  U = [[x, -conj(y)], [y, conj(x)]] / r.
// Then U^H (x, y)^T = (r, 0)^T.  Returns false when x = y = 0.
bool unit_first_column(cd x, cd y, cd U[2][2]) {
  const double r = std::sqrt(std::norm(x) + std::norm(y));
  if (!(r > 0.0)) return false;
  U[0][0] = x / r;
  U[1][0] = y / r;
  U[0][1] = -std::conj(y) / r;
  U[1][1] = std::conj(x) / r;
  return true;
}

// Householder reduction of a real matrix (column-major, n x n) to upper
// Hessenberg form H = Q^T A Q; returns H and Q as complex matrices.
void hessenberg(int n, const double* A, int64_t lda, CMat& H, CMat& Q) {
  std::vector<double> M((size_t)n * n), Qr((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) M[(size_t)j * n + i] = A[(size_t)j * lda + i];
  for (int i = 0; i < n; ++i) Qr[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += M[(size_t)k * n + i] * M[(size_t)k * n + i];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    const double x0 = M[(size_t)k * n + k + 1];
    const double beta = x0 >= 0 ? -alpha : alpha;  // new subdiagonal entry
    std::fill(v.begin(), v.end(), 0.0);
    v[k + 1] = x0 - beta;
    for (int i = k + 2; i < n; ++i) v[i] = M[(size_t)k * n + i];
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    // M <- (I - tau v v^T) M (I - tau v v^T); Q <- Q (I - tau v v^T)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * M[(size_t)j * n + i];
      s *= tau;
      for (int i = k + 1; i < n; ++i) M[(size_t)j * n + i] -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += M[(size_t)j * n + i] * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) M[(size_t)j * n + i] -= s * v[j];
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += Qr[(size_t)j * n + i] * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) Qr[(size_t)j * n + i] -= s * v[j];
    }
    M[(size_t)k * n + k + 1] = beta;
    for (int i = k + 2; i < n; ++i) M[(size_t)k * n + i] = 0.0;
  }
  for (size_t e = 0; e < M.size(); ++e) {
    H.a[e] = cd(M[e], 0.0);
    Q.a[e] = cd(Qr[e], 0.0);
  }
}

// Complex Schur form of the Hessenberg matrix T in place (T <- Z^H T Z,
// upper triangular), accumulating the unitary transformations into Z.
bool complex_qr(CMat& T, CMat& Z, std::string& err) {
  const int n = T.n;
  const double eps = 2.220446049250313e-16;
  double nrm = 0.0;
  for (const cd& x : T.a) nrm = std::max(nrm, std::abs(x));
  if (nrm == 0.0) return true;
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      double s = std::abs(T(lo, lo)) + std::abs(T(lo - 1, lo - 1));
      if (s == 0.0) s = nrm;
      if (std::abs(T(lo, lo - 1)) <= eps * s) {
        T(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {  // a converged eigenvalue at the bottom of the active block
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 60 * n) {
      err = "complex QR iteration did not converge";
      return false;
    }
    ++iter;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closer to T(hi, hi);
    // an exceptional shift every tenth iteration without deflation
    cd mu;
    if (iter % 10 == 0) {
      mu = T(hi, hi) + 0.75 * std::abs(T(hi, hi - 1));
    } else {
      const cd a = T(hi - 1, hi - 1), b = T(hi - 1, hi), c = T(hi, hi - 1), d = T(hi, hi);
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    // implicit single-shift QR step on rows/columns lo..hi (bulge chase)
    cd x = T(lo, lo) - mu, y = T(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      cd U[2][2];
      if (!unit_first_column(x, y, U)) {
        U[0][0] = U[1][1] = 1.0;
        U[0][1] = U[1][0] = 0.0;
      }
      rows_apply(T, k, U, k > lo ? k - 1 : lo);
      cols_apply(T, k, U, std::min(k + 2, hi) + 1);
      cols_apply(Z, k, U, n);
      if (k > lo) T(k + 1, k - 1) = 0.0;
      if (k + 1 < hi) {
        x = T(k + 1, k);
        y = T(k + 2, k);
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) T(i, j) = 0.0;
  return true;
}

// Swap the adjacent diagonal entries i, i+1 of the upper triangular T.
void swap_diag(CMat& T, CMat& Z, int i) {
  const cd a = T(i, i), b = T(i + 1, i + 1), t = T(i, i + 1);
  cd U[2][2];
  // eigenvector of [[a, t], [0, b]] for b: (t, b - a)
  if (!unit_first_column(t, b - a, U)) return;  // a == b and t == 0: nothing to swap
  rows_apply(T, i, U, i);
  cols_apply(T, i, U, i + 2);
  cols_apply(Z, i, U, T.n);
  T(i + 1, i) = 0.0;
  T(i, i) = b;
  T(i + 1, i + 1) = a;
}

}  // namespace

int schur_select(int n, const double* Hm, int64_t ldh, int k, std::vector<double>& W,
                 std::vector<double>& Hk, std::vector<double>& ritz_re, std::vector<double>& ritz_im,
                 std::string& err) {
  W.clear();
  Hk.clear();
  ritz_re.assign(n, 0.0);
  ritz_im.assign(n, 0.0);
  if (n <= 0 || k <= 0) return 0;
  k = std::min(k, n);
  CMat T(n), Z(n);
  hessenberg(n, Hm, ldh, T, Z);
  if (!complex_qr(T, Z, err)) return -1;
  std::vector<cd> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = T(i, i);
  // Ritz values by decreasing modulus
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return std::abs(ev[a]) > std::abs(ev[b]); });
  for (int r = 0; r < n; ++r) {
    ritz_re[r] = ev[order[r]].real();
    ritz_im[r] = ev[order[r]].imag();
  }
  // keep the k of largest modulus, minus one when the k-th is a complex value
  // whose conjugate is the (k+1)-th (the cut would split the pair); then every
  // value whose modulus ties the last kept one (within a relative 1e-10), so
  // that the kept set is a well-defined invariant subspace
  double scale = 0.0;
  for (const cd& e : ev) scale = std::max(scale, std::abs(e));
  int kk = k;
  if (kk < n) {
    const cd a = ev[order[kk - 1]], b = ev[order[kk]];
    if (std::abs(a.imag()) > 1e-10 * std::max(scale, 1e-300) &&
        std::abs(a - std::conj(b)) <= 1e-8 * std::max(1.0, std::abs(a)))
      --kk;
  }
  std::vector<char> sel(n, 0);
  if (kk > 0) {
    const double cut = std::abs(ev[order[kk - 1]]) * (1.0 - 1e-10);
    for (int r = 0; r < n; ++r)
      if (r < kk || std::abs(ev[order[r]]) >= cut) sel[order[r]] = 1;
  }
  // a kept complex value whose conjugate partner (the nearest eigenvalue to
  // its conjugate) is not kept cannot be part of a real invariant subspace
  for (int r = n - 1; r >= 0; --r) {
    const int i = order[r];
    if (!sel[i] || std::abs(ev[i].imag()) <= 1e-10 * std::max(scale, 1e-300)) continue;
    int partner = -1;
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double d = std::abs(ev[j] - std::conj(ev[i]));
      if (partner < 0 || d < best) {
        partner = j;
        best = d;
      }
    }
    if (partner >= 0 && !sel[partner]) sel[i] = 0;
  }
  int kept = 0;
  for (int i = 0; i < n; ++i) kept += sel[i];
  if (kept == 0) return 0;
  // bring the selected eigenvalues to the leading positions
  int front = 0;
  for (int i = 0; i < n; ++i) {
    if (!sel[i]) continue;
    for (int p = i; p > front; --p) {
      swap_diag(T, Z, p - 1);
      std::swap(sel[p - 1], sel[p]);
    }
    ++front;
  }
  // real orthonormal basis of span(Z[:, :kept]) (closed under conjugation):
  // column-pivoted Gram-Schmidt (two passes) on [Re Z_k, Im Z_k]
  const int nc = 2 * kept;
  std::vector<double> M((size_t)n * nc);
  for (int j = 0; j < kept; ++j)
    for (int i = 0; i < n; ++i) {
      M[(size_t)j * n + i] = Z(i, j).real();
      M[(size_t)(kept + j) * n + i] = Z(i, j).imag();
    }
  std::vector<double> norm0(nc);
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += M[(size_t)c * n + i] * M[(size_t)c * n + i];
    norm0[c] = std::sqrt(s);
  }
  std::vector<char> used(nc, 0);
  W.assign((size_t)n * kept, 0.0);
  for (int j = 0; j < kept; ++j) {
    int piv = -1;
    double best = -1.0;
    for (int c = 0; c < nc; ++c) {
      if (used[c]) continue;
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += M[(size_t)c * n + i] * M[(size_t)c * n + i];
      if (s > best) {
        best = s;
        piv = c;
      }
    }
    if (piv < 0 || !(best > 1e-24)) {
      err = "selected Schur subspace is rank deficient";
      return -1;
    }
    used[piv] = 1;
    double* w = &W[(size_t)j * n];
    for (int i = 0; i < n; ++i) w[i] = M[(size_t)piv * n + i];
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l < j; ++l) {
        const double* u = &W[(size_t)l * n];
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += u[i] * w[i];
        for (int i = 0; i < n; ++i) w[i] -= d * u[i];
      }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += w[i] * w[i];
    s = std::sqrt(s);
    if (!(s > 0.0)) {
      err = "selected Schur subspace is rank deficient";
      return -1;
    }
    for (int i = 0; i < n; ++i) w[i] /= s;
    // remove the new direction from the remaining candidates
    for (int c = 0; c < nc; ++c) {
      if (used[c]) continue;
      double* mc = &M[(size_t)c * n];
      double d = 0.0;
      for (int i = 0; i < n; ++i) d += w[i] * mc[i];
      for (int i = 0; i < n; ++i) mc[i] -= d * w[i];
    }
  }
  // the candidates left over lie in the span (conjugation closure)
  for (int c = 0; c < nc; ++c) {
    if (used[c]) continue;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += M[(size_t)c * n + i] * M[(size_t)c * n + i];
    if (std::sqrt(s) > 1e-6 * std::max(norm0[c], 1.0)) {
      err = "selected eigenvalues are not closed under conjugation";
      return -1;
    }
  }
  // H_k = W^T H_m W
  std::vector<double> HW((size_t)n * kept, 0.0);
  for (int j = 0; j < kept; ++j)
    for (int l = 0; l < n; ++l) {
      const double wl = W[(size_t)j * n + l];
      if (wl == 0.0) continue;
      for (int i = 0; i < n; ++i) HW[(size_t)j * n + i] += Hm[(size_t)l * ldh + i] * wl;
    }
  Hk.assign((size_t)kept * kept, 0.0);
  for (int j = 0; j < kept; ++j)
    for (int i = 0; i < kept; ++i) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += W[(size_t)i * n + l] * HW[(size_t)j * n + l];
      Hk[(size_t)j * kept + i] = s;
    }
  return kept;
}

}  // namespace pslr
