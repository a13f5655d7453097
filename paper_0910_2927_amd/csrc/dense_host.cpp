// Small dense complex FP64 linear algebra on the host, for the setup-time
// eigensolver of the deflation space (Sect. 4 needs the m critical
// eigenpairs; the paper takes them as given): Hessenberg reduction, the
// shifted QR algorithm for the complex Schur form, reordering of a Schur
// form, LU solves and the Newton iteration for the matrix sign function
// (Roberts' method, which Sect. 6 names for sign(H_k)).
//
// Matrices are column-major, element (i, j) at a[i + j*n].  Sizes are the
// Krylov-Schur basis size (<= 512), so O(n^3) host work is negligible next
// to the device work of a restart.
#include "dense_host.h"

#include <algorithm>
#include <cmath>

namespace sk {
namespace dense {

using cd = std::complex<double>;

static inline cd& at(std::vector<cd>& a, int n, int i, int j) { return a[i + (size_t)j * n]; }

// Householder reduction to upper Hessenberg form: A = Q H Q^H (in place).
void hessenberg(int n, std::vector<cd>& A, std::vector<cd>& Q) {
  Q.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) at(Q, n, i, i) = 1.0;
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha2 = 0.0;
    for (int i = k + 1; i < n; ++i) alpha2 += std::norm(at(A, n, i, k));
    double xnorm = std::sqrt(alpha2);
    if (xnorm == 0.0) continue;
    cd x0 = at(A, n, k + 1, k);
    cd ph = (std::abs(x0) == 0.0) ? cd(1.0) : x0 / std::abs(x0);
    // v = x + ph * ||x|| e1, H = I - 2 v v^H / (v^H v)
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = at(A, n, i, k);
    v[k + 1] += ph * xnorm;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // A <- H A
    for (int j = 0; j < n; ++j) {
      cd s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * at(A, n, i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) at(A, n, i, j) -= v[i] * s;
    }
    // A <- A H, Q <- Q H
    for (int i = 0; i < n; ++i) {
      cd s = 0.0, t = 0.0;
      for (int j = k + 1; j < n; ++j) {
        s += at(A, n, i, j) * v[j];
        t += at(Q, n, i, j) * v[j];
      }
      s *= 2.0 / vn;
      t *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) {
        at(A, n, i, j) -= s * std::conj(v[j]);
        at(Q, n, i, j) -= t * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < n; ++i) at(A, n, i, k) = 0.0;
  }
}

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G^H [a; b] = [r; 0].
static void givens(cd a, cd b, double& c, cd& s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (aa == 0.0) {
    c = 0.0;
    s = std::conj(b / bb);   // [0; b] -> [|b|; 0]
    return;
  }
  const double r = std::hypot(aa, bb);
  c = aa / r;
  s = (a / aa) * std::conj(b) / r;
}

// rows p, q of A (columns j0..j1-1) <- [[c, s], [-conj(s), c]] applied from the left
static void rot_rows(std::vector<cd>& A, int n, int p, int q, double c, cd s, int j0, int j1) {
  for (int j = j0; j < j1; ++j) {
    cd x = at(A, n, p, j), y = at(A, n, q, j);
    at(A, n, p, j) = c * x + s * y;
    at(A, n, q, j) = -std::conj(s) * x + c * y;
  }
}
// columns p, q of A (rows i0..i1-1) <- A [[c, -s], [conj(s), c]]  (the adjoint rotation)
static void rot_cols(std::vector<cd>& A, int n, int p, int q, double c, cd s, int i0, int i1) {
  for (int i = i0; i < i1; ++i) {
    cd x = at(A, n, i, p), y = at(A, n, i, q);
    at(A, n, i, p) = c * x + std::conj(s) * y;
    at(A, n, i, q) = -s * x + c * y;
  }
}

// Complex Schur form of a Hessenberg matrix by single-shift QR with
// Wilkinson shifts and deflation; H <- T (upper triangular), Q <- Q Z.
bool schur_hessenberg(int n, std::vector<cd>& H, std::vector<cd>& Q, int max_sweeps) {
  int hi = n - 1;
  int iter = 0;
  const double eps = 2.220446049250313e-16;
  while (hi > 0) {
    // find the active block [lo, hi]
    int lo = hi;
    while (lo > 0) {
      double sub = std::abs(at(H, n, lo, lo - 1));
      double d = std::abs(at(H, n, lo, lo)) + std::abs(at(H, n, lo - 1, lo - 1));
      if (sub <= eps * (d == 0.0 ? 1.0 : d)) {
        at(H, n, lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > max_sweeps) return false;
    // Wilkinson shift from the trailing 2x2 of the block
    cd a = at(H, n, hi - 1, hi - 1), b = at(H, n, hi - 1, hi), c = at(H, n, hi, hi - 1),
       d = at(H, n, hi, hi);
    cd tr = a + d, det = a * d - b * c;
    cd disc = std::sqrt(tr * tr - 4.0 * det);
    cd e1 = 0.5 * (tr + disc), e2 = 0.5 * (tr - disc);
    cd mu = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
    if (iter % 11 == 10) mu = d + cd(std::abs(at(H, n, hi, hi - 1)), 0.0);   // exceptional shift
    // implicit single-shift QR sweep on the block (bulge chase)
    cd x = at(H, n, lo, lo) - mu, y = at(H, n, lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      double cs;
      cd sn;
      givens(x, y, cs, sn);
      const int j0 = std::max(lo, k - 1);
      rot_rows(H, n, k, k + 1, cs, sn, j0, n);
      rot_cols(H, n, k, k + 1, cs, sn, 0, std::min(hi, k + 2) + 1);
      rot_cols(Q, n, k, k + 1, cs, sn, 0, n);
      if (k > lo) at(H, n, k + 1, k - 1) = 0.0;
      if (k + 1 < hi) {
        x = at(H, n, k + 1, k);
        y = at(H, n, k + 2, k);
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) at(H, n, i, j) = 0.0;
  return true;
}

bool schur(int n, std::vector<cd>& A, std::vector<cd>& Q) {
  hessenberg(n, A, Q);
  return schur_hessenberg(n, A, Q, 100 * n + 100);
}

// Swap diagonal entries k, k+1 of an upper triangular T (T <- G^H T G,
// Q <- Q G) keeping it triangular.
static void swap_adjacent(int n, std::vector<cd>& T, std::vector<cd>& Q, int k) {
  cd t11 = at(T, n, k, k), t22 = at(T, n, k + 1, k + 1), t12 = at(T, n, k, k + 1);
  if (t11 == t22) return;
  // the rotation takes the eigenvector of t22, [t12; t22 - t11], to e1
  double cs;
  cd sn;
  givens(t12, t22 - t11, cs, sn);
  rot_rows(T, n, k, k + 1, cs, sn, k, n);
  rot_cols(T, n, k, k + 1, cs, sn, 0, k + 2);
  rot_cols(Q, n, k, k + 1, cs, sn, 0, n);
  at(T, n, k + 1, k) = 0.0;
}

// Stable reordering: the entries with the `count` smallest keys first, in
// increasing key order (bubble of adjacent swaps).
void reorder_schur(int n, std::vector<cd>& T, std::vector<cd>& Q,
                   const std::function<double(cd)>& key, int count) {
  for (int pos = 0; pos < count && pos < n; ++pos) {
    int best = pos;
    double bk = key(at(T, n, pos, pos));
    for (int i = pos + 1; i < n; ++i) {
      double ki = key(at(T, n, i, i));
      if (ki < bk) {
        bk = ki;
        best = i;
      }
    }
    for (int i = best - 1; i >= pos; --i) swap_adjacent(n, T, Q, i);
  }
}

// Solve A X = B (A n x n, B n x r) by LU with partial pivoting; false if singular.
bool lu_solve(int n, std::vector<cd> A, std::vector<cd>& B, int r) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(at(A, n, k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(at(A, n, i, k)) > best) {
        best = std::abs(at(A, n, i, k));
        p = i;
      }
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(at(A, n, k, j), at(A, n, p, j));
      for (int j = 0; j < r; ++j) std::swap(at(B, n, k, j), at(B, n, p, j));
    }
    for (int i = k + 1; i < n; ++i) {
      cd l = at(A, n, i, k) / at(A, n, k, k);
      at(A, n, i, k) = l;
      for (int j = k + 1; j < n; ++j) at(A, n, i, j) -= l * at(A, n, k, j);
      for (int j = 0; j < r; ++j) at(B, n, i, j) -= l * at(B, n, k, j);
    }
  }
  for (int j = 0; j < r; ++j)
    for (int i = n - 1; i >= 0; --i) {
      cd s = at(B, n, i, j);
      for (int l = i + 1; l < n; ++l) s -= at(A, n, i, l) * at(B, n, l, j);
      at(B, n, i, j) = s / at(A, n, i, i);
    }
  return true;
}

bool inverse(int n, const std::vector<cd>& A, std::vector<cd>& X) {
  X.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) at(X, n, i, i) = 1.0;
  return lu_solve(n, A, X, n);
}

// sign(A) by Newton's iteration X <- (X + X^{-1}) / 2 (Roberts' method).
bool newton_sign(int n, const std::vector<cd>& A, std::vector<cd>& S, double tol, int maxit) {
  S = A;
  std::vector<cd> Xi;
  for (int it = 0; it < maxit; ++it) {
    if (!inverse(n, S, Xi)) return false;
    double diff = 0.0, nrm = 0.0;
    for (size_t e = 0; e < S.size(); ++e) {
      cd nx = 0.5 * (S[e] + Xi[e]);
      diff += std::norm(nx - S[e]);
      nrm += std::norm(nx);
      S[e] = nx;
    }
    if (std::sqrt(diff) <= tol * std::sqrt(nrm)) return true;
  }
  return false;
}

void matmul(int m, int k, int n, const std::vector<cd>& A, const std::vector<cd>& B,
            std::vector<cd>& C, bool conjA) {
  // C (m x n) = op(A) (m x k) * B (k x n); op(A) = A or A^H (A stored k x m then)
  C.assign((size_t)m * n, cd(0.0));
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const cd b = B[l + (size_t)j * k];
      if (b == cd(0.0)) continue;
      for (int i = 0; i < m; ++i) {
        const cd a = conjA ? std::conj(A[l + (size_t)i * k]) : A[i + (size_t)l * m];
        C[i + (size_t)j * m] += a * b;
      }
    }
}

}  // namespace dense
}  // namespace sk
