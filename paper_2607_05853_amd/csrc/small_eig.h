// Host-side dense linear algebra for small complex Hermitian problems
// (Rayleigh-Ritz of the block eigensolver, tridiagonal resolvents of the
// spectrum's VJP).  Plain C++ so it also builds with the host compiler for
// CPU tests.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <vector>

namespace bse {
namespace small {

using cd = std::complex<double>;

// Cyclic Jacobi for a complex Hermitian n x n matrix A (row-major, destroyed).
// Each rotation first removes the phase of a_pq with a diagonal unitary, then
// applies the real symmetric Schur rotation of Golub & Van Loan (Alg. 8.4.1).
// On return w holds the eigenvalues ascending and V (row-major, V[i*n+j] =
// component i of eigenvector j) the orthonormal eigenvectors.
inline int jacobi_herm(int n, std::vector<cd>& A, std::vector<double>& w, std::vector<cd>& V,
                       int max_sweeps = 100) {
  V.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  double fro = 0.0;
  for (auto& z : A) fro += std::norm(z);
  fro = std::sqrt(fro);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(at(p, q));
    if (std::sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double r = std::abs(at(p, q));
        if (r <= 1e-300) continue;
        const cd ph = at(p, q) / r;  // e^{i theta}
        const double al = at(p, p).real(), ga = at(q, q).real();
        const double tau = (ga - al) / (2.0 * r);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        const cd eq = std::conj(ph);  // e^{-i theta}
        // A <- A U : col_p' = c col_p - s e^{-i theta} col_q ; col_q' = s col_p + c e^{-i theta} col_q
        for (int k = 0; k < n; ++k) {
          const cd ap = at(k, p), aq = at(k, q);
          at(k, p) = c * ap - s * eq * aq;
          at(k, q) = s * ap + c * eq * aq;
          const cd vp = V[(size_t)k * n + p], vq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vp - s * eq * vq;
          V[(size_t)k * n + q] = s * vp + c * eq * vq;
        }
        // A <- U^H A : row_p' = c row_p - s e^{i theta} row_q ; row_q' = s row_p + c e^{i theta} row_q
        for (int k = 0; k < n; ++k) {
          const cd ap = at(p, k), aq = at(q, k);
          at(p, k) = c * ap - s * ph * aq;
          at(q, k) = s * ap + c * ph * aq;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        at(p, p) = at(p, p).real();
        at(q, q) = at(q, q).real();
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = at(i, i).real();
  // sort ascending
  for (int i = 0; i < n; ++i) {
    int m = i;
    for (int j = i + 1; j < n; ++j)
      if (w[j] < w[m]) m = j;
    if (m != i) {
      std::swap(w[i], w[m]);
      for (int k = 0; k < n; ++k) std::swap(V[(size_t)k * n + i], V[(size_t)k * n + m]);
    }
  }
  return sweep;
}

// Cholesky of a Hermitian positive definite matrix: G = L L^H (row-major, lower).
// Returns false if a pivot is not positive.
inline bool cholesky(int n, const std::vector<cd>& G, std::vector<cd>& L) {
  L.assign((size_t)n * n, cd(0, 0));
  for (int j = 0; j < n; ++j) {
    double d = G[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[(size_t)j * n + k]);
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cd s = G[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * std::conj(L[(size_t)j * n + k]);
      L[(size_t)i * n + j] = s / ljj;
    }
  }
  return true;
}

// Inverse of a lower-triangular matrix (row-major).
inline void tri_lower_inverse(int n, const std::vector<cd>& L, std::vector<cd>& Li) {
  Li.assign((size_t)n * n, cd(0, 0));
  for (int j = 0; j < n; ++j) {
    Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      cd s = 0;
      for (int k = j; k < i; ++k) s -= L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = s / L[(size_t)i * n + i];
    }
  }
}

// Generalised Hermitian-definite problem A x = lambda G x via G = L L^H:
// eigenvalues ascending in w, eigenvectors (G-orthonormal) as columns of X.
// Returns false when G is not numerically positive definite.
inline bool gen_eig(int n, const std::vector<cd>& A, const std::vector<cd>& G, std::vector<double>& w,
                    std::vector<cd>& X) {
  std::vector<cd> L, Li;
  if (!cholesky(n, G, L)) return false;
  tri_lower_inverse(n, L, Li);
  // C = Li A Li^H
  std::vector<cd> T((size_t)n * n, cd(0, 0)), C((size_t)n * n, cd(0, 0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int k = 0; k <= i; ++k) s += Li[(size_t)i * n + k] * A[(size_t)k * n + j];
      T[(size_t)i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int k = 0; k <= j; ++k) s += T[(size_t)i * n + k] * std::conj(Li[(size_t)j * n + k]);
      C[(size_t)i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {  // symmetrise against rounding
      const cd m = 0.5 * (C[(size_t)i * n + j] + std::conj(C[(size_t)j * n + i]));
      C[(size_t)i * n + j] = m;
      C[(size_t)j * n + i] = std::conj(m);
    }
  std::vector<cd> V;
  jacobi_herm(n, C, w, V);
  // X = Li^H V
  X.assign((size_t)n * n, cd(0, 0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int k = i; k < n; ++k) s += std::conj(Li[(size_t)k * n + i]) * V[(size_t)k * n + j];
      X[(size_t)i * n + j] = s;
    }
  return true;
}

// Rank-revealing variant of gen_eig for a Gram matrix G that may be singular:
// G = U diag(g) U^H, directions with g_i <= thr * max(g) are dropped, the rest
// are whitened (Z = U_r g_r^-1/2) and A is diagonalised in that basis.
// Returns the rank r; w[0..r) ascending, X (n x r, row-major) G-orthonormal.
inline int gen_eig_robust(int n, const std::vector<cd>& A, const std::vector<cd>& G, std::vector<double>& w,
                          std::vector<cd>& X, double thr = 1e-12) {
  std::vector<cd> Gc = G, U;
  std::vector<double> g;
  jacobi_herm(n, Gc, g, U);
  const double gmax = g.empty() ? 0.0 : g.back();
  std::vector<int> keep;
  for (int i = 0; i < n; ++i)
    if (g[i] > thr * gmax && g[i] > 0.0) keep.push_back(i);
  const int r = (int)keep.size();
  if (r == 0) return 0;
  std::vector<cd> Z((size_t)n * r);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < r; ++j) Z[(size_t)i * r + j] = U[(size_t)i * n + keep[j]] / std::sqrt(g[keep[j]]);
  std::vector<cd> AZ((size_t)n * r, cd(0, 0)), Ar((size_t)r * r, cd(0, 0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < r; ++j) {
      cd s = 0;
      for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * Z[(size_t)k * r + j];
      AZ[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      cd s = 0;
      for (int k = 0; k < n; ++k) s += std::conj(Z[(size_t)k * r + i]) * AZ[(size_t)k * r + j];
      Ar[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) {
      const cd m = 0.5 * (Ar[(size_t)i * r + j] + std::conj(Ar[(size_t)j * r + i]));
      Ar[(size_t)i * r + j] = m;
      Ar[(size_t)j * r + i] = std::conj(m);
    }
  std::vector<cd> V;
  jacobi_herm(r, Ar, w, V);
  X.assign((size_t)n * r, cd(0, 0));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < r; ++j) {
      cd s = 0;
      for (int k = 0; k < r; ++k) s += Z[(size_t)i * r + k] * V[(size_t)k * r + j];
      X[(size_t)i * r + j] = s;
    }
  return r;
}

// Solve (z - T) s = b0 e_1 for the m x m Hermitian tridiagonal T with diagonal
// a[0..m-1] and off-diagonal b[1..m-1] (Thomas algorithm, complex z).
inline void tridiag_resolvent(int m, const double* a, const double* b, double b0, cd z, cd* s) {
  std::vector<cd> cp(m), dp(m);
  // rows: -b_{i} s_{i-1} + (z - a_i) s_i - b_{i+1} s_{i+1} = rhs_i
  cd diag = z - a[0];
  cp[0] = (m > 1 ? -b[1] : 0.0) / diag;
  dp[0] = cd(b0, 0.0) / diag;
  for (int i = 1; i < m; ++i) {
    const cd lo = -b[i];
    diag = (z - a[i]) - lo * cp[i - 1];
    cp[i] = (i + 1 < m ? -b[i + 1] : 0.0) / diag;
    dp[i] = (0.0 - lo * dp[i - 1]) / diag;
  }
  s[m - 1] = dp[m - 1];
  for (int i = m - 2; i >= 0; --i) s[i] = dp[i] - cp[i] * s[i + 1];
}

// Eigenvalues of the real symmetric tridiagonal matrix with diagonal d[0..n-1] and off-diagonal
// e[0..n-2] (e[i] couples i and i + 1), with the first component of each normalised eigenvector
// (the Gauss-quadrature weights of a Lanczos tridiagonal): implicit QL iteration with a shift from the
// leading 2 x 2 block (Bowdler, Martin, Reinsch & Wilkinson, Numer. Math. 11, 1968), the rotations
// applied to the first row of the eigenvector matrix only.  On return w is ascending and z[i] belongs
// to w[i].  Returns false if an eigenvalue needs more than 64 iterations.
inline bool tridiag_eig_first(int n, const double* d_in, const double* e_in, std::vector<double>& w,
                              std::vector<double>& z) {
  std::vector<double> d(d_in, d_in + n), e((size_t)n + 1, 0.0), q(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
  if (n > 0) q[0] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      while (m + 1 < n && std::fabs(e[m]) > eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) ++m;
      if (m == l) break;
      if (iter >= 64) return false;
      // shift: the eigenvalue of [[d_l, e_l], [e_l, d_l+1]] nearer to d_l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // the rotation underflowed: the matrix splits at i + 1
          d[i + 1] -= p;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        const double t = q[i + 1];
        q[i + 1] = s * q[i] + c * t;
        q[i] = c * q[i] - s * t;
      }
      if (split) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  z.resize(n);
  for (int i = 0; i < n; ++i) {
    w[i] = d[idx[i]];
    z[i] = q[idx[i]];
  }
  return true;
}

}  // namespace small
}  // namespace bse
