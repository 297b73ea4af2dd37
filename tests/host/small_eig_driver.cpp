// CPU driver for the host-side small eigensolvers (reads stdin, writes stdout).
// mode 0: n, A(n*n complex) -> w, V        (Jacobi)
// mode 1: n, A, G            -> w, X        (generalised, Cholesky + Jacobi)
// mode 2: m, a(m), b(m), b0, zr, zi -> s(m) (tridiagonal resolvent)
// mode 3: n, A, G            -> r, w(r), X(n*r) (rank-revealing generalised)
// mode 4: n, d(n), e(n-1)     -> w(n), z(n)   (symmetric tridiagonal, first eigenvector components)
#include <cstdio>
#include <vector>

#include "../../paper_2607_05853_amd/csrc/small_eig.h"

using bse::small::cd;

static std::vector<cd> read_mat(int n) {
  std::vector<cd> M((size_t)n * n);
  for (auto& z : M) {
    double re, im;
    if (scanf("%lf %lf", &re, &im) != 2) return {};
    z = cd(re, im);
  }
  return M;
}

int main() {
  int mode, n;
  if (scanf("%d %d", &mode, &n) != 2) return 1;
  if (mode == 4) {
    std::vector<double> d(n), e(n > 0 ? n - 1 : 0), w, z;
    for (auto& x : d) scanf("%lf", &x);
    for (auto& x : e) scanf("%lf", &x);
    if (!bse::small::tridiag_eig_first(n, d.data(), e.data(), w, z)) return 3;
    for (double x : w) printf("%.17g\n", x);
    for (double x : z) printf("%.17g\n", x);
    return 0;
  }
  if (mode == 3) {
    std::vector<cd> A = read_mat(n), G = read_mat(n), X;
    std::vector<double> w;
    const int r = bse::small::gen_eig_robust(n, A, G, w, X);
    printf("%d\n", r);
    for (int i = 0; i < r; ++i) printf("%.17g\n", w[i]);
    for (auto& z : X) printf("%.17g %.17g\n", z.real(), z.imag());
    return 0;
  }
  if (mode == 0 || mode == 1) {
    std::vector<cd> A = read_mat(n), G, V;
    std::vector<double> w;
    if (mode == 0) {
      bse::small::jacobi_herm(n, A, w, V);
    } else {
      G = read_mat(n);
      if (!bse::small::gen_eig(n, A, G, w, V)) return 2;
    }
    for (double x : w) printf("%.17g\n", x);
    for (auto& z : V) printf("%.17g %.17g\n", z.real(), z.imag());
  } else {
    std::vector<double> a(n), b(n);
    for (auto& x : a) scanf("%lf", &x);
    for (auto& x : b) scanf("%lf", &x);
    double b0, zr, zi;
    scanf("%lf %lf %lf", &b0, &zr, &zi);
    std::vector<cd> s(n);
    bse::small::tridiag_resolvent(n, a.data(), b.data(), b0, cd(zr, zi), s.data());
    for (auto& z : s) printf("%.17g %.17g\n", z.real(), z.imag());
  }
  return 0;
}
