// Drivers on top of the apply: block LOBPCG for the lowest excitons (Knyazev
// 2001; Rayleigh-Ritz in FP64 on the host) and the vector-Jacobian product of
// the Haydock spectrum through the stored Lanczos basis.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bse_internal.h"
#include "small_eig.h"

namespace bse {
namespace {

using small::cd;

// counter-based start block: splitmix64 of (row, column), uniform in [-1, 1)
__global__ void random_block_kernel(long long N, int nb, unsigned long long seed, double* __restrict__ X) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  auto mix = [](unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const unsigned long long h1 = mix(seed ^ (2 * (unsigned long long)t));
  const unsigned long long h2 = mix(seed ^ (2 * (unsigned long long)t + 1));
  X[2 * t] = (double)(h1 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  X[2 * t + 1] = (double)(h2 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// R = AX - X diag(lambda);  W = R / max(d_I - lambda_j, tau_j)
__global__ void residual_precond_kernel(long long N, int nb, int nv, int nc, const double* __restrict__ eps,
                                        const double* __restrict__ lam, const double* __restrict__ X,
                                        const double* __restrict__ AX, double* __restrict__ R,
                                        double* __restrict__ W) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  const int j = (int)(t % nb);
  const long long I = t / nb;
  const int v = (int)(I % nv);
  const long long kc = I / nv;
  const int c = (int)(kc % nc);
  const long long k = kc / nc;
  const double d = eps[k * (nv + nc) + nv + c] - eps[k * (nv + nc) + v];
  const double rr = AX[2 * t] - lam[j] * X[2 * t], ri = AX[2 * t + 1] - lam[j] * X[2 * t + 1];
  R[2 * t] = rr;
  R[2 * t + 1] = ri;
  // positive definite preconditioner (D - lambda_j)^-1 clamped below at tau_j = 0.02 |lambda_j|:
  // components with transition energies below the Ritz value are not amplified without bound
  const double tau = 0.02 * fmax(fabs(lam[j]), 1e-12);
  double den = d - lam[j];
  if (den < tau) den = tau;
  W[2 * t] = rr / den;
  W[2 * t + 1] = ri / den;
}

__global__ void add_kernel(long long n, const double* __restrict__ in, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += in[i];
}

__global__ void reduce_parts(int nsplit, int n, const double* __restrict__ part, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sr = 0, si = 0;
  for (int s = 0; s < nsplit; ++s) {
    sr += part[2 * ((long long)s * n + i)];
    si += part[2 * ((long long)s * n + i) + 1];
  }
  out[2 * i] = sr;
  out[2 * i + 1] = si;
}

// Rayleigh-Ritz drops basis directions whose Gram eigenvalue is below thr times the largest: the
// whitening multiplies the error of the projected operator by 1 / g, so the threshold follows the
// rounding of the apply (FP64 ~1e-15; FP32 and BF16x3 ~1e-8 relative, where 1e-12 would let that error
// grow to spurious Ritz values of 1e4 |A| and beyond)
double rr_threshold(const Plan* p) { return p->prec == BSE_F64 ? 1e-12 : 1e-6; }

struct Work {
  std::vector<double*> bufs;
  ~Work() {
    for (double* p : bufs) dfree(p);
  }
  bse_status get(double** p, size_t bytes) {
    BSE_TRY(dmalloc((void**)p, bytes));
    bufs.push_back(*p);
    return BSE_OK;
  }
};

// out (device, c128 [a][b]) = U^H V for U [N][a], V [N][b] (row-major blocks), split over rows
bse_status gram_dev(const double* U, int a, const double* V, int b, long long N, double* part, int nsplit,
                    double* out, hipStream_t st) {
  const long long Ks = (N + nsplit - 1) / nsplit;
  // use whole chunks only: the remainder rows go through a second GEMM
  const int full = (int)(N / Ks);
  GemmArgs g;
  g.batch = full;
  g.M = a;
  g.N = b;
  g.K = (int)Ks;
  g.A = U;
  g.a_sb = Ks * a;
  g.a_si = 1;
  g.a_sk = a;
  g.conjA = 1;
  g.B = V;
  g.b_sb = Ks * b;
  g.b_sk = b;
  g.b_sj = 1;
  g.C = part;
  g.c_sb = (long long)a * b;
  g.c_si = b;
  g.c_sj = 1;
  BSE_TRY(cgemm(g, AR_F64, true, true, st));
  int used = full;
  const long long rem = N - (long long)full * Ks;
  if (rem > 0) {
    GemmArgs h = g;
    h.batch = 1;
    h.K = (int)rem;
    h.A = U + 2 * (long long)full * Ks * a;
    h.B = V + 2 * (long long)full * Ks * b;
    h.C = part + 2 * (long long)full * a * b;
    BSE_TRY(cgemm(h, AR_F64, true, true, st));
    ++used;
  }
  const int n = a * b;
  hipLaunchKernelGGL(reduce_parts, dim3((n + 255) / 256), dim3(256), 0, st, used, n, part, out);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// out [N][nc] (+)= U [N][a] C [a][nc]   (C on the device)
bse_status combine(const double* U, int a, const double* Cd, int ncol, long long N, double* out, int beta,
                   hipStream_t st) {
  GemmArgs g;
  g.M = (int)N;
  g.N = ncol;
  g.K = a;
  g.A = U;
  g.a_si = a;
  g.a_sk = 1;
  g.B = Cd;
  g.b_sk = ncol;
  g.b_sj = 1;
  g.C = out;
  g.c_si = ncol;
  g.c_sj = 1;
  g.beta = beta;
  return cgemm(g, AR_F64, true, true, st);
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" bse_status bse_lowest_excitons(bse_plan* plan, int32_t n_block, int32_t max_iter, double tol,
                                          const void* X0, double* omega, void* x_out, int32_t* iters,
                                          void* hip_stream) {
  set_error("");
  if (!plan || !omega || n_block <= 0 || max_iter <= 0 || !(tol > 0.0)) {
    set_error("bse_lowest_excitons: invalid argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  const int nb = n_block;
  if (nb > p->max_nb || 3LL * nb > p->N) {
    set_error("bse_lowest_excitons: need n_block <= max_nb and 3*n_block <= N");
    return BSE_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long long N = p->N;
  const size_t blk = 16 * (size_t)N * nb;
  Work wk;
  double *X, *AX, *W, *AW, *P, *AP, *R, *T1, *T2, *part, *gsm, *cdev, *lam;
  BSE_TRY(wk.get(&X, blk));
  BSE_TRY(wk.get(&AX, blk));
  BSE_TRY(wk.get(&W, blk));
  BSE_TRY(wk.get(&AW, blk));
  BSE_TRY(wk.get(&P, blk));
  BSE_TRY(wk.get(&AP, blk));
  BSE_TRY(wk.get(&R, blk));
  BSE_TRY(wk.get(&T1, blk));
  BSE_TRY(wk.get(&T2, blk));
  const int nsplit = (int)std::max<long long>(1, std::min<long long>(256, N / 64));
  BSE_TRY(wk.get(&part, 16 * (size_t)(nsplit + 1) * nb * nb));
  BSE_TRY(wk.get(&gsm, 16 * (size_t)12 * nb * nb));
  BSE_TRY(wk.get(&cdev, 16 * (size_t)3 * nb * nb));
  BSE_TRY(wk.get(&lam, 8 * (size_t)nb));

  if (X0)
    BSE_HIP(hipMemcpyAsync(X, X0, blk, hipMemcpyDeviceToDevice, st));
  else
    hipLaunchKernelGGL(random_block_kernel, dim3((unsigned)((N * nb + 255) / 256)), dim3(256), 0, st, N, nb,
                       0x2607058530000001ull, X);
  BSE_CHECK_LAUNCH();

  auto fetch = [&](int count, std::vector<cd>& h) -> bse_status {
    h.resize((size_t)count * nb * nb);
    BSE_HIP(hipMemcpyAsync(h.data(), gsm, 16 * h.size(), hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    return BSE_OK;
  };
  auto put_coeffs = [&](const std::vector<cd>& c) -> bse_status {
    BSE_HIP(hipMemcpyAsync(cdev, c.data(), 16 * c.size(), hipMemcpyHostToDevice, st));
    return BSE_OK;
  };
  const size_t nn = (size_t)nb * nb;

  // Rayleigh-Ritz on the start block (orthonormalises it as well)
  BSE_TRY(bse_apply(plan, X, AX, nb, hip_stream));
  BSE_TRY(gram_dev(X, nb, AX, nb, N, part, nsplit, gsm, st));
  BSE_TRY(gram_dev(X, nb, X, nb, N, part, nsplit, gsm + 2 * nn, st));
  std::vector<cd> h, GA(nn), GB(nn), C;
  std::vector<double> w;
  BSE_TRY(fetch(2, h));
  for (size_t i = 0; i < nn; ++i) {
    GA[i] = h[i];
    GB[i] = h[nn + i];
  }
  for (int i = 0; i < nb; ++i)
    for (int j = i + 1; j < nb; ++j) {
      GA[(size_t)j * nb + i] = std::conj(GA[(size_t)i * nb + j]);
      GB[(size_t)j * nb + i] = std::conj(GB[(size_t)i * nb + j]);
    }
  if (small::gen_eig_robust(nb, GA, GB, w, C, rr_threshold(p)) < nb) {
    set_error("bse_lowest_excitons: start block is rank deficient");
    return BSE_ESHAPE;
  }
  BSE_TRY(put_coeffs(C));
  BSE_TRY(combine(X, nb, cdev, nb, N, T1, 0, st));
  BSE_TRY(combine(AX, nb, cdev, nb, N, T2, 0, st));
  std::swap(X, T1);
  std::swap(AX, T2);
  std::vector<double> lamh(w.begin(), w.begin() + nb);
  bool haveP = false;
  int it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    BSE_HIP(hipMemcpyAsync(lam, lamh.data(), 8 * nb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(residual_precond_kernel, dim3((unsigned)((N * nb + 255) / 256)), dim3(256), 0, st, N, nb,
                       p->d.nv, p->d.nc, p->eps, lam, X, AX, R, W);
    BSE_CHECK_LAUNCH();
    BSE_TRY(gram_dev(R, nb, R, nb, N, part, nsplit, gsm, st));
    BSE_TRY(fetch(1, h));
    double worst = 0.0;
    for (int j = 0; j < nb; ++j)
      worst = std::max(worst, std::sqrt(std::max(h[(size_t)j * nb + j].real(), 0.0)) /
                                  std::max(std::fabs(lamh[j]), 1e-300));
    if (worst <= tol) {
      converged = true;
      break;
    }
    BSE_TRY(bse_apply(plan, W, AW, nb, hip_stream));
    // blocks of the basis S = [X, W, P] and of A S
    const double* Sb[3] = {X, W, P};
    const double* ASb[3] = {AX, AW, AP};
    const int nblk = haveP ? 3 : 2;
    int slot = 0;
    for (int i = 0; i < nblk; ++i)
      for (int j = i; j < nblk; ++j) {
        BSE_TRY(gram_dev(Sb[i], nb, ASb[j], nb, N, part, nsplit, gsm + 2 * nn * slot, st));
        ++slot;
        BSE_TRY(gram_dev(Sb[i], nb, Sb[j], nb, N, part, nsplit, gsm + 2 * nn * slot, st));
        ++slot;
      }
    BSE_TRY(fetch(slot, h));
    int rank = 0;
    auto solve = [&](int nbk) -> bool {
      const int n = nbk * nb;
      GA.assign((size_t)n * n, cd(0, 0));
      GB.assign((size_t)n * n, cd(0, 0));
      int s = 0;
      for (int i = 0; i < nblk; ++i)
        for (int j = i; j < nblk; ++j) {
          const cd* ga = h.data() + nn * s;
          const cd* gb = h.data() + nn * (s + 1);
          s += 2;
          if (i >= nbk || j >= nbk) continue;
          for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c) {
              const size_t ij = (size_t)(i * nb + r) * n + (j * nb + c);
              const size_t ji = (size_t)(j * nb + c) * n + (i * nb + r);
              GA[ij] = ga[(size_t)r * nb + c];
              GB[ij] = gb[(size_t)r * nb + c];
              GA[ji] = std::conj(ga[(size_t)r * nb + c]);
              GB[ji] = std::conj(gb[(size_t)r * nb + c]);
            }
        }
      // diagonal scaling for conditioning
      std::vector<double> sc(n);
      for (int i = 0; i < n; ++i) sc[i] = 1.0 / std::sqrt(std::max(GB[(size_t)i * n + i].real(), 1e-300));
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          GA[(size_t)i * n + j] *= sc[i] * sc[j];
          GB[(size_t)i * n + j] *= sc[i] * sc[j];
        }
      rank = small::gen_eig_robust(n, GA, GB, w, C, rr_threshold(p));
      if (rank < nb) return false;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < rank; ++j) C[(size_t)i * rank + j] *= sc[i];
      return true;
    };
    int used = nblk;
    if (!solve(used)) {
      used = 2;  // restart without the search directions
      if (!solve(used)) {
        set_error("bse_lowest_excitons: basis [X, W] lost rank");
        return BSE_ESHAPE;
      }
    }
    // coefficient blocks of the lowest nb Ritz vectors: rows [X | W | P], C is (used*nb) x rank
    std::vector<cd> cx(nn), cw(nn), cp(nn);
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) {
        cx[(size_t)r * nb + c] = C[(size_t)r * rank + c];
        cw[(size_t)r * nb + c] = C[(size_t)(nb + r) * rank + c];
        cp[(size_t)r * nb + c] = used == 3 ? C[(size_t)(2 * nb + r) * rank + c] : cd(0, 0);
      }
    std::vector<cd> all(3 * nn);
    std::copy(cx.begin(), cx.end(), all.begin());
    std::copy(cw.begin(), cw.end(), all.begin() + nn);
    std::copy(cp.begin(), cp.end(), all.begin() + 2 * nn);
    BSE_TRY(put_coeffs(all));
    double* dcx = cdev;
    double* dcw = cdev + 2 * nn;
    double* dcp = cdev + 4 * nn;
    // P' = W cw + P cp, AP' = AW cw + AP cp;  X' = X cx + P', AX' = AX cx + AP'
    BSE_TRY(combine(W, nb, dcw, nb, N, T1, 0, st));
    BSE_TRY(combine(AW, nb, dcw, nb, N, T2, 0, st));
    if (used == 3) {
      BSE_TRY(combine(P, nb, dcp, nb, N, T1, 1, st));
      BSE_TRY(combine(AP, nb, dcp, nb, N, T2, 1, st));
    }
    std::swap(P, T1);
    std::swap(AP, T2);
    BSE_TRY(combine(X, nb, dcx, nb, N, T1, 0, st));
    BSE_TRY(combine(AX, nb, dcx, nb, N, T2, 0, st));
    {
      const long long n2 = 2 * N * nb;
      hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, P, T1);
      hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, AP, T2);
      BSE_CHECK_LAUNCH();
    }
    std::swap(X, T1);
    std::swap(AX, T2);
    haveP = true;
    for (int j = 0; j < nb; ++j) lamh[j] = w[j];
  }
  for (int j = 0; j < nb; ++j) omega[j] = lamh[j];
  if (iters) *iters = converged ? it : max_iter;
  if (x_out) BSE_HIP(hipMemcpyAsync(x_out, X, blk, hipMemcpyDeviceToDevice, st));
  BSE_HIP(hipStreamSynchronize(st));
  if (!converged) {
    set_error("bse_lowest_excitons: not converged within max_iter");
    return BSE_INFO_NOT_CONVERGED;
  }
  return BSE_OK;
}

extern "C" bse_status bse_haydock_vjp(bse_plan* plan, const void* basis, const double* a, const double* b,
                                      const int32_t* steps, int32_t nb, int32_t n_steps, const double* omega,
                                      int32_t n_w, double eta, const double* gamma, void* g_WR, void* g_Wq,
                                      double* g_eps, void* hip_stream) {
  set_error("");
  if (!plan || !basis || !a || !b || !steps || !omega || !gamma || nb <= 0 || n_steps <= 0 || n_w <= 0 ||
      !(eta > 0.0)) {
    set_error("bse_haydock_vjp: invalid argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (g_WR && p->R.empty()) {
    set_error("bse_haydock_vjp: g_WR requested but bse_plan_set_R was not called");
    return BSE_EINVAL;
  }
  for (int i = 0; i < nb; ++i)
    if (steps[i] < 0 || steps[i] > n_steps) {
      set_error("bse_haydock_vjp: steps out of range");
      return BSE_EINVAL;
    }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long long N = p->N;
  const int na = p->d.n_aux;
  const int chunk = std::min<int>(p->max_nb, n_w);
  const int m = n_steps;
  Work wk;
  double *Xp, *Yp, *cy, *cyt;
  BSE_TRY(wk.get(&Xp, 16 * (size_t)N * chunk));
  BSE_TRY(wk.get(&Yp, 16 * (size_t)N * chunk));
  BSE_TRY(wk.get(&cy, 16 * (size_t)m * chunk));
  BSE_TRY(wk.get(&cyt, 16 * (size_t)m * chunk));
  double* gq = (double*)g_Wq;
  if (!gq && g_WR) {
    if (!p->gq_acc) BSE_TRY(plan_alloc(p, (void**)&p->gq_acc, 16 * (size_t)p->Nk * na * na));
    gq = p->gq_acc;
  }
  const bool want_w = gq != nullptr;
  if (want_w) BSE_TRY(zero_fill(gq, 16 * (size_t)p->Nk * na * na, st));
  if (g_eps) BSE_TRY(zero_fill(g_eps, 8 * (size_t)p->Nk * p->nbnd, st));
  const double pref = 1.0 / (M_PI * (double)p->Nk);
  std::vector<cd> sy((size_t)m * chunk), syt((size_t)m * chunk), col(m);
  for (int ch = 0; ch < nb; ++ch) {
    const int ns = steps[ch];
    if (ns <= 0) continue;
    const double* ac = a + (size_t)ch * m;
    const double* bc = b + (size_t)ch * (m + 1);
    for (int w0 = 0; w0 < n_w; w0 += chunk) {
      const int nw = std::min(chunk, n_w - w0);
      for (int iw = 0; iw < nw; ++iw) {
        const double wv = omega[w0 + iw];
        const double gm = gamma[(size_t)ch * n_w + w0 + iw];
        small::tridiag_resolvent(ns, ac, bc, bc[0], cd(wv, eta), col.data());
        for (int j = 0; j < ns; ++j) sy[(size_t)j * nw + iw] = col[j];
        small::tridiag_resolvent(ns, ac, bc, bc[0], cd(wv, -eta), col.data());
        const cd f = cd(0.0, -gm * pref);  // Ybar = -(i gamma / (pi N_k)) yt
        for (int j = 0; j < ns; ++j) syt[(size_t)j * nw + iw] = f * col[j];
      }
      BSE_HIP(hipMemcpyAsync(cy, sy.data(), 16 * (size_t)ns * nw, hipMemcpyHostToDevice, st));
      BSE_HIP(hipMemcpyAsync(cyt, syt.data(), 16 * (size_t)ns * nw, hipMemcpyHostToDevice, st));
      for (int which = 0; which < 2; ++which) {
        GemmArgs g;  // out[I][w] = sum_j basis[ch][j][I] coef[j][w]
        g.M = (int)N;
        g.N = nw;
        g.K = ns;
        g.A = (const double*)basis + 2 * (long long)ch * m * N;
        g.a_si = 1;
        g.a_sk = N;
        g.B = which == 0 ? cy : cyt;
        g.b_sk = nw;
        g.b_sj = 1;
        g.C = which == 0 ? Xp : Yp;
        g.c_si = nw;
        g.c_sj = 1;
        BSE_TRY(cgemm(g, AR_F64, true, true, st));
      }
      if (g_eps) BSE_TRY(adjoint_eps(p, Yp, Xp, nw, g_eps, true, st));
      if (want_w) BSE_TRY(adjoint_direct(p, Yp, Xp, nw, gq, true, st));
      // the host coefficient buffers are reused by the next chunk
      BSE_HIP(hipStreamSynchronize(st));
    }
  }
  if (g_WR) {
    const std::vector<double> q = plan_kfrac(p);
    BSE_TRY(interp_adjoint(na, (int)p->wR.size(), p->R.data(), p->wR.data(), p->Nk, q.data(), gq,
                           (double*)g_WR, st));
  }
  return BSE_OK;
}

// ---------------------------------------------------------------------------
// Lowest positive excitations of the full BSE.  With J = diag(I, -I) and
// M = J H = [[A, B], [B*, A*]] positive definite, H z = Omega z is the
// Hermitian-definite pencil J z = (1/Omega) M z, and the smallest positive
// Omega belong to its largest eigenvalues: block LOBPCG on that pencil, with
// Rayleigh-Ritz of S^H J S against S^H M S = S^H J (H S) (one full apply per
// block and iteration), the preconditioner 1 / max(d - Omega, tau) on the X part
// and -1 / (d + Omega) on the Y part (the inverse of diag(d, -d) - Omega, d the
// transition energies).
// ---------------------------------------------------------------------------
namespace bse {
namespace {

// out = J in for blocks [2N][nb] (rows N.. negated)
__global__ void jflip_kernel(long long N, int nb, const double* __restrict__ in, double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * N * nb) return;
  const double s = t / nb < N ? 1.0 : -1.0;
  out[2 * t] = s * in[2 * t];
  out[2 * t + 1] = s * in[2 * t + 1];
}

__global__ void full_residual_precond_kernel(long long N, int nb, int nv, int nc, const double* __restrict__ eps,
                                             const double* __restrict__ lam, const double* __restrict__ X,
                                             const double* __restrict__ HX, double* __restrict__ R,
                                             double* __restrict__ W) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * N * nb) return;
  const int j = (int)(t % nb);
  const long long I2 = t / nb;
  const bool top = I2 < N;
  const long long I = top ? I2 : I2 - N;
  const int v = (int)(I % nv);
  const long long kc = I / nv;
  const int c = (int)(kc % nc);
  const long long k = kc / nc;
  const double d = eps[k * (nv + nc) + nv + c] - eps[k * (nv + nc) + v];
  const double rr = HX[2 * t] - lam[j] * X[2 * t], ri = HX[2 * t + 1] - lam[j] * X[2 * t + 1];
  R[2 * t] = rr;
  R[2 * t + 1] = ri;
  const double tau = 0.02 * fmax(fabs(lam[j]), 1e-12);
  // (H - Omega)^-1 of the diagonal part diag(d, -d): the Y rows take -1 / (d + Omega)
  const double den = top ? fmax(d - lam[j], tau) : -(d + fmax(lam[j], 0.0));
  W[2 * t] = rr / den;
  W[2 * t + 1] = ri / den;
}

// random top block, zero bottom block: a start in the positive branch (x^H x > 0, x^H A x > 0)
__global__ void top_only_kernel(long long N, int nb, double* __restrict__ X) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  X[2 * (N * nb + t)] = 0.0;
  X[2 * (N * nb + t) + 1] = 0.0;
}

__global__ void scale_cols_kernel(long long rows, int nb, const double* __restrict__ s, double* __restrict__ X) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * nb) return;
  const double f = s[t % nb];
  X[2 * t] *= f;
  X[2 * t + 1] *= f;
}

}  // namespace
}  // namespace bse

extern "C" bse_status bse_full_lowest(bse_plan* plan, int32_t n_block, int32_t max_iter, double tol, const void* X0,
                                      double* omega, void* xy_out, int32_t* iters, void* hip_stream) {
  set_error("");
  if (!plan || !omega || n_block <= 0 || max_iter <= 0 || !(tol > 0.0)) {
    set_error("bse_full_lowest: invalid argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  const int nb = n_block;
  if (2 * nb > p->max_nb || 3LL * nb > 2 * p->N) {
    set_error("bse_full_lowest: need 2 n_block <= max_nb and 3 n_block <= 2N");
    return BSE_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long long N = p->N, L = 2 * N;
  const size_t blk = 16 * (size_t)L * nb;
  const unsigned gL = (unsigned)((L * nb + 255) / 256);
  Work wk;
  double *X, *HX, *W, *HW, *P, *HP, *R, *T1, *T2, *JS, *JHS, *part, *gsm, *cdev, *lam;
  BSE_TRY(wk.get(&X, blk));
  BSE_TRY(wk.get(&HX, blk));
  BSE_TRY(wk.get(&W, blk));
  BSE_TRY(wk.get(&HW, blk));
  BSE_TRY(wk.get(&P, blk));
  BSE_TRY(wk.get(&HP, blk));
  BSE_TRY(wk.get(&R, blk));
  BSE_TRY(wk.get(&T1, blk));
  BSE_TRY(wk.get(&T2, blk));
  BSE_TRY(wk.get(&JS, blk));
  BSE_TRY(wk.get(&JHS, blk));
  const int nsplit = (int)std::max<long long>(1, std::min<long long>(256, L / 64));
  BSE_TRY(wk.get(&part, 16 * (size_t)(nsplit + 1) * nb * nb));
  BSE_TRY(wk.get(&gsm, 16 * (size_t)12 * nb * nb));
  BSE_TRY(wk.get(&cdev, 16 * (size_t)3 * nb * nb));
  BSE_TRY(wk.get(&lam, 8 * (size_t)nb));

  if (X0) {
    BSE_HIP(hipMemcpyAsync(X, X0, blk, hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(random_block_kernel, dim3((unsigned)((N * nb + 255) / 256)), dim3(256), 0, st, N, nb,
                       0x2607058530000002ull, X);
    hipLaunchKernelGGL(top_only_kernel, dim3((unsigned)((N * nb + 255) / 256)), dim3(256), 0, st, N, nb, X);
  }
  BSE_CHECK_LAUNCH();
  const size_t nn = (size_t)nb * nb;
  auto fetch = [&](int count, std::vector<cd>& h) -> bse_status {
    h.resize((size_t)count * nn);
    BSE_HIP(hipMemcpyAsync(h.data(), gsm, 16 * h.size(), hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    return BSE_OK;
  };
  auto put_coeffs = [&](const std::vector<cd>& c) -> bse_status {
    BSE_HIP(hipMemcpyAsync(cdev, c.data(), 16 * c.size(), hipMemcpyHostToDevice, st));
    return BSE_OK;
  };
  auto jflip = [&](const double* in, double* out) -> bse_status {
    hipLaunchKernelGGL(jflip_kernel, dim3(gL), dim3(256), 0, st, N, nb, in, out);
    BSE_CHECK_LAUNCH();
    return BSE_OK;
  };

  // Rayleigh-Ritz on the start block: S^H J S y = lambda S^H J H S y, largest lambda = 1 / smallest Omega
  BSE_TRY(bse_apply_full(plan, X, HX, nb, hip_stream));
  BSE_TRY(jflip(X, JS));
  BSE_TRY(jflip(HX, JHS));
  BSE_TRY(gram_dev(X, nb, JS, nb, L, part, nsplit, gsm, st));
  BSE_TRY(gram_dev(X, nb, JHS, nb, L, part, nsplit, gsm + 2 * nn, st));
  std::vector<cd> h, GA(nn), GB(nn), C;
  std::vector<double> w;
  BSE_TRY(fetch(2, h));
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {  // Hermitian parts (the grams are Hermitian up to rounding)
      GA[(size_t)i * nb + j] = 0.5 * (h[(size_t)i * nb + j] + std::conj(h[(size_t)j * nb + i]));
      GB[(size_t)i * nb + j] = 0.5 * (h[nn + (size_t)i * nb + j] + std::conj(h[nn + (size_t)j * nb + i]));
    }
  int rank0 = small::gen_eig_robust(nb, GA, GB, w, C, rr_threshold(p));
  if (rank0 < nb || !(w[0] > 0.0)) {
    set_error("bse_full_lowest: start block is rank deficient or not in the positive branch");
    return BSE_ESHAPE;
  }
  {
    std::vector<cd> Cr(nn);
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) Cr[(size_t)r * nb + c] = C[(size_t)r * rank0 + (rank0 - 1 - c)];
    BSE_TRY(put_coeffs(Cr));
  }
  BSE_TRY(combine(X, nb, cdev, nb, L, T1, 0, st));
  BSE_TRY(combine(HX, nb, cdev, nb, L, T2, 0, st));
  std::swap(X, T1);
  std::swap(HX, T2);
  std::vector<double> lamh(nb);
  for (int j = 0; j < nb; ++j) lamh[j] = 1.0 / w[rank0 - 1 - j];
  bool haveP = false;
  int it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    BSE_HIP(hipMemcpyAsync(lam, lamh.data(), 8 * nb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(full_residual_precond_kernel, dim3(gL), dim3(256), 0, st, N, nb, p->d.nv, p->d.nc, p->eps,
                       lam, X, HX, R, W);
    BSE_CHECK_LAUNCH();
    BSE_TRY(gram_dev(R, nb, R, nb, L, part, nsplit, gsm, st));
    BSE_TRY(gram_dev(X, nb, X, nb, L, part, nsplit, gsm + 2 * nn, st));
    BSE_TRY(fetch(2, h));
    double worst = 0.0;
    for (int j = 0; j < nb; ++j)
      worst = std::max(worst, std::sqrt(std::max(h[(size_t)j * nb + j].real(), 0.0)) /
                                  (std::max(std::fabs(lamh[j]), 1e-300) *
                                   std::sqrt(std::max(h[nn + (size_t)j * nb + j].real(), 1e-300))));
    if (worst <= tol) {
      converged = true;
      break;
    }
    BSE_TRY(bse_apply_full(plan, W, HW, nb, hip_stream));
    const double* Sb[3] = {X, W, P};
    const double* HSb[3] = {HX, HW, HP};
    const int nblk = haveP ? 3 : 2;
    int slot = 0;
    for (int j = 0; j < nblk; ++j) {
      BSE_TRY(jflip(Sb[j], JS));
      BSE_TRY(jflip(HSb[j], JHS));
      for (int i = 0; i <= j; ++i) {
        BSE_TRY(gram_dev(Sb[i], nb, JS, nb, L, part, nsplit, gsm + 2 * nn * slot, st));
        ++slot;
        BSE_TRY(gram_dev(Sb[i], nb, JHS, nb, L, part, nsplit, gsm + 2 * nn * slot, st));
        ++slot;
      }
    }
    BSE_TRY(fetch(slot, h));
    int rank = 0;
    auto solve = [&](int nbk) -> bool {
      const int n = nbk * nb;
      GA.assign((size_t)n * n, cd(0, 0));
      GB.assign((size_t)n * n, cd(0, 0));
      int s = 0;
      for (int j = 0; j < nblk; ++j)
        for (int i = 0; i <= j; ++i) {
          const cd* ga = h.data() + nn * s;
          const cd* gb = h.data() + nn * (s + 1);
          s += 2;
          if (i >= nbk || j >= nbk) continue;
          for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c) {
              const size_t ij = (size_t)(i * nb + r) * n + (j * nb + c);
              const size_t ji = (size_t)(j * nb + c) * n + (i * nb + r);
              GA[ij] = ga[(size_t)r * nb + c];
              GB[ij] = gb[(size_t)r * nb + c];
              GA[ji] = std::conj(ga[(size_t)r * nb + c]);
              GB[ji] = std::conj(gb[(size_t)r * nb + c]);
            }
        }
      for (int i = 0; i < n; ++i) {  // the diagonal of a Hermitian gram is real
        GA[(size_t)i * n + i] = GA[(size_t)i * n + i].real();
        GB[(size_t)i * n + i] = GB[(size_t)i * n + i].real();
      }
      std::vector<double> sc(n);
      for (int i = 0; i < n; ++i) sc[i] = 1.0 / std::sqrt(std::max(GB[(size_t)i * n + i].real(), 1e-300));
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          GA[(size_t)i * n + j] *= sc[i] * sc[j];
          GB[(size_t)i * n + j] *= sc[i] * sc[j];
        }
      rank = small::gen_eig_robust(n, GA, GB, w, C, rr_threshold(p));
      if (rank < nb || !(w[rank - nb] > 0.0)) return false;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < rank; ++j) C[(size_t)i * rank + j] *= sc[i];
      return true;
    };
    int used = nblk;
    if (!solve(used)) {
      used = 2;
      if (!solve(used)) {
        set_error("bse_full_lowest: basis [X, W] lost rank");
        return BSE_ESHAPE;
      }
    }
    // the nb largest pencil eigenvalues, in descending order (ascending Omega)
    std::vector<cd> all(3 * nn, cd(0, 0));
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) {
        const int col = rank - 1 - c;
        all[(size_t)r * nb + c] = C[(size_t)r * rank + col];
        all[nn + (size_t)r * nb + c] = C[(size_t)(nb + r) * rank + col];
        if (used == 3) all[2 * nn + (size_t)r * nb + c] = C[(size_t)(2 * nb + r) * rank + col];
      }
    BSE_TRY(put_coeffs(all));
    double* dcx = cdev;
    double* dcw = cdev + 2 * nn;
    double* dcp = cdev + 4 * nn;
    BSE_TRY(combine(W, nb, dcw, nb, L, T1, 0, st));
    BSE_TRY(combine(HW, nb, dcw, nb, L, T2, 0, st));
    if (used == 3) {
      BSE_TRY(combine(P, nb, dcp, nb, L, T1, 1, st));
      BSE_TRY(combine(HP, nb, dcp, nb, L, T2, 1, st));
    }
    std::swap(P, T1);
    std::swap(HP, T2);
    BSE_TRY(combine(X, nb, dcx, nb, L, T1, 0, st));
    BSE_TRY(combine(HX, nb, dcx, nb, L, T2, 0, st));
    {
      const long long n2 = 2 * L * nb;
      hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, P, T1);
      hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, n2, HP, T2);
      BSE_CHECK_LAUNCH();
    }
    std::swap(X, T1);
    std::swap(HX, T2);
    haveP = true;
    for (int j = 0; j < nb; ++j) lamh[j] = 1.0 / w[rank - 1 - j];
  }
  for (int j = 0; j < nb; ++j) omega[j] = lamh[j];
  if (iters) *iters = converged ? it : max_iter;
  if (xy_out) {
    // Ritz vectors are M-orthonormal (z^H M z = 1, so z^H J z = 1 / Omega): rescale to X^H X - Y^H Y = 1
    std::vector<double> s(nb);
    for (int j = 0; j < nb; ++j) s[j] = std::sqrt(std::max(lamh[j], 0.0));
    BSE_HIP(hipMemcpyAsync(lam, s.data(), 8 * nb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(scale_cols_kernel, dim3(gL), dim3(256), 0, st, L, nb, lam, X);
    BSE_CHECK_LAUNCH();
    BSE_HIP(hipMemcpyAsync(xy_out, X, blk, hipMemcpyDeviceToDevice, st));
  }
  BSE_HIP(hipStreamSynchronize(st));
  if (!converged) {
    set_error("bse_full_lowest: not converged within max_iter");
    return BSE_INFO_NOT_CONVERGED;
  }
  return BSE_OK;
}
