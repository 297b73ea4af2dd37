// Full BSE: the coupling block B of Eq. (Hamiltonian), the full Hamiltonian
// H = [[A, B], [-B*, -A*]] applied matrix-free, and the absorption spectrum of
// Eq. (full_BSE_epsilon2) from a structure-preserving Lanczos recurrence.
//
// With J = diag(I, -I), M = J H = [[A, B], [B*, A*]] is Hermitian and, for a
// stable ground state, positive definite; H is then self-adjoint in the inner
// product <x, y>_M = x^H M y = (H x)^H J y.  Lanczos in that inner product,
// started from v = [p; p*] (p the velocity-form start vector), needs one apply
// of H per step when H q_j is kept beside every basis vector q_j; it builds a
// real symmetric tridiagonal T whose diagonal vanishes (the Krylov vectors
// alternate between the two parities of z -> [z_2*; z_1*]), so its Ritz values
// come in exact +- pairs.  The spectrum over the positive excitations,
//   S(omega) = (1/N_k) sum_S |p^H X^S - p^T Y^S|^2 L(omega - Omega_S)
//            = (1/N_k) v^H J g(H) v,   g(x) = L(omega - x) [x > 0],
// equals (1/N_k) <v, H^{-1} g(H) v>_M and is evaluated by Gauss quadrature on T:
//   S(omega) ~ (|v|_M^2 / N_k) sum_{theta_i > 0} z_i^2 L(omega - theta_i) / theta_i
// with theta_i, z_i the eigenvalues of T and the first components of its
// eigenvectors (exact once the Krylov space is invariant).
#include <algorithm>
#include <cmath>
#include <vector>

#include "bse_internal.h"
#include "small_eig.h"

namespace bse {
namespace {

constexpr int FB = 256;  // threads per reduction block

// Z[I][b] = F[off1 + I][b],  Z[I][nb + b] = conj(F[off2 + I][b])   (F: [2N][nb], Z: [N][2 nb])
__global__ void fb_pack(long long N, int nb, const double* __restrict__ F, long long off1, long long off2,
                        double* __restrict__ Z) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < N * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const long long I = t / nb;
    const int b = (int)(t % nb);
    const double* a = F + 2 * ((off1 + I) * nb + b);
    const double* c = F + 2 * ((off2 + I) * nb + b);
    double* z = Z + 2 * (I * 2 * nb);
    z[2 * b] = a[0];
    z[2 * b + 1] = a[1];
    z[2 * (nb + b)] = c[0];
    z[2 * (nb + b) + 1] = -c[1];
  }
}

// out[I][b] = RA[I][b] + RB[I][b],  out[N + I][b] = -conj(RA[I][nb + b]) - conj(RB[I][nb + b])
__global__ void fb_combine(long long N, int nb, const double* __restrict__ RA, const double* __restrict__ RB,
                           double* __restrict__ out) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < N * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const long long I = t / nb;
    const int b = (int)(t % nb);
    const double* ra = RA + 2 * (I * 2 * nb);
    const double* rb = RB + 2 * (I * 2 * nb);
    double* top = out + 2 * (I * nb + b);
    double* bot = out + 2 * ((N + I) * nb + b);
    top[0] = ra[2 * b] + rb[2 * b];
    top[1] = ra[2 * b + 1] + rb[2 * b + 1];
    bot[0] = -ra[2 * (nb + b)] - rb[2 * (nb + b)];
    bot[1] = ra[2 * (nb + b) + 1] + rb[2 * (nb + b) + 1];
  }
}

__device__ __forceinline__ void fb_block_sum(double& a) {
  __shared__ double sa[FB];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int s = FB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
    __syncthreads();
  }
  a = sa[0];
  __syncthreads();
}

// rows[bi][I] <-> block[I][bi] for vectors of length L = 2N
__global__ void fb_rows_from_block(long long L, int nb, const double* __restrict__ blk, double* __restrict__ rows) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < L * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const long long I = t / nb;
    const int bi = (int)(t % nb);
    rows[2 * (bi * L + I)] = blk[2 * t];
    rows[2 * (bi * L + I) + 1] = blk[2 * t + 1];
  }
}

__global__ void fb_block_from_rows(long long L, int nb, const double* __restrict__ rows, double* __restrict__ blk) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < L * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const long long I = t / nb;
    const int bi = (int)(t % nb);
    blk[2 * t] = rows[2 * (bi * L + I)];
    blk[2 * t + 1] = rows[2 * (bi * L + I) + 1];
  }
}

// start vectors v = [p; p*] as rows [nb][2N] and as a block [2N][nb]
__global__ void fb_start(long long N, int nb, const double* __restrict__ P, double* __restrict__ rows,
                         double* __restrict__ blk) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < N * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const long long I = t / nb;
    const int bi = (int)(t % nb);
    const double pr = P[2 * t], pi = P[2 * t + 1];
    const long long L = 2 * N;
    rows[2 * (bi * L + I)] = pr;
    rows[2 * (bi * L + I) + 1] = pi;
    rows[2 * (bi * L + N + I)] = pr;
    rows[2 * (bi * L + N + I) + 1] = -pi;
    blk[2 * (I * nb + bi)] = pr;
    blk[2 * (I * nb + bi) + 1] = pi;
    blk[2 * ((N + I) * nb + bi)] = pr;
    blk[2 * ((N + I) * nb + bi) + 1] = -pi;
  }
}

// out[bi * ostride] = Re sum_I conj(x[bi][I]) J_I y[bi][I] (J = +1 on the first N entries, -1 after);
// mode 1 stores sqrt(max(., 0)).  One block per chain.
__global__ void fb_jdot(long long N, const double* __restrict__ x, long long xs, const double* __restrict__ y,
                        long long ys, double* __restrict__ out, long long ostride, int mode) {
  const int bi = blockIdx.x;
  const double* xb = x + 2 * bi * xs;
  const double* yb = y + 2 * bi * ys;
  double s = 0.0;
  for (long long I = threadIdx.x; I < 2 * N; I += FB) {
    const double v = xb[2 * I] * yb[2 * I] + xb[2 * I + 1] * yb[2 * I + 1];
    s += I < N ? v : -v;
  }
  fb_block_sum(s);
  if (threadIdx.x == 0) out[bi * ostride] = mode == 1 ? sqrt(fmax(s, 0.0)) : s;
}

// h[bi][i] = sum_I conj(W[bi][i][I]) J_I r[bi][I]  for i < j   (grid j x nb)
__global__ void fb_project(long long N, int m, const double* __restrict__ W, const double* __restrict__ r,
                           double* __restrict__ h) {
  const int i = blockIdx.x, bi = blockIdx.y;
  const long long L = 2 * N;
  const double* w = W + 2 * ((long long)bi * m * L + (long long)i * L);
  const double* rb = r + 2 * (long long)bi * L;
  double sr = 0.0, si = 0.0;
  for (long long I = threadIdx.x; I < L; I += FB) {
    const double ar = w[2 * I], ai = -w[2 * I + 1], br = rb[2 * I], bim = rb[2 * I + 1];
    const double tr = ar * br - ai * bim, ti = ar * bim + ai * br;
    sr += I < N ? tr : -tr;
    si += I < N ? ti : -ti;
  }
  fb_block_sum(sr);
  fb_block_sum(si);
  if (threadIdx.x == 0) {
    h[2 * ((long long)bi * m + i)] = sr;
    h[2 * ((long long)bi * m + i) + 1] = si;
  }
}

// r -= sum_{i<j} Q_i h_i  (grid ceil(L/256) x nb)
__global__ void fb_subtract(long long L, int m, int j, const double* __restrict__ Q, const double* __restrict__ h,
                            double* __restrict__ r) {
  extern __shared__ double hs[];
  const int bi = blockIdx.y;
  for (int i = threadIdx.x; i < 2 * j; i += blockDim.x) hs[i] = h[2 * (long long)bi * m + i];
  __syncthreads();
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= L) return;
  double sr = 0.0, si = 0.0;
  const double* q = Q + 2 * ((long long)bi * m * L + I);
  for (int i = 0; i < j; ++i) {
    const double qr = q[2 * (long long)i * L], qi = q[2 * (long long)i * L + 1];
    sr += qr * hs[2 * i] - qi * hs[2 * i + 1];
    si += qr * hs[2 * i + 1] + qi * hs[2 * i];
  }
  r[2 * (bi * L + I)] -= sr;
  r[2 * (bi * L + I) + 1] -= si;
}

// r = W_j - a_j Q_j - b_j Q_{j-1}   (b_j couples q_{j-1} and q_j; none for j = 0)
__global__ void fb_three_term(long long L, int m, int j, const double* __restrict__ a, const double* __restrict__ b,
                              const double* __restrict__ Q, const double* __restrict__ W, double* __restrict__ r) {
  const int bi = blockIdx.y;
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= L) return;
  const double aj = a[(long long)bi * m + j];
  const long long base = (long long)bi * m * L;
  double vr = W[2 * (base + (long long)j * L + I)] - aj * Q[2 * (base + (long long)j * L + I)];
  double vi = W[2 * (base + (long long)j * L + I) + 1] - aj * Q[2 * (base + (long long)j * L + I) + 1];
  if (j > 0) {
    const double bj = b[(long long)bi * (m + 1) + j];
    vr -= bj * Q[2 * (base + (long long)(j - 1) * L + I)];
    vi -= bj * Q[2 * (base + (long long)(j - 1) * L + I) + 1];
  }
  r[2 * (bi * L + I)] = vr;
  r[2 * (bi * L + I) + 1] = vi;
}

// basis row j of Q and W: x / s and y / s per chain (s = b[bi][sidx]); a chain that fb_mark stopped, now
// or before, gets zero rows
__global__ void fb_store(long long L, int nb, int m, int j, int sidx, const double* __restrict__ b,
                         const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ Q,
                         double* __restrict__ W, const int* __restrict__ active) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < L * nb;
       t += (long long)gridDim.x * blockDim.x) {
    const int bi = (int)(t / L);
    const long long I = t % L;
    const double s = b[(long long)bi * (m + 1) + sidx];
    const bool ok = active[bi] != 0 && s > 0.0;
    const double f = ok ? 1.0 / s : 0.0;
    const long long o = 2 * ((long long)bi * m * L + (long long)j * L + I);
    Q[o] = x[2 * t] * f;
    Q[o + 1] = x[2 * t + 1] * f;
    W[o] = y[2 * t] * f;
    W[o + 1] = y[2 * t + 1] * f;
  }
}

// breakdown test, one thread per chain.  sidx = 0: the start vector (its M-norm b_0 must be positive).
// sidx >= 1: b_sidx <= tol * s with s = max(|a_0|, .., |a_{sidx-1}|, b_1, .., b_{sidx-1}), the largest
// recurrence coefficient so far (kept in scale[bi]); the coefficients are in the units of H, b_0 carries the
// start vector's size and does not enter.  A chain that stops records its step count j.
__global__ void fb_mark(int nb, int m, int j, int sidx, double tol, const double* __restrict__ a,
                        const double* __restrict__ b, double* __restrict__ scale, int* __restrict__ active,
                        int* __restrict__ steps) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= nb || !active[bi]) return;
  const double s = b[(long long)bi * (m + 1) + sidx];
  bool ok = s > 0.0;
  if (sidx > 0) {
    double sc = fmax(scale[bi], fabs(a[(long long)bi * m + sidx - 1]));
    if (sidx > 1) sc = fmax(sc, b[(long long)bi * (m + 1) + sidx - 1]);
    scale[bi] = sc;
    ok = ok && s > tol * sc;
  }
  if (!ok) {
    active[bi] = 0;
    steps[bi] = j;
  }
}

unsigned grid_of(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65536)); }

bse_status full_buffers(Plan* p) {
  // each buffer on its own, so that a call after a failed allocation completes the set
  const size_t bytes = 16 * (size_t)p->N * p->max_nb;
  if (!p->fz) BSE_TRY(plan_alloc(p, (void**)&p->fz, bytes));
  if (!p->fra) BSE_TRY(plan_alloc(p, (void**)&p->fra, bytes));
  if (!p->frb) BSE_TRY(plan_alloc(p, (void**)&p->frb, bytes));
  return BSE_OK;
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" {

bse_status bse_apply_coupling(bse_plan* plan, const void* X, void* Y, int32_t nb, void* hip_stream) {
  set_error("");
  if (!plan || !X || !Y) {
    set_error("bse_apply_coupling: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || nb > p->max_nb) {
    set_error("bse_apply_coupling: nb must be in [1, max_nb]");
    return BSE_EINVAL;
  }
  if (X == Y) {
    set_error("bse_apply_coupling: X and Y must not alias");
    return BSE_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  BSE_TRY(zero_fill(Y, 16 * (size_t)p->N * nb, st));
  BSE_TRY(apply_exchange(p, (const double*)X, (double*)Y, nb, st, true));
  BSE_TRY(apply_coupling_direct(p, (const double*)X, (double*)Y, nb, st));
  return BSE_OK;
}

bse_status bse_apply_full(bse_plan* plan, const void* XY, void* out, int32_t nb, void* hip_stream) {
  set_error("");
  if (!plan || !XY || !out) {
    set_error("bse_apply_full: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || 2 * nb > p->max_nb) {
    set_error("bse_apply_full: need 1 <= nb and 2 nb <= max_nb");
    return BSE_EINVAL;
  }
  if (XY == out) {
    set_error("bse_apply_full: input and output must not alias");
    return BSE_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  BSE_TRY(full_buffers(p));
  const long long N = p->N;
  const unsigned g = grid_of(N * nb);
  // A on [X | conj Y]
  hipLaunchKernelGGL(fb_pack, dim3(g), dim3(256), 0, st, N, nb, (const double*)XY, 0LL, N, p->fz);
  BSE_CHECK_LAUNCH();
  BSE_TRY(bse_apply(plan, p->fz, p->fra, 2 * nb, hip_stream));
  // B on [Y | conj X]
  hipLaunchKernelGGL(fb_pack, dim3(g), dim3(256), 0, st, N, nb, (const double*)XY, N, 0LL, p->fz);
  BSE_CHECK_LAUNCH();
  BSE_TRY(bse_apply_coupling(plan, p->fz, p->frb, 2 * nb, hip_stream));
  hipLaunchKernelGGL(fb_combine, dim3(g), dim3(256), 0, st, N, nb, p->fra, p->frb, (double*)out);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bse_status bse_full_spectrum(bse_plan* plan, const void* P, int32_t nb, int32_t n_steps, const double* omega,
                             int32_t n_w, double eta, double* S, double* a, double* b, int32_t* steps_done,
                             void* hip_stream) {
  set_error("");
  if (!plan || !P || !omega || !S || !a || !b || !steps_done) {
    set_error("bse_full_spectrum: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || 2 * nb > p->max_nb || n_steps < 2 || n_w <= 0 || !(eta > 0.0)) {
    set_error("bse_full_spectrum: need 1 <= nb, 2 nb <= max_nb, n_steps >= 2, n_w > 0, eta > 0");
    return BSE_EINVAL;
  }
  if ((long long)n_steps > 2 * p->N) {
    set_error("bse_full_spectrum: n_steps exceeds the dimension 2N");
    return BSE_ESHAPE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long long N = p->N, L = 2 * N;
  const int m = n_steps;
  const double tol = 1e-12;
  struct Bufs {
    double *Q = nullptr, *W = nullptr, *blk = nullptr, *hblk = nullptr, *r = nullptr, *hr = nullptr,
           *da = nullptr, *db = nullptr, *h = nullptr, *scl = nullptr;
    int *act = nullptr, *stp = nullptr;
    ~Bufs() {
      dfree(scl);
      dfree(Q);
      dfree(W);
      dfree(blk);
      dfree(hblk);
      dfree(r);
      dfree(hr);
      dfree(da);
      dfree(db);
      dfree(h);
      dfree(act);
      dfree(stp);
    }
  } B;
  BSE_TRY(dmalloc((void**)&B.Q, 16 * (size_t)nb * m * L));
  BSE_TRY(dmalloc((void**)&B.W, 16 * (size_t)nb * m * L));
  BSE_TRY(dmalloc((void**)&B.blk, 16 * (size_t)L * nb));
  BSE_TRY(dmalloc((void**)&B.hblk, 16 * (size_t)L * nb));
  BSE_TRY(dmalloc((void**)&B.r, 16 * (size_t)L * nb));
  BSE_TRY(dmalloc((void**)&B.hr, 16 * (size_t)L * nb));
  BSE_TRY(dmalloc((void**)&B.da, 8 * (size_t)nb * m));
  BSE_TRY(dmalloc((void**)&B.db, 8 * (size_t)nb * (m + 1)));
  BSE_TRY(dmalloc((void**)&B.h, 16 * (size_t)nb * m));
  BSE_TRY(dmalloc((void**)&B.scl, 8 * (size_t)nb));
  BSE_TRY(dmalloc((void**)&B.act, sizeof(int) * nb));
  BSE_TRY(dmalloc((void**)&B.stp, sizeof(int) * nb));
  BSE_TRY(zero_fill(B.da, 8 * (size_t)nb * m, st));
  BSE_TRY(zero_fill(B.db, 8 * (size_t)nb * (m + 1), st));
  BSE_TRY(zero_fill(B.scl, 8 * (size_t)nb, st));
  {
    std::vector<int> one(nb, 1), full(nb, m);
    BSE_HIP(hipMemcpyAsync(B.act, one.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    BSE_HIP(hipMemcpyAsync(B.stp, full.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    BSE_HIP(hipStreamSynchronize(st));
  }
  const unsigned gL = grid_of(L * nb);
  const dim3 gV((unsigned)((L + 255) / 256), (unsigned)nb);
  // v = [p; p*], H v, |v|_M = sqrt(Re (H v)^H J v)
  hipLaunchKernelGGL(fb_start, dim3(grid_of(N * nb)), dim3(256), 0, st, N, nb, (const double*)P, B.r, B.blk);
  BSE_CHECK_LAUNCH();
  BSE_TRY(bse_apply_full(plan, B.blk, B.hblk, nb, hip_stream));
  hipLaunchKernelGGL(fb_rows_from_block, dim3(gL), dim3(256), 0, st, L, nb, B.hblk, B.hr);
  hipLaunchKernelGGL(fb_jdot, dim3(nb), dim3(FB), 0, st, N, B.hr, L, B.r, L, B.db, (long long)(m + 1), 1);
  hipLaunchKernelGGL(fb_mark, dim3((nb + 63) / 64), dim3(64), 0, st, nb, m, 0, 0, tol, B.da, B.db, B.scl, B.act,
                     B.stp);
  hipLaunchKernelGGL(fb_store, dim3(gL), dim3(256), 0, st, L, nb, m, 0, 0, B.db, B.r, B.hr, B.Q, B.W, B.act);
  BSE_CHECK_LAUNCH();
  for (int j = 0; j < m; ++j) {
    {
      StageMark sm_(p, BSE_STAGE_LANCZOS, st);
      // a_j = Re <q_j, H q_j>_M = Re (H q_j)^H J (H q_j)
      hipLaunchKernelGGL(fb_jdot, dim3(nb), dim3(FB), 0, st, N, B.W + 2 * (long long)j * L, (long long)m * L,
                         B.W + 2 * (long long)j * L, (long long)m * L, B.da + j, (long long)m, 0);
      BSE_CHECK_LAUNCH();
      if (j == m - 1) break;
      hipLaunchKernelGGL(fb_three_term, gV, dim3(256), 0, st, L, m, j, B.da, B.db, B.Q, B.W, B.r);
      for (int pass = 0; pass < 2; ++pass) {  // <q_i, r>_M = (H q_i)^H J r for i <= j
        hipLaunchKernelGGL(fb_project, dim3(j + 1, nb), dim3(FB), 0, st, N, m, B.W, B.r, B.h);
        hipLaunchKernelGGL(fb_subtract, gV, dim3(256), 16 * (size_t)(j + 1), st, L, m, j + 1, B.Q, B.h, B.r);
      }
      hipLaunchKernelGGL(fb_block_from_rows, dim3(gL), dim3(256), 0, st, L, nb, B.r, B.blk);
      BSE_CHECK_LAUNCH();
    }
    BSE_TRY(bse_apply_full(plan, B.blk, B.hblk, nb, hip_stream));
    {
      StageMark sm_(p, BSE_STAGE_LANCZOS, st);
      hipLaunchKernelGGL(fb_rows_from_block, dim3(gL), dim3(256), 0, st, L, nb, B.hblk, B.hr);
      // b_{j+1} = |r|_M
      hipLaunchKernelGGL(fb_jdot, dim3(nb), dim3(FB), 0, st, N, B.hr, L, B.r, L, B.db + (j + 1), (long long)(m + 1), 1);
      hipLaunchKernelGGL(fb_mark, dim3((nb + 63) / 64), dim3(64), 0, st, nb, m, j + 1, j + 1, tol, B.da, B.db,
                         B.scl, B.act, B.stp);
      hipLaunchKernelGGL(fb_store, dim3(gL), dim3(256), 0, st, L, nb, m, j + 1, j + 1, B.db, B.r, B.hr, B.Q, B.W,
                         B.act);
      BSE_CHECK_LAUNCH();
    }
  }
  BSE_HIP(hipMemcpyAsync(a, B.da, 8 * (size_t)nb * m, hipMemcpyDeviceToHost, st));
  BSE_HIP(hipMemcpyAsync(b, B.db, 8 * (size_t)nb * (m + 1), hipMemcpyDeviceToHost, st));
  BSE_HIP(hipMemcpyAsync(steps_done, B.stp, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
  BSE_HIP(hipStreamSynchronize(st));
  // Gauss quadrature on the leading even-sized tridiagonal of each chain
  bool broke = false;
  for (int bi = 0; bi < nb; ++bi) {
    double* Sb = S + (long long)bi * n_w;
    for (int iw = 0; iw < n_w; ++iw) Sb[iw] = 0.0;
    int n = std::min(steps_done[bi], m);
    if (n < m) broke = true;
    n -= n % 2;
    const double b0 = b[(long long)bi * (m + 1)];
    if (n <= 0 || !(b0 > 0.0)) continue;
    std::vector<double> d(a + (long long)bi * m, a + (long long)bi * m + n), e(n > 1 ? n - 1 : 0), w, z;
    for (int i = 0; i + 1 < n; ++i) e[i] = b[(long long)bi * (m + 1) + i + 1];
    if (!small::tridiag_eig_first(n, d.data(), e.data(), w, z)) {
      set_error("bse_full_spectrum: tridiagonal eigensolver did not converge");
      return BSE_EDEVICE;
    }
    const double thr = 1e-10 * std::max(std::fabs(w.front()), std::fabs(w.back()));
    for (int i = 0; i < n; ++i) {
      if (!(w[i] > thr)) continue;
      const double f = b0 * b0 * z[i] * z[i] / (w[i] * (double)p->Nk);
      for (int iw = 0; iw < n_w; ++iw) {
        const double x = omega[iw] - w[i];
        Sb[iw] += f * (eta / M_PI) / (x * x + eta * eta);
      }
    }
  }
  return broke ? BSE_INFO_BREAKDOWN : BSE_OK;
}

}  // extern "C"
