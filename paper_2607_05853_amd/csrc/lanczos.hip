// Haydock recurrence for the absorption spectrum: nb independent Lanczos chains
// share one block apply per step; the recurrence, the full re-orthogonalisation
// (classical Gram-Schmidt twice) and the continued fraction run in FP64 on the
// device.  Breakdown is masked per chain on the device, so the host loop never
// synchronises until the end.
#include <cmath>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr int RB = 256;  // threads per reduction block

__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[RB], sb[RB];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
}

// part[bi][blk] = sum over the block's slice of conj(x[bi][I]) y[bi][I]
__global__ void dotc_partial(long long N, const double* __restrict__ x, long long xs, const double* __restrict__ y,
                             long long ys, double* __restrict__ part) {
  const int bi = blockIdx.y, nblk = gridDim.x;
  const double* xb = x + 2 * bi * xs;
  const double* yb = y + 2 * bi * ys;
  double sr = 0, si = 0;
  for (long long I = (long long)blockIdx.x * RB + threadIdx.x; I < N; I += (long long)nblk * RB) {
    const double ar = xb[2 * I], ai = -xb[2 * I + 1], br = yb[2 * I], bi_ = yb[2 * I + 1];
    sr += ar * br - ai * bi_;
    si += ar * bi_ + ai * br;
  }
  block_sum2(sr, si);
  if (threadIdx.x == 0) {
    part[2 * ((long long)bi * nblk + blockIdx.x)] = sr;
    part[2 * ((long long)bi * nblk + blockIdx.x) + 1] = si;
  }
}

// mode 0: out[bi*ostride] = Re(sum)      mode 1: out = sqrt(Re(sum))
__global__ void dot_finalize(int nblk, const double* __restrict__ part, double* __restrict__ out, long long ostride,
                             int mode) {
  const int bi = blockIdx.x;
  double sr = 0, si = 0;
  for (int i = threadIdx.x; i < nblk; i += RB) {
    sr += part[2 * ((long long)bi * nblk + i)];
    si += part[2 * ((long long)bi * nblk + i) + 1];
  }
  block_sum2(sr, si);
  if (threadIdx.x == 0) out[bi * ostride] = mode == 1 ? sqrt(fmax(sr, 0.0)) : sr;
}

// start: q_1 = p / b_0 into the basis row 0 and the apply block
__global__ void lz_init(long long N, int nb, int m, const double* __restrict__ P, const double* __restrict__ b,
                        double* __restrict__ basis, double* __restrict__ Qcur, int* __restrict__ active,
                        int* __restrict__ steps) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nb) {
    active[t] = b[t * (m + 1)] > 0.0 ? 1 : 0;
    steps[t] = b[t * (m + 1)] > 0.0 ? m : 0;
  }
  if (t >= N * nb) return;
  const long long I = t / nb;
  const int bi = (int)(t % nb);
  const double b0 = b[(long long)bi * (m + 1)];
  const double s = b0 > 0.0 ? 1.0 / b0 : 0.0;
  const double vr = P[2 * t] * s, vi = P[2 * t + 1] * s;
  Qcur[2 * t] = vr;
  Qcur[2 * t + 1] = vi;
  double* row = basis + 2 * ((long long)bi * m * N + I);
  row[0] = vr;
  row[1] = vi;
}

// w[bi][I] = Wblk[I][bi] (transpose the apply result into per-chain rows)
__global__ void lz_gather(long long N, int nb, const double* __restrict__ Wblk, double* __restrict__ w) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  const long long I = t / nb;
  const int bi = (int)(t % nb);
  w[2 * (bi * N + I)] = Wblk[2 * t];
  w[2 * (bi * N + I) + 1] = Wblk[2 * t + 1];
}

// w -= a_j q_j + b_{j-1} q_{j-1}
__global__ void lz_three_term(long long N, int m, int j, const double* __restrict__ a, const double* __restrict__ b,
                              const double* __restrict__ basis, double* __restrict__ w) {
  const int bi = blockIdx.y;
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const double aj = a[(long long)bi * m + (j - 1)];
  const double* qj = basis + 2 * ((long long)bi * m * N + (long long)(j - 1) * N + I);
  double* wi = w + 2 * (bi * N + I);
  double wr = wi[0] - aj * qj[0], wim = wi[1] - aj * qj[1];
  if (j > 1) {
    const double bp = b[(long long)bi * (m + 1) + (j - 1)];
    const double* qp = basis + 2 * ((long long)bi * m * N + (long long)(j - 2) * N + I);
    wr -= bp * qp[0];
    wim -= bp * qp[1];
  }
  wi[0] = wr;
  wi[1] = wim;
}

// h[bi][i] = q_i^H w for i < j   (grid: j x nb blocks)
__global__ void lz_project(long long N, int m, const double* __restrict__ basis, const double* __restrict__ w,
                           double* __restrict__ h) {
  const int i = blockIdx.x, bi = blockIdx.y;
  const double* q = basis + 2 * ((long long)bi * m * N + (long long)i * N);
  const double* wb = w + 2 * (long long)bi * N;
  double sr = 0, si = 0;
  for (long long I = threadIdx.x; I < N; I += RB) {
    const double ar = q[2 * I], ai = -q[2 * I + 1], br = wb[2 * I], bi_ = wb[2 * I + 1];
    sr += ar * br - ai * bi_;
    si += ar * bi_ + ai * br;
  }
  block_sum2(sr, si);
  if (threadIdx.x == 0) {
    h[2 * ((long long)bi * m + i)] = sr;
    h[2 * ((long long)bi * m + i) + 1] = si;
  }
}

// w -= sum_{i<j} q_i h_i
__global__ void lz_subtract(long long N, int m, int j, const double* __restrict__ basis, const double* __restrict__ h,
                            double* __restrict__ w) {
  extern __shared__ double hs[];
  const int bi = blockIdx.y;
  for (int i = threadIdx.x; i < 2 * j; i += blockDim.x) hs[i] = h[2 * (long long)bi * m + i];
  __syncthreads();
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  double sr = 0, si = 0;
  const double* q = basis + 2 * ((long long)bi * m * N + I);
  for (int i = 0; i < j; ++i) {
    const double qr = q[2 * (long long)i * N], qi = q[2 * (long long)i * N + 1];
    const double hr = hs[2 * i], hi = hs[2 * i + 1];
    sr += qr * hr - qi * hi;
    si += qr * hi + qi * hr;
  }
  w[2 * (bi * N + I)] -= sr;
  w[2 * (bi * N + I) + 1] -= si;
}

// breakdown test of step j, one thread per chain: b_j <= tol * s_j with s_j = max(|a_1|, .., |a_j|,
// b_1, .., b_{j-1}), the largest recurrence coefficient of the chain so far (kept in scale[bi]).  b_j is in
// the units of A (the q_j are unit vectors); b_0 = |p| is the start vector's size and does not enter, so the
// test does not depend on how p is scaled.  A chain that breaks down records steps = j and goes inactive.
__global__ void lz_decide(int nb, int m, int j, double tol, const double* __restrict__ a,
                          const double* __restrict__ b, double* __restrict__ scale, int* __restrict__ active,
                          int* __restrict__ steps) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= nb || !active[bi]) return;
  double sc = fmax(scale[bi], fabs(a[(long long)bi * m + j - 1]));
  if (j > 1) sc = fmax(sc, b[(long long)bi * (m + 1) + j - 1]);
  scale[bi] = sc;
  const double bj = b[(long long)bi * (m + 1) + j];
  if (!(bj > tol * sc)) {
    active[bi] = 0;
    steps[bi] = j;
  }
}

// q_{j+1} = w / b_j on the chains still active after step j's test (zero on the others)
__global__ void lz_next(long long N, int nb, int m, int j, const double* __restrict__ b,
                        const double* __restrict__ w, double* __restrict__ basis, double* __restrict__ Qcur,
                        const int* __restrict__ active) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  const long long I = t / nb;
  const int bi = (int)(t % nb);
  double vr = 0, vi = 0;
  if (active[bi]) {
    const double bj = b[(long long)bi * (m + 1) + j];
    vr = w[2 * (bi * N + I)] / bj;
    vi = w[2 * (bi * N + I) + 1] / bj;
  }
  Qcur[2 * t] = vr;
  Qcur[2 * t + 1] = vi;
  if (j < m) {
    double* row = basis + 2 * ((long long)bi * m * N + (long long)j * N + I);
    row[0] = vr;
    row[1] = vi;
  }
}

// continued fraction, one thread per (chain, frequency)
__global__ void cont_frac(int nb, int m, int n_w, const double* __restrict__ a, const double* __restrict__ b,
                          const int* __restrict__ steps, const double* __restrict__ omega, double eta, double scale,
                          double* __restrict__ S) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * n_w) return;
  const int bi = t / n_w, iw = t % n_w;
  const int n = steps[bi];
  if (n <= 0) {
    S[t] = 0.0;
    return;
  }
  const double zr = omega[iw], zi = eta;
  const double* ab = a + (long long)bi * m;
  const double* bb = b + (long long)bi * (m + 1);
  double gr = zr - ab[n - 1], gi = zi;
  for (int j = n - 1; j >= 1; --j) {
    const double den = gr * gr + gi * gi;
    const double b2 = bb[j] * bb[j];
    // g = z - a_j - b_j^2 / g
    const double qr = b2 * gr / den, qi = -b2 * gi / den;
    gr = zr - ab[j - 1] - qr;
    gi = zi - qi;
  }
  const double den = gr * gr + gi * gi;
  const double fi = -bb[0] * bb[0] * gi / den;  // Im(b0^2 / g)
  S[t] = -fi * scale;
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" bse_status bse_haydock_spectrum(bse_plan* plan, const void* P, int32_t nb, int32_t n_steps,
                                           const double* omega, int32_t n_w, double eta, double* S, double* a,
                                           double* b, int32_t* steps_done, void* basis_out, void* hip_stream) {
  set_error("");
  if (!plan || !P || !omega || !S || !a || !b || !steps_done) {
    set_error("bse_haydock_spectrum: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || nb > p->max_nb || n_steps <= 0 || n_w <= 0 || !(eta > 0.0)) {
    set_error("bse_haydock_spectrum: need 1 <= nb <= max_nb, n_steps > 0, n_w > 0, eta > 0");
    return BSE_EINVAL;
  }
  if ((long long)n_steps > p->N) {
    set_error("bse_haydock_spectrum: n_steps exceeds the dimension");
    return BSE_ESHAPE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const long long N = p->N;
  const int m = n_steps;
  const double tol = 1e-12;
  const int nblk = (int)std::min<long long>(1024, (N + RB - 1) / RB);

  struct Bufs {
    double *basis = nullptr, *Q = nullptr, *Wb = nullptr, *w = nullptr, *da = nullptr, *db = nullptr, *h = nullptr,
           *part = nullptr, *dom = nullptr, *dS = nullptr, *scl = nullptr;
    int *act = nullptr, *stp = nullptr;
    bool own_basis = false;
    ~Bufs() {
      if (own_basis) dfree(basis);
      dfree(Q);
      dfree(Wb);
      dfree(w);
      dfree(da);
      dfree(db);
      dfree(h);
      dfree(part);
      dfree(dom);
      dfree(dS);
      dfree(scl);
      dfree(act);
      dfree(stp);
    }
  } B;
  if (basis_out) {
    B.basis = (double*)basis_out;
  } else {
    BSE_TRY(dmalloc((void**)&B.basis, 16 * (size_t)nb * m * N));
    B.own_basis = true;
  }
  BSE_TRY(dmalloc((void**)&B.Q, 16 * (size_t)N * nb));
  BSE_TRY(dmalloc((void**)&B.Wb, 16 * (size_t)N * nb));
  BSE_TRY(dmalloc((void**)&B.w, 16 * (size_t)N * nb));
  BSE_TRY(dmalloc((void**)&B.da, 8 * (size_t)nb * m));
  BSE_TRY(dmalloc((void**)&B.db, 8 * (size_t)nb * (m + 1)));
  BSE_TRY(dmalloc((void**)&B.h, 16 * (size_t)nb * m));
  BSE_TRY(dmalloc((void**)&B.part, 16 * (size_t)nb * nblk));
  BSE_TRY(dmalloc((void**)&B.dom, 8 * (size_t)n_w));
  BSE_TRY(dmalloc((void**)&B.dS, 8 * (size_t)nb * n_w));
  BSE_TRY(dmalloc((void**)&B.scl, 8 * (size_t)nb));
  BSE_TRY(dmalloc((void**)&B.act, sizeof(int) * nb));
  BSE_TRY(dmalloc((void**)&B.stp, sizeof(int) * nb));
  BSE_TRY(zero_fill(B.da, 8 * (size_t)nb * m, st));
  BSE_TRY(zero_fill(B.db, 8 * (size_t)nb * (m + 1), st));
  BSE_TRY(zero_fill(B.scl, 8 * (size_t)nb, st));
  BSE_HIP(hipMemcpyAsync(B.dom, omega, 8 * (size_t)n_w, hipMemcpyHostToDevice, st));

  const unsigned gN = (unsigned)((N * nb + 255) / 256);
  const dim3 gV((unsigned)((N + 255) / 256), nb);
  // b_0 = |p|   (P is [N][nb]: chain stride 1, element stride nb -> gather first)
  hipLaunchKernelGGL(lz_gather, dim3(gN), dim3(256), 0, st, N, nb, (const double*)P, B.w);
  hipLaunchKernelGGL(dotc_partial, dim3(nblk, nb), dim3(RB), 0, st, N, B.w, N, B.w, N, B.part);
  hipLaunchKernelGGL(dot_finalize, dim3(nb), dim3(RB), 0, st, nblk, B.part, B.db, (long long)(m + 1), 1);
  hipLaunchKernelGGL(lz_init, dim3(gN), dim3(256), 0, st, N, nb, m, (const double*)P, B.db, B.basis, B.Q, B.act,
                     B.stp);
  BSE_CHECK_LAUNCH();
  for (int j = 1; j <= m; ++j) {
    BSE_TRY(bse_apply(plan, B.Q, B.Wb, nb, hip_stream));
    StageMark sm_(p, BSE_STAGE_LANCZOS, st);
    hipLaunchKernelGGL(lz_gather, dim3(gN), dim3(256), 0, st, N, nb, B.Wb, B.w);
    // a_j = Re q_j^H w
    hipLaunchKernelGGL(dotc_partial, dim3(nblk, nb), dim3(RB), 0, st, N, B.basis + 2 * (long long)(j - 1) * N,
                       (long long)m * N, B.w, N, B.part);
    hipLaunchKernelGGL(dot_finalize, dim3(nb), dim3(RB), 0, st, nblk, B.part, B.da + (j - 1), (long long)m, 0);
    hipLaunchKernelGGL(lz_three_term, gV, dim3(256), 0, st, N, m, j, B.da, B.db, B.basis, B.w);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(lz_project, dim3(j, nb), dim3(RB), 0, st, N, m, B.basis, B.w, B.h);
      hipLaunchKernelGGL(lz_subtract, gV, dim3(256), 16 * (size_t)j, st, N, m, j, B.basis, B.h, B.w);
    }
    hipLaunchKernelGGL(dotc_partial, dim3(nblk, nb), dim3(RB), 0, st, N, B.w, N, B.w, N, B.part);
    hipLaunchKernelGGL(dot_finalize, dim3(nb), dim3(RB), 0, st, nblk, B.part, B.db + j, (long long)(m + 1), 1);
    hipLaunchKernelGGL(lz_decide, dim3((nb + 63) / 64), dim3(64), 0, st, nb, m, j, tol, B.da, B.db, B.scl, B.act,
                       B.stp);
    hipLaunchKernelGGL(lz_next, dim3(gN), dim3(256), 0, st, N, nb, m, j, B.db, B.w, B.basis, B.Q, B.act);
    BSE_CHECK_LAUNCH();
  }
  {
    const int n = nb * n_w;
    hipLaunchKernelGGL(cont_frac, dim3((n + 255) / 256), dim3(256), 0, st, nb, m, n_w, B.da, B.db, B.stp, B.dom, eta,
                       1.0 / (M_PI * (double)p->Nk), B.dS);
    BSE_CHECK_LAUNCH();
  }
  BSE_HIP(hipMemcpyAsync(S, B.dS, 8 * (size_t)nb * n_w, hipMemcpyDeviceToHost, st));
  BSE_HIP(hipMemcpyAsync(a, B.da, 8 * (size_t)nb * m, hipMemcpyDeviceToHost, st));
  BSE_HIP(hipMemcpyAsync(b, B.db, 8 * (size_t)nb * (m + 1), hipMemcpyDeviceToHost, st));
  BSE_HIP(hipMemcpyAsync(steps_done, B.stp, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
  BSE_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nb; ++i)
    if (steps_done[i] < m) return BSE_INFO_BREAKDOWN;
  return BSE_OK;
}

// k-offset averaging (Sec. IV.A, k-point convergence): independent Haydock spectra on shifted dense meshes,
// S = sum_j w_j S_j.  Every plan must describe the same problem sizes (they differ in their bands).
extern "C" bse_status bse_offset_spectrum(bse_plan* const* plans, const void* const* P, const double* weights,
                                          int32_t n_off, int32_t nb, int32_t n_steps, const double* omega,
                                          int32_t n_w, double eta, double* S, int32_t* steps_done,
                                          void* hip_stream) {
  set_error("");
  if (!plans || !P || !weights || !omega || !S || n_off <= 0 || nb <= 0 || n_steps <= 0 || n_w <= 0) {
    set_error("bse_offset_spectrum: NULL argument or non-positive size");
    return BSE_EINVAL;
  }
  for (int j = 0; j < n_off; ++j) {
    if (!plans[j] || !P[j] || !std::isfinite(weights[j])) {
      set_error("bse_offset_spectrum: NULL plan / start block or non-finite weight at offset " + std::to_string(j));
      return BSE_EINVAL;
    }
    const bse_dims& a = plans[0]->impl.d;
    const bse_dims& b = plans[j]->impl.d;
    if (a.nk[0] != b.nk[0] || a.nk[1] != b.nk[1] || a.nk[2] != b.nk[2] || a.n_ao != b.n_ao || a.nv != b.nv ||
        a.nc != b.nc || a.n_aux != b.n_aux) {
      set_error("bse_offset_spectrum: the plans describe different problem sizes");
      return BSE_ESHAPE;
    }
  }
  const size_t ns = (size_t)nb * n_w;
  std::vector<double> Sj(ns), a((size_t)nb * n_steps), b((size_t)nb * (n_steps + 1));
  std::vector<int32_t> steps(nb);
  for (size_t i = 0; i < ns; ++i) S[i] = 0.0;
  bool breakdown = false;
  for (int j = 0; j < n_off; ++j) {
    const bse_status s = bse_haydock_spectrum(plans[j], P[j], nb, n_steps, omega, n_w, eta, Sj.data(), a.data(),
                                              b.data(), steps.data(), nullptr, hip_stream);
    if (s != BSE_OK && s != BSE_INFO_BREAKDOWN) return s;
    breakdown = breakdown || s == BSE_INFO_BREAKDOWN;
    for (size_t i = 0; i < ns; ++i) S[i] += weights[j] * Sj[i];
    if (steps_done)
      for (int i = 0; i < nb; ++i) steps_done[(size_t)j * nb + i] = steps[i];
  }
  return breakdown ? BSE_INFO_BREAKDOWN : BSE_OK;
}

// the paper's offset set: the four classes of a 3x3x3 grid of offsets (units of the mesh spacing)
extern "C" bse_status bse_offset_set(int32_t* n, double* offsets, double* weights) {
  set_error("");
  if (!n) {
    set_error("bse_offset_set: NULL argument");
    return BSE_EINVAL;
  }
  static const double off[4][3] = {{0.0, 0.0, 0.0}, {1.0 / 3, 0.0, 0.0}, {1.0 / 3, 1.0 / 3, 0.0}, {2.0 / 3, 1.0 / 3, 0.0}};
  static const double wts[4] = {1.0 / 27, 8.0 / 27, 6.0 / 27, 12.0 / 27};
  *n = 4;
  for (int j = 0; j < 4; ++j) {
    if (offsets)
      for (int i = 0; i < 3; ++i) offsets[3 * j + i] = off[j][i];
    if (weights) weights[j] = wts[j];
  }
  return BSE_OK;
}
