// C ABI of the BSE library: argument validation (before any HIP call), plan
// construction and the apply / adjoint / start-vector entry points.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>

#include "bse_internal.h"

namespace bse {

namespace {
thread_local std::string g_err;
int g_alloc_count = 0;
std::string g_fail_spec;  // the value of BSE_TEST_FAIL_ALLOC the count started from
}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

bse_status dmalloc(void** p, size_t bytes) {
  *p = nullptr;
  // fault injection for tests: BSE_TEST_FAIL_ALLOC=n fails the n-th device allocation counted from the
  // first one made under that value (a new value starts the count again)
  const char* f = std::getenv("BSE_TEST_FAIL_ALLOC");
  if (g_fail_spec != (f ? f : "")) {
    g_fail_spec = f ? f : "";
    g_alloc_count = 0;
  }
  ++g_alloc_count;
  if (f && std::atoi(f) == g_alloc_count) {
    set_error("device allocation failed (BSE_TEST_FAIL_ALLOC)");
    return BSE_ENOMEM;
  }
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    return BSE_ENOMEM;
  }
  return BSE_OK;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

namespace {
bool pool_event(Plan* p, hipEvent_t* e) {
  if (!p->ev_pool.empty()) {
    *e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return true;
  }
  if (hipEventCreate(e) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}
}  // namespace

StageMark::StageMark(Plan* p_, int stage, hipStream_t s) : p(p_), st(s) {
  if (!p->timing) return;
  Plan::StageRec r{stage, nullptr, nullptr};
  if (!pool_event(p, &r.a)) return;
  if (!pool_event(p, &r.b)) {
    p->ev_pool.push_back(r.a);
    return;
  }
  (void)hipEventRecord(r.a, st);
  p->recs.push_back(r);
  idx = (int)p->recs.size() - 1;
}

StageMark::~StageMark() {
  if (idx >= 0) (void)hipEventRecord(p->recs[idx].b, st);
}

bse_status collect_stage_times(Plan* p) {
  bse_status s = BSE_OK;
  for (auto& r : p->recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p->stage_ms[r.stage] += ms;
      p->stage_n[r.stage] += 1;
    } else {
      (void)hipGetLastError();
      set_error("stage timing: event query failed");
      s = BSE_EDEVICE;
    }
    p->ev_pool.push_back(r.a);
    p->ev_pool.push_back(r.b);
  }
  p->recs.clear();
  return s;
}

std::vector<double> plan_kfrac(const Plan* p) {
  std::vector<double> q(3 * (size_t)p->Nk);
  const int n1 = p->d.nk[0], n2 = p->d.nk[1], n3 = p->d.nk[2];
  for (int k = 0; k < p->Nk; ++k) {
    q[3 * k] = (double)(k / (n2 * n3)) / n1;
    q[3 * k + 1] = (double)((k / n3) % n2) / n2;
    q[3 * k + 2] = (double)(k % n3) / n3;
  }
  return q;
}

bse_status plan_alloc(Plan* p, void** ptr, size_t bytes) {
  BSE_TRY(dmalloc(ptr, bytes));
  p->owned.push_back(DevBuf{*ptr, bytes});
  p->bytes += bytes;
  return BSE_OK;
}

namespace {

// ---------------------------------------------------------------------------
// plan-construction kernels
// ---------------------------------------------------------------------------
// rho[k][c][v][mu] = sum_t Bc[k][c][mu][t] psi[k][v][t]   (chunk of k, FP64)
// two-centre coefficients (Bv not NULL): + conj(sum_t Bv[k][v][mu][t] psi[k][nv+c][t]), the pair
// density of the reversed pair with its band indices exchanged
__global__ void rho_kernel(int kcount, int k0, int nv, int nc, int nbnd, int n_ao, int n_aux,
                           const double* __restrict__ Bc, const double* __restrict__ psi,
                           const double* __restrict__ Bv, double* __restrict__ rho) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)kcount * nc * n_aux;
  if (t >= total) return;
  const int mu = (int)(t % n_aux);
  const long long kc = t / n_aux;
  const int c = (int)(kc % nc);
  const int kl = (int)(kc / nc);
  const int k = k0 + kl;
  const double* brow = Bc + 2 * (((long long)kl * nc + c) * n_aux + mu) * n_ao;
  for (int v = 0; v < nv; ++v) {
    const double* pv = psi + 2 * ((long long)k * nbnd + v) * n_ao;
    double sr = 0, si = 0;
    for (int s = 0; s < n_ao; ++s) {
      const double ar = brow[2 * s], ai = brow[2 * s + 1], br = pv[2 * s], bi = pv[2 * s + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    if (Bv) {
      const double* vrow = Bv + 2 * (((long long)kl * nv + v) * n_aux + mu) * n_ao;
      const double* pc = psi + 2 * ((long long)k * nbnd + nv + c) * n_ao;
      double tr = 0, ti = 0;
      for (int s = 0; s < n_ao; ++s) {
        const double ar = vrow[2 * s], ai = vrow[2 * s + 1], br = pc[2 * s], bi = pc[2 * s + 1];
        tr += ar * br - ai * bi;
        ti += ar * bi + ai * br;
      }
      sr += tr;
      si -= ti;
    }
    double* o = rho + 2 * ((((long long)k * nc + c) * nv + v) * n_aux + mu);
    o[0] = sr;
    o[1] = si;
  }
}

// P[(k c v)] = sum_s conj(psi[k][nv+c][s]) psi[k][v][s]: <u_c^{k+Q}|u_v^k> with the conduction rows of psi
// at k + Q, one thread per transition
__global__ void density_kernel(long long N, int nv, int nc, int n_ao, const double* __restrict__ psi,
                               double* __restrict__ P) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= N) return;
  const int v = (int)(I % nv);
  const long long kc = I / nv;
  const int c = (int)(kc % nc);
  const long long k = kc / nc;
  const double* pc = psi + 2 * ((k * (nv + nc) + nv + c) * n_ao);
  const double* pv = psi + 2 * ((k * (nv + nc) + v) * n_ao);
  double sr = 0, si = 0;
  for (int s = 0; s < n_ao; ++s) {
    const double ar = pc[2 * s], ai = pc[2 * s + 1], br = pv[2 * s], bi = pv[2 * s + 1];
    sr += ar * br + ai * bi;
    si += ar * bi - ai * br;
  }
  P[2 * I] = sr;
  P[2 * I + 1] = si;
}

__global__ void velocity_kernel(long long N, int nv, int nc, int nb, long long Nk, const double* __restrict__ vel,
                                const double* __restrict__ eks, const double* __restrict__ pol,
                                double* __restrict__ P) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  const int b = (int)(t % nb);
  const long long I = t / nb;
  const int v = (int)(I % nv);
  const long long kc = I / nv;
  const int c = (int)(kc % nc);
  const long long k = kc / nc;
  const double de = eks[k * (nv + nc) + nv + c] - eks[k * (nv + nc) + v];
  double sr = 0, si = 0;
  for (int a = 0; a < 3; ++a) {
    const double* e = vel + 2 * (((a * Nk + k) * nc + c) * nv + v);
    sr += pol[3 * b + a] * e[0];
    si += pol[3 * b + a] * e[1];
  }
  P[2 * t] = sr / de;
  P[2 * t + 1] = si / de;
}

// two-centre halves as one FP64 GEMM of depth n_R * n_ao per k:
//   B^mu_n(k)[t] = sum_{r, s} A[k][n][(r s)] Bst[(mu t)][(r s)]
//   A[k][n][(r s)] = conj(psi_ns(k)) exp(-2 pi i k_n.R_r),   Bst[(mu t)][(r s)] = C^mu_ts(R_r)
// so that B^mu_n(k) = psi_n(k)^H C^mu(-k_n)^T with C^mu(k) = sum_R C^mu(R) exp(+2 pi i k.R)
__global__ void tc_stack_C(int nR, int na, int no, const double* __restrict__ C_R, double* __restrict__ Bst) {
  const long long n = (long long)na * no * nR * no;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(i % no);
    const int r = (int)((i / no) % nR);
    const long long row = i / ((long long)no * nR);  // mu * no + t
    const int mu = (int)(row / no), t = (int)(row % no);
    Bst[2 * i] = C_R[(((long long)r * na + mu) * no + t) * no + s];
    Bst[2 * i + 1] = 0.0;
  }
}

__global__ void tc_stack_psi(int kn, int k0, int Nk, int nv, int nbnd, int nR, int no, const double* __restrict__ psi,
                             const double* __restrict__ ph, double* __restrict__ A) {
  const long long n = (long long)kn * nbnd * nR * no;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(i % no);
    const int r = (int)((i / no) % nR);
    const int b = (int)((i / ((long long)no * nR)) % nbnd);
    const int k = k0 + (int)(i / ((long long)no * nR * nbnd));
    const double* ps = psi + 2 * (((long long)k * nbnd + b) * no + s);
    const double* pp = ph + 2 * (((long long)(b < nv ? 0 : 1) * Nk + k) * nR + r);
    A[2 * i] = ps[0] * pp[0] + ps[1] * pp[1];
    A[2 * i + 1] = ps[0] * pp[1] - ps[1] * pp[0];
  }
}

bool bad_ptr(const void* p) { return p == nullptr; }

bse_status validate_dims(const bse_dims* d) {
  if (!d) {
    set_error("dims is NULL");
    return BSE_EINVAL;
  }
  for (int i = 0; i < 3; ++i)
    if (d->nk[i] <= 0) {
      set_error("nk must be positive");
      return BSE_EINVAL;
    }
  if (d->n_ao <= 0 || d->nv <= 0 || d->nc <= 0 || d->n_aux <= 0) {
    set_error("n_ao, nv, nc, n_aux must be positive");
    return BSE_EINVAL;
  }
  if (!std::isfinite(d->alpha)) {
    set_error("alpha must be finite");
    return BSE_EINVAL;
  }
  const long long Nk = (long long)d->nk[0] * d->nk[1] * d->nk[2];
  if (Nk > (1 << 20) || (long long)d->nv * d->nc > 4096 || d->n_aux > 16384 || d->n_ao > 16384) {
    set_error("dimensions exceed the supported range");
    return BSE_ESHAPE;
  }
  const long long N = Nk * d->nv * d->nc;
  if (N > std::numeric_limits<int>::max() / 2) {
    set_error("transition space too large");
    return BSE_ESHAPE;
  }
  return BSE_OK;
}

bool valid_prec(int p) { return p == BSE_F64 || p == BSE_F32 || p == BSE_BF16X3; }

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// workspace bytes per q of a batch: Gv, P, T, and the conduction pair densities Mc unless the plan is
// split (the BF16x3 apply never forms them; its adjoint allocates them on first use)
size_t per_q_bytes(const Plan* p) {
  const long long Nk = p->Nk, nv = p->d.nv, nc = p->d.nc, na = p->d.n_aux;
  const size_t tc = p->two_centre ? (size_t)(p->prec == BSE_F64 ? 16 : 8) * 2 * (size_t)(Nk * (nv * nv + nc * nc) * na)
                                  : 0;
  return p->esz * (size_t)(Nk * nv * nv * na * 2 + (p->mc_direct ? Nk * nc * nc * na : 0) + Nk * nc * nc * nv * nv) +
         tc;
}

// BF16X3 conduction side: estimated time per pair of forming M_cc' (pair-density GEMM, T = M_c P^T on
// 128 x 128 tiles, M_cc' written and read once) against the B_c(k) contraction (U = B_c^T P^T on tiles
// of 64 or 128 AO rows and 128 columns holding floor(128 / n_v^2) whole q, then psi_c'(k') on the
// matrix cores), both with the tile padding they execute; 250 TFLOP/s and 4 TB/s are the measured
// orders of the kernels (16^3 / N_ao = 128: 0.42 against 1.09 us per pair; 12^3 / N_ao = 96: 0.45
// against 0.65; 8^3 / N_ao = 64: U at 0.075)
bool prefer_mc(const bse_dims& d) {
  const double na = d.n_aux, no = d.n_ao, nv = d.nv, nc = d.nc;
  auto up = [](double x, double t) { return std::ceil(x / t) * t; };
  const double t_mc = 8.0 * (na * no * nc * nc + up(nc * nc, 128) * up(nv * nv, 128) * na) / 250e12 +
                      16.0 * nc * nc * na / 4e12;
  const double cols = 128.0 / std::floor(128.0 / (nv * nv));  // tile columns per pair
  const double t_u = 8.0 * (nc * up(no, 64) * na * cols + nc * nc * no * nv * nv) / 250e12;
  return t_mc < t_u;
}

// max |A_ij - conj A_ji| and max |A_ij| (per component) over nmat complex n x n matrices, as the bit
// patterns of the non-negative doubles
__global__ void herm_check(const double* __restrict__ A, long long nmat, int n, unsigned long long* __restrict__ out) {
  double dmax = 0.0, amax = 0.0;
  const long long per = (long long)n * n;
  const long long tot = per * nmat;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    const long long m = i / per, e = i % per;
    const long long et = (e % n) * n + e / n;
    const double2 a = reinterpret_cast<const double2*>(A)[i];
    const double2 t = reinterpret_cast<const double2*>(A)[m * per + et];
    dmax = fmax(dmax, fmax(fabs(t.x - a.x), fabs(t.y + a.y)));
    amax = fmax(amax, fmax(fabs(a.x), fabs(a.y)));
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmax(dmax, __shfl_down(dmax, o));
    amax = fmax(amax, __shfl_down(amax, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(dmax));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(amax));
  }
}

// Every C^mu (k-independent coefficients; C == nullptr skips them) and Vbar Hermitian to 1e-12 of their
// largest element, checked on the device; BSE_ENOTHERM otherwise.  The direct term reads
// M^mu_v'v(k',k) as conj M^mu_vv'(k,k') and the exchange term M^nu_v'c'(k',k') as conj rho, both of which
// hold only for Hermitian C^mu, so a plan on other coefficients would apply a different operator.
bse_status check_hermitian(const void* C, const void* Vbar, const bse_dims* d, hipStream_t st) {
  unsigned long long* dout = nullptr;
  BSE_TRY(dmalloc((void**)&dout, 32));
  unsigned long long hout[4] = {0, 0, 0, 0};
  bse_status s = BSE_OK;
  if (hipMemsetAsync(dout, 0, 32, st) != hipSuccess) s = BSE_EDEVICE;
  if (s == BSE_OK && C)
    hipLaunchKernelGGL(herm_check, dim3(1024), dim3(256), 0, st, (const double*)C, (long long)d->n_aux, d->n_ao,
                       dout);
  if (s == BSE_OK)
    hipLaunchKernelGGL(herm_check, dim3(256), dim3(256), 0, st, (const double*)Vbar, 1LL, d->n_aux, dout + 2);
  if (s == BSE_OK && (hipGetLastError() != hipSuccess ||
                      hipMemcpyAsync(hout, dout, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
                      hipStreamSynchronize(st) != hipSuccess))
    s = BSE_EDEVICE;
  dfree(dout);
  if (s != BSE_OK) {
    set_error("Hermiticity check of C and Vbar failed on the device");
    return s;
  }
  double v[4];
  std::memcpy(v, hout, sizeof(v));
  if (C && !(v[0] <= 1e-12 * v[1])) {
    set_error("C^mu is not Hermitian: max |C - C^H| = " + std::to_string(v[0]) + " against max |C| = " +
              std::to_string(v[1]));
    return BSE_ENOTHERM;
  }
  if (!(v[2] <= 1e-12 * v[3])) {
    set_error("Vbar is not Hermitian: max |V - V^H| = " + std::to_string(v[2]) + " against max |V| = " +
              std::to_string(v[3]));
    return BSE_ENOTHERM;
  }
  return BSE_OK;
}

void destroy_plan(Plan* p) {
  (void)collect_stage_times(p);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  p->ev_pool.clear();
  for (auto& b : p->owned) dfree(b.p);
  p->owned.clear();
}

// max |W[-q] - conj W[q]|, max |W|, and max |W[q] - W[q]^H| over all q and elements (non-negative
// doubles compared as their bit patterns)
__global__ void w_pair_check(int na, int Nk, const int* __restrict__ neg, const double* __restrict__ W,
                             unsigned long long* __restrict__ out) {
  double dmax = 0.0, wmax = 0.0, hmax = 0.0;
  const long long per_q = (long long)na * na;
  const long long n = per_q * Nk;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long q = i / per_q, e = i % per_q;
    const long long et = (e % na) * na + e / na;
    const double2 a = reinterpret_cast<const double2*>(W)[i];
    const double2 b = reinterpret_cast<const double2*>(W)[(long long)neg[q] * per_q + e];
    const double2 t = reinterpret_cast<const double2*>(W)[q * per_q + et];
    dmax = fmax(dmax, fmax(fabs(b.x - a.x), fabs(b.y + a.y)));
    wmax = fmax(wmax, fmax(fabs(a.x), fabs(a.y)));
    hmax = fmax(hmax, fmax(fabs(t.x - a.x), fabs(t.y + a.y)));
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmax(dmax, __shfl_down(dmax, o));
    wmax = fmax(wmax, __shfl_down(wmax, o));
    hmax = fmax(hmax, __shfl_down(hmax, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(dmax));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(wmax));
    atomicMax(&out[2], (unsigned long long)__double_as_longlong(hmax));
  }
}

// out block j = in block order[j] for each of nplanes planes (blocks of blk 2-byte units)
__global__ void permute_blocks(const unsigned short* __restrict__ in, unsigned short* __restrict__ out,
                               const int* __restrict__ order, int nblk, long long blk, int nplanes, long long plane) {
  const long long n = (long long)nblk * blk * nplanes;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long pl = i / ((long long)nblk * blk), r = i % ((long long)nblk * blk);
    const long long j = r / blk, e = r % blk;
    out[pl * plane + j * blk + e] = in[pl * plane + (long long)order[j] * blk + e];
  }
}

// two-centre LRI coefficients as given to plan creation
struct TwoCentreIn {
  int nR = 0;
  const int32_t* R = nullptr;   // host [nR][3]
  const double* C_R = nullptr;  // device f64 [nR][n_aux][n_ao][n_ao]
  const double* kf = nullptr;   // host f64 [2][Nk][3]: k of the valence bands, then of the conduction bands
};

bse_status build_plan(Plan* p, const bse_dims* d, const double* eps_qp, const void* psi, const void* C,
                      const TwoCentreIn* tc, const void* Vbar, const void* W_q, bse_prec prec, int max_nb,
                      uint32_t flags, hipStream_t st) {
  p->d = *d;
  p->two_centre = tc ? 1 : 0;
  p->Nk = d->nk[0] * d->nk[1] * d->nk[2];
  p->nbnd = d->nv + d->nc;
  p->nt = d->nv * d->nc;
  p->N = (long long)p->Nk * p->nt;
  p->prec = prec;
  p->max_nb = max_nb;
  p->esz = prec == BSE_F64 ? 16 : 8;
  BSE_HIP(hipGetDevice(&p->device));
  const int Nk = p->Nk, nv = d->nv, nc = d->nc, na = d->n_aux, no = d->n_ao, nbnd = p->nbnd;
  const bool f64 = prec == BSE_F64;

  // copies of the inputs
  BSE_TRY(plan_alloc(p, (void**)&p->eps, sizeof(double) * Nk * nbnd));
  BSE_HIP(hipMemcpyAsync(p->eps, eps_qp, sizeof(double) * Nk * nbnd, hipMemcpyDeviceToDevice, st));
  const long long npsi = (long long)Nk * nbnd * no;
  BSE_TRY(plan_alloc(p, (void**)&p->psi64, 16 * npsi));
  BSE_HIP(hipMemcpyAsync(p->psi64, psi, 16 * npsi, hipMemcpyDeviceToDevice, st));
  BSE_TRY(plan_alloc(p, (void**)&p->vbar, 16 * (size_t)na * na));
  BSE_HIP(hipMemcpyAsync(p->vbar, Vbar, 16 * (size_t)na * na, hipMemcpyDeviceToDevice, st));
  const long long nw = (long long)Nk * na * na;
  p->split = prec == BSE_BF16X3;
  if (f64) {
    p->psi = p->psi64;
    BSE_TRY(plan_alloc(p, &p->Wq, 16 * nw));
    BSE_HIP(hipMemcpyAsync(p->Wq, W_q, 16 * nw, hipMemcpyDeviceToDevice, st));
  } else if (p->split) {
    BSE_TRY(plan_alloc(p, &p->psi, 8 * npsi));
    BSE_TRY(split_planes(p->psi64, true, (__bf16*)p->psi, npsi, npsi, st));
    BSE_TRY(plan_alloc(p, &p->Wq, 8 * nw));
    BSE_TRY(split_planes_T(W_q, true, (__bf16*)p->Wq, Nk, na, na, nw, st));
    BSE_TRY(plan_alloc(p, (void**)&p->psi32, 8 * npsi));
    BSE_TRY(convert_c128_to_c64(p->psi64, p->psi32, npsi, st));
  } else {
    BSE_TRY(plan_alloc(p, &p->psi, 8 * npsi));
    BSE_TRY(convert_c128_to_c64(p->psi64, (float*)p->psi, npsi, st));
    BSE_TRY(plan_alloc(p, &p->Wq, 8 * nw));
    // transposed per q (W[q][nu][mu]), as for BF16X3: the W step reads columns nu contiguous in mu
    BSE_TRY(convert_c128_to_c64_T((const double*)W_q, (float*)p->Wq, Nk, na, na, st));
  }

  // halves B^mu_n(k) = psi_n(k)^H C^mu, computed in FP64; rho from the FP64 halves
  const long long hv = (long long)Nk * nv * na * no, hc = (long long)Nk * nc * na * no;
  p->ps_psi = npsi;
  p->ps_W = nw;
  p->ps_Bv = hv;
  p->ps_Bc = hc;
  // BF16X3 halves in fragment order where every pair-density product of the plan runs on the streaming
  // kernel: K = N_ao of 64 or 128, columns in whole 32-blocks, split results (k-independent coefficients,
  // and the k-major adjoint's alignment)
  p->frag_halves = (p->split && !tc && (no == 64 || no == 128) && na % 32 == 0 && (nv * nv) % 8 == 0 &&
                    na % 8 == 0 && frag_halves_enabled())
                       ? 1
                       : 0;
  BSE_TRY(plan_alloc(p, &p->Bv, p->esz * hv));
  BSE_TRY(plan_alloc(p, &p->Bc, p->esz * hc));
  if (p->split) BSE_TRY(plan_alloc(p, &p->BcT, 8 * hc));
  BSE_TRY(plan_alloc(p, (void**)&p->rho, 16 * (size_t)p->N * na));
  long long* colt = nullptr;
  {
    std::vector<long long> h((size_t)na * no);
    for (int m = 0; m < na; ++m)
      for (int t = 0; t < no; ++t) h[(size_t)m * no + t] = (long long)m * no * no + t;
    BSE_TRY(dmalloc((void**)&colt, sizeof(long long) * h.size()));
    hipError_t e = hipMemcpyAsync(colt, h.data(), sizeof(long long) * h.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      dfree(colt);
      set_error(std::string("plan tables: ") + hipGetErrorString(e));
      return BSE_EDEVICE;
    }
  }
  bse_status s = BSE_OK;
  double* tmp = nullptr;
  const long long per_k = (long long)nbnd * na * no;  // complex elements of both halves at one k
  int kc = Nk;
  if (!f64) {
    const long long budget = 1LL << 31;  // 2 GiB of FP64 staging
    kc = (int)std::max(1LL, std::min<long long>(Nk, budget / (16 * per_k)));
    s = dmalloc((void**)&tmp, 16 * (size_t)kc * per_k);
  }
  // two-centre: the stacked coefficients and phases of the half GEMM (depth n_R * n_ao)
  const int nR = tc ? tc->nR : 0;
  double* bst = nullptr;
  double* dph = nullptr;
  double* astk = nullptr;
  if (tc && s == BSE_OK) {
    s = dmalloc((void**)&bst, 16 * (size_t)na * no * nR * no);
    if (s == BSE_OK) s = dmalloc((void**)&dph, 16 * (size_t)2 * Nk * nR);
    if (s == BSE_OK) s = dmalloc((void**)&astk, 16 * (size_t)kc * nbnd * nR * no);
    if (s == BSE_OK) {
      // exp(-2 pi i k.R) with k.R reduced to [0, 1) first
      std::vector<double> hph((size_t)4 * Nk * nR);
      for (int set = 0; set < 2; ++set)
        for (int k = 0; k < Nk; ++k)
          for (int r = 0; r < nR; ++r) {
            const double* kk = tc->kf + 3 * ((size_t)set * Nk + k);
            double x = kk[0] * tc->R[3 * r] + kk[1] * tc->R[3 * r + 1] + kk[2] * tc->R[3 * r + 2];
            x -= std::floor(x);
            const size_t o = 2 * (((size_t)set * Nk + k) * nR + r);
            hph[o] = std::cos(2.0 * M_PI * x);
            hph[o + 1] = -std::sin(2.0 * M_PI * x);
          }
      hipError_t e = hipMemcpyAsync(dph, hph.data(), 8 * hph.size(), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(tc_stack_C, dim3(4096), dim3(256), 0, st, nR, na, no, tc->C_R, bst);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipStreamSynchronize(st);  // hph is released at the end of this block
      if (e != hipSuccess) {
        set_error(std::string("two-centre coefficients: ") + hipGetErrorString(e));
        s = BSE_EDEVICE;
      }
    }
  }
  for (int k0 = 0; s == BSE_OK && k0 < Nk; k0 += kc) {
    const int kn = std::min(kc, Nk - k0);
    double* dv = f64 ? (double*)p->Bv + 2LL * k0 * nv * na * no : tmp;
    double* dc = f64 ? (double*)p->Bc + 2LL * k0 * nc * na * no : tmp + 2LL * kn * nv * na * no;
    if (tc) {
      hipLaunchKernelGGL(tc_stack_psi, dim3(2048), dim3(256), 0, st, kn, k0, Nk,
                         nv, nbnd, nR, no, p->psi64, dph, astk);
      if (hipGetLastError() != hipSuccess) {
        set_error("two-centre halves: launch failed");
        s = BSE_EDEVICE;
        break;
      }
    }
    for (int part = 0; part < 2 && s == BSE_OK; ++part) {
      const int nb_ = part == 0 ? nv : nc;
      GemmArgs g;
      g.batch = kn;
      g.M = nb_;
      g.N = na * no;
      g.C = part == 0 ? dv : dc;
      g.c_sb = (long long)nb_ * na * no;
      g.c_si = (long long)na * no;
      g.c_sj = 1;
      if (tc) {
        g.K = nR * no;
        g.A = astk + 2LL * (part == 0 ? 0 : nv) * nR * no;
        g.a_sb = (long long)nbnd * nR * no;
        g.a_si = (long long)nR * no;
        g.a_sk = 1;
        g.B = bst;
        g.b_sj = (long long)nR * no;
        g.b_sk = 1;
      } else {
        g.K = no;
        g.A = (const double*)p->psi64 + 2 * ((long long)k0 * nbnd + (part == 0 ? 0 : nv)) * no;
        g.a_sb = (long long)nbnd * no;
        g.a_si = no;
        g.a_sk = 1;
        g.conjA = 1;
        g.B = C;
        g.b_tab = colt;
        g.b_sk = no;
      }
      s = cgemm(g, AR_F64, true, true, st);
    }
    if (s != BSE_OK) break;
    {
      const long long tot = (long long)kn * nc * na;
      hipLaunchKernelGGL(rho_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, kn, k0, nv, nc, nbnd,
                         no, na, dc, p->psi64, tc ? dv : nullptr, p->rho);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        set_error(std::string("rho kernel: ") + hipGetErrorString(e));
        s = BSE_EDEVICE;
        break;
      }
    }
    if (p->split && p->frag_halves) {
      s = split_planes_frag(dv, (__bf16*)p->Bv + (long long)k0 * nv * na * no, kn, nv * na, no, hv, st);
      if (s == BSE_OK)
        s = split_planes_frag(dc, (__bf16*)p->Bc + (long long)k0 * nc * na * no, kn, nc * na, no, hc, st);
      if (s == BSE_OK)
        s = split_planes_T(dc, true, (__bf16*)p->BcT + (long long)k0 * nc * no * na, kn * nc, na, no, hc, st);
    } else if (p->split) {
      s = split_planes(dv, true, (__bf16*)p->Bv + (long long)k0 * nv * na * no, (long long)kn * nv * na * no, hv, st);
      if (s == BSE_OK)
        s = split_planes(dc, true, (__bf16*)p->Bc + (long long)k0 * nc * na * no, (long long)kn * nc * na * no, hc,
                         st);
      if (s == BSE_OK)
        s = split_planes_T(dc, true, (__bf16*)p->BcT + (long long)k0 * nc * no * na, kn * nc, na, no, hc, st);
    } else if (!f64) {
      s = convert_c128_to_c64(dv, (float*)p->Bv + 2LL * k0 * nv * na * no, (long long)kn * nv * na * no, st);
      if (s == BSE_OK)
        s = convert_c128_to_c64(dc, (float*)p->Bc + 2LL * k0 * nc * na * no, (long long)kn * nc * na * no, st);
    }
    if (!f64 && s == BSE_OK) {
      hipError_t e = hipStreamSynchronize(st);  // tmp is reused by the next chunk
      if (e != hipSuccess) {
        set_error(std::string("plan halves: ") + hipGetErrorString(e));
        s = BSE_EDEVICE;
      }
    }
  }
  {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess && s == BSE_OK) {
      set_error(std::string("plan halves: ") + hipGetErrorString(e));
      s = BSE_EDEVICE;
    }
  }
  dfree(tmp);
  dfree(colt);
  dfree(bst);
  dfree(dph);
  dfree(astk);
  if (s != BSE_OK) return s;

  // k + q table, and the q order of the pair symmetry
  {
    std::vector<int> h((size_t)Nk * Nk), neg(Nk);
    const int n1 = d->nk[0], n2 = d->nk[1], n3 = d->nk[2];
    for (int k = 0; k < Nk; ++k) {
      const int a1 = k / (n2 * n3), a2 = (k / n3) % n2, a3 = k % n3;
      for (int q = 0; q < Nk; ++q) {
        const int b1 = q / (n2 * n3), b2 = (q / n3) % n2, b3 = q % n3;
        h[(size_t)k * Nk + q] = (((a1 + b1) % n1) * n2 + (a2 + b2) % n2) * n3 + (a3 + b3) % n3;
      }
      neg[k] = (((n1 - a1) % n1) * n2 + (n2 - a2) % n2) * n3 + (n3 - a3) % n3;
    }
    BSE_TRY(plan_alloc(p, (void**)&p->kq, sizeof(int) * h.size()));
    BSE_HIP(hipMemcpyAsync(p->kq, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, st));
    if (p->two_centre) {
      std::vector<int> hi((size_t)Nk * Nk);
      for (int k = 0; k < Nk; ++k)
        for (int q = 0; q < Nk; ++q) hi[(size_t)k * Nk + q] = h[(size_t)k * Nk + neg[q]];
      BSE_TRY(plan_alloc(p, (void**)&p->kqinv, sizeof(int) * hi.size()));
      BSE_HIP(hipMemcpyAsync(p->kqinv, hi.data(), sizeof(int) * hi.size(), hipMemcpyHostToDevice, st));
      BSE_HIP(hipStreamSynchronize(st));  // hi is released at the end of this block
    }
    // self-conjugate q (q = -q on the mesh) first, then the smaller index of each pair, then partners
    std::vector<int> order;
    order.reserve(Nk);
    for (int q = 0; q < Nk; ++q)
      if (neg[q] == q) order.push_back(q);
    const int nself = (int)order.size();
    for (int q = 0; q < Nk; ++q)
      if (q < neg[q]) order.push_back(q);
    const int nhalf = (int)order.size();
    for (int j = nself; j < nhalf; ++j) order.push_back(neg[order[j]]);
    bool use = !(flags & BSE_ALL_PAIRS) && nhalf < Nk;
    if (use) {
      // W_q(-q) = conj W_q(q) elementwise, to 1e-12 of the largest element
      int* dneg = nullptr;
      unsigned long long* dout = nullptr;
      BSE_TRY(dmalloc((void**)&dneg, sizeof(int) * Nk));
      bse_status s = dmalloc((void**)&dout, 24);
      unsigned long long hout[3] = {0, 0, 0};
      if (s == BSE_OK) {
        (void)hipMemcpyAsync(dneg, neg.data(), sizeof(int) * Nk, hipMemcpyHostToDevice, st);
        (void)hipMemsetAsync(dout, 0, 24, st);
        hipLaunchKernelGGL(w_pair_check, dim3(1024), dim3(256), 0, st, na, Nk, dneg, (const double*)W_q, dout);
        (void)hipMemcpyAsync(hout, dout, 24, hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess) s = BSE_EDEVICE;
      }
      dfree(dneg);
      dfree(dout);
      BSE_TRY(s);
      double dmax, wmax, hmax;
      std::memcpy(&dmax, &hout[0], 8);
      std::memcpy(&wmax, &hout[1], 8);
      std::memcpy(&hmax, &hout[2], 8);
      use = dmax <= 1e-12 * wmax;
      // the coupling block's transpose relation D_B(k', k) = D_B(k, k')^T needs W(-q) = W(q)^T as well,
      // i.e. (with the relation above) a Hermitian W(q)
      p->b_pairs = use && hmax <= 1e-12 * wmax;
    }
    if (use) {
      std::vector<int> hp((size_t)Nk * Nk), hm((size_t)Nk * Nk);
      for (int k = 0; k < Nk; ++k)
        for (int j = 0; j < Nk; ++j) {
          hp[(size_t)k * Nk + j] = h[(size_t)k * Nk + order[j]];
          hm[(size_t)k * Nk + j] = h[(size_t)k * Nk + neg[order[j]]];
        }
      BSE_TRY(plan_alloc(p, (void**)&p->kqp, sizeof(int) * hp.size()));
      BSE_TRY(plan_alloc(p, (void**)&p->kqm, sizeof(int) * hm.size()));
      BSE_HIP(hipMemcpyAsync(p->kqp, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, st));
      BSE_HIP(hipMemcpyAsync(p->kqm, hm.data(), sizeof(int) * hm.size(), hipMemcpyHostToDevice, st));
      BSE_TRY(plan_alloc(p, (void**)&p->qord, sizeof(int) * Nk));
      BSE_HIP(hipMemcpyAsync(p->qord, order.data(), sizeof(int) * Nk, hipMemcpyHostToDevice, st));
      // the W step reads W(q) in this order: permute the plan's copy once
      int* dorder = nullptr;
      void* tmp = nullptr;
      BSE_TRY(dmalloc((void**)&dorder, sizeof(int) * Nk));
      const size_t wbytes = (p->split ? 8 : (size_t)p->esz) * (size_t)nw;
      bse_status s = dmalloc(&tmp, wbytes);
      if (s == BSE_OK) {
        (void)hipMemcpyAsync(dorder, order.data(), sizeof(int) * Nk, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(tmp, p->Wq, wbytes, hipMemcpyDeviceToDevice, st);
        // bf16 planes: 4 planes of Nk blocks of na^2 * 2 bytes; complex: one plane of na^2 * esz bytes
        const int nplanes = p->split ? 4 : 1;
        const long long blk = (long long)na * na * (p->split ? 2 : p->esz) / 2;
        hipLaunchKernelGGL(permute_blocks, dim3(4096), dim3(256), 0, st, (const unsigned short*)tmp,
                           (unsigned short*)p->Wq, dorder, Nk, blk, nplanes, blk * Nk);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
          set_error("pair symmetry: permuting W(q) failed");
          s = BSE_EDEVICE;
        }
      }
      dfree(dorder);
      dfree(tmp);
      BSE_TRY(s);
      p->herm_half = 1;
      p->nself = nself;
      p->nhalf = nhalf;
    }
    BSE_HIP(hipStreamSynchronize(st));
  }

  // conduction side of the direct term
  if (p->split) {
    const bool u_ok = (long long)nv * nv <= 128 && no <= 128;
    if (p->two_centre) {
      p->mc_direct = 1;  // the second centre puts mu on the psi_c'(k') side: no B_c(k) contraction
    } else if (flags & BSE_CONDUCTION_U) {
      p->mc_direct = 0;
    } else if (flags & BSE_CONDUCTION_MC) {
      p->mc_direct = 1;
    } else {
      p->mc_direct = (!u_ok || prefer_mc(*d)) ? 1 : 0;
    }
  }

  p->fused_wt = (p->split && p->mc_direct && nv == 8 && nc == 8 && na % 256 == 0 && Nk % 2 == 0) ? 1 : 0;

  // direct-term workspaces: at least 12 GiB, more where 16 q per batch need it and 40 % of the free
  // device memory allows (short q batches leave the pair-density tiles mostly empty)
  {
    const size_t pq = per_q_bytes(p);
    size_t budget = (size_t)12 << 30;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
      budget = std::max(budget, std::min<size_t>(16 * pq, (size_t)(0.4 * (double)free_b)));
    else
      (void)hipGetLastError();
    if (const char* e = std::getenv("BSE_WORKSPACE_GB")) budget = (size_t)(std::atof(e) * (double)(1ull << 30));
    long long qb = (long long)(budget / std::max<size_t>(pq, 1));
    if (const char* e = std::getenv("BSE_QBATCH")) qb = std::atoll(e);
    qb = std::max(1LL, std::min<long long>(qb, Nk));
    p->qb = (int)qb;
    const long long nq = qb;
    BSE_TRY(plan_alloc(p, &p->Mv, p->esz * (size_t)(nq * Nk * nv * nv * na)));
    p->ps_Mv = nq * Nk * nv * nv * na;
    p->ps_Mc = nq * Nk * nc * nc * na;
    p->ps_T = nq * Nk * nc * nc * nv * nv;
    BSE_TRY(plan_alloc(p, &p->P, p->esz * (size_t)(nq * Nk * nv * nv * na)));
    if (p->mc_direct) BSE_TRY(plan_alloc(p, &p->Mc, p->esz * (size_t)(nq * Nk * nc * nc * na)));
    BSE_TRY(plan_alloc(p, &p->T, p->esz * (size_t)(nq * Nk * nc * nc * nv * nv)));
    if (p->two_centre) {
      const size_t nn = (size_t)(f64 ? 16 : 8) * (size_t)(nq * Nk * (nv * nv + nc * nc) * na);
      BSE_TRY(plan_alloc(p, &p->Nt, nn));
      BSE_TRY(plan_alloc(p, &p->Nt2, nn));
    }
    BSE_TRY(plan_alloc(p, (void**)&p->tab_psi_v, sizeof(long long) * (size_t)(nq * Nk * nv)));
    BSE_TRY(plan_alloc(p, (void**)&p->tab_mv, sizeof(long long) * (size_t)(nq * Nk * nv)));
    BSE_TRY(plan_alloc(p, (void**)&p->tab_psi_c, sizeof(long long) * (size_t)(nq * Nk * nc)));
    BSE_TRY(plan_alloc(p, (void**)&p->tab_mc, sizeof(long long) * (size_t)(nq * Nk * nc)));
  }
  // exchange split-K: chunks of whole k points
  {
    int gk = 1;
    while (gk < Nk && (long long)(Nk / gk) > 512) {
      ++gk;
      while (Nk % gk) ++gk;
    }
    p->xsplit = Nk / gk;
    BSE_TRY(plan_alloc(p, (void**)&p->xt, 16 * (size_t)(p->xsplit + 1) * na * max_nb));
    BSE_TRY(plan_alloc(p, (void**)&p->xu, 16 * (size_t)na * max_nb));
  }
  BSE_TRY(plan_alloc(p, (void**)&p->txp, 16 * (size_t)TX_CHUNKS * p->N * max_nb));
  return BSE_OK;
}

}  // namespace
}  // namespace bse

using namespace bse;

extern "C" {

const char* bse_version(void) { return "bse-gfx950 0.1"; }

const char* bse_status_string(bse_status s) {
  switch (s) {
    case BSE_OK: return "ok";
    case BSE_EINVAL: return "invalid argument";
    case BSE_ESHAPE: return "inconsistent shape";
    case BSE_ENOMEM: return "out of device memory";
    case BSE_EDEVICE: return "HIP device error";
    case BSE_ENOTHERM: return "input not Hermitian";
    case BSE_INFO_BREAKDOWN: return "Lanczos breakdown (information)";
    case BSE_INFO_NOT_CONVERGED: return "iteration limit reached (information)";
  }
  return "unknown status";
}

const char* bse_last_error(void) { return last_error(); }

bse_status bse_interpolate_W(int32_t n_aux, int32_t n_R, const void* W_R, const int32_t* R, const double* w_R,
                             int32_t n_q, const double* q_frac, void* W_q, bse_prec out_prec, void* hip_stream) {
  set_error("");
  if (n_aux <= 0 || n_R <= 0 || n_q <= 0) {
    set_error("bse_interpolate_W: sizes must be positive");
    return BSE_EINVAL;
  }
  if (bad_ptr(W_R) || bad_ptr(R) || bad_ptr(w_R) || bad_ptr(q_frac) || bad_ptr(W_q)) {
    set_error("bse_interpolate_W: NULL pointer");
    return BSE_EINVAL;
  }
  if (!valid_prec(out_prec)) {
    set_error("bse_interpolate_W: unknown precision");
    return BSE_EINVAL;
  }
  if ((long long)n_aux * n_aux > std::numeric_limits<int>::max()) {
    set_error("bse_interpolate_W: n_aux too large");
    return BSE_ESHAPE;
  }
  return interp_forward(n_aux, n_R, (const double*)W_R, R, w_R, n_q, q_frac, W_q, out_prec == BSE_F64,
                        S(hip_stream));
}

bse_status bse_interpolate_W_adjoint(int32_t n_aux, int32_t n_R, const int32_t* R, const double* w_R, int32_t n_q,
                                     const double* q_frac, const void* g_Wq, void* g_WR, void* hip_stream) {
  set_error("");
  if (n_aux <= 0 || n_R <= 0 || n_q <= 0) {
    set_error("bse_interpolate_W_adjoint: sizes must be positive");
    return BSE_EINVAL;
  }
  if (bad_ptr(R) || bad_ptr(w_R) || bad_ptr(q_frac) || bad_ptr(g_Wq) || bad_ptr(g_WR)) {
    set_error("bse_interpolate_W_adjoint: NULL pointer");
    return BSE_EINVAL;
  }
  return interp_adjoint(n_aux, n_R, R, w_R, n_q, q_frac, (const double*)g_Wq, (double*)g_WR, S(hip_stream));
}

}  // extern "C"

namespace bse {
namespace {
bse_status plan_create(const char* fn, const bse_dims* d, const double* eps_qp, const void* psi, const void* C,
                       const TwoCentreIn* tc, const void* Vbar, const void* W_q, bse_prec prec, int32_t max_nb,
                       uint32_t flags, void* hip_stream, bse_plan** out) {
  const std::string f(fn);
  set_error("");
  if (!out) {
    set_error(f + ": out is NULL");
    return BSE_EINVAL;
  }
  *out = nullptr;
  BSE_TRY(validate_dims(d));
  if (bad_ptr(eps_qp) || bad_ptr(psi) || (!tc && bad_ptr(C)) || bad_ptr(Vbar) || bad_ptr(W_q)) {
    set_error(f + ": NULL input pointer");
    return BSE_EINVAL;
  }
  if (tc && (tc->nR <= 0 || bad_ptr(tc->R) || bad_ptr(tc->C_R) || bad_ptr(tc->kf))) {
    set_error(f + ": two-centre coefficients need n_RC > 0 and non-NULL RC, C_R and k_frac");
    return BSE_EINVAL;
  }
  if (!valid_prec(prec)) {
    set_error(f + ": unknown precision");
    return BSE_EINVAL;
  }
  if (max_nb <= 0) {
    set_error(f + ": max_nb must be positive");
    return BSE_EINVAL;
  }
  if ((long long)d->nv * d->nc * max_nb > 2048) {
    set_error(f + ": nv*nc*max_nb must not exceed 2048");
    return BSE_ESHAPE;
  }
  {
    // the direct term stages one (nc nv)^2 block and one X slice per pair in LDS
    const long long nt = (long long)d->nv * d->nc;
    if (nt * nt * 16 + nt * max_nb * 16 > 150 * 1024) {
      set_error(f + ": (nv*nc)^2 + nv*nc*max_nb too large for the LDS-staged pair block");
      return BSE_ESHAPE;
    }
  }
  if ((flags & BSE_CONDUCTION_MC) && (flags & BSE_CONDUCTION_U)) {
    set_error(f + ": BSE_CONDUCTION_MC and BSE_CONDUCTION_U exclude each other");
    return BSE_EINVAL;
  }
  if (flags & ~(BSE_CHECK_HERMITIAN | BSE_ALL_PAIRS | BSE_CONDUCTION_MC | BSE_CONDUCTION_U)) {
    set_error(f + ": unknown flags");
    return BSE_EINVAL;
  }
  if (flags & BSE_CONDUCTION_U) {
    if (prec != BSE_BF16X3) {
      set_error(f + ": BSE_CONDUCTION_U applies to BSE_BF16X3 only");
      return BSE_EINVAL;
    }
    if (tc) {
      set_error(f + ": BSE_CONDUCTION_U needs k-independent coefficients");
      return BSE_EINVAL;
    }
    if ((long long)d->nv * d->nv > 128 || d->n_ao > 128) {
      set_error(f + ": BSE_CONDUCTION_U needs nv^2 <= 128 and n_ao <= 128");
      return BSE_ESHAPE;
    }
  }
  BSE_TRY(check_hermitian(tc ? nullptr : C, Vbar, d, S(hip_stream)));
  bse_plan* h = new (std::nothrow) bse_plan();
  if (!h) {
    set_error(f + ": host allocation failed");
    return BSE_ENOMEM;
  }
  bse_status s = build_plan(&h->impl, d, eps_qp, psi, C, tc, Vbar, W_q, prec, max_nb, flags, S(hip_stream));
  if (s != BSE_OK) {
    destroy_plan(&h->impl);
    delete h;
    return s;
  }
  *out = h;
  return BSE_OK;
}
}  // namespace
}  // namespace bse

extern "C" {

bse_status bse_plan_create(const bse_dims* d, const double* eps_qp, const void* psi, const void* C,
                           const void* Vbar, const void* W_q, bse_prec prec, int32_t max_nb, uint32_t flags,
                           void* hip_stream, bse_plan** out) {
  return bse::plan_create("bse_plan_create", d, eps_qp, psi, C, nullptr, Vbar, W_q, prec, max_nb, flags, hip_stream,
                          out);
}

bse_status bse_plan_create_2c(const bse_dims* d, const double* eps_qp, const void* psi, int32_t n_RC,
                              const int32_t* RC, const double* C_R, const double* k_frac, const void* Vbar,
                              const void* W_q, bse_prec prec, int32_t max_nb, uint32_t flags, void* hip_stream,
                              bse_plan** out) {
  bse::TwoCentreIn tc;
  tc.nR = n_RC;
  tc.R = RC;
  tc.C_R = C_R;
  tc.kf = k_frac;
  return bse::plan_create("bse_plan_create_2c", d, eps_qp, psi, nullptr, &tc, Vbar, W_q, prec, max_nb, flags,
                          hip_stream, out);
}

bse_status bse_plan_pairs(const bse_plan* plan, int64_t* formed, int64_t* total) {
  if (!plan || bad_ptr(formed) || bad_ptr(total)) {
    set_error("bse_plan_pairs: NULL argument");
    return BSE_EINVAL;
  }
  const Plan& p = plan->impl;
  *formed = p.herm_half ? p.nhalf : p.Nk;
  *total = p.Nk;
  return BSE_OK;
}

bse_status bse_plan_conduction(const bse_plan* plan, int32_t* forms_mc) {
  if (!plan || bad_ptr(forms_mc)) {
    set_error("bse_plan_conduction: NULL argument");
    return BSE_EINVAL;
  }
  *forms_mc = plan->impl.mc_direct;
  return BSE_OK;
}

bse_status bse_plan_fused(const bse_plan* plan, int32_t* fused) {
  if (!plan || bad_ptr(fused)) {
    set_error("bse_plan_fused: NULL argument");
    return BSE_EINVAL;
  }
  *fused = (plan->impl.fused_wt && fused_wstep_enabled()) ? 1 : 0;
  return BSE_OK;
}

bse_status bse_plan_frag(const bse_plan* plan, int32_t* frag) {
  if (!plan || bad_ptr(frag)) {
    set_error("bse_plan_frag: NULL argument");
    return BSE_EINVAL;
  }
  *frag = plan->impl.frag_halves ? 1 : 0;
  return BSE_OK;
}

bse_status bse_plan_destroy(bse_plan* plan) {
  if (!plan) return BSE_OK;
  destroy_plan(&plan->impl);
  delete plan;
  return BSE_OK;
}

bse_status bse_plan_set_R(bse_plan* plan, int32_t n_R, const int32_t* R, const double* w_R) {
  set_error("");
  if (!plan || n_R <= 0 || bad_ptr(R) || bad_ptr(w_R)) {
    set_error("bse_plan_set_R: invalid argument");
    return BSE_EINVAL;
  }
  plan->impl.R.assign(R, R + 3 * (size_t)n_R);
  plan->impl.wR.assign(w_R, w_R + n_R);
  return BSE_OK;
}

bse_status bse_plan_set_eps(bse_plan* plan, const double* eps_qp, void* hip_stream) {
  set_error("");
  if (!plan || bad_ptr(eps_qp)) {
    set_error("bse_plan_set_eps: invalid argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  BSE_HIP(hipMemcpyAsync(p->eps, eps_qp, sizeof(double) * p->Nk * p->nbnd, hipMemcpyDeviceToDevice,
                         S(hip_stream)));
  return BSE_OK;
}

bse_status bse_plan_bytes(const bse_plan* plan, uint64_t* bytes) {
  if (!plan || !bytes) {
    set_error("bse_plan_bytes: invalid argument");
    return BSE_EINVAL;
  }
  *bytes = plan->impl.bytes;
  return BSE_OK;
}

bse_status bse_plan_set_timing(bse_plan* plan, int enable) {
  set_error("");
  if (!plan) {
    set_error("bse_plan_set_timing: NULL plan");
    return BSE_EINVAL;
  }
  plan->impl.timing = enable != 0;
  return BSE_OK;
}

bse_status bse_plan_stage_times(bse_plan* plan, double* ms, int64_t* launches, int reset) {
  set_error("");
  if (!plan || !ms || !launches) {
    set_error("bse_plan_stage_times: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  bse_status s = collect_stage_times(p);
  for (int i = 0; i < BSE_NSTAGES; ++i) {
    ms[i] = p->stage_ms[i];
    launches[i] = p->stage_n[i];
    if (reset) {
      p->stage_ms[i] = 0;
      p->stage_n[i] = 0;
    }
  }
  return s;
}

bse_status bse_apply(bse_plan* plan, const void* X, void* Y, int32_t nb, void* hip_stream) {
  set_error("");
  if (!plan || bad_ptr(X) || bad_ptr(Y)) {
    set_error("bse_apply: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || nb > p->max_nb) {
    set_error("bse_apply: nb must be in [1, max_nb]");
    return BSE_EINVAL;
  }
  if (X == Y) {
    set_error("bse_apply: X and Y must not alias");
    return BSE_EINVAL;
  }
  hipStream_t st = S(hip_stream);
  BSE_TRY(apply_diag(p, (const double*)X, (double*)Y, nb, st));
  BSE_TRY(apply_exchange(p, (const double*)X, (double*)Y, nb, st));
  BSE_TRY(apply_direct(p, (const double*)X, (double*)Y, nb, st));
  return BSE_OK;
}

bse_status bse_apply_adjoint(bse_plan* plan, const void* Ybar, const void* X, int32_t nb, void* g_WR, void* g_Wq,
                             double* g_eps, void* hip_stream) {
  set_error("");
  if (!plan || bad_ptr(Ybar) || bad_ptr(X)) {
    set_error("bse_apply_adjoint: NULL argument");
    return BSE_EINVAL;
  }
  Plan* p = &plan->impl;
  if (nb <= 0 || nb > p->max_nb) {
    set_error("bse_apply_adjoint: nb must be in [1, max_nb]");
    return BSE_EINVAL;
  }
  if (g_WR && p->R.empty()) {
    set_error("bse_apply_adjoint: g_WR requested but bse_plan_set_R was not called");
    return BSE_EINVAL;
  }
  hipStream_t st = S(hip_stream);
  if (g_eps) BSE_TRY(adjoint_eps(p, (const double*)Ybar, (const double*)X, nb, g_eps, false, st));
  if (!g_WR && !g_Wq) return BSE_OK;
  const int na = p->d.n_aux;
  double* gq = (double*)g_Wq;
  if (!gq) {
    if (!p->gq_acc) BSE_TRY(plan_alloc(p, (void**)&p->gq_acc, 16 * (size_t)p->Nk * na * na));
    gq = p->gq_acc;
  }
  BSE_TRY(adjoint_direct(p, (const double*)Ybar, (const double*)X, nb, gq, false, st));
  if (g_WR) {
    const int nR = (int)p->wR.size();
    const std::vector<double> q = plan_kfrac(p);
    BSE_TRY(interp_adjoint(na, nR, p->R.data(), p->wR.data(), p->Nk, q.data(), gq, (double*)g_WR, st));
  }
  return BSE_OK;
}

bse_status bse_density_start(const bse_plan* plan, const void* psi, void* P, void* hip_stream) {
  set_error("");
  if (!plan || bad_ptr(psi) || bad_ptr(P)) {
    set_error("bse_density_start: invalid argument");
    return BSE_EINVAL;
  }
  const Plan* p = &plan->impl;
  hipStream_t st = S(hip_stream);
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, st, p->N, p->d.nv,
                     p->d.nc, p->d.n_ao, (const double*)psi, (double*)P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("bse_density_start: ") + hipGetErrorString(e));
    return BSE_EDEVICE;
  }
  return BSE_OK;
}

bse_status bse_velocity_start(const bse_plan* plan, const void* vel, const double* eps_ks, int32_t nb,
                              const double* pol, void* P, void* hip_stream) {
  set_error("");
  if (!plan || bad_ptr(vel) || bad_ptr(eps_ks) || bad_ptr(pol) || bad_ptr(P) || nb <= 0) {
    set_error("bse_velocity_start: invalid argument");
    return BSE_EINVAL;
  }
  const Plan* p = &plan->impl;
  hipStream_t st = S(hip_stream);
  double* dpol = nullptr;
  BSE_HIP(hipMallocAsync((void**)&dpol, sizeof(double) * 3 * nb, st));
  BSE_HIP(hipMemcpyAsync(dpol, pol, sizeof(double) * 3 * nb, hipMemcpyHostToDevice, st));
  const long long n = p->N * nb;
  hipLaunchKernelGGL(velocity_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p->N, p->d.nv, p->d.nc,
                     nb, (long long)p->Nk, (const double*)vel, eps_ks, dpol, (double*)P);
  hipError_t e = hipGetLastError();
  (void)hipFreeAsync(dpol, st);
  if (e != hipSuccess) {
    set_error(std::string("bse_velocity_start: ") + hipGetErrorString(e));
    return BSE_EDEVICE;
  }
  return BSE_OK;
}

}  // extern "C"
