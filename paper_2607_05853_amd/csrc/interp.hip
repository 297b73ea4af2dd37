// Dual-k-mesh Fourier interpolation of the screened interaction (Sec. III.B):
//   W_q[q] = sum_R w_R W_R[R] exp(+2 pi i q.R)
// as one complex GEMM  [n_q x n_R] (phases) x [n_R x n_aux^2] (W_R)  on the FP64
// matrix cores, and its conjugate transpose for gradients.
#include "bse_internal.h"

namespace bse {
namespace {

// phase[q][r] = w_r exp(+2 pi i q.R_r); the argument q.R is reduced to [-1/2, 1/2)
// before sincospi so the phase keeps full FP64 accuracy for large |R|.
__global__ void phase_kernel(int n_q, int n_R, const double* __restrict__ q, const int* __restrict__ R,
                             const double* __restrict__ w, double* __restrict__ ph) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_q * n_R) return;
  const int iq = (int)(t / n_R), ir = (int)(t % n_R);
  double x = q[3 * iq] * R[3 * ir] + q[3 * iq + 1] * R[3 * ir + 1] + q[3 * iq + 2] * R[3 * ir + 2];
  x -= rint(x);
  double s, c;
  sincospi(2.0 * x, &s, &c);
  ph[2 * t] = w[ir] * c;
  ph[2 * t + 1] = w[ir] * s;
}

// Workspace of one interpolation: q [3 n_q] f64, R [3 n_R] int32, w [n_R] f64 and the phase table
// [n_q][n_R] c128, each at a 256-byte aligned offset.
struct Ws {
  double* q;
  int* R;
  double* w;
  double* ph;
};

size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

Ws carve(void* base, int n_q, int n_R) {
  char* b = static_cast<char*>(base);
  Ws ws;
  ws.q = reinterpret_cast<double*>(b);
  b += up256(sizeof(double) * 3 * (size_t)n_q);
  ws.R = reinterpret_cast<int*>(b);
  b += up256(sizeof(int) * 3 * (size_t)n_R);
  ws.w = reinterpret_cast<double*>(b);
  b += up256(sizeof(double) * (size_t)n_R);
  ws.ph = reinterpret_cast<double*>(b);
  return ws;
}

// the host tables go to the workspace (stream-ordered copies) and the phase kernel fills the table
bse_status make_phases(const Ws& t, int n_R, const int32_t* R, const double* w_R, int n_q, const double* q,
                       hipStream_t st) {
  BSE_HIP(hipMemcpyAsync(t.q, q, sizeof(double) * 3 * n_q, hipMemcpyHostToDevice, st));
  BSE_HIP(hipMemcpyAsync(t.R, R, sizeof(int) * 3 * n_R, hipMemcpyHostToDevice, st));
  BSE_HIP(hipMemcpyAsync(t.w, w_R, sizeof(double) * n_R, hipMemcpyHostToDevice, st));
  const long long n = (long long)n_q * n_R;
  hipLaunchKernelGGL(phase_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_q, n_R, t.q,
                     t.R, t.w, t.ph);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// a workspace allocated on the stream and freed stream-ordered after the work that uses it
struct StreamBuf {
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~StreamBuf() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

}  // namespace

size_t interp_scratch_bytes(int n_q, int n_R) {
  return up256(sizeof(double) * 3 * (size_t)n_q) + up256(sizeof(int) * 3 * (size_t)n_R) +
         up256(sizeof(double) * (size_t)n_R) + up256(sizeof(double) * 2 * (size_t)n_q * n_R);
}

bse_status interp_forward_ws(int n_aux, int n_R, const double* W_R, const int32_t* R, const double* w_R,
                             int n_q, const double* q, void* W_q, bool out_f64, void* ws, hipStream_t st) {
  const Ws t = carve(ws, n_q, n_R);
  BSE_TRY(make_phases(t, n_R, R, w_R, n_q, q, st));
  const long long a2 = (long long)n_aux * n_aux;
  GemmArgs g;
  g.M = n_q;
  g.N = (int)a2;
  g.K = n_R;
  g.A = t.ph;
  g.a_si = n_R;
  g.a_sk = 1;
  g.B = W_R;
  g.b_sj = 1;
  g.b_sk = a2;
  g.C = W_q;
  g.c_si = a2;
  g.c_sj = 1;
  return cgemm(g, AR_F64, true, out_f64, st);
}

bse_status interp_forward(int n_aux, int n_R, const double* W_R, const int32_t* R, const double* w_R,
                          int n_q, const double* q, void* W_q, bool out_f64, hipStream_t st) {
  StreamBuf buf;
  buf.st = st;
  BSE_HIP(hipMallocAsync(&buf.p, interp_scratch_bytes(n_q, n_R), st));
  return interp_forward_ws(n_aux, n_R, W_R, R, w_R, n_q, q, W_q, out_f64, buf.p, st);
}

bse_status interp_adjoint(int n_aux, int n_R, const int32_t* R, const double* w_R, int n_q,
                          const double* q, const double* g_Wq, double* g_WR, hipStream_t st) {
  StreamBuf buf;
  buf.st = st;
  BSE_HIP(hipMallocAsync(&buf.p, interp_scratch_bytes(n_q, n_R), st));
  const Ws t = carve(buf.p, n_q, n_R);
  BSE_TRY(make_phases(t, n_R, R, w_R, n_q, q, st));
  const long long a2 = (long long)n_aux * n_aux;
  GemmArgs g;
  g.M = n_R;
  g.N = (int)a2;
  g.K = n_q;
  g.A = t.ph;  // A[r][q] = conj(phase[q][r])
  g.a_si = 1;
  g.a_sk = n_R;
  g.conjA = 1;
  g.B = g_Wq;
  g.b_sj = 1;
  g.b_sk = a2;
  g.C = g_WR;
  g.c_si = a2;
  g.c_sj = 1;
  return cgemm(g, AR_F64, true, true, st);
}

}  // namespace bse
