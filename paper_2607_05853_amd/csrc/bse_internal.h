// Internal declarations of the gfx950 BSE library: plan layout, error
// plumbing and the batched complex GEMM engine shared by the stages.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bse.h"

namespace bse {

// ---------------------------------------------------------------------------
// error handling: a thread-local message, status codes, no exceptions across
// the C ABI
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error();

#define BSE_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::bse::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return BSE_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

#define BSE_CHECK_LAUNCH()                                                     \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) {                                                    \
      ::bse::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));\
      return BSE_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

#define BSE_TRY(expr)                                                          \
  do {                                                                         \
    bse_status s_ = (expr);                                                    \
    if (s_ != BSE_OK) return s_;                                               \
  } while (0)

// device allocation with a test hook: BSE_TEST_FAIL_ALLOC=n makes the n-th
// allocation of the process fail (n >= 1), so ENOMEM paths are testable.
bse_status dmalloc(void** p, size_t bytes);
void dfree(void* p);

// ---------------------------------------------------------------------------
// batched complex GEMM on the matrix cores
//   C_b[i][j] = alpha * sum_k opA(A_b[i][k]) opB(B_b[k][j])  (+ C_b[i][j] if beta)
// Offsets are in complex elements.  Row offsets of A and C and column offsets
// of B are either affine (b*sb + i*si) or read from a device table indexed by
// i (tab_pb = 0) or by b*M + i (tab_pb = 1); the K strides are uniform.
// ---------------------------------------------------------------------------
enum Arith { AR_F64 = 0, AR_F32 = 1, AR_BF16X3 = 2 };

struct GemmArgs {
  int M = 0, N = 0, K = 0, batch = 1;
  const void* A = nullptr;
  long long a_sb = 0, a_si = 0, a_sk = 0;
  const long long* a_tab = nullptr;
  int a_tab_pb = 0, conjA = 0;
  const void* B = nullptr;
  long long b_sb = 0, b_sj = 0, b_sk = 0;
  const long long* b_tab = nullptr;
  int b_tab_pb = 0, conjB = 0;
  void* C = nullptr;
  long long c_sb = 0, c_si = 0, c_sj = 0;
  const long long* c_tab = nullptr;
  int c_tab_pb = 0;
  double alpha = 1.0;
  int beta = 0;
  // plane strides (elements) of operands stored pre-split as four bf16 planes
  long long a_ps = 0, b_ps = 0, c_ps = 0;
  // set by the caller when every table offset (a_tab, b_tab) is a multiple of 8 elements
  int tab_aligned = 0;
  // k-major kernel with a c128 result: batch entry b of the product is stored at C batch c_bidx[b]
  const int* c_bidx = nullptr;
  // B pre-split in fragment order (split_planes_frag; b_sb per batch entry, b_ps per plane, column j and
  // k as that layout places them; b_sj and b_sk unused): only the streaming pair-density kernel reads it
  int b_frag = 0;
};

// in_f64: A and B are c128 (else c64); out_f64: C is c128 (else c64).
// AR_F64 requires in_f64.  AR_F32 / AR_BF16X3 require c64 inputs.
bse_status cgemm(const GemmArgs& g, Arith ar, bool in_f64, bool out_f64, hipStream_t st);
// BF16X3 on the large-tile kernel with any of A, B, C pre-split into bf16 planes
// (Re hi, Re lo, Im hi, Im lo at plane strides a_ps / b_ps / c_ps); non-split
// operands are c64 (A, B) and c64 / c128 (C, per out_f64).
bse_status cgemm_split(const GemmArgs& g, bool a_split, bool b_split, bool c_split, bool out_f64, hipStream_t st);
// BF16x3 W step and direct block in one kernel (64 rows per pair on both band sides, N_aux a multiple of
// 256): P = conj(Gv) W(q) as g describes it (A = Gv planes with conjA, B = W(q) planes, M = 64 N_k per q,
// N = K = N_aux), stays on chip, and T[b][k] = Mc[b][k] P[b][k]^T is written as c64 [b][k][64][64] (stride
// t_sb per batch entry); Mc planes at mc (stride mc_sb per batch entry, plane stride mc_ps, rows of N_aux)
bse_status wstep_dblock(const GemmArgs& g, const __bf16* mc, long long mc_sb, long long mc_ps, float* t, long long t_sb,
                        hipStream_t st);
// BSE_FUSED_WSTEP=0 in the environment selects the two GEMMs (read at every call)
bool fused_wstep_enabled();
// Fragment order of a pre-split B operand for the streaming pair-density kernel: each batch entry's
// N x K matrix (N a multiple of 32, K of 16) as [N/32][K/16][64 lanes][8], lane 32 h + c of block (jb, s)
// holding column 32 jb + c, k = 16 s + 8 h .. 16 s + 8 h + 7 -- the 16 bytes that lane passes to one 32x32x16
// MFMA, so a wave reads each fragment as one contiguous KiB.  in: c128 [batch][N][K]; out: four planes of
// batch * N * K bf16 at plane_stride.
bse_status split_planes_frag(const double* in, __bf16* out, int batch, int N, int K, long long plane_stride,
                             hipStream_t st);
// the plan stores its BF16X3 halves in fragment order when its shape allows it; BSE_FRAG_HALVES=0 in the
// environment at plan creation keeps the row order
bool frag_halves_enabled();
// split c64 / c128 arrays into four bf16 planes (util.hip); n complex elements,
// optionally transposing each of `batch` rows x cols matrices
bse_status split_planes(const void* in, bool in_f64, __bf16* out, long long n, long long plane_stride,
                        hipStream_t st);
bse_status split_planes_T(const void* in, bool in_f64, __bf16* out, int batch, int rows, int cols,
                          long long plane_stride, hipStream_t st);
// out[b][c][r] = complex64(in[b][r][c]) for batch complex128 rows x cols matrices
bse_status convert_c128_to_c64_T(const double* in, float* out, int batch, int rows, int cols, hipStream_t st);

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// q chunks of the T.X stage (each block sums its chunk; a second pass adds the chunks in order)
constexpr int TX_CHUNKS = 16;

struct Plan {
  bse_dims d{};
  int Nk = 0, nt = 0, nbnd = 0;
  long long N = 0;
  bse_prec prec = BSE_F64;
  int max_nb = 0;
  int device = 0;
  size_t esz = 16;  // bytes per complex element of the plan precision
  bool split = false;  // BF16X3: psi, halves, W_q and the valence pair densities are stored as
                       // four bf16 planes (Re hi, Re lo, Im hi, Im lo); W_q transposed per q
  long long ps_psi = 0, ps_W = 0, ps_Bv = 0, ps_Bc = 0, ps_Mv = 0, ps_Mc = 0, ps_T = 0;  // plane strides (elements)

  // FP64 data
  double* eps = nullptr;      // [Nk][nv+nc]
  double* psi64 = nullptr;    // c128 [Nk][nv+nc][n_ao]
  double* rho = nullptr;      // c128 [N][n_aux]   rho[I][mu] = M^mu_cv(k,k)
  double* vbar = nullptr;     // c128 [n_aux][n_aux]
  // plan-precision data (c128 for F64, c64 otherwise)
  void* psi = nullptr;        // [Nk][nv+nc][n_ao]
  void* Bv = nullptr;         // [Nk][nv][n_aux][n_ao]   B^mu_v(k)
  void* Bc = nullptr;         // [Nk][nc][n_aux][n_ao]   B^mu_c(k)
  void* Wq = nullptr;         // [Nk][n_aux][n_aux]
  void* BcT = nullptr;        // BF16X3 only: planes [Nk][nc][n_ao][n_aux] (B^nu_ct(k), t-major)
  float* psi32 = nullptr;     // BF16X3 only: c64 [Nk][nv+nc][n_ao]

  // q-batch workspaces of the direct term (plan precision)
  int qb = 0;                 // q values per batch
  void* Mv = nullptr;         // [qb][Nk][nv][nv][n_aux]  M^mu_{v v'}(k, k+q)  (row (v', v) after conj)
  void* Mc = nullptr;         // [qb][Nk][nc][nc][n_aux]  M^nu_{c c'}(k, k+q)
  void* P = nullptr;          // [qb][Nk][nv][nv][n_aux]
  void* T = nullptr;          // [qb][Nk][nc*nc][nv*nv]   direct block per pair
  long long* tab_psi_v = nullptr;   // [Nk][qb*nv]  row offsets of psi_v(k+q)
  long long* tab_psi_c = nullptr;   // [Nk][qb*nc]
  long long* tab_mv = nullptr;      // [Nk][qb*nv]  row offsets into Mv
  long long* tab_mc = nullptr;      // [Nk][qb*nc]
  int* kq = nullptr;                // [Nk][Nk] k + q index table (k, q) -> k'
  // pair symmetry of the apply: q order with the self-conjugate q first, then one q of each pair
  // {q, -q}, then their partners; kqp[k][j] = k + q_j, kqm[k][j] = k - q_j in that order
  int herm_half = 0, nself = 0, nhalf = 0;
  // conduction side: 1 = form M_cc' and T = M_c P^T (FP64 / FP32 always), 0 = B_c(k) contraction (BF16X3)
  int mc_direct = 1;
  int fused_wt = 0;  // the shape admits the fused W step + direct block (BF16X3, M_cc' route, n_v = n_c = 8)
  int frag_halves = 0;  // BF16X3 halves Bv, Bc stored in fragment order (split_planes_frag)
  int* kqp = nullptr;
  int* kqm = nullptr;
  int* qord = nullptr;              // [Nk] dense-mesh index of the j-th q of that order
  // two-centre LRI coefficients: the halves hold psi_n(k)^H C^mu(-k_n)^T, and every pair density is
  // the one-sided product N(k, k') plus conj N(k', k) with the band indices exchanged; Nt / Nt2 hold
  // N for the pairs of a q batch and for their reverses (GEMM output type: c128 on F64, else c64)
  int two_centre = 0;
  void* Nt = nullptr;               // [qb][Nk][nv][nv][n_aux] then [qb][Nk][nc][nc][n_aux]
  void* Nt2 = nullptr;              // same layout, pair (k + q, k) stored at slot (q, k + q)
  int* kqinv = nullptr;             // [Nk][Nk] (k, q) -> k - q, the reverse of kq

  // coupling block B of the full BSE (allocated on the first coupling apply), per pair (k, k' = k + q):
  //   Gb[c'][v][mu] = conj M^mu_{c'v}(k', k),  Pb = conj(Gb) W(q),  M2[v'][c][nu] = M^nu_{cv'}(k, k'),
  //   Tb[(v' c)][(c' v)] = sum_nu M2 Pb,  B_d X = -(1/N_k) sum_q Tb X(k')
  int b_pairs = 0;                  // 1: the coupling block forms the q of the pair-symmetric order only
  int qbB = 0;
  void* Gb = nullptr;               // [qbB][Nk][nc][nv][n_aux]
  void* Pb = nullptr;               // [qbB][Nk][nc][nv][n_aux]
  void* M2 = nullptr;               // [qbB][Nk][nv][nc][n_aux]
  void* Tb = nullptr;               // [qbB][Nk][nt][nt]
  long long ps_Gb = 0;              // plane stride of Gb, Pb and M2
  void* Btc[4] = {};                // two-centre: one-sided Gb and M2 products of the pairs and of their reverses
  long long* tabB_psi_c = nullptr;  // [Nk][qbB*nc]
  long long* tabB_psi_v = nullptr;  // [Nk][qbB*nv]
  long long* tabB_g = nullptr;      // [Nk][qbB*nc]
  long long* tabB_m2 = nullptr;     // [Nk][qbB*nv]
  // full BSE apply: packed [N][2 nb] operands and results (allocated on first use)
  double* fz = nullptr;
  double* fra = nullptr;
  double* frb = nullptr;

  // exchange / misc workspaces (FP64)
  double* xt = nullptr;       // c128 split-K partials [nsplit][n_aux][max_nb]
  double* xu = nullptr;       // c128 [n_aux][max_nb]
  int xsplit = 1;
  double* txp = nullptr;      // c128 T.X partial sums [TX_CHUNKS][N][max_nb] (one per q chunk)

  // adjoint
  std::vector<int32_t> R;
  std::vector<double> wR;
  double* gq_acc = nullptr;   // c128 [Nk][n_aux][n_aux]

  std::vector<DevBuf> owned;
  size_t bytes = 0;

  // stage timing
  struct StageRec {
    int stage;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<StageRec> recs;
  std::vector<hipEvent_t> ev_pool;   // events reused across stages (created once)
  double stage_ms[BSE_NSTAGES] = {};
  long long stage_n[BSE_NSTAGES] = {};
};

// RAII stage marker: records a start event now and the end event on destruction
// (only when the plan's timing is enabled)
struct StageMark {
  Plan* p;
  int idx = -1;
  hipStream_t st;
  StageMark(Plan* p_, int stage, hipStream_t s);
  ~StageMark();
};
bse_status collect_stage_times(Plan* p);

bse_status plan_alloc(Plan* p, void** ptr, size_t bytes);

// stage launchers (apply.hip)
bse_status apply_direct(Plan* p, const double* X, double* Y, int nb, hipStream_t st);
bse_status apply_exchange(Plan* p, const double* X, double* Y, int nb, hipStream_t st, bool transpose = false);
bse_status apply_coupling_direct(Plan* p, const double* X, double* Y, int nb, hipStream_t st);
bse_status apply_diag(Plan* p, const double* X, double* Y, int nb, hipStream_t st);
bse_status adjoint_direct(Plan* p, const double* Ybar, const double* X, int nb, double* gWq, bool acc,
                          hipStream_t st);
bse_status direct_u_b3(Plan* p, int q0, int nq, const int* kq, hipStream_t st);
bse_status adjoint_eps(Plan* p, const double* Ybar, const double* X, int nb, double* geps, bool acc,
                       hipStream_t st);
// the dense-mesh k list of a plan (fractional coordinates, host)
std::vector<double> plan_kfrac(const Plan* p);

// interpolation (interp.hip); interp_forward allocates its workspace on the stream, interp_forward_ws takes
// one of at least interp_scratch_bytes(n_q, n_R) bytes (256-byte aligned)
size_t interp_scratch_bytes(int n_q, int n_R);
bse_status interp_forward(int n_aux, int n_R, const double* W_R, const int32_t* R, const double* w_R,
                          int n_q, const double* q, void* W_q, bool out_f64, hipStream_t st);
bse_status interp_forward_ws(int n_aux, int n_R, const double* W_R, const int32_t* R, const double* w_R,
                             int n_q, const double* q, void* W_q, bool out_f64, void* ws, hipStream_t st);
bse_status interp_adjoint(int n_aux, int n_R, const int32_t* R, const double* w_R, int n_q,
                          const double* q, const double* g_Wq, double* g_WR, hipStream_t st);

// small streaming kernels (util.hip)
bse_status convert_c128_to_c64(const double* in, float* out, long long n, hipStream_t st);
bse_status zero_fill(void* p, size_t bytes, hipStream_t st);

}  // namespace bse

struct bse_plan {
  bse::Plan impl;
};
