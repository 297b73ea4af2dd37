// Batched complex GEMM on the gfx950 matrix cores.
//
// A complex product C = A B is evaluated as one real GEMM of doubled depth and
// width:  A is read as the real M x 2K matrix its interleaved storage already is
// (column 2k = Re A_ik, 2k+1 = Im A_ik) and B is expanded on the fly to the real
// 2K x 2N matrix  [[Re B, Im B], [-Im B, Re B]]  (row 2k / 2k+1, column 2j / 2j+1),
// so the real output is the interleaved complex C.  That is the 4-real-product
// form of the complex product (8 real flops per complex MAC), with no separate
// real/imaginary accumulators and a natural interleaved store.
//
//  FP64 : v_mfma_f64_16x16x4f64, FP32 : v_mfma_f32_16x16x4f32.  Each wave owns a
//         TM x TN grid of 16 x 16 real output tiles; A and B tiles are staged in
//         LDS with a one-tile register prefetch of the next K slice.
//  BF16X3: v_mfma_f32_16x16x32_bf16.  Operands are split once when staged into
//         LDS (hi = bf16(x), lo = bf16(x - hi)); every tile step issues
//         hi*hi + hi*lo + lo*hi with FP32 accumulation.
#include "bse_internal.h"
#include "mfma_common.h"

#include <cstdlib>

namespace bse {
namespace {

template <typename T>
struct V4;
template <>
struct V4<double> {
  using t = d4v;
};
template <>
struct V4<float> {
  using t = f4v;
};

__device__ __forceinline__ d4v mma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


// wait until at most N vector-memory ops of this wave are outstanding and its LDS
// ops are done, then barrier
template <int N>
__device__ __forceinline__ void vm_lds_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> ldc(const T* p, long long off) {
  C2<T> r;
  if constexpr (sizeof(T) == 8) {
    const double2 v = *reinterpret_cast<const double2*>(p + 2 * off);
    r.x = v.x;
    r.y = v.y;
  } else {
    const float2 v = *reinterpret_cast<const float2*>(p + 2 * off);
    r.x = v.x;
    r.y = v.y;
  }
  return r;
}

// ----------------------------------------------------------------------------
// FP64 / FP32 kernel
// ----------------------------------------------------------------------------
// at least two waves per SIMD: the 64 x 64 tile otherwise takes 244 VGPRs + 64 AGPRs (one wave), which
// leaves the load and LDS latencies of its single-stage loop exposed; at 247 VGPRs it keeps no spills
template <typename T, typename TC, int WM, int WN, int TM, int TN, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void cgemm_real(GemmArgs g) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int BM = WM * TM * 16;   // complex rows per block
  constexpr int BNR = WN * TN * 16;  // real output columns per block
  constexpr int BN = BNR / 2;        // complex columns per block
  constexpr int AE = (BM * BK + 255) / 256;
  constexpr int BE = (BK * BN + 255) / 256;
  constexpr int PA = (sizeof(T) == 8) ? 1 : 1;
  constexpr int PB = (sizeof(T) == 8) ? 2 : 4;
  __shared__ T As[BM][2 * BK + PA];
  __shared__ T Bs[BK][BNR + PB];
  using acc_t = typename V4<T>::t;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const T* __restrict__ A = (const T*)g.A;
  const T* __restrict__ B = (const T*)g.B;
  TC* __restrict__ C = (TC*)g.C;
  const bool a_kf = (g.a_sk == 1);
  const bool b_kf = (g.b_sk == 1);
  const int r = (lane >> 4) & 1, s = lane & 1;
  const int bcomp = (r != s) ? 1 : 0;
  const T bsgn = (r == 1 && s == 0) ? T(-1) : T(1);
  const T asg = g.conjA ? T(-1) : T(1);
  const T bsg = g.conjB ? T(-1) : T(1);

  for (int b = blockIdx.z; b < g.batch; b += gridDim.z) {
    long long aoff[AE];
    int ai[AE], ak[AE];
    bool aok[AE];
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + 256 * e;
      if (a_kf) {
        ak[e] = idx % BK;
        ai[e] = idx / BK;
      } else {
        ai[e] = idx % BM;
        ak[e] = idx / BM;
      }
      const int row = m0 + ai[e];
      aok[e] = (idx < BM * BK) && (row < g.M);
      aoff[e] = aok[e] ? off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, row) : 0;
    }
    long long boff[BE];
    int bj[BE], bk[BE];
    bool bok[BE];
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + 256 * e;
      if (b_kf) {
        bk[e] = idx % BK;
        bj[e] = idx / BK;
      } else {
        bj[e] = idx % BN;
        bk[e] = idx / BN;
      }
      const int col = n0 + bj[e];
      bok[e] = (idx < BK * BN) && (col < g.N);
      boff[e] = bok[e] ? off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, col) : 0;
    }

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    C2<T> ra[AE], rb[BE];
    auto gload = [&](int k0) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int kk = k0 + ak[e];
        if (aok[e] && kk < g.K) {
          ra[e] = ldc<T>(A, aoff[e] + (long long)kk * g.a_sk);
          ra[e].y *= asg;
        } else {
          ra[e].x = T(0);
          ra[e].y = T(0);
        }
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        const int kk = k0 + bk[e];
        if (bok[e] && kk < g.K) {
          rb[e] = ldc<T>(B, boff[e] + (long long)kk * g.b_sk);
          rb[e].y *= bsg;
        } else {
          rb[e].x = T(0);
          rb[e].y = T(0);
        }
      }
    };
    gload(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        if (tid + 256 * e < BM * BK) {
          As[ai[e]][2 * ak[e]] = ra[e].x;
          As[ai[e]][2 * ak[e] + 1] = ra[e].y;
        }
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        if (tid + 256 * e < BK * BN) {
          Bs[bk[e]][2 * bj[e]] = rb[e].x;
          Bs[bk[e]][2 * bj[e] + 1] = rb[e].y;
        }
      }
      __syncthreads();
      if (k0 + BK < g.K) gload(k0 + BK);
#pragma unroll
      for (int kk4 = 0; kk4 < (2 * BK) / 4; ++kk4) {
        const int kk = kk4 * 4 + (lane >> 4);
        const int kc = kk >> 1;
        T av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = As[wm * TM * 16 + i * 16 + (lane & 15)][kk];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int jj = wn * TN * 16 + j * 16 + (lane & 15);
          bv[j] = bsgn * Bs[kc][(jj & ~1) + bcomp];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mma16(av[i], bv[j], acc[i][j]);
      }
      __syncthreads();
    }

    // epilogue: register q of a lane holds real column lane%16 of row
    //   4*(lane/16) + q  (f32 16x16x4)   or   4*q + lane/16  (f64 16x16x4)
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rin = (sizeof(T) == 8) ? (4 * q + (lane >> 4)) : (4 * (lane >> 4) + q);
        const int row = m0 + wm * TM * 16 + i * 16 + rin;
        if (row >= g.M) continue;
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int jj = wn * TN * 16 + j * 16 + (lane & 15);
          const int col = n0 + (jj >> 1);
          if (col >= g.N) continue;
          const long long o = 2 * (ro + (long long)col * g.c_sj) + (jj & 1);
          double v = g.alpha * (double)acc[i][j][q];
          if (g.beta) v += (double)C[o];
          C[o] = (TC)v;
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// FP32, large tiles: interleaved c64 operands staged straight into LDS, 32x32x2 MFMA
// ----------------------------------------------------------------------------
// The wide tile (128 x 256 complex, eight waves of 64 x 64, three 48 KiB LDS stages of 16 complex k, the
// ping-pong schedule of wide_tile_kloop) for FP32 plans, whose operands are interleaved complex64.  An LDS
// row holds the 16 k of one operand row (128 bytes, eight 16-byte chunks of two complex values); chunk c of
// row r is stored at c ^ ((r / 2) % 8), so the 16-byte fragment reads of 32 consecutive rows spread over
// the banks.  A lane of half h (lane / 32) reads chunk 2 g + h for k group g (four complex k), i.e. k =
// 4 g + 2 h + m for m = 0, 1 in its two complex values; one 32x32x2 product per (g, m) then sums the k of both
// halves, the same split for A and B.  Each complex k step is four real products with FP32 accumulation:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br   (conj A / conj B negate Ai / Bi).
// 256 FP32 products per k step per wave (8192 matrix-core cycles), so the 48 KiB of operands per stage are
// far from limiting.  The result is written from the registers (each row of 32 lanes is 256 contiguous bytes).
constexpr int FW_BM = 128, FW_BN = 256, FW_BK = 16, FW_NS = 3;
constexpr int FW_STAGE = (FW_BM + FW_BN) * FW_BK * 2;  // floats per stage
constexpr size_t FW_LDS = (size_t)FW_NS * FW_STAGE * sizeof(float);  // 144 KiB

template <int CJA, int CJB, typename TC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void cgemm_f32_dma_w(GemmArgs g) {
  constexpr int BM = FW_BM, BN = FW_BN, BK = FW_BK, NS = FW_NS, STAGE = FW_STAGE;
  constexpr int RBLK = (BM + BN) / 8;  // 8-row DMA blocks per stage: 16 of A, 32 of B
  extern __shared__ __attribute__((aligned(1024))) float smem_f[];
  float* smem = smem_f;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int h = lane >> 5, l32 = lane & 31;
  const int nK = g.K / BK;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  // DMA: block rb (of 48) -> wave rb % 8; lane -> row 8 (rb') + lane / 8, stored chunk lane % 8, which holds
  // source chunk (lane % 8) ^ ((row / 2) % 8); rows past the edge re-load a valid row (never stored)
  const float* src[RBLK / 8];
  int ldo[RBLK / 8];
#pragma unroll
  for (int u = 0; u < RBLK / 8; ++u) {
    const int rb = wave + 8 * u;
    const bool isA = rb < BM / 8;
    const int r = 8 * (isA ? rb : rb - BM / 8) + (lane >> 3);
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    if (isA) {
      const int row = (m0 + r < g.M) ? m0 + r : m0;
      src[u] = (const float*)g.A + 2 * off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, row) + 4 * c;
      ldo[u] = 8 * rb * BK * 2;
    } else {
      const int col = (n0 + r < g.N) ? n0 + r : n0;
      src[u] = (const float*)g.B + 2 * off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, col) + 4 * c;
      ldo[u] = BM * BK * 2 + 8 * (rb - BM / 8) * BK * 2;
    }
  }
  auto issue = [&](int kt) {
    if (kt >= nK) return;
    float* st = smem + (kt % NS) * STAGE;
#pragma unroll
    for (int u = 0; u < RBLK / 8; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(src[u] + 2 * BK * kt),
                                       (__attribute__((address_space(3))) void*)(st + ldo[u]), 16, 0, 0);
  };
  f16v accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[i][j][r] = 0.f;
        accI[i][j][r] = 0.f;
      }
  issue(0);
  issue(1);
  f4v a[2][4], bb[2][4];
  auto frags = [&](int kt) {
    const float* sa = smem + (kt % NS) * STAGE;
    const float* sb = sa + BM * BK * 2;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 64 + i * 32 + l32;
#pragma unroll
      for (int gk = 0; gk < 4; ++gk)
        a[i][gk] = *reinterpret_cast<const f4v*>(sa + row * BK * 2 + 4 * ((2 * gk + h) ^ ((row >> 1) & 7)));
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 64 + j * 32 + l32;
#pragma unroll
      for (int gk = 0; gk < 4; ++gk)
        bb[j][gk] = *reinterpret_cast<const f4v*>(sb + col * BK * 2 + 4 * ((2 * gk + h) ^ ((col >> 1) & 7)));
    }
  };
  auto mma = [&]() {
#pragma unroll
    for (int gk = 0; gk < 4; ++gk)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float ar = a[i][gk][2 * m];
          const float ai = CJA ? -a[i][gk][2 * m + 1] : a[i][gk][2 * m + 1];
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const float br = bb[j][gk][2 * m];
            const float bi = CJB ? -bb[j][gk][2 * m + 1] : bb[j][gk][2 * m + 1];
            accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, accR[i][j], 0, 0, 0);
            accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, accI[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, accI[i][j], 0, 0, 0);
          }
        }
  };
  // ping-pong as in wide_tile_kloop (six loads per wave per stage)
  auto bar = [&](int n) {
    if (n >= 2)
      vm_lds_barrier<12>();
    else if (n == 1)
      vm_lds_barrier<6>();
    else
      vm_lds_barrier<0>();
  };
  auto last = [&](int kt) { return kt < nK - 1 ? kt : nK - 1; };
  const bool late = wave >= 4;
  if (late) bar(last(1) - 0);
  for (int kt = 0; kt < nK; ++kt) {
    bar(last(kt + 1) - kt);
    issue(kt + 2);
    frags(kt);
    if (late)
      bar(last(kt + 2) - (kt + 1));
    else
      bar(last(kt + 2) - kt);
    mma();
  }
  if (!late) bar(0);
  // result: register r of a 32 x 32 tile holds row 8 (r / 4) + 4 h + r % 4, column l32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      if (row >= g.M) continue;
      const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn * 64 + j * 32 + l32;
        if (col >= g.N) continue;
        TC* o = (TC*)g.C + 2 * (ro + (long long)col * g.c_sj);
        double vr = g.alpha * (double)accR[i][j][r], vi = g.alpha * (double)accI[i][j][r];
        if (g.beta) {
          vr += (double)o[0];
          vi += (double)o[1];
        }
        o[0] = (TC)vr;
        o[1] = (TC)vi;
      }
    }
}

// The same products on 64 x 64 tiles for small per-pair matrices (the FP32 direct block T = M_c P^T has
// n_c^2 x n_v^2 entries per pair, K = N_aux): four waves of one 32 x 32 tile each, three 16 KiB
// direct-to-LDS stages (16 complex k of 64 rows of A and 64 of B, the chunk swizzle of the wide tile), loads
// of stage kt + 2 in flight while stage kt is multiplied, three blocks per CU.
constexpr int F64T_BM = 64, F64T_BN = 64, F64T_BK = 16, F64T_NS = 3;

template <int CJA, int CJB, typename TC>
__global__ __launch_bounds__(256) void cgemm_f32_dma64(GemmArgs g) {
  constexpr int BM = F64T_BM, BN = F64T_BN, BK = F64T_BK, NS = F64T_NS;
  constexpr int STAGE = (BM + BN) * BK * 2;  // floats per stage
  constexpr int RBLK = (BM + BN) / 8;        // 8-row DMA blocks per stage: 8 of A, 8 of B
  __shared__ __attribute__((aligned(1024))) float smem[NS * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const int nK = g.K / BK;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  // DMA: block rb (of 16) -> wave rb % 4; lane -> row 8 (rb') + lane / 8, stored chunk lane % 8, which holds
  // source chunk (lane % 8) ^ ((row / 2) % 8); rows past the edge re-load a valid row (never stored)
  const float* src[RBLK / 4];
  int ldo[RBLK / 4];
#pragma unroll
  for (int u = 0; u < RBLK / 4; ++u) {
    const int rb = wave + 4 * u;
    const bool isA = rb < BM / 8;
    const int r = 8 * (isA ? rb : rb - BM / 8) + (lane >> 3);
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    if (isA) {
      const int row = (m0 + r < g.M) ? m0 + r : m0;
      src[u] = (const float*)g.A + 2 * off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, row) + 4 * c;
      ldo[u] = 8 * rb * BK * 2;
    } else {
      const int col = (n0 + r < g.N) ? n0 + r : n0;
      src[u] = (const float*)g.B + 2 * off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, col) + 4 * c;
      ldo[u] = BM * BK * 2 + 8 * (rb - BM / 8) * BK * 2;
    }
  }
  auto issue = [&](int kt) {
    if (kt >= nK) return;
    float* st = smem + (kt % NS) * STAGE;
#pragma unroll
    for (int u = 0; u < RBLK / 4; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(src[u] + 2 * BK * kt),
                                       (__attribute__((address_space(3))) void*)(st + ldo[u]), 16, 0, 0);
  };
  f16v accR, accI;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] = 0.f;
    accI[r] = 0.f;
  }
  issue(0);
  issue(1);
  for (int kt = 0; kt < nK; ++kt) {
    // stage kt has landed (the four loads of stage kt + 1 may still be in flight) and every wave is done
    // with stage kt - 1, whose slot the next issue overwrites
    if (kt + 1 < nK)
      vm_lds_barrier<RBLK / 4>();
    else
      vm_lds_barrier<0>();
    issue(kt + 2);
    const float* sa = smem + (kt % NS) * STAGE;
    const float* sb = sa + BM * BK * 2;
    f4v a[4], bb[4];
    const int row = wm * 32 + l32, col = wn * 32 + l32;
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
      a[gk] = *reinterpret_cast<const f4v*>(sa + row * BK * 2 + 4 * ((2 * gk + h) ^ ((row >> 1) & 7)));
      bb[gk] = *reinterpret_cast<const f4v*>(sb + col * BK * 2 + 4 * ((2 * gk + h) ^ ((col >> 1) & 7)));
    }
#pragma unroll
    for (int gk = 0; gk < 4; ++gk)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const float ar = a[gk][2 * m];
        const float ai = CJA ? -a[gk][2 * m + 1] : a[gk][2 * m + 1];
        const float br = bb[gk][2 * m];
        const float bi = CJB ? -bb[gk][2 * m + 1] : bb[gk][2 * m + 1];
        accR = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, accI, 0, 0, 0);
      }
  }
  // result: register r holds row 8 (r / 4) + 4 h + r % 4, column l32 of the wave's 32 x 32 tile
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
    const int col = n0 + wn * 32 + l32;
    if (row >= g.M || col >= g.N) continue;
    const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
    TC* o = (TC*)g.C + 2 * (ro + (long long)col * g.c_sj);
    double vr = g.alpha * (double)accR[r], vi = g.alpha * (double)accI[r];
    if (g.beta) {
      vr += (double)o[0];
      vi += (double)o[1];
    }
    o[0] = (TC)vr;
    o[1] = (TC)vi;
  }
}

// ----------------------------------------------------------------------------
// BF16x3 kernel (c64 inputs, split into bf16 hi/lo when staged to LDS)
// ----------------------------------------------------------------------------

template <typename TC, int WM, int WN, int TM, int TN, int BK>
__global__ __launch_bounds__(256) void cgemm_bf16x3(GemmArgs g) {
  static_assert(WM * WN == 4, "4 waves");
  static_assert(BK % 16 == 0, "BK multiple of 16 complex (32 real)");
  constexpr int BM = WM * TM * 16;
  constexpr int BNR = WN * TN * 16;
  constexpr int BN = BNR / 2;
  constexpr int KR = 2 * BK;        // real depth of a tile
  constexpr int LD = KR + 8;        // bf16 row length in LDS (16 B aligned rows)
  constexpr int AE = (BM * BK + 255) / 256;
  constexpr int BE = (BK * BN + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM * LD];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM * LD];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BNR * LD];   // expanded B, transposed: [jj][kk]
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BNR * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
  const float* __restrict__ A = (const float*)g.A;
  const float* __restrict__ B = (const float*)g.B;
  TC* __restrict__ C = (TC*)g.C;
  const bool a_kf = (g.a_sk == 1);
  const bool b_kf = (g.b_sk == 1);
  const float asg = g.conjA ? -1.f : 1.f;
  const float bsg = g.conjB ? -1.f : 1.f;

  for (int b = blockIdx.z; b < g.batch; b += gridDim.z) {
    long long aoff[AE];
    int ai[AE], ak[AE];
    bool aok[AE];
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + 256 * e;
      if (a_kf) {
        ak[e] = idx % BK;
        ai[e] = idx / BK;
      } else {
        ai[e] = idx % BM;
        ak[e] = idx / BM;
      }
      const int row = m0 + ai[e];
      aok[e] = (idx < BM * BK) && (row < g.M);
      aoff[e] = aok[e] ? off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, row) : 0;
    }
    long long boff[BE];
    int bj[BE], bk[BE];
    bool bok[BE];
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + 256 * e;
      if (b_kf) {
        bk[e] = idx % BK;
        bj[e] = idx / BK;
      } else {
        bj[e] = idx % BN;
        bk[e] = idx / BN;
      }
      const int col = n0 + bj[e];
      bok[e] = (idx < BK * BN) && (col < g.N);
      boff[e] = bok[e] ? off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, col) : 0;
    }
    f4v acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = f4v{0, 0, 0, 0};

    C2<float> ra[AE], rb[BE];
    auto gload = [&](int k0) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int kk = k0 + ak[e];
        if (aok[e] && kk < g.K) {
          ra[e] = ldc<float>(A, aoff[e] + (long long)kk * g.a_sk);
          ra[e].y *= asg;
        } else {
          ra[e].x = 0.f;
          ra[e].y = 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        const int kk = k0 + bk[e];
        if (bok[e] && kk < g.K) {
          rb[e] = ldc<float>(B, boff[e] + (long long)kk * g.b_sk);
          rb[e].y *= bsg;
        } else {
          rb[e].x = 0.f;
          rb[e].y = 0.f;
        }
      }
    };
    gload(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        if (tid + 256 * e < BM * BK) {
          __bf16 h, l;
          split_bf16(ra[e].x, h, l);
          Ah[ai[e] * LD + 2 * ak[e]] = h;
          Al[ai[e] * LD + 2 * ak[e]] = l;
          split_bf16(ra[e].y, h, l);
          Ah[ai[e] * LD + 2 * ak[e] + 1] = h;
          Al[ai[e] * LD + 2 * ak[e] + 1] = l;
        }
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        if (tid + 256 * e < BK * BN) {
          // real rows 2k, 2k+1 and columns 2j, 2j+1 of [[Br, Bi], [-Bi, Br]]
          __bf16 rh, rl, ih, il, nh, nl;
          split_bf16(rb[e].x, rh, rl);
          split_bf16(rb[e].y, ih, il);
          split_bf16(-rb[e].y, nh, nl);
          const int c0 = (2 * bj[e]) * LD + 2 * bk[e];
          const int c1 = (2 * bj[e] + 1) * LD + 2 * bk[e];
          Bh[c0] = rh;
          Bl[c0] = rl;
          Bh[c0 + 1] = nh;
          Bl[c0 + 1] = nl;
          Bh[c1] = ih;
          Bl[c1] = il;
          Bh[c1 + 1] = rh;
          Bl[c1 + 1] = rl;
        }
      }
      __syncthreads();
      if (k0 + BK < g.K) gload(k0 + BK);
#pragma unroll
      for (int ks = 0; ks < KR / 32; ++ks) {
        const int kb = ks * 32 + 8 * (lane >> 4);
        bf8v ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int row = wm * TM * 16 + i * 16 + (lane & 15);
          ah[i] = *reinterpret_cast<const bf8v*>(&Ah[row * LD + kb]);
          al[i] = *reinterpret_cast<const bf8v*>(&Al[row * LD + kb]);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int jj = wn * TN * 16 + j * 16 + (lane & 15);
          bh[j] = *reinterpret_cast<const bf8v*>(&Bh[jj * LD + kb]);
          bl[j] = *reinterpret_cast<const bf8v*>(&Bl[jj * LD + kb]);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wm * TM * 16 + i * 16 + 4 * (lane >> 4) + q;
        if (row >= g.M) continue;
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int jj = wn * TN * 16 + j * 16 + (lane & 15);
          const int col = n0 + (jj >> 1);
          if (col >= g.N) continue;
          const long long o = 2 * (ro + (long long)col * g.c_sj) + (jj & 1);
          double v = g.alpha * (double)acc[i][j][q];
          if (g.beta) v += (double)C[o];
          C[o] = (TC)v;
        }
      }
    }
  }
}


// ----------------------------------------------------------------------------
// BF16X3, large tiles: planar hi/lo operands and 32x32x16 MFMA
//
// Block tile 128 x 128 complex, K step 16 complex, 4 waves in 2 x 2, each wave
// 2 x 2 tiles of 32 x 32 complex.  Every thread stages one (row, 8 k) slice of A
// and of B per K step: the 8 complex values are split once into four bf16 planes
// (Re hi, Re lo, Im hi, Im lo) and written to LDS as 16-byte vectors, so the
// MFMA operands are single ds_read_b128 loads.  Complex products use four real
// products per plane pair with separate Re / Im accumulators:
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br,  each as hi*hi + hi*lo + lo*hi.
// LDS is double buffered with one barrier per K step.
// ----------------------------------------------------------------------------

// A, B: AS / BS = true when the operand is stored pre-split as four bf16 planes
// (Re hi, Re lo, Im hi, Im lo; plane p at base + p * ps, same element offsets as
// the complex array); otherwise complex64 and split while staging.
// CS = true writes C pre-split the same way (alpha applied, beta ignored).
template <bool AS, bool BS, bool CS, typename TC>
__global__ __launch_bounds__(256) void cgemm_b3_big(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = 16;
  constexpr int PL = BM * BK;  // bf16 elements per plane
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][4][PL];
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][4][BN * BK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const float asg = g.conjA ? -1.f : 1.f;
  const float bsg = g.conjB ? -1.f : 1.f;
  // staging slice of this thread: row / column tid/2, k half tid%2
  const int sr = tid >> 1, sh = tid & 1;
  const int nK = (g.K + BK - 1) / BK;
  // 1-D grid over (batch, row tile, column tile), XCD-aware (one batch entry per XCD)
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  const long long total = per_batch * g.batch;

  for (long long L = blockIdx.x; L < total; L += gridDim.x) {
    long long bl, t;
    xcd_map(L, per_batch, g.batch, bl, t);
    const int b = (int)bl;
    int m0, n0;
    tile_of(t, gxn, gyn, BM, BN, m0, n0);
    const bool aok = (m0 + sr) < g.M;
    const bool bok = (n0 + sr) < g.N;
    const long long aoff = aok ? off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, m0 + sr) : 0;
    const long long boff = bok ? off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, n0 + sr) : 0;
    // staged operand slices: 4 planes x 8 bf16
    bf8v pa[4], pb[4];
    auto load_split = [&](const __bf16* base, long long ps, long long off, long long sk, bool ok, int kb,
                          float sg, bf8v* out) {
      const bool fast = ok && sk == 1 && ((off + kb) & 7) == 0 && kb + 8 <= g.K;
      if (fast) {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) out[pl] = *reinterpret_cast<const bf8v*>(base + pl * ps + off + kb);
      } else {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            out[pl][e] = (ok && kb + e < g.K) ? base[pl * ps + off + (long long)(kb + e) * sk] : (__bf16)0.f;
      }
      if (sg < 0.f) {
        out[2] = neg8(out[2]);
        out[3] = neg8(out[3]);
      }
    };
    auto load_c64 = [&](const float* base, long long off, long long sk, bool ok, int kb, float sg, bf8v* out) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float re = 0.f, im = 0.f;
        if (ok && kb + e < g.K) {
          const float2 v = *reinterpret_cast<const float2*>(base + 2 * (off + (long long)(kb + e) * sk));
          re = v.x;
          im = sg * v.y;
        }
        __bf16 h, l;
        split_bf16(re, h, l);
        out[0][e] = h;
        out[1][e] = l;
        split_bf16(im, h, l);
        out[2][e] = h;
        out[3][e] = l;
      }
    };
    auto gload = [&](int kt) {
      const int kb = kt * BK + 8 * sh;
      if constexpr (AS)
        load_split((const __bf16*)g.A, g.a_ps, aoff, g.a_sk, aok, kb, asg, pa);
      else
        load_c64((const float*)g.A, aoff, g.a_sk, aok, kb, asg, pa);
      if constexpr (BS)
        load_split((const __bf16*)g.B, g.b_ps, boff, g.b_sk, bok, kb, bsg, pb);
      else
        load_c64((const float*)g.B, boff, g.b_sk, bok, kb, bsg, pb);
    };
    auto lstore = [&](int st) {
      const int o = sr * BK + 8 * sh;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        *reinterpret_cast<bf8v*>(&sA[st][pl][o]) = pa[pl];
        *reinterpret_cast<bf8v*>(&sB[st][pl][o]) = pb[pl];
      }
    };

    f16v accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          accR[i][j][r] = 0.f;
          accI[i][j][r] = 0.f;
        }

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nK; ++kt) {
      const int st = kt & 1;
      if (kt + 1 < nK) gload(kt + 1);
      const int fo = 8 * (lane >> 5);
      bf8v a[2][4], bb[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm * 64 + i * 32 + (lane & 31);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) a[i][pl] = *reinterpret_cast<const bf8v*>(&sA[st][pl][row * BK + fo]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wn * 64 + j * 32 + (lane & 31);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) bb[j][pl] = *reinterpret_cast<const bf8v*>(&sB[st][pl][col * BK + fo]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          f16v cr = accR[i][j], ci = accI[i][j];
          cmma_b3(a[i], nih, nil, bb[j], cr, ci);
          accR[i][j] = cr;
          accI[i][j] = ci;
        }
      }
      if (kt + 1 < nK) lstore(st ^ 1);
      __syncthreads();
    }
    // epilogue: register r of a lane holds row 8*(r/4) + 4*(lane/32) + r%4, column lane%32
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= g.M) continue;
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = n0 + wn * 64 + j * 32 + (lane & 31);
          if (col >= g.N) continue;
          const long long co = ro + (long long)col * g.c_sj;
          if constexpr (CS) {
            __bf16* o = (__bf16*)g.C + co;
            const float vr = (float)(g.alpha * (double)accR[i][j][r]);
            const float vi = (float)(g.alpha * (double)accI[i][j][r]);
            __bf16 h, l;
            split_bf16(vr, h, l);
            o[0] = h;
            o[g.c_ps] = l;
            split_bf16(vi, h, l);
            o[2 * g.c_ps] = h;
            o[3 * g.c_ps] = l;
          } else {
            TC* o = (TC*)g.C + 2 * co;
            double vr = g.alpha * (double)accR[i][j][r], vi = g.alpha * (double)accI[i][j][r];
            if (g.beta) {
              vr += (double)o[0];
              vi += (double)o[1];
            }
            o[0] = (TC)vr;
            o[1] = (TC)vi;
          }
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// BF16X3 with both operands pre-split: direct-to-LDS staging
//
// Same tile (128 x 128 complex, K step 16, 4 waves of 2 x 2 32x32 tiles) and the
// same per-accumulator MFMA order as cgemm_b3_big, so results are identical.
// Operands go from global memory straight into LDS with global_load_lds_dwordx4
// (no register staging): wave w fills rows 32w .. 32w+31 of every plane, one
// 16-byte k chunk per lane, and the two chunks of a row are XOR-swizzled by bit 3
// of the row so the ds_read_b128 fragment loads are free of bank conflicts.  Two
// LDS stages; the loads of stage kt+1 are in flight while stage kt is multiplied.
// A split C is staged through LDS and written with 16-byte stores.
// ----------------------------------------------------------------------------


template <int CJA, int CJB, bool CS, typename TC>
__global__ __launch_bounds__(256) void cgemm_b3_dma(GemmArgs g) {
  constexpr int BM = 128, BN = 128, BK = 16, NS = 2;
  constexpr int PL = BM * BK;    // bf16 per plane per operand per stage
  constexpr int STAGE = 8 * PL;  // A planes 0..3, B planes 4..7
  __shared__ __attribute__((aligned(1024))) __bf16 smem[NS * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nK = g.K / BK;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  // this lane's DMA slot: row 32*wave + lane/2, stored chunk position lane%2 holds k chunk
  // (lane%2) ^ ((row >> 3) & 1).  Rows past the matrix edge re-load a valid row: those
  // products only reach output rows / columns that are never stored.
  const int drow = 32 * wave + (lane >> 1);
  const int dch = (lane & 1) ^ ((drow >> 3) & 1);
  const int arow = (m0 + drow < g.M) ? m0 + drow : m0;
  const int bcol = (n0 + drow < g.N) ? n0 + drow : n0;
  const __bf16* ga = (const __bf16*)g.A + off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, arow) + 8 * dch;
  const __bf16* gb = (const __bf16*)g.B + off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, bcol) + 8 * dch;
  auto issue = [&](int kt) {
    __bf16* st = smem + (kt % NS) * STAGE + 32 * wave * BK;
    const int kb = kt * BK;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      __builtin_amdgcn_global_load_lds((const void*)(ga + pl * g.a_ps + kb),
                                       (__attribute__((address_space(3))) void*)(st + pl * PL), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(gb + pl * g.b_ps + kb),
                                       (__attribute__((address_space(3))) void*)(st + (4 + pl) * PL), 16, 0, 0);
    }
  };
  f16v accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[i][j][r] = 0.f;
        accI[i][j][r] = 0.f;
      }
  issue(0);
  const int ch = lane >> 5;
  for (int kt = 0; kt < nK; ++kt) {
    // stage kt has landed once only the 8 loads of stage kt+1 (if issued) may be outstanding; the
    // barrier also guarantees that every wave has finished reading stage kt-1, whose buffer is refilled next
    vm_lds_barrier<0>();
    if (kt + 1 < nK) issue(kt + 1);
    const __bf16* sa = smem + (kt % NS) * STAGE;
    const __bf16* sb = sa + 4 * PL;
    bf8v a[2][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 64 + i * 32 + (lane & 31);
      const int o = row * BK + 8 * (ch ^ ((row >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[i][pl] = *reinterpret_cast<const bf8v*>(sa + pl * PL + o);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 64 + j * 32 + (lane & 31);
      const int o = col * BK + 8 * (ch ^ ((col >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) bb[j][pl] = *reinterpret_cast<const bf8v*>(sb + pl * PL + o);
      if (CJB) {
        bb[j][2] = neg8(bb[j][2]);
        bb[j][3] = neg8(bb[j][3]);
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br, with Ai -> -Ai for conj(A); rh/rl carry the sign of
      // Im A in the real part, ih/il in the imaginary part
      const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
      const bf8v rh = CJA ? a[i][2] : nih, rl = CJA ? a[i][3] : nil;
      const bf8v ih = CJA ? nih : a[i][2], il = CJA ? nil : a[i][3];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        f16v& cr = accR[i][j];
        f16v& ci = accI[i][j];
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bb[j][0], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bb[j][2], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][1], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][3], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bb[j][2], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bb[j][0], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][3], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][1], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][0], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][2], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][2], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][0], ci, 0, 0, 0);
      }
    }
  }
  vm_lds_barrier<0>();  // all waves are done with the stages before the epilogue reuses LDS
  if constexpr (CS) {
    // one row half (64 rows) at a time through LDS as planes [4][64][128], then 16-byte stores
    __bf16* sC = smem;
    const float al = (float)g.alpha;
    for (int h = 0; h < 2; ++h) {
      if (wm == h) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int row = i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
              const int col = wn * 64 + j * 32 + (lane & 31);
              __bf16 hh, ll;
              split_bf16(al * accR[i][j][r], hh, ll);
              sC[(0 * 64 + row) * 128 + col] = hh;
              sC[(1 * 64 + row) * 128 + col] = ll;
              split_bf16(al * accI[i][j][r], hh, ll);
              sC[(2 * 64 + row) * 128 + col] = hh;
              sC[(3 * 64 + row) * 128 + col] = ll;
            }
      }
      vm_lds_barrier<63>();
#pragma unroll 4
      for (int it = 0; it < 16; ++it) {
        const int id = tid + 256 * it;
        const int c8 = id & 15, row = (id >> 4) & 63, pl = id >> 10;
        const int grow = m0 + h * 64 + row, gcol = n0 + c8 * 8;
        if (grow < g.M && gcol < g.N) {
          const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, grow);
          __bf16* o = (__bf16*)g.C + pl * g.c_ps + ro + gcol;
          const bf8v v = *reinterpret_cast<const bf8v*>(&sC[(pl * 64 + row) * 128 + c8 * 8]);
          if (gcol + 8 <= g.N && ((ro + gcol) & 7) == 0) {
            *reinterpret_cast<bf8v*>(o) = v;
          } else {
            for (int e = 0; e < 8 && gcol + e < g.N; ++e) o[e] = v[e];
          }
        }
      }
      vm_lds_barrier<63>();
    }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= g.M) continue;
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = n0 + wn * 64 + j * 32 + (lane & 31);
          if (col >= g.N) continue;
          TC* o = (TC*)g.C + 2 * (ro + (long long)col * g.c_sj);
          double vr = g.alpha * (double)accR[i][j][r], vi = g.alpha * (double)accI[i][j][r];
          if (g.beta) {
            vr += (double)o[0];
            vi += (double)o[1];
          }
          o[0] = (TC)vr;
          o[1] = (TC)vi;
        }
      }
    }
  }
}

// 64 x 128 tiles of the same product with the result written pre-split (CS), for the long-K products
// (the W step, K = N_aux): four waves of 32 x 64 hold 64 accumulator registers, so three blocks of
// 48 KiB LDS share a CU (three waves per SIMD) where the 128 x 128 tile runs one.  A's two and B's four
// 32-row DMA blocks go to waves 0..3 and 0..1.  Each accumulator receives the same MFMA sequence as in
// cgemm_b3_dma, so the results are identical.
template <int CJA, int CJB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void cgemm_b3_dma_m64(GemmArgs g) {
  constexpr int BM = 64, BN = 128, BK = 16;
  constexpr int PA = BM * BK, PB = BN * BK;  // bf16 per plane per stage
  constexpr int STAGE = 4 * (PA + PB);
  constexpr int RBA = BM / 32, RB = (BM + BN) / 32;
  __shared__ __attribute__((aligned(1024))) __bf16 smem[2 * STAGE];
  static_assert(4 * 32 * BN <= 2 * STAGE, "epilogue staging must fit in the stages");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nK = g.K / BK;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  // DMA slot of 32-row block rb: lane -> row 32 rb' + lane / 2, 16-byte chunk (lane % 2) ^ bit 3 of the
  // row; rows past the matrix edge re-load a valid row (their products are never stored)
  auto slot = [&](int rb, const __bf16*& src, int& lo, long long& ps, int& pstride) {
    const bool isA = rb < RBA;
    const int r = 32 * (isA ? rb : rb - RBA) + (lane >> 1);
    const int chunk = (lane & 1) ^ ((r >> 3) & 1);
    if (isA) {
      const int arow = (m0 + r < g.M) ? m0 + r : m0;
      src = (const __bf16*)g.A + off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, arow) + 8 * chunk;
      lo = 32 * rb * BK;
      ps = g.a_ps;
      pstride = PA;
    } else {
      const int bcol = (n0 + r < g.N) ? n0 + r : n0;
      src = (const __bf16*)g.B + off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, bcol) + 8 * chunk;
      lo = 4 * PA + 32 * (rb - RBA) * BK;
      ps = g.b_ps;
      pstride = PB;
    }
  };
  const __bf16 *src0 = nullptr, *src1 = nullptr;
  int lo0 = 0, lo1 = 0, pst0 = 0, pst1 = 0;
  long long ps0 = 0, ps1 = 0;
  slot(wave, src0, lo0, ps0, pst0);
  const bool two = wave + 4 < RB;
  if (two) slot(wave + 4, src1, lo1, ps1, pst1);
  auto issue = [&](int kt) {
    __bf16* st = smem + (kt & 1) * STAGE;
    const int kb = kt * BK;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      __builtin_amdgcn_global_load_lds((const void*)(src0 + pl * ps0 + kb),
                                       (__attribute__((address_space(3))) void*)(st + lo0 + pl * pst0), 16, 0, 0);
    if (two) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        __builtin_amdgcn_global_load_lds((const void*)(src1 + pl * ps1 + kb),
                                         (__attribute__((address_space(3))) void*)(st + lo1 + pl * pst1), 16, 0, 0);
    }
  };
  f16v accR[2], accI[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accR[j][r] = 0.f;
      accI[j][r] = 0.f;
    }
  issue(0);
  const int ch = lane >> 5;
  for (int kt = 0; kt < nK; ++kt) {
    vm_lds_barrier<0>();
    if (kt + 1 < nK) issue(kt + 1);
    const __bf16* sa = smem + (kt & 1) * STAGE;
    const __bf16* sb = sa + 4 * PA;
    bf8v a[4], bb[2][4];
    {
      const int row = wm * 32 + (lane & 31);
      const int o = row * BK + 8 * (ch ^ ((row >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const bf8v*>(sa + pl * PA + o);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 64 + j * 32 + (lane & 31);
      const int o = col * BK + 8 * (ch ^ ((col >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) bb[j][pl] = *reinterpret_cast<const bf8v*>(sb + pl * PB + o);
      if (CJB) {
        bb[j][2] = neg8(bb[j][2]);
        bb[j][3] = neg8(bb[j][3]);
      }
    }
    const bf8v nih = neg8(a[2]), nil = neg8(a[3]);
    const bf8v rh = CJA ? a[2] : nih, rl = CJA ? a[3] : nil;
    const bf8v ih = CJA ? nih : a[2], il = CJA ? nil : a[3];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f16v& cr = accR[j];
      f16v& ci = accI[j];
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[j][0], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[j][2], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[j][1], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[j][3], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bb[j][2], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bb[j][0], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][3], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][1], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[j][0], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[j][2], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][2], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][0], ci, 0, 0, 0);
    }
  }
  vm_lds_barrier<0>();  // every wave is done with the stages before the epilogue reuses LDS
  // one row half (32 rows) at a time through LDS as planes [4][32][128], then 16-byte stores
  __bf16* sC = smem;
  const float al = (float)g.alpha;
  for (int h = 0; h < 2; ++h) {
    if (wm == h) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int col = wn * 64 + j * 32 + (lane & 31);
          __bf16 hh, ll;
          split_bf16(al * accR[j][r], hh, ll);
          sC[(0 * 32 + row) * BN + col] = hh;
          sC[(1 * 32 + row) * BN + col] = ll;
          split_bf16(al * accI[j][r], hh, ll);
          sC[(2 * 32 + row) * BN + col] = hh;
          sC[(3 * 32 + row) * BN + col] = ll;
        }
    }
    vm_lds_barrier<63>();
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int id = tid + 256 * it;
      const int c8 = id & 15, row = (id >> 4) & 31, pl = id >> 9;
      const int grow = m0 + h * 32 + row, gcol = n0 + c8 * 8;
      if (grow < g.M && gcol < g.N) {
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, grow);
        __bf16* o = (__bf16*)g.C + pl * g.c_ps + ro + gcol;
        const bf8v v = *reinterpret_cast<const bf8v*>(&sC[(pl * 32 + row) * BN + c8 * 8]);
        if (gcol + 8 <= g.N && ((ro + gcol) & 7) == 0) {
          *reinterpret_cast<bf8v*>(o) = v;
        } else {
          for (int e = 0; e < 8 && gcol + e < g.N; ++e) o[e] = v[e];
        }
      }
    }
    vm_lds_barrier<63>();
  }
}

// 128 x 256 tiles of the same product with the result written pre-split, for long-K products with a wide
// B (the W step: K = N = N_aux).  Eight waves of 64 x 64 (two per SIMD, one block per CU) and three LDS
// stages of 48 KiB: the loads of stage kt + 2 are issued while stage kt is multiplied, so two k steps of
// matrix work cover the latency of each operand fetch, where the 64 x 128 tile's two stages cover one.
// The A panel of 128 rows is shared by both column tiles of N = 512 and W(q) by every row tile of its
// batch entry.  A's four and B's eight 32-row DMA blocks go to waves 0..7 and 0..3.  Each accumulator
// receives the same MFMA sequence as in cgemm_b3_dma, so the results are identical.
constexpr int WB_BM = 128, WB_BN = 256, WB_NS = 3, WB_BK = 16;
#ifndef WB_MIN_K
#define WB_MIN_K 256  // shortest K given to the wide tile
#endif
#ifndef WB_PINGPONG
#define WB_PINGPONG 1  // wide-tile main loop with the two wave groups taking turns on the matrix cores
#endif
#ifndef WT_AH
#define WT_AH 1  // Mc k steps requested ahead in the fused direct block
#endif
constexpr int WB_STAGE = 4 * (WB_BM + WB_BN) * WB_BK;  // bf16 per stage
constexpr size_t WB_LDS = (size_t)WB_NS * WB_STAGE * sizeof(__bf16);  // 144 KiB

// The main loop of the wide tile: rows m0 .. m0 + 127, columns n0 .. n0 + 255 of batch entry b, all of K.
// Wave (wm, wn) = (wave / 4, wave % 4) ends with the 64 x 64 block at rows 64 wm, columns 64 wn of the
// tile in accR / accI ([i][j]: 32 x 32 sub-tiles); every wave has finished with LDS on return.
template <int CJA, int CJB>
__device__ __forceinline__ void wide_tile_kloop(const GemmArgs& g, __bf16* smem, int b, int m0, int n0,
                                                f16v (&accR)[2][2], f16v (&accI)[2][2]) {
  constexpr int BM = WB_BM, BN = WB_BN, BK = WB_BK, NS = WB_NS;
  constexpr int PA = BM * BK, PB = BN * BK;  // bf16 per plane per stage
  constexpr int STAGE = WB_STAGE;
  constexpr int RBA = BM / 32, RB = (BM + BN) / 32;
  static_assert(RB <= 16 && RB > 8, "two DMA blocks at most per wave");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int nK = g.K / BK;
  // DMA slot of 32-row block rb: lane -> row 32 rb' + lane / 2, 16-byte chunk (lane % 2) ^ bit 3 of the
  // row; rows past the matrix edge re-load a valid row (their products are never stored)
  auto slot = [&](int rb, const __bf16*& src, int& lo, long long& ps, int& pstride) {
    const bool isA = rb < RBA;
    const int r = 32 * (isA ? rb : rb - RBA) + (lane >> 1);
    const int chunk = (lane & 1) ^ ((r >> 3) & 1);
    if (isA) {
      const int arow = (m0 + r < g.M) ? m0 + r : m0;
      src = (const __bf16*)g.A + off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, arow) + 8 * chunk;
      lo = 32 * rb * BK;
      ps = g.a_ps;
      pstride = PA;
    } else {
      const int bcol = (n0 + r < g.N) ? n0 + r : n0;
      src = (const __bf16*)g.B + off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, bcol) + 8 * chunk;
      lo = 4 * PA + 32 * (rb - RBA) * BK;
      ps = g.b_ps;
      pstride = PB;
    }
  };
  const __bf16 *src0 = nullptr, *src1 = nullptr;
  int lo0 = 0, lo1 = 0, pst0 = 0, pst1 = 0;
  long long ps0 = 0, ps1 = 0;
  slot(wave, src0, lo0, ps0, pst0);
  const bool two = wave + 8 < RB;
  if (two) slot(wave + 8, src1, lo1, ps1, pst1);
  auto issue = [&](int kt) {
    __bf16* st = smem + (kt % NS) * STAGE;
    const int kb = kt * BK;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      __builtin_amdgcn_global_load_lds((const void*)(src0 + pl * ps0 + kb),
                                       (__attribute__((address_space(3))) void*)(st + lo0 + pl * pst0), 16, 0, 0);
    if (two) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        __builtin_amdgcn_global_load_lds((const void*)(src1 + pl * ps1 + kb),
                                         (__attribute__((address_space(3))) void*)(st + lo1 + pl * pst1), 16, 0, 0);
    }
  };
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[i][j][r] = 0.f;
        accI[i][j][r] = 0.f;
      }
  issue(0);
  if (nK > 1) issue(1);
  const int ch = lane >> 5;
  bf8v a[2][4], bb[2][4];
  auto frags = [&](int kt) {
    const __bf16* sa = smem + (kt % NS) * STAGE;
    const __bf16* sb = sa + 4 * PA;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 64 + i * 32 + (lane & 31);
      const int o = row * BK + 8 * (ch ^ ((row >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[i][pl] = *reinterpret_cast<const bf8v*>(sa + pl * PA + o);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 64 + j * 32 + (lane & 31);
      const int o = col * BK + 8 * (ch ^ ((col >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) bb[j][pl] = *reinterpret_cast<const bf8v*>(sb + pl * PB + o);
    }
  };
  auto mma = [&]() {
    if (CJB) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bb[j][2] = neg8(bb[j][2]);
        bb[j][3] = neg8(bb[j][3]);
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
      const bf8v rh = CJA ? a[i][2] : nih, rl = CJA ? a[i][3] : nil;
      const bf8v ih = CJA ? nih : a[i][2], il = CJA ? nil : a[i][3];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        f16v& cr = accR[i][j];
        f16v& ci = accI[i][j];
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bb[j][0], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bb[j][2], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][1], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][3], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bb[j][2], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bb[j][0], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][3], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][1], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][0], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bb[j][2], ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[j][2], cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[j][0], ci, 0, 0, 0);
      }
    }
  };
  // barrier after waiting until at most `n` of this wave's most recent stages are in flight
  auto bar = [&](int n) {
    if (two) {
      if (n >= 2)
        vm_lds_barrier<16>();
      else if (n == 1)
        vm_lds_barrier<8>();
      else
        vm_lds_barrier<0>();
    } else {
      if (n >= 2)
        vm_lds_barrier<8>();
      else if (n == 1)
        vm_lds_barrier<4>();
      else
        vm_lds_barrier<0>();
    }
  };
  auto last = [&](int kt) { return kt < nK - 1 ? kt : nK - 1; };  // last stage issued by step kt
#if WB_PINGPONG
  // Ping-pong: waves 0..3 and 4..7 (one of each per SIMD) take turns on the matrix cores.  Both groups run
  // "barrier, fragments of stage kt, barrier, products" per step, the second group one barrier behind, so
  // that between consecutive barriers one group reads LDS while the other multiplies.  With barriers
  // B0, B1, ...: group 0 reads stage kt between B(2kt) and B(2kt+1), group 1 between B(2kt+1) and B(2kt+2),
  // so every wave waits for its loads of stage kt before B(2kt), all reads of stage kt are done at
  // B(2kt+2), and the loads of stage kt + 2 (into stage kt - 1's buffer) are issued after B(2kt).
  const bool late = wave >= 4;
  if (late) bar(last(1) - 0);
  for (int kt = 0; kt < nK; ++kt) {
    bar(last(kt + 1) - kt);  // stage kt has landed (group 0 reads it next)
    if (kt + 2 < nK) issue(kt + 2);
    frags(kt);
    if (late)
      bar(last(kt + 2) - (kt + 1));  // stage kt + 1 has landed (group 0 reads it after this barrier)
    else
      bar(last(kt + 2) - kt);
    mma();
  }
  if (!late) bar(0);
#else
  for (int kt = 0; kt < nK; ++kt) {
    bar(last(kt + 1) - kt);  // stage kt has landed; every wave is done with stage kt - 1
    if (kt + 2 < nK) issue(kt + 2);
    frags(kt);
    mma();
  }
#endif
  vm_lds_barrier<0>();  // every wave is done with the stages before the caller reuses LDS
}

template <int CJA, int CJB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void cgemm_b3_dma_w(GemmArgs g) {
  constexpr int BM = WB_BM, BN = WB_BN;
  extern __shared__ __attribute__((aligned(1024))) __bf16 smem_w[];
  __bf16* smem = smem_w;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  f16v accR[2][2], accI[2][2];
  wide_tile_kloop<CJA, CJB>(g, smem, b, m0, n0, accR, accI);
  // the real parts, then the imaginary parts, of the whole tile through LDS as two planes (hi, lo) of
  // [128][256], then 16-byte stores; the real accumulators are dead before the imaginary ones are staged
  static_assert(2 * BM * BN <= WB_NS * WB_STAGE, "epilogue staging must fit in the stages");
  __bf16* sC = smem;
  const float al = (float)g.alpha;
#pragma unroll
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int col = wn * 64 + j * 32 + (lane & 31);
          __bf16 hh, ll;
          split_bf16(al * (part ? accI[i][j][r] : accR[i][j][r]), hh, ll);
          sC[row * BN + col] = hh;
          sC[(BM + row) * BN + col] = ll;
        }
    vm_lds_barrier<63>();
#pragma unroll 2
    for (int it = 0; it < 16; ++it) {
      const int id = tid + 512 * it;
      const int c8 = id & 31, row = (id >> 5) & 127, pl = id >> 12;
      const int grow = m0 + row, gcol = n0 + c8 * 8;
      if (grow < g.M && gcol < g.N) {
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, grow);
        __bf16* o = (__bf16*)g.C + (2 * part + pl) * g.c_ps + ro + gcol;
        const bf8v v = *reinterpret_cast<const bf8v*>(&sC[(pl * BM + row) * BN + c8 * 8]);
        if (gcol + 8 <= g.N && ((ro + gcol) & 7) == 0) {
          *reinterpret_cast<bf8v*>(o) = v;
        } else {
          for (int e = 0; e < 8 && gcol + e < g.N; ++e) o[e] = v[e];
        }
      }
    }
    vm_lds_barrier<63>();
  }
}

// The W step and the direct block of the BF16x3 apply in one kernel, for 64 rows per pair on both band
// sides (n_v = n_c = 8) and N_aux a multiple of 256.  A workgroup takes the pairs (k0, k0 + 1) of one q
// (batch entry b, rows m0 = 64 k0 .. m0 + 127 of Gv) and, for each 256-column tile n0 of P,
//   P[(v'v)][nu] = sum_mu conj(Gv[(v'v)][mu]) W(q)[mu][nu]      (the wide-tile main loop)
//   T[(c'c)][(v'v)] += sum_{nu in the tile} Mc[(c'c)][nu] P[(v'v)][nu]
// P never reaches HBM.  After the main loop it is split into bf16 planes in LDS in two rounds: round s
// stages rows (v'v) = 32 s .. 32 s + 31 of both pairs (every wave's sub-tile i = s, so the accumulators of
// round 0 are dead before round 1), and the round's T columns are formed on 16x16x32 MFMA: wave w takes
// pair w / 4, rows (c'c) 16 (w % 4) .. + 15, both 16-column blocks, with its Mc rows read from global
// memory (the A operand, one k step ahead).  Partial T tiles are kept in the output between rounds and
// column tiles (16 + 16 registers would not fit beside the main loop).  LDS slab [plane][64 rows][256 nu],
// 16-byte chunk c of row r stored at position c ^ (r % 16).
struct WTArgs {
  GemmArgs g;              // the W step: A = Gv planes (conj), B = W(q) planes; M = 64 N_k, N = K = N_aux
  const __bf16* mc;        // Mc planes: element (b, k, r, nu) at b mc_sb + (64 k + r) N_aux + nu
  long long mc_sb, mc_ps;  // per batch entry stride, plane stride (elements)
  float* t;                // T c64: element (b, k, r, c) at b t_sb + 4096 k + 64 r + c
  long long t_sb;
};

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void wstep_dblock_fused(WTArgs w) {
  const GemmArgs& g = w.g;
  constexpr int BM = WB_BM, BN = WB_BN;
  constexpr int SR = 64;          // slab rows: 32 (v'v) of each pair
  constexpr int SPL = SR * BN;    // bf16 per plane of the slab
  extern __shared__ __attribute__((aligned(1024))) __bf16 smem_w[];
  __bf16* smem = smem_w;
  static_assert(4 * SPL <= WB_NS * WB_STAGE, "slab staging must fit in the stages");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int gyn = g.M / BM;
  long long bl, t;
  xcd_map(blockIdx.x, gyn, g.batch, bl, t);
  const int b = (int)bl;
  const int m0 = (int)t * BM, k0 = m0 / 64;
  const int na = g.N;
  const int nN = g.N / BN;
#pragma unroll 1
  for (int nt = 0; nt < nN; ++nt) {
    const int n0 = nt * BN;
    f16v accR[2][2], accI[2][2];
    wide_tile_kloop<1, 0>(g, smem, b, m0, n0, accR, accI);
    // the index math of the T phase is derived from an opaque copy of the lane id, so that none of it is
    // hoisted above the main loop (it would be live there and spilled)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    // this wave's T rows and the lane's place in the 16x16x32 operands / results
    const int wp = wave >> 2, mb = wave & 3;
    const int l16 = ln & 15, q4 = ln >> 4;
    // Mc row 16 mb + l16 of pair wp, nu chunk 8 q4 of each k step (plane 0; planes at mc_ps)
    const __bf16* mcl =
        w.mc + (long long)b * w.mc_sb + (long long)(m0 + 64 * wp + 16 * mb + l16) * na + 8 * q4 + n0;
    // T element (row 16 mb + 4 q4 + e, column 32 s + 16 jb + l16) of pair wp
    float* tl = w.t + 2 * ((long long)b * w.t_sb + (long long)(k0 + wp) * 4096 + (16 * mb + 4 * q4) * 64 + l16);
    // slab writes: element (j, r) of this wave's sub-tile goes to row 32 wm + 8 (r / 4) + 4 h + r % 4,
    // column 64 wn + 32 j + lane % 32 (chunk 8 wn + 4 j + x, x = (lane % 32) / 8, stored at chunk ^ (row % 16))
    const int h = ln >> 5, x = (ln & 31) >> 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // stage rows 32 s .. 32 s + 31 of each pair (sub-tile i = s of every wave)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * wm + 8 * (r >> 2) + 4 * h + (r & 3);
          const int chunk = (8 * wn + 4 * j + x) ^ (row & 15);
          const int o = row * BN + 8 * chunk + (ln & 7);
          __bf16 hh, ll;
          split_bf16(accR[s][j][r], hh, ll);
          smem[o] = hh;
          smem[SPL + o] = ll;
          split_bf16(accI[s][j][r], hh, ll);
          smem[2 * SPL + o] = hh;
          smem[3 * SPL + o] = ll;
        }
      // the round's first Mc k steps and the parked T tiles are requested once the slab is written (the
      // staged accumulators are dead by then), before the barrier; later k steps are requested four ahead
      constexpr int NKS = BN / 32, AH = WT_AH;
      bf8v mf[AH][4];
#pragma unroll
      for (int ks = 0; ks < AH; ++ks)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          mf[ks][pl] = *reinterpret_cast<const bf8v*>(mcl + pl * w.mc_ps + 32 * ks);
      f4v tR[2], tI[2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float2 v = make_float2(0.f, 0.f);
          if (nt > 0) v = *reinterpret_cast<const float2*>(tl + 2 * (e * 64 + 32 * s + 16 * jb));
          tR[jb][e] = v.x;
          tI[jb][e] = v.y;
        }
      vm_lds_barrier<0>();  // the slab is staged (and the requested Mc and T have landed)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        bf8v a[4];
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) a[pl] = mf[ks % AH][pl];
        if (ks + AH < NKS) {
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            mf[ks % AH][pl] = *reinterpret_cast<const bf8v*>(mcl + pl * w.mc_ps + 32 * (ks + AH));
        }
        const bf8v nih = neg8(a[2]), nil = neg8(a[3]);
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
          const int row = 32 * wp + 16 * jb + l16;
          const int o = row * BN + 8 * ((4 * ks + q4) ^ (row & 15));
          bf8v bb[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) bb[pl] = *reinterpret_cast<const bf8v*>(smem + pl * SPL + o);
          f4v& cr = tR[jb];
          f4v& ci = tI[jb];
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bb[0], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bb[2], ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bb[1], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bb[3], ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, bb[2], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3], bb[0], ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bb[3], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], bb[1], ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bb[0], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bb[2], ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, bb[2], cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], bb[0], ci, 0, 0, 0);
        }
        // keep each k step's LDS reads with its products (hoisting them all would spill)
        __builtin_amdgcn_sched_barrier(0);
      }
      // park the round's T tiles (the final values after the last column tile)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          *reinterpret_cast<float2*>(tl + 2 * (e * 64 + 32 * s + 16 * jb)) = make_float2(tR[jb][e], tI[jb][e]);
      vm_lds_barrier<0>();  // every wave is done with the slab before it is restaged
    }
  }
}

// Short-K split products with a small A, on persistent blocks: the pair densities (A = psi rows of one k's
// q batch, K = N_ao; B = that k's halves, N = n_band N_aux; the result written pre-split).  One block of
// eight waves per CU keeps a 128-row block of A in LDS while it runs over the 256-column tiles of its batch
// entry; each wave takes 32 columns and all 128 rows, reads its B fragments straight from global memory
// PD_AHEAD k steps ahead (the first ones of the next tile during this tile's epilogue, so about 64 KiB per
// CU stay in flight) and writes its 128 x 32 result through a private 4 KiB LDS buffer with 16-byte stores:
// no block barrier separates one tile from the next.  Each accumulator receives the MFMA sequence of
// cgemm_b3_dma over k in order, so the results are identical to those of the other split kernels.
// A in LDS as [plane][128 rows][K], 16-byte chunk c of row r stored at c ^ (r % (K / 8)).  FRAG: B in fragment
// order (split_planes_frag), so that each of a wave's fragment loads reads one contiguous KiB instead of 16
// or 32 bytes of 32 different columns.
constexpr int PD_BM = 128, PD_BN = 256, PD_KMAX = 128, PD_AHEAD = 2;
constexpr size_t PD_LDS = (size_t)4 * PD_BM * PD_KMAX * sizeof(__bf16) + 8 * 4096;  // 160 KiB

template <int NK, bool FRAG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void cgemm_b3_stream(GemmArgs g) {
  constexpr int K = 16 * NK, CPR = K / 8;  // k, 16-byte chunks per A row
  constexpr int APL = PD_BM * K;           // bf16 per A plane
  static_assert(K <= PD_KMAX && (CPR & (CPR - 1)) == 0, "K of 64 or 128");
  static_assert(NK % PD_AHEAD == 0, "the fragment ring restarts at slot 0 on every tile");
  extern __shared__ __attribute__((aligned(1024))) __bf16 smem_s[];
  __bf16* sA = smem_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __bf16* sE = smem_s + 4 * APL + wave * 2048;  // this wave's epilogue buffer [2][32][32]
  const int h = lane >> 5, l32 = lane & 31;
  const int gyn = (g.M + PD_BM - 1) / PD_BM, gxn = (g.N + PD_BN - 1) / PD_BN;
  const long long items = (long long)g.batch * gyn * gxn;
  const long long per = (items + gridDim.x - 1) / gridDim.x;
  const long long it0 = (long long)blockIdx.x * per;
  const long long it1 = it0 + per < items ? it0 + per : items;
  if (it0 >= it1) return;  // uniform over the block
  // B fragments of tile `it`, k step kt: column n0 + 32 wave + l32 (a valid column past the edge), k 16 kt + 8 h
  // (FRAG: the wave's 32-column block, the last one past the edge)
  auto bsrc = [&](long long it) -> const __bf16* {
    const long long bm = it / gxn;
    const int b = (int)(bm / gyn), n0 = (int)(it % gxn) * PD_BN;
    if constexpr (FRAG) {
      const int last = g.N / 32 - 1, jb = n0 / 32 + wave;
      return (const __bf16*)g.B + (long long)b * g.b_sb + (long long)(jb < last ? jb : last) * (NK * 512) + 8 * lane;
    } else {
      const int col = n0 + 32 * wave + l32;
      return (const __bf16*)g.B + off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, col < g.N ? col : g.N - 1) +
             8 * h;
    }
  };
  bf8v bq[PD_AHEAD][4];
  constexpr int BSTEP = FRAG ? 512 : 16;  // bf16 between the fragments of consecutive k steps
  auto load_b = [&](const __bf16* src, int kt, bf8v* dst) {
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) dst[pl] = *reinterpret_cast<const bf8v*>(src + pl * g.b_ps + BSTEP * kt);
  };
  const __bf16* bs = bsrc(it0);
#pragma unroll
  for (int s = 0; s < PD_AHEAD; ++s)
    if (s < NK) load_b(bs, s, bq[s]);
  long long cur_bm = -1;
  for (long long it = it0; it < it1; ++it) {
    const long long bm = it / gxn;
    const int b = (int)(bm / gyn), m0 = (int)(bm % gyn) * PD_BM, n0 = (int)(it % gxn) * PD_BN;
    if (bm != cur_bm) {
      // restage A: rows m0 .. m0 + 127 of batch entry b (a valid row past the edge); every wave is past its
      // last A read of the previous block of rows at the first barrier
      __syncthreads();
      constexpr int RPI = 64 / CPR;  // rows per DMA instruction (1 KiB)
      for (int ins = wave; ins < 4 * PD_BM / RPI; ins += 8) {
        const int pl = ins / (PD_BM / RPI), r = (ins % (PD_BM / RPI)) * RPI + lane / CPR;
        const int ph = lane % CPR, lc = ph ^ (r % CPR);
        const int arow = (m0 + r < g.M) ? m0 + r : g.M - 1;
        const __bf16* src = (const __bf16*)g.A + off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, arow) +
                            pl * g.a_ps + 8 * lc;
        __builtin_amdgcn_global_load_lds((const void*)src,
                                         (__attribute__((address_space(3))) void*)(sA + pl * APL +
                                                                                   (ins % (PD_BM / RPI)) * RPI * K),
                                         16, 0, 0);
      }
      vm_lds_barrier<0>();
      cur_bm = bm;
    }
    f16v accR[4], accI[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[i][r] = 0.f;
        accI[i][r] = 0.f;
      }
    // the next tile's fragments are requested as this tile's last k steps retire
    const __bf16* bn = (it + 1 < it1) ? bsrc(it + 1) : bs;
#pragma unroll
    for (int kt = 0; kt < NK; ++kt) {
      bf8v bb[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) bb[pl] = bq[kt % PD_AHEAD][pl];
      if (kt + PD_AHEAD < NK)
        load_b(bs, kt + PD_AHEAD, bq[kt % PD_AHEAD]);
      else if (it + 1 < it1)
        load_b(bn, kt + PD_AHEAD - NK, bq[kt % PD_AHEAD]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 32 * i + l32;
        const int o = row * K + 8 * ((2 * kt + h) ^ (row % CPR));
        bf8v a[4];
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const bf8v*>(sA + pl * APL + o);
        // B fragments as the MFMA's first operand: the lane's registers 4 g .. 4 g + 3 hold four
        // consecutive columns of one row, which the epilogue packs into 8-byte writes
        cmma_b3_t(a, neg8(a[2]), neg8(a[3]), bb, accR[i], accI[i]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    bs = bn;
    // epilogue: per row sub-tile and part (Re, Im), hi and lo planes of 32 x 32 through the wave's buffer.
    // Lane l holds row 32 i + l % 32, register 4 g + e column 8 g + 4 (l / 32) + e; the buffer keeps each
    // row's 16-byte chunk c at c ^ ((row / 4) % 4), so the 8-byte writes of a wave meet every bank twice
    // and the 16-byte reads once
    const float al = (float)g.alpha;
    const int col0 = n0 + 32 * wave;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          f4v x;
#pragma unroll
          for (int e = 0; e < 4; ++e) x[e] = al * (part ? accI[i][4 * gq + e] : accR[i][4 * gq + e]);
          // split_bf16 on four values at once (pairs share one conversion instruction)
          const bf4v hv = __builtin_convertvector(x, bf4v);
          const bf4v lv = __builtin_convertvector(x - __builtin_convertvector(hv, f4v), bf4v);
          const int o = l32 * 32 + 8 * (gq ^ ((l32 >> 2) & 3)) + 4 * h;
          *reinterpret_cast<bf4v*>(sE + o) = hv;
          *reinterpret_cast<bf4v*>(sE + 1024 + o) = lv;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int id = lane + 64 * j;
          const int pl = id >> 7, row = (id >> 2) & 31, c4 = id & 3;
          const bf8v v = *reinterpret_cast<const bf8v*>(sE + pl * 1024 + row * 32 + 8 * (c4 ^ ((row >> 2) & 3)));
          const int grow = m0 + 32 * i + row, gcol = col0 + 8 * c4;
          if (grow < g.M && gcol < g.N) {
            const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, grow);
            __bf16* o = (__bf16*)g.C + (2 * part + pl) * g.c_ps + ro + gcol;
            if (gcol + 8 <= g.N && ((ro + gcol) & 7) == 0) {
              *reinterpret_cast<bf8v*>(o) = v;
            } else {
              for (int e = 0; e < 8 && gcol + e < g.N; ++e) o[e] = v[e];
            }
          }
        }
      }
  }
}

// 64 x 64 tiles of the same product for small per-pair matrices (the direct block T = M_c P^T has
// n_c^2 x n_v^2 entries, 64 x 64 at n_c = n_v = 8, where a 128 x 128 tile would be three quarters
// empty): four waves of one 32 x 32 tile each, waves 0 and 1 stage the A rows, 2 and 3 the B columns.
// Each accumulator receives the same MFMA sequence as in cgemm_b3_dma, so the results are identical.
// CS writes C pre-split, as cgemm_b3_dma<.., true, ..> does; at 85 registers five blocks share a CU,
// which hides the staging and the epilogue of products with a short K (the pair densities, K = N_ao).
template <typename TC, bool CS = false>
__global__ __launch_bounds__(256) void cgemm_b3_dma64(GemmArgs g) {
  constexpr int BM = 64, BN = 64, BK = 16, NS = 2;
  constexpr int PL = BM * BK;
  constexpr int STAGE = 8 * PL;
  __shared__ __attribute__((aligned(1024))) __bf16 smem[NS * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nK = g.K / BK;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per_batch = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per_batch, g.batch, bl, t);
  const int b = (int)bl;
  int m0, n0;
  tile_of(t, gxn, gyn, BM, BN, m0, n0);
  // DMA slot: row 32 (wave % 2) + lane / 2 of A (waves 0, 1) or of B (waves 2, 3), 16-byte chunk as above
  const bool isB = wave >= 2;
  const int drow = 32 * (wave & 1) + (lane >> 1);
  const int dch = (lane & 1) ^ ((drow >> 3) & 1);
  const __bf16* src;
  long long ps;
  if (!isB) {
    const int arow = (m0 + drow < g.M) ? m0 + drow : m0;
    src = (const __bf16*)g.A + off_of(g.a_tab, g.a_tab_pb, g.a_sb, g.a_si, b, g.M, arow) + 8 * dch;
    ps = g.a_ps;
  } else {
    const int bcol = (n0 + drow < g.N) ? n0 + drow : n0;
    src = (const __bf16*)g.B + off_of(g.b_tab, g.b_tab_pb, g.b_sb, g.b_sj, b, g.N, bcol) + 8 * dch;
    ps = g.b_ps;
  }
  const int loff = (isB ? 4 * PL : 0) + 32 * (wave & 1) * BK;
  auto issue = [&](int kt) {
    __bf16* st = smem + (kt % NS) * STAGE + loff;
    const int kb = kt * BK;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      __builtin_amdgcn_global_load_lds((const void*)(src + pl * ps + kb),
                                       (__attribute__((address_space(3))) void*)(st + pl * PL), 16, 0, 0);
  };
  f16v accR, accI;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accR[r] = 0.f;
    accI[r] = 0.f;
  }
  issue(0);
  const int ch = lane >> 5;
  for (int kt = 0; kt < nK; ++kt) {
    vm_lds_barrier<0>();
    if (kt + 1 < nK) issue(kt + 1);
    const __bf16* sa = smem + (kt % NS) * STAGE;
    const __bf16* sb = sa + 4 * PL;
    bf8v a[4], bb[4];
    {
      const int row = wm * 32 + (lane & 31);
      const int o = row * BK + 8 * (ch ^ ((row >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const bf8v*>(sa + pl * PL + o);
    }
    {
      const int col = wn * 32 + (lane & 31);
      const int o = col * BK + 8 * (ch ^ ((col >> 3) & 1));
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) bb[pl] = *reinterpret_cast<const bf8v*>(sb + pl * PL + o);
      if (g.conjB) {
        bb[2] = neg8(bb[2]);
        bb[3] = neg8(bb[3]);
      }
    }
    const bf8v nih = neg8(a[2]), nil = neg8(a[3]);
    const bf8v rh = g.conjA ? a[2] : nih, rl = g.conjA ? a[3] : nil;
    const bf8v ih = g.conjA ? nih : a[2], il = g.conjA ? nil : a[3];
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[0], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[2], accI, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[1], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[3], accI, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bb[2], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bb[0], accI, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[3], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[1], accI, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[0], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[2], accI, 0, 0, 0);
    accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bb[2], accR, 0, 0, 0);
    accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bb[0], accI, 0, 0, 0);
  }
  // register r holds row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of the wave's tile
  if constexpr (CS) {
    // planes [4][64][64] through LDS (free once every wave is past its last stage read), then 16-byte stores
    vm_lds_barrier<0>();
    __bf16* sC = smem;
    const float al = (float)g.alpha;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = wn * 32 + (lane & 31);
      __bf16 hh, ll;
      split_bf16(al * accR[r], hh, ll);
      sC[(0 * 64 + row) * 64 + col] = hh;
      sC[(1 * 64 + row) * 64 + col] = ll;
      split_bf16(al * accI[r], hh, ll);
      sC[(2 * 64 + row) * 64 + col] = hh;
      sC[(3 * 64 + row) * 64 + col] = ll;
    }
    vm_lds_barrier<63>();
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int id = tid + 256 * it;
      const int c8 = id & 7, row = (id >> 3) & 63, pl = id >> 9;
      const int grow = m0 + row, gcol = n0 + c8 * 8;
      if (grow < g.M && gcol < g.N) {
        const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, grow);
        __bf16* o = (__bf16*)g.C + pl * g.c_ps + ro + gcol;
        const bf8v v = *reinterpret_cast<const bf8v*>(&sC[(pl * 64 + row) * 64 + c8 * 8]);
        if (gcol + 8 <= g.N && ((ro + gcol) & 7) == 0) {
          *reinterpret_cast<bf8v*>(o) = v;
        } else {
          for (int e = 0; e < 8 && gcol + e < g.N; ++e) o[e] = v[e];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int col = n0 + wn * 32 + (lane & 31);
    if (row >= g.M || col >= g.N) continue;
    const long long ro = off_of(g.c_tab, g.c_tab_pb, g.c_sb, g.c_si, b, g.M, row);
    TC* o = (TC*)g.C + 2 * (ro + (long long)col * g.c_sj);
    double vr = g.alpha * (double)accR[r], vi = g.alpha * (double)accI[r];
    if (g.beta) {
      vr += (double)o[0];
      vi += (double)o[1];
    }
    o[0] = (TC)vr;
    o[1] = (TC)vi;
  }
}

// ----------------------------------------------------------------------------
// BF16X3, both operands pre-split and k-major:  C[b][m][n] = sum_k A[b][k][m] B[b][k][n]
//
// For reductions over a long row index (the gradient of W(q) sums over every
// pair of a q).  Rows k of A and B are contiguous in m / n, so the MFMA operand
// layout (8 consecutive k per lane) needs a transpose: each thread loads an 8 x 8
// (k x column) block of one plane with eight 16-byte loads, transposes it in
// registers and writes eight 16-byte column vectors to LDS.  LDS rows are the
// tile's columns (16 k each, two 8-k halves); within each group of 8 rows the
// row is XOR-permuted by the group index so that the eight rows a thread writes
// per instruction, and the rows of different threads, spread over the banks, and
// the two halves swap places in every other group (bit 3 of the row) so that the
// fragment reads of rows r and r + 8 do not share banks.
// Same tile and MFMA order as the other BF16x3 kernels.  The K range can be
// split over blocks (split s covers [s kc, (s+1) kc)): partial sums go to a
// FP64 buffer part[b][s][m][n] and are added in split order by tn_reduce.
// CS writes C pre-split instead (one split only).
// ----------------------------------------------------------------------------
__device__ __forceinline__ int tn_row(int m) { return (m & ~7) | ((m ^ (m >> 3)) & 7); }

// TM = 32-row tiles per wave in m: BM = 64 TM (TM = 1 for products of at most 64 rows, such as the n_v^2
// rows of Z at n_v = 8, which would leave half of a 128-row tile empty)
template <bool CS, int TM>
__global__ __launch_bounds__(256) void cgemm_b3_tn(GemmArgs g, int nsplit, int kc, double* __restrict__ part) {
  constexpr int BM = 64 * TM, BN = 128, BK = 16;
  constexpr int PLA = BM * BK, PLB = BN * BK;  // bf16 per plane per stage of A and of B
  constexpr int SS = 4 * (PLA + PLB);
  __shared__ __attribute__((aligned(16))) __bf16 smem[2 * SS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int gxn = (g.N + BN - 1) / BN, gyn = (g.M + BM - 1) / BM;
  const long long per = (long long)gxn * gyn;
  long long bl, t;
  xcd_map(blockIdx.x, per, (long long)g.batch * nsplit, bl, t);
  const int b = (int)(bl / nsplit), s = (int)(bl % nsplit);
  const int m0 = (int)(t / gxn) * BM, n0 = (int)(t % gxn) * BN;
  const int k_lo = s * kc, k_hi = min(g.K, k_lo + kc);
  const int nK = (k_hi - k_lo + BK - 1) / BK;

  // staging role (wave-uniform operand): threads 0 .. BM-1 stage A, the next 128 B (the last wave idles
  // when TM = 1); plane pl, k half kh (rows 8 kh .. 8 kh + 7 of the step), columns 8 cb .. 8 cb + 7
  const int isB = tid >= BM ? 1 : 0;
  const bool active = tid < BM + 128;
  const int u = isB ? tid - BM : tid;
  const int per_plane = isB ? 32 : 16 * TM;
  const int pl = u / per_plane, w = u % per_plane;
  const int kh = (w >> 3) & 1, cb = (w & 7) | ((w >> 4) << 3);  // 16 lanes: 16 distinct bank slots
  const int c0 = (isB ? n0 : m0) + 8 * cb;
  const bool cok = active && c0 < (isB ? g.N : g.M);
  const long long ld = isB ? g.b_sk : g.a_sk;
  const __bf16* src = (const __bf16*)(isB ? g.B : g.A) + (isB ? g.b_ps : g.a_ps) * pl +
                      (long long)b * (isB ? g.b_sb : g.a_sb) + (cok ? c0 : 0);
  const unsigned flip = ((isB ? g.conjB : g.conjA) && pl >= 2) ? 0x80008000u : 0u;  // conj: -Im planes
  // the two 8-k halves of a row are swapped in every other group of 8 rows (bit 3 of the row), as in the
  // direct-to-LDS kernels: the fragment reads of rows r and r + 8 then fall on different banks
  __bf16* const dst0 = smem + (isB ? 4 * PLA + pl * PLB : pl * PLA) + 8 * (kh ^ (cb & 1));

  u4v v[8];
  auto gload = [&](int kt) {
    const int kb = k_lo + kt * BK + 8 * kh;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (cok && kb + r < k_hi)
        v[r] = *reinterpret_cast<const u4v*>(src + (long long)(kb + r) * ld);
      else
        v[r] = u4v{0u, 0u, 0u, 0u};
    }
  };
  auto lstore = [&](int st) {
    if (!active) return;
    __bf16* dst = dst0 + st * SS;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      // column c of the 8 x 8 block: dword j holds rows 2j (low half) and 2j + 1 (high half)
      u4v w;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned lo = v[2 * j][c >> 1], hi = v[2 * j + 1][c >> 1];
        w[j] = (c & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
      }
      w ^= flip;
      *reinterpret_cast<u4v*>(dst + tn_row(8 * cb + c) * BK) = w;
    }
  };

  f16v accR[TM][2], accI[TM][2];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[i][j][r] = 0.f;
        accI[i][j][r] = 0.f;
      }
  if (nK > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nK; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < nK) gload(kt + 1);
    const __bf16* sa = smem + st * SS;
    const __bf16* sb = sa + 4 * PLA;
    bf8v a[TM][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = tn_row(wm * 32 * TM + i * 32 + (lane & 31));
      const int o = r * BK + 8 * ((lane >> 5) ^ ((r >> 3) & 1));
#pragma unroll
      for (int q = 0; q < 4; ++q) a[i][q] = *reinterpret_cast<const bf8v*>(sa + q * PLA + o);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int r = tn_row(wn * 64 + j * 32 + (lane & 31));
      const int o = r * BK + 8 * ((lane >> 5) ^ ((r >> 3) & 1));
#pragma unroll
      for (int q = 0; q < 4; ++q) bb[j][q] = *reinterpret_cast<const bf8v*>(sb + q * PLB + o);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
#pragma unroll
      for (int j = 0; j < 2; ++j) cmma_b3(a[i], nih, nil, bb[j], accR[i][j], accI[i][j]);
    }
    if (kt + 1 < nK) lstore(st ^ 1);
    __syncthreads();
  }
  // register r of a lane holds row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32 of its 32 x 32 tile
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wm * 32 * TM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (row >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn * 64 + j * 32 + (lane & 31);
        if (col >= g.N) continue;
        if constexpr (CS) {
          __bf16* o = (__bf16*)g.C + (long long)b * g.c_sb + (long long)row * g.c_si + (long long)col * g.c_sj;
          __bf16 h, l;
          split_bf16((float)(g.alpha * (double)accR[i][j][r]), h, l);
          o[0] = h;
          o[g.c_ps] = l;
          split_bf16((float)(g.alpha * (double)accI[i][j][r]), h, l);
          o[2 * g.c_ps] = h;
          o[3 * g.c_ps] = l;
        } else {
          double* o = part + 2 * ((((long long)b * nsplit + s) * g.M + row) * g.N + col);
          *reinterpret_cast<double2*>(o) = make_double2((double)accR[i][j][r], (double)accI[i][j][r]);
        }
      }
    }
  }
}

// C[b'][m][n] = alpha * sum_s part[b][s][m][n] (+ C if beta), splits added in order; C is c128 and
// b' = c_bidx[b] when a batch index table is given
__global__ void tn_reduce(GemmArgs g, int nsplit, const double* __restrict__ part) {
  const long long mn = (long long)g.M * g.N, n = mn * g.batch;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / mn, e = i % mn;
    const int row = (int)(e / g.N), col = (int)(e % g.N);
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const double2 v = reinterpret_cast<const double2*>(part)[(b * nsplit + s) * mn + e];
      sr += v.x;
      si += v.y;
    }
    const long long bo = g.c_bidx ? (long long)g.c_bidx[b] : b;
    double* o = (double*)g.C + 2 * (bo * g.c_sb + (long long)row * g.c_si + (long long)col * g.c_sj);
    double vr = g.alpha * sr, vi = g.alpha * si;
    if (g.beta) {
      vr += o[0];
      vi += o[1];
    }
    o[0] = vr;
    o[1] = vi;
  }
}

template <typename K>
bse_status launch(K kern, const GemmArgs& g, int BM, int BN, hipStream_t st) {
  const long long gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
  if (gy > 65535) {
    set_error("cgemm: too many row tiles");
    return BSE_ESHAPE;
  }
  const int gz = g.batch < 65535 ? g.batch : 65535;
  hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(256), 0, st, g);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// 1-D launch of the XCD-aware large-tile kernel (it loops if the grid is capped)
template <typename K>
bse_status launch_1d(K kern, const GemmArgs& g, int BM, int BN, hipStream_t st) {
  const long long tiles = (long long)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * g.batch;
  const long long cap = 1LL << 30;
  const unsigned gx = (unsigned)(tiles < cap ? tiles : cap);
  hipLaunchKernelGGL(kern, dim3(gx), dim3(256), 0, st, g);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// shape classes: wide (64 x 64), narrow-N (64 x 16), narrow-M (16 x 64)
enum Shape { SH_WIDE, SH_NARROW_N, SH_NARROW_M };
Shape pick(const GemmArgs& g) {
  if (g.N <= 16 && g.M > 16) return SH_NARROW_N;
  if (g.M <= 16 && g.N > 16) return SH_NARROW_M;
  return SH_WIDE;
}

bool dma_ok(const GemmArgs& g);
bool wide_tiles_enabled();

template <typename TC>
bse_status launch_f32_wide(const GemmArgs& g, hipStream_t st) {
  const long long tiles = (long long)((g.N + FW_BN - 1) / FW_BN) * ((g.M + FW_BM - 1) / FW_BM) * g.batch;
  const dim3 grid((unsigned)tiles), block(512);
  auto go = [&](auto kern) -> bse_status {
    BSE_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FW_LDS));
    hipLaunchKernelGGL(kern, grid, block, FW_LDS, st, g);
    BSE_CHECK_LAUNCH();
    return BSE_OK;
  };
  if (g.conjA && g.conjB) return go(cgemm_f32_dma_w<1, 1, TC>);
  if (g.conjA) return go(cgemm_f32_dma_w<1, 0, TC>);
  if (g.conjB) return go(cgemm_f32_dma_w<0, 1, TC>);
  return go(cgemm_f32_dma_w<0, 0, TC>);
}

template <typename T, typename TC>
bse_status run_real(const GemmArgs& g, hipStream_t st) {
  constexpr int BK = 16;  // 16 complex k per stage: the FP32 tile spills at two waves per SIMD with 32
  if constexpr (sizeof(T) == 4) {
    // FP32 products with enough rows and columns for the wide tile (direct-to-LDS operands)
    const long long tiles = (long long)((g.N + FW_BN - 1) / FW_BN) * ((g.M + FW_BM - 1) / FW_BM) * g.batch;
    if (g.M >= FW_BM && g.N >= FW_BN && g.K % FW_BK == 0 && dma_ok(g) && tiles < (1LL << 31) &&
        wide_tiles_enabled())
      return launch_f32_wide<TC>(g, st);
    // small per-pair products with a long K (the direct block): 64 x 64 tiles, one per batch entry, where
    // they are at least a quarter full (narrower products keep the 64 x 16 tiles below)
    if (g.M <= F64T_BM && g.N <= F64T_BN && g.M > 32 && g.N > 32 && g.K % F64T_BK == 0 &&
        g.K >= 4 * F64T_BK && dma_ok(g) && wide_tiles_enabled()) {
      const dim3 grid((unsigned)g.batch), block(256);
      if (g.conjA && g.conjB)
        hipLaunchKernelGGL((cgemm_f32_dma64<1, 1, TC>), grid, block, 0, st, g);
      else if (g.conjA)
        hipLaunchKernelGGL((cgemm_f32_dma64<1, 0, TC>), grid, block, 0, st, g);
      else if (g.conjB)
        hipLaunchKernelGGL((cgemm_f32_dma64<0, 1, TC>), grid, block, 0, st, g);
      else
        hipLaunchKernelGGL((cgemm_f32_dma64<0, 0, TC>), grid, block, 0, st, g);
      BSE_CHECK_LAUNCH();
      return BSE_OK;
    }
  }
  switch (pick(g)) {
    case SH_NARROW_N:
      return launch(cgemm_real<T, TC, 4, 1, 1, 2, BK>, g, 64, 16, st);
    case SH_NARROW_M:
      return launch(cgemm_real<T, TC, 1, 4, 1, 2, BK>, g, 16, 64, st);
    default:
      return launch(cgemm_real<T, TC, 2, 2, 2, 4, BK>, g, 64, 64, st);
  }
}

template <typename TC>
bse_status run_bf16(const GemmArgs& g, hipStream_t st) {
  if (g.M >= 64 && g.N >= 64) return launch_1d(cgemm_b3_big<false, false, false, TC>, g, 128, 128, st);
  switch (pick(g)) {
    case SH_NARROW_N:
      return launch(cgemm_bf16x3<TC, 4, 1, 1, 2, 32>, g, 64, 16, st);
    case SH_NARROW_M:
      return launch(cgemm_bf16x3<TC, 1, 4, 1, 2, 32>, g, 16, 64, st);
    default:
      return launch(cgemm_bf16x3<TC, 2, 2, 2, 4, 32>, g, 64, 64, st);
  }
}

// BSE_WIDE_TILES=0 keeps long-K split-output products on the 64 x 128 tiles (identical results; read at
// every launch so that one process can time and compare both)
bool wide_tiles_enabled() {
  const char* e = std::getenv("BSE_WIDE_TILES");
  return !(e && e[0] == '0');
}

// BSE_STREAM_PD=0 keeps the short-K split products on the tiled kernels (identical results; read at every
// launch)
bool stream_enabled() {
  const char* e = std::getenv("BSE_STREAM_PD");
  return !(e && e[0] == '0');
}

// the direct-to-LDS kernel needs unit k stride, whole K steps and 16-byte aligned operand rows
bool dma_ok(const GemmArgs& g) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (g.a_sk != 1 || g.b_sk != 1 || g.K % 16 != 0) return false;
  if (!al(g.A) || !al(g.B) || (g.a_ps & 7) || (g.b_ps & 7)) return false;
  if (g.a_tab ? !g.tab_aligned : ((g.a_sb & 7) || (g.a_si & 7))) return false;
  if (g.b_tab ? !g.tab_aligned : ((g.b_sb & 7) || (g.b_sj & 7))) return false;
  const long long tiles = (long long)((g.N + 127) / 128) * ((g.M + 127) / 128) * g.batch;
  return tiles < (1LL << 31);
}

template <bool CS, typename TC>
bse_status launch_dma(const GemmArgs& g, hipStream_t st) {
  const long long tiles = (long long)((g.N + 127) / 128) * ((g.M + 127) / 128) * g.batch;
  const dim3 grid((unsigned)tiles), block(256);
  if (g.conjA && g.conjB)
    hipLaunchKernelGGL((cgemm_b3_dma<1, 1, CS, TC>), grid, block, 0, st, g);
  else if (g.conjA)
    hipLaunchKernelGGL((cgemm_b3_dma<1, 0, CS, TC>), grid, block, 0, st, g);
  else if (g.conjB)
    hipLaunchKernelGGL((cgemm_b3_dma<0, 1, CS, TC>), grid, block, 0, st, g);
  else
    hipLaunchKernelGGL((cgemm_b3_dma<0, 0, CS, TC>), grid, block, 0, st, g);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// the k-major kernel: unit m / n strides, 16-byte aligned rows of whole 8-column chunks, no tables
bool tn_ok(const GemmArgs& g) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (g.a_si != 1 || g.b_sj != 1 || g.a_tab || g.b_tab || g.c_tab) return false;
  if (!al(g.A) || !al(g.B) || (g.M & 7) || (g.N & 7)) return false;
  if ((g.a_sk & 7) || (g.b_sk & 7) || (g.a_sb & 7) || (g.b_sb & 7) || (g.a_ps & 7) || (g.b_ps & 7)) return false;
  const long long tiles = (long long)((g.N + 127) / 128) * ((g.M + 127) / 128) * g.batch;
  return tiles < (1LL << 24);
}

// split K over enough blocks to fill the chip (about 2048 blocks, at least 1024 k per split)
bse_status launch_tn(const GemmArgs& g, bool c_split, hipStream_t st) {
  const bool small = g.M <= 64;  // 64-row tiles
  const long long tiles = (long long)((g.N + 127) / 128) * ((g.M + (small ? 63 : 127)) / (small ? 64 : 128)) * g.batch;
  if (c_split) {
    if (g.c_bidx) {
      set_error("cgemm_b3_tn: a batch index table needs a c128 result");
      return BSE_EINVAL;
    }
    if (small)
      hipLaunchKernelGGL((cgemm_b3_tn<true, 1>), dim3((unsigned)tiles), dim3(256), 0, st, g, 1, g.K, (double*)nullptr);
    else
      hipLaunchKernelGGL((cgemm_b3_tn<true, 2>), dim3((unsigned)tiles), dim3(256), 0, st, g, 1, g.K, (double*)nullptr);
    BSE_CHECK_LAUNCH();
    return BSE_OK;
  }
  long long ns = (2048 + tiles - 1) / tiles;
  ns = std::max(1LL, std::min<long long>(ns, g.K / 1024));
  const int kc = (int)(((g.K + ns - 1) / ns + 15) / 16 * 16);
  const int nsplit = (g.K + kc - 1) / kc;
  double* part = nullptr;
  const size_t bytes = 16 * (size_t)g.batch * nsplit * g.M * g.N;
  BSE_HIP(hipMallocAsync((void**)&part, bytes, st));
  if (small)
    hipLaunchKernelGGL((cgemm_b3_tn<false, 1>), dim3((unsigned)(tiles * nsplit)), dim3(256), 0, st, g, nsplit, kc, part);
  else
    hipLaunchKernelGGL((cgemm_b3_tn<false, 2>), dim3((unsigned)(tiles * nsplit)), dim3(256), 0, st, g, nsplit, kc, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const long long n = (long long)g.batch * g.M * g.N;
    hipLaunchKernelGGL(tn_reduce, dim3((unsigned)std::min<long long>((n + 255) / 256, 65536)), dim3(256), 0, st, g,
                       nsplit, (const double*)part);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(part, st);
  if (e != hipSuccess) {
    set_error(std::string("cgemm_b3_tn: ") + hipGetErrorString(e));
    return BSE_EDEVICE;
  }
  return BSE_OK;
}

}  // namespace

bse_status wstep_dblock(const GemmArgs& g, const __bf16* mc, long long mc_sb, long long mc_ps, float* t, long long t_sb,
                        hipStream_t st) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (g.M <= 0 || g.batch <= 0) return BSE_OK;
  if (g.M % WB_BM || g.N % WB_BN || g.K % WB_BK || g.N != g.K || !g.conjA || g.conjB || g.a_tab || g.b_tab ||
      g.a_sk != 1 || g.b_sk != 1 || !al(g.A) || !al(g.B) || !al(mc) || (g.a_sb & 7) || (g.a_si & 7) ||
      (g.b_sb & 7) || (g.b_sj & 7) || (g.a_ps & 7) || (g.b_ps & 7) || (mc_sb & 7) || (mc_ps & 7)) {
    set_error("wstep_dblock: unsupported operand shape or alignment");
    return BSE_ESHAPE;
  }
  const long long tiles = (long long)(g.M / WB_BM) * g.batch;
  if (tiles >= (1LL << 31)) {
    set_error("wstep_dblock: too many tiles");
    return BSE_ESHAPE;
  }
  WTArgs w;
  w.g = g;
  w.mc = mc;
  w.mc_sb = mc_sb;
  w.mc_ps = mc_ps;
  w.t = t;
  w.t_sb = t_sb;
  BSE_HIP(hipFuncSetAttribute((const void*)wstep_dblock_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)WB_LDS));
  hipLaunchKernelGGL(wstep_dblock_fused, dim3((unsigned)tiles), dim3(512), WB_LDS, st, w);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

template <int NK, bool FRAG>
bse_status launch_stream(const GemmArgs& g, hipStream_t st) {
  int dev = 0, ncu = 0;
  BSE_HIP(hipGetDevice(&dev));
  BSE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const long long items = (long long)g.batch * ((g.M + PD_BM - 1) / PD_BM) * ((g.N + PD_BN - 1) / PD_BN);
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(items, ncu));
  BSE_HIP(hipFuncSetAttribute((const void*)cgemm_b3_stream<NK, FRAG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)PD_LDS));
  hipLaunchKernelGGL((cgemm_b3_stream<NK, FRAG>), dim3(grid), dim3(512), PD_LDS, st, g);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bse_status cgemm_split(const GemmArgs& g, bool a_split, bool b_split, bool c_split, bool out_f64, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return BSE_OK;
  if (g.K <= 0) {
    set_error("cgemm_split: K must be positive");
    return BSE_ESHAPE;
  }
  if (g.c_bidx) {  // only the k-major kernel scatters its batches
    if (a_split && b_split && !c_split && out_f64 && !dma_ok(g) && tn_ok(g)) return launch_tn(g, false, st);
    set_error("cgemm_split: a batch index table needs the k-major kernel");
    return BSE_EINVAL;
  }
  if (g.b_frag) {  // a B operand in fragment order: only the streaming kernel reads that layout
    if (!(a_split && b_split && c_split && dma_ok(g) && (g.K == 64 || g.K == 128) && g.N % 32 == 0 && !g.conjA &&
          !g.conjB && !g.b_tab)) {
      set_error("cgemm_split: a fragment-order B needs split operands and result, K of 64 or 128, N a multiple "
                "of 32");
      return BSE_EINVAL;
    }
    return g.K == 64 ? launch_stream<4, true>(g, st) : launch_stream<8, true>(g, st);
  }
  if (a_split && b_split && dma_ok(g)) {
    if (!c_split && g.M <= 64 && g.N <= 64) {  // small per-pair products: quarter-size tiles
      const long long tiles = (long long)g.batch;
      if (out_f64)
        hipLaunchKernelGGL(cgemm_b3_dma64<double>, dim3((unsigned)tiles), dim3(256), 0, st, g);
      else
        hipLaunchKernelGGL(cgemm_b3_dma64<float>, dim3((unsigned)tiles), dim3(256), 0, st, g);
      BSE_CHECK_LAUNCH();
      return BSE_OK;
    }
    if (c_split && g.K <= 64) {  // short K: 64 x 64 tiles, five blocks per CU
      const long long tiles = (long long)((g.N + 63) / 64) * ((g.M + 63) / 64) * g.batch;
      if (tiles < (1LL << 31)) {
        hipLaunchKernelGGL((cgemm_b3_dma64<float, true>), dim3((unsigned)tiles), dim3(256), 0, st, g);
        BSE_CHECK_LAUNCH();
        return BSE_OK;
      }
    }
    if (c_split && (g.K == 64 || g.K == 128) && g.M <= 2 * PD_BM && g.N >= 4 * PD_BN && !g.conjA && !g.conjB &&
        stream_enabled()) {
      // short K, few rows, many columns (the pair densities): persistent streaming blocks, one per CU
      return g.K == 64 ? launch_stream<4, false>(g, st) : launch_stream<8, false>(g, st);
    }
    if (c_split && g.K >= WB_MIN_K && g.N >= 256 && g.M >= 128 && wide_tiles_enabled()) {
      // long K and a wide B (the W step): 128 x 256 tiles, three LDS stages
      const long long tiles = (long long)((g.N + WB_BN - 1) / WB_BN) * ((g.M + WB_BM - 1) / WB_BM) * g.batch;
      if (tiles < (1LL << 31)) {
        const dim3 grid((unsigned)tiles), block(512);
        auto go = [&](auto kern) -> bse_status {
          BSE_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)WB_LDS));
          hipLaunchKernelGGL(kern, grid, block, WB_LDS, st, g);
          BSE_CHECK_LAUNCH();
          return BSE_OK;
        };
        if (g.conjA && g.conjB) return go(cgemm_b3_dma_w<1, 1>);
        if (g.conjA) return go(cgemm_b3_dma_w<1, 0>);
        if (g.conjB) return go(cgemm_b3_dma_w<0, 1>);
        return go(cgemm_b3_dma_w<0, 0>);
      }
    }
    if (c_split) {  // longer K: 64 x 128 tiles, three blocks per CU
      const long long tiles = (long long)((g.N + 127) / 128) * ((g.M + 63) / 64) * g.batch;
      if (tiles < (1LL << 31)) {
        const dim3 grid((unsigned)tiles), block(256);
        if (g.conjA && g.conjB)
          hipLaunchKernelGGL((cgemm_b3_dma_m64<1, 1>), grid, block, 0, st, g);
        else if (g.conjA)
          hipLaunchKernelGGL((cgemm_b3_dma_m64<1, 0>), grid, block, 0, st, g);
        else if (g.conjB)
          hipLaunchKernelGGL((cgemm_b3_dma_m64<0, 1>), grid, block, 0, st, g);
        else
          hipLaunchKernelGGL((cgemm_b3_dma_m64<0, 0>), grid, block, 0, st, g);
        BSE_CHECK_LAUNCH();
        return BSE_OK;
      }
      return launch_dma<true, float>(g, st);
    }
    return out_f64 ? launch_dma<false, double>(g, st) : launch_dma<false, float>(g, st);
  }
  if (a_split && b_split && (c_split || out_f64) && tn_ok(g)) return launch_tn(g, c_split, st);
#define BSE_SPLIT_CASE(AS, BS, CS)                                                              \
  if (a_split == AS && b_split == BS && c_split == CS)                                           \
    return out_f64 ? launch_1d(cgemm_b3_big<AS, BS, CS, double>, g, 128, 128, st)                \
                   : launch_1d(cgemm_b3_big<AS, BS, CS, float>, g, 128, 128, st);
  BSE_SPLIT_CASE(true, true, true)
  BSE_SPLIT_CASE(true, true, false)
  BSE_SPLIT_CASE(true, false, false)
  BSE_SPLIT_CASE(false, true, false)
  BSE_SPLIT_CASE(false, false, false)
  BSE_SPLIT_CASE(false, true, true)
  BSE_SPLIT_CASE(false, false, true)
#undef BSE_SPLIT_CASE
  set_error("cgemm_split: unsupported operand combination");
  return BSE_EINVAL;
}

bse_status cgemm(const GemmArgs& g, Arith ar, bool in_f64, bool out_f64, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return BSE_OK;
  if (g.c_bidx) {
    set_error("cgemm: batch index tables are for the k-major split kernel only");
    return BSE_EINVAL;
  }
  if (g.K <= 0) {
    set_error("cgemm: K must be positive");
    return BSE_ESHAPE;
  }
  if (ar == AR_F64) {
    if (!in_f64) {
      set_error("cgemm: FP64 arithmetic needs c128 operands");
      return BSE_EINVAL;
    }
    return out_f64 ? run_real<double, double>(g, st) : run_real<double, float>(g, st);
  }
  if (in_f64) {
    set_error("cgemm: reduced-precision arithmetic needs c64 operands");
    return BSE_EINVAL;
  }
  if (ar == AR_F32) return out_f64 ? run_real<float, double>(g, st) : run_real<float, float>(g, st);
  return out_f64 ? run_bf16<double>(g, st) : run_bf16<float>(g, st);
}

}  // namespace bse
