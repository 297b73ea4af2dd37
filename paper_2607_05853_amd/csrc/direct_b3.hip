// Conduction side of the direct term on the BF16x3 path, without forming the
// conduction pair densities.  With M^nu_{cc'}(k,k') = sum_t B^nu_{ct}(k) psi_{c't}(k'):
//
//   T(k,k')[(c'c)][(v'v)] = sum_nu M^nu_{cc'}(k,k') P(k,k')[(v'v)][nu]
//                         = sum_t psi_{c't}(k') U(k,k')[(c,t)][(v'v)],
//   U(k,k')[(c,t)][(v'v)] = sum_nu B^nu_{ct}(k) P(k,k')[(v'v)][nu].
//
// One block owns one k, one conduction band c and a group of q: U is a
// complex GEMM (rows t, columns (q, v'v), depth nu) on the 32x32x16 BF16 MFMA
// with pre-split operands; its epilogue stages U in LDS and contracts the AO
// index t with psi(k+q) on the vector units, writing the direct blocks T.
// Nothing of size N_k^2 x n_aux leaves the chip.
#include "bse_internal.h"
#include "mfma_common.h"

namespace bse {
namespace {

__device__ __forceinline__ void vm_wait_barrier0() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ __forceinline__ void lds_wait_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

struct UArgs {
  int Nk, nq, q0, nv, nc, nbnd, no, na, qg;
  const __bf16* BcT;   // planes [Nk][nc][no][na] (K = nu contiguous)
  long long ps_BcT;
  const __bf16* P;     // planes [nq][Nk][nv*nv][na]
  long long ps_P;
  const float* psi;    // c64 [Nk][nbnd][no]
  const int* kq;       // [Nk][Nk]
  float* T;            // c64 [nq][Nk][nc*nc][nv*nv]
  const __bf16* psis;  // planes [Nk][nbnd][no] (pre-split psi) for the matrix-core epilogue
  long long ps_psi;
  int mfma_epi;        // 1: contract t on the matrix cores (needs nv^2 <= 64 and n_ao % 8 == 0)
};

// one complex step of the BF16x3 product on 16x16x32 MFMA (no conjugation):
//   cr += ar br - ai bi,  ci += ar bi + ai br   (each as hi*hi + hi*lo + lo*hi)
__device__ __forceinline__ void cmma16_b3(const bf8v* a, const bf8v* b, f4v& cr, f4v& ci) {
  const bf8v nih = neg8(a[2]), nil = neg8(a[3]);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[2], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[3], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nil, b[2], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3], b[0], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[3], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[1], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nih, b[2], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], ci, 0, 0, 0);
}

template <int TMW>
__global__ __launch_bounds__(256) void u_direct_b3(UArgs u) {
  constexpr int BM = 2 * TMW * 32, BN = 128, BK = 16, HN = 64;
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][4][BM * BK];
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][4][BN * BK];
  __shared__ float2 Us[BM * HN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nv2 = u.nv * u.nv;
  // 1-D grid over (k, q group, c), XCD-aware: all blocks of one k share B_c(k) and P(k, .); the n_c
  // blocks that read one column group of P run back to back
  const int nqg = (u.nq + u.qg - 1) / u.qg;
  long long kl, t;
  xcd_map(blockIdx.x, (long long)u.nc * nqg, u.Nk, kl, t);
  const int k = (int)kl, c = (int)(t % u.nc);
  const int qbase = (int)(t / u.nc) * u.qg;  // batch-local index of the first q of the group
  const int ncol = min(u.qg, u.nq - qbase) * nv2;
  const int na = u.na, no = u.no, Nk = u.Nk;

  // staging slices: rows / columns tid/2, k half tid%2
  const int sr = tid >> 1, sh = tid & 1;
  const bool a_thread = sr < BM;
  const bool aok = a_thread && sr < no;
  const long long aoff = aok ? ((long long)(k * u.nc + c) * no + sr) * na : 0;
  const bool bok = sr < ncol;
  long long boff = 0;
  if (bok) {
    const int ql = sr / nv2, r = sr % nv2;
    boff = ((long long)(qbase + ql) * Nk + k) * nv2 * na + (long long)r * na;
  }
  const int nK = (na + BK - 1) / BK;
  bf8v pa[4], pb[4];
  auto load = [&](const __bf16* base, long long ps, long long off, bool ok, int kb, bf8v* out) {
    if (ok && ((off + kb) & 7) == 0 && kb + 8 <= na) {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) out[pl] = *reinterpret_cast<const bf8v*>(base + pl * ps + off + kb);
    } else {
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
#pragma unroll
        for (int e = 0; e < 8; ++e) out[pl][e] = (ok && kb + e < na) ? base[pl * ps + off + kb + e] : (__bf16)0.f;
    }
  };
  auto gload = [&](int kt) {
    const int kb = kt * BK + 8 * sh;
    if (a_thread) load(u.BcT, u.ps_BcT, aoff, aok, kb, pa);
    load(u.P, u.ps_P, boff, bok, kb, pb);
  };
  auto lstore = [&](int st) {
    const int o = sr * BK + 8 * sh;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      if (a_thread) *reinterpret_cast<bf8v*>(&sA[st][pl][o]) = pa[pl];
      *reinterpret_cast<bf8v*>(&sB[st][pl][o]) = pb[pl];
    }
  };

  f16v accR[TMW][2], accI[TMW][2];
#pragma unroll
  for (int i = 0; i < TMW; ++i)
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
    bf8v a[TMW][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < TMW; ++i) {
      const int row = wm * TMW * 32 + i * 32 + (lane & 31);
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
    for (int i = 0; i < TMW; ++i) {
      const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
#pragma unroll
      for (int j = 0; j < 2; ++j) cmma_b3(a[i], nih, nil, bb[j], accR[i][j], accI[i][j]);
    }
    if (kt + 1 < nK) lstore(st ^ 1);
    __syncthreads();
  }

  // epilogue, one half of the columns at a time: U -> LDS, then T = psi(k+q) U over t
  const int nc = u.nc;
  for (int h = 0; h < 2; ++h) {
    if (wn == h) {
#pragma unroll
      for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = wm * TMW * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int col = j * 32 + (lane & 31);
            Us[row * HN + col] = make_float2(accR[i][j][r], accI[i][j][r]);
          }
    }
    __syncthreads();
    // outputs (c', col) of this half: col -> (q, v'v)
    for (int o = tid; o < nc * HN; o += 256) {
      const int col = o % HN, cp = o / HN;
      const int gcol = h * HN + col;
      if (gcol >= ncol) continue;
      const int ql = gcol / nv2, r = gcol % nv2;
      const int qi = qbase + ql;
      const int kp = u.kq[(long long)k * Nk + u.q0 + qi];
      const float* ps = u.psi + 2 * ((long long)kp * u.nbnd + u.nv + cp) * no;
      float sr_ = 0.f, si_ = 0.f;
      for (int t = 0; t < no; ++t) {
        const float2 uv = Us[t * HN + col];
        const float pr = ps[2 * t], pi = ps[2 * t + 1];
        sr_ += pr * uv.x - pi * uv.y;
        si_ += pr * uv.y + pi * uv.x;
      }
      float* out = u.T + 2 * ((((long long)qi * Nk + k) * nc * nc + (long long)cp * nc + c) * nv2 + r);
      out[0] = sr_;
      out[1] = si_;
    }
    __syncthreads();
  }
}


// Same computation with direct-to-LDS staging of both operands (global_load_lds_dwordx4,
// two stages, XOR-swizzled 16-byte k chunks as in the split GEMM); needs N_aux % 16 == 0.
// MEPI picks the epilogue at compile time: with both in one kernel the accumulators stay live across
// the matrix-core epilogue and spill.  The 64-row tile (N_ao <= 64) fits 168 VGPRs and 48 KiB of LDS,
// so three blocks share a CU (three waves per SIMD) to cover the per-stage barrier.
template <int TMW, bool MEPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TMW == 1 ? 3 : 1, TMW == 1 ? 3 : 1))) void u_direct_b3_dma(UArgs u) {
  constexpr int BM = 2 * TMW * 32, BN = 128, BK = 16, HN = 64;
  constexpr int PA = BM * BK, PB = BN * BK;  // bf16 per plane per stage
  constexpr int STAGE = 4 * (PA + PB);
  constexpr int RBA = BM / 32, RB = (BM + BN) / 32;  // 32-row blocks of A, of A and B together
  __shared__ __attribute__((aligned(1024))) __bf16 smem[2 * STAGE];
  float2* Us = reinterpret_cast<float2*>(smem);  // epilogue: [BM][HN] (reuses the stages)
  static_assert(BM * HN * 8 <= 2 * STAGE * 2, "epilogue staging must fit in the stages");

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nv2 = u.nv * u.nv;
  const int nqg = (u.nq + u.qg - 1) / u.qg;
  long long kl, t;
  xcd_map(blockIdx.x, (long long)u.nc * nqg, u.Nk, kl, t);
  const int k = (int)kl, c = (int)(t % u.nc);  // c fastest: the n_c blocks of one P column group in a row
  const int qbase = (int)(t / u.nc) * u.qg;
  const int ncol = min(u.qg, u.nq - qbase) * nv2;
  const int na = u.na, no = u.no, Nk = u.Nk;
  const int nK = na / BK;

  // DMA slots: 32-row block rb (A rows first, then B columns) is loaded by wave rb % 4, so a wave owns
  // row blocks wave and wave + 4; lane -> row 32 rb' + lane / 2, 16-byte chunk (lane % 2) ^ bit 3 of the row
  auto slot = [&](int rb, const __bf16*& src, int& lo, long long& ps, int& pstride) {
    const bool isA = rb < RBA;
    const int r = 32 * (isA ? rb : rb - RBA) + (lane >> 1);
    const int chunk = (lane & 1) ^ ((r >> 3) & 1);
    if (isA) {
      const int tr = r < no ? r : 0;  // rows past N_ao re-load row 0; those U rows are never used
      src = u.BcT + ((long long)(k * u.nc + c) * no + tr) * na + 8 * chunk;
      lo = 32 * rb * BK;
      ps = u.ps_BcT;
      pstride = PA;
    } else {
      const int cc = r < ncol ? r : 0;  // columns past the group re-load column 0; never stored
      const int ql = cc / nv2, rr = cc % nv2;
      src = u.P + ((long long)(qbase + ql) * Nk + k) * nv2 * na + (long long)rr * na + 8 * chunk;
      lo = 4 * PA + 32 * (rb - RBA) * BK;
      ps = u.ps_P;
      pstride = PB;
    }
  };
  const __bf16 *src0 = nullptr, *src1 = nullptr;
  int lo0 = 0, lo1 = 0, pst0 = 0, pst1 = 0;
  long long ps0 = 0, ps1 = 0;
  slot(wave, src0, lo0, ps0, pst0);  // RB >= 6 > wave always
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

  f16v accR[TMW][2], accI[TMW][2];
#pragma unroll
  for (int i = 0; i < TMW; ++i)
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
    vm_wait_barrier0();
    if (kt + 1 < nK) issue(kt + 1);
    const __bf16* sa = smem + (kt & 1) * STAGE;
    const __bf16* sb = sa + 4 * PA;
    bf8v a[TMW][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < TMW; ++i) {
      const int row = wm * TMW * 32 + i * 32 + (lane & 31);
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
#pragma unroll
    for (int i = 0; i < TMW; ++i) {
      const bf8v nih = neg8(a[i][2]), nil = neg8(a[i][3]);
#pragma unroll
      for (int j = 0; j < 2; ++j) cmma_b3(a[i], nih, nil, bb[j], accR[i][j], accI[i][j]);
    }
  }
  vm_wait_barrier0();

  const int nc = u.nc;
  if constexpr (MEPI) {
    // T_q = Psi_q U_q for every q of the group, on 16x16x32 MFMA: U is split into bf16 planes in LDS,
    // [plane][column][t] with row stride TPAD (zero for t >= n_ao), one pass per PW columns holding whole q
    constexpr int PW = 64, TPAD = BM + 8, UPL = PW * TPAD;
    __shared__ __attribute__((aligned(16))) __bf16 ubx[TMW == 2 ? 4 * UPL : 8];
    __bf16* Ub = TMW == 2 ? ubx : smem;
    const int qpp = PW / nv2;  // whole q per pass
    const int nql = min(u.qg, u.nq - qbase);
    const int NT = (nv2 + 15) / 16, MT = (nc + 15) / 16, KP = (no + 31) / 32 * 32;
    for (int pq0 = 0; pq0 < nql; pq0 += qpp) {
      const int qcount = min(qpp, nql - pq0);
      const int pc0 = pq0 * nv2, pcn = qcount * nv2;  // tile columns [pc0, pc0 + pcn) in this pass
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int pc = wn * 64 + j * 32 + (lane & 31) - pc0;
        if (pc < 0 || pc >= pcn) continue;
#pragma unroll
        for (int i = 0; i < TMW; ++i)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int t0 = wm * TMW * 32 + i * 32 + 8 * r4 + 4 * (lane >> 5);
            typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
            bf4v rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool ok = t0 + e < no;
              __bf16 hh, ll;
              split_bf16(ok ? accR[i][j][4 * r4 + e] : 0.f, hh, ll);
              rh[e] = hh;
              rl[e] = ll;
              split_bf16(ok ? accI[i][j][4 * r4 + e] : 0.f, hh, ll);
              ih[e] = hh;
              il[e] = ll;
            }
            __bf16* o = Ub + pc * TPAD + t0;
            *reinterpret_cast<bf4v*>(o) = rh;
            *reinterpret_cast<bf4v*>(o + UPL) = rl;
            *reinterpret_cast<bf4v*>(o + 2 * UPL) = ih;
            *reinterpret_cast<bf4v*>(o + 3 * UPL) = il;
          }
      }
      lds_wait_barrier();
      const int nunits = qcount * NT * MT;
      for (int un = wave; un < nunits; un += 4) {
        const int ql = un / (NT * MT), nt = (un / MT) % NT, mt = un % MT;
        const int qi = qbase + pq0 + ql;
        const int kp = u.kq[(long long)k * Nk + u.q0 + qi];
        const int cpa = mt * 16 + (lane & 15);  // A row (conduction band c') of this lane
        const int n = nt * 16 + (lane & 15);    // B column (v'v) of this lane
        const int pcb = min(ql * nv2 + n, PW - 1);
        const __bf16* pa = u.psis + ((long long)kp * u.nbnd + u.nv + (cpa < nc ? cpa : 0)) * no;
        f4v cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < KP; kk += 32) {
          const int t = kk + 8 * (lane >> 4);
          bf8v af[4], bfr[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) {
            if (cpa < nc && t < no)
              af[pl] = *reinterpret_cast<const bf8v*>(pa + pl * u.ps_psi + t);
            else
              af[pl] = bf8v{};
            bfr[pl] = *reinterpret_cast<const bf8v*>(Ub + pl * UPL + pcb * TPAD + t);
          }
          cmma16_b3(af, bfr, cr, ci);
        }
        // lane holds rows c' = 16 mt + 4 (lane / 16) + e, column n
        if (n < nv2) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int cp = mt * 16 + 4 * (lane >> 4) + e;
            if (cp >= nc) continue;
            float* out = u.T + 2 * ((((long long)qi * Nk + k) * nc * nc + (long long)cp * nc + c) * nv2 + n);
            out[0] = cr[e];
            out[1] = ci[e];
          }
        }
      }
      lds_wait_barrier();
    }
  } else {
  for (int h = 0; h < 2; ++h) {
    if (wn == h) {
#pragma unroll
      for (int i = 0; i < TMW; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = wm * TMW * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int col = j * 32 + (lane & 31);
            Us[row * HN + col] = make_float2(accR[i][j][r], accI[i][j][r]);
          }
    }
    lds_wait_barrier();
    for (int o = tid; o < nc * HN; o += 256) {
      const int col = o % HN, cp = o / HN;
      const int gcol = h * HN + col;
      if (gcol >= ncol) continue;
      const int ql = gcol / nv2, r = gcol % nv2;
      const int qi = qbase + ql;
      const int kp = u.kq[(long long)k * Nk + u.q0 + qi];
      const float* ps = u.psi + 2 * ((long long)kp * u.nbnd + u.nv + cp) * no;
      float sr_ = 0.f, si_ = 0.f;
      for (int tt = 0; tt < no; ++tt) {
        const float2 uv = Us[tt * HN + col];
        const float pr = ps[2 * tt], pi = ps[2 * tt + 1];
        sr_ += pr * uv.x - pi * uv.y;
        si_ += pr * uv.y + pi * uv.x;
      }
      float* out = u.T + 2 * ((((long long)qi * Nk + k) * nc * nc + (long long)cp * nc + c) * nv2 + r);
      out[0] = sr_;
      out[1] = si_;
    }
    lds_wait_barrier();
  }
  }
}

}  // namespace

bse_status direct_u_b3(Plan* p, int q0, int nq, const int* kq, hipStream_t st) {
  const bse_dims& d = p->d;
  UArgs u;
  u.Nk = p->Nk;
  u.nq = nq;
  u.q0 = q0;
  u.nv = d.nv;
  u.nc = d.nc;
  u.nbnd = p->nbnd;
  u.no = d.n_ao;
  u.na = d.n_aux;
  const int nv2 = d.nv * d.nv;
  if (nv2 > 128 || d.n_ao > 128) {
    set_error("direct_u_b3: needs nv^2 <= 128 and n_ao <= 128");
    return BSE_ESHAPE;
  }
  u.qg = 128 / nv2;
  u.BcT = (const __bf16*)p->BcT;
  u.ps_BcT = p->ps_Bc;
  u.P = (const __bf16*)p->P;
  u.ps_P = p->ps_Mv;
  u.psi = p->psi32;
  u.kq = kq;
  u.T = (float*)p->T;
  u.psis = (const __bf16*)p->psi;
  u.ps_psi = p->ps_psi;
  u.mfma_epi = nv2 <= 64 && d.n_ao % 8 == 0 && p->ps_psi % 8 == 0 &&
               (reinterpret_cast<uintptr_t>(p->psi) & 15) == 0;
  const dim3 grid((unsigned)((long long)((nq + u.qg - 1) / u.qg) * d.nc * p->Nk));
  const bool dma = d.n_aux % 16 == 0 && u.ps_BcT % 8 == 0 && u.ps_P % 8 == 0 &&
                   (reinterpret_cast<uintptr_t>(u.BcT) & 15) == 0 && (reinterpret_cast<uintptr_t>(u.P) & 15) == 0;
  if (dma) {
    if (d.n_ao <= 64) {
      if (u.mfma_epi)
        hipLaunchKernelGGL((u_direct_b3_dma<1, true>), grid, dim3(256), 0, st, u);
      else
        hipLaunchKernelGGL((u_direct_b3_dma<1, false>), grid, dim3(256), 0, st, u);
    } else {
      if (u.mfma_epi)
        hipLaunchKernelGGL((u_direct_b3_dma<2, true>), grid, dim3(256), 0, st, u);
      else
        hipLaunchKernelGGL((u_direct_b3_dma<2, false>), grid, dim3(256), 0, st, u);
    }
    BSE_CHECK_LAUNCH();
    return BSE_OK;
  }
  if (d.n_ao <= 64)
    hipLaunchKernelGGL(u_direct_b3<1>, grid, dim3(256), 0, st, u);
  else
    hipLaunchKernelGGL(u_direct_b3<2>, grid, dim3(256), 0, st, u);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

}  // namespace bse
