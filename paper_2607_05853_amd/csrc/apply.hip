// Matrix-free action of the TDA Hamiltonian A (Eq. (Hamiltonian) with the LRI
// kernel of Eq. (W_LRI)) and its vector-Jacobian product.
//
// Direct term, per pair (k, k' = k + q), with the halves B^mu_n(k) = psi_n(k)^H C^mu:
//   Gv[v'][v][mu]   = sum_t psi_v'(k')_t B^mu_vt(k)        = conj M^mu_{v'v}(k', k)
//   Mc[c'][c][nu]   = sum_t psi_c'(k')_t B^nu_ct(k)        = M^nu_{cc'}(k, k')
//   P[v'v][nu]      = sum_mu conj(Gv[v'v][mu]) W_munu(q)   (W on the smaller band side)
//   T[c'c][v'v]     = sum_nu Mc[c'c][nu] P[v'v][nu]        = -N_k * direct block
//   Y(k)           -= (1/N_k) sum_q T(k, q) X(k + q)
// All four contractions are batched complex GEMMs on the matrix cores; pairs are
// processed in batches of qb momentum transfers q so that W(q) is read once per
// batch and the per-pair intermediates stay within a fixed workspace.
#include "bse_internal.h"
#include "mfma_common.h"

#include <cstdlib>
#include <type_traits>

namespace bse {
namespace {

// tables of one q batch (q0 .. q0+nq-1), per-batch layout [k][nq*nband]
__global__ void tables_kernel(int Nk, int nq, int q0, int nv, int nc, int nbnd, int n_ao, int n_aux,
                              const int* __restrict__ kq, long long* __restrict__ tpv,
                              long long* __restrict__ tpc, long long* __restrict__ tmv,
                              long long* __restrict__ tmc) {
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < nq * (nv + nc); t += blockDim.x) {
    if (t < nq * nv) {
      const int qi = t / nv, v = t % nv;
      const int kp = kq[(long long)k * Nk + q0 + qi];
      tpv[(long long)k * nq * nv + t] = ((long long)kp * nbnd + v) * n_ao;
      tmv[(long long)k * nq * nv + t] = ((long long)qi * Nk + k) * nv * nv * n_aux + (long long)v * nv * n_aux;
    } else {
      const int u = t - nq * nv;
      const int qi = u / nc, c = u % nc;
      const int kp = kq[(long long)k * Nk + q0 + qi];
      tpc[(long long)k * nq * nc + u] = ((long long)kp * nbnd + nv + c) * n_ao;
      tmc[(long long)k * nq * nc + u] = ((long long)qi * Nk + k) * nc * nc * n_aux + (long long)c * nc * n_aux;
    }
  }
}

// part[chunk][k][(c v)][b] = sum_{qi in chunk} sum_{c'v'} T[qi][k][(c' c)][(v' v)] X[k'][(c' v')][b],
// k' = k + q_j with j = q0 + qi in the order of kqp (block (k, chunk), chunks of qlen consecutive q).
// For j >= nself the partner block is added too: D(k, k - q) = D(k - q, k)^dagger, i.e.
//   part += sum_{c'v'} conj(T[qi][k''][(c c')][(v v')]) X[k''][(c' v')][b],   k'' = kqm[k][j] = k - q_j.
// The (q, pass) items of a chunk are staged in LDS `group` at a time (one T block and one X slice each,
// 16-byte loads where the block size allows), so one pair of barriers serves several items; every
// thread adds the items in the same order as one item at a time.
constexpr size_t TX_STAGE_BYTES = 12 * 1024;  // LDS budget of the staged T.X items per block (occupancy first)

template <typename TT, int SLOTS>
__global__ __launch_bounds__(256) void direct_tx_kernel(int Nk, int nq, int q0, int nv, int nc, int nb, int qlen,
                                                        const int* __restrict__ kqp, const int* __restrict__ kqm,
                                                        int nself, int group, int x16, const TT* __restrict__ T,
                                                        const double* __restrict__ X, double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sbytes[];
  const int k = blockIdx.x, chunk = blockIdx.y;
  const int nt = nc * nv, nt2 = nt * nt;
  const int tbytes = nt2 * 2 * (int)sizeof(TT);
  const int tstride = (tbytes + 15) & ~15;
  const int item_bytes = tstride + nt * nb * 16;
  const bool t16 = (tbytes & 15) == 0;  // T blocks are then 16-byte aligned in global memory as well
  const int nout = nt * nb;  // SLOTS outputs per thread: nt * nb <= SLOTS * 256
  double accr[SLOTS], acci[SLOTS];
#pragma unroll
  for (int r = 0; r < SLOTS; ++r) accr[r] = acci[r] = 0.0;
  const int qa = chunk * qlen, qe = min(nq, qa + qlen);
  // items in order: (qi, pass 0), then (qi, pass 1) when q0 + qi >= nself
  int qi = qa, pass = 0;
  while (qi < qe) {
    // stage up to `group` items
    int cnt = 0, sq = qi, sp = pass;
    __syncthreads();
    while (cnt < group && sq < qe) {
      const int j = q0 + sq;
      const int kb = sp == 0 ? k : kqm[(long long)k * Nk + j];  // block row of the stored T
      const int kx = sp == 0 ? kqp[(long long)k * Nk + j] : kb;  // k-point of the X slice
      const TT* Tg = T + 2 * ((long long)sq * Nk + kb) * nt2;
      const double* Xg = X + 2 * (long long)kx * nt * nb;
      unsigned char* slot = sbytes + (size_t)cnt * item_bytes;
      if (t16) {
        for (int i = threadIdx.x; i < tbytes / 16; i += blockDim.x)
          reinterpret_cast<uint4*>(slot)[i] = reinterpret_cast<const uint4*>(Tg)[i];
      } else {
        for (int i = threadIdx.x; i < tbytes / 8; i += blockDim.x)
          reinterpret_cast<uint2*>(slot)[i] = reinterpret_cast<const uint2*>(Tg)[i];
      }
      if (x16) {
        for (int i = threadIdx.x; i < nout; i += blockDim.x)
          reinterpret_cast<uint4*>(slot + tstride)[i] = reinterpret_cast<const uint4*>(Xg)[i];
      } else {  // X given at 8-byte alignment only
        for (int i = threadIdx.x; i < 2 * nout; i += blockDim.x)
          reinterpret_cast<uint2*>(slot + tstride)[i] = reinterpret_cast<const uint2*>(Xg)[i];
      }
      ++cnt;
      if (sp == 0 && j >= nself) {
        sp = 1;
      } else {
        sp = 0;
        ++sq;
      }
    }
    __syncthreads();
    for (int it = 0; it < cnt; ++it) {
      const TT* Ts = reinterpret_cast<const TT*>(sbytes + (size_t)it * item_bytes);
      const double* Xs = reinterpret_cast<const double*>(sbytes + (size_t)it * item_bytes + tstride);
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        const int o = threadIdx.x + r * blockDim.x;
        if (o >= nout) break;
        const int cv = o / nb, b = o % nb;
        const int c = cv / nv, v = cv % nv;
        double sr = 0, si = 0;
        for (int cp = 0; cp < nc; ++cp) {
          const double* xrow = Xs + 2 * ((cp * nv) * nb + b);
          if (pass == 0) {
            const TT* trow = Ts + 2 * ((cp * nc + c) * (nv * nv) + v);
            for (int vp = 0; vp < nv; ++vp) {
              const double tr = (double)trow[2 * vp * nv], ti = (double)trow[2 * vp * nv + 1];
              const double xr = xrow[2 * vp * nb], xi = xrow[2 * vp * nb + 1];
              sr += tr * xr - ti * xi;
              si += tr * xi + ti * xr;
            }
          } else {
            const TT* trow = Ts + 2 * ((c * nc + cp) * (nv * nv) + v * nv);
            for (int vp = 0; vp < nv; ++vp) {
              const double tr = (double)trow[2 * vp], ti = -(double)trow[2 * vp + 1];
              const double xr = xrow[2 * vp * nb], xi = xrow[2 * vp * nb + 1];
              sr += tr * xr - ti * xi;
              si += tr * xi + ti * xr;
            }
          }
        }
        accr[r] += sr;
        acci[r] += si;
      }
      // advance (qi, pass) in step with the staging order
      if (pass == 0 && q0 + qi >= nself) {
        pass = 1;
      } else {
        pass = 0;
        ++qi;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < SLOTS; ++r) {
    const int o = threadIdx.x + r * blockDim.x;
    if (o >= nout) break;
    double* y = part + 2 * (((long long)chunk * Nk + k) * nout + o);
    y[0] = accr[r];
    y[1] = acci[r];
  }
}

// The same sums on the matrix cores for c64 T (FP32 and BF16x3 plans).  Per staged (q, pass) item the block
// forms the complex product Y_k[(c v)][b] = sum_(c'v') T'[(c v)][(c' v')] X[(c' v')][b] as one real product
// of the interleaved T' ([nt][2 nt]) and X expanded to [2 nt][2 nb] (row 2j: [Re, Im], row 2j + 1: [-Im, Re]
// per column pair) on FP32 16x16x4 MFMA, the X slice rounded to FP32 as it is staged.  Each item's product
// is added to FP64 accumulators, so the sum over the items of a chunk stays FP64.  T' is T[(c' c)][(v' v)]
// on the first pass and conj T[(c c')][(v v')] of the partner block on the second.  The block's output
// tiles (16 rows x 16 real columns) go round-robin to the four waves, at most TX_MAXT each.  FP64 plans
// keep the vector-unit kernel above.
constexpr int TX_MAXT = 8;

__global__ __launch_bounds__(256) void direct_tx_mfma(int Nk, int nq, int q0, int nv, int nc, int nb, int qlen,
                                                      const int* __restrict__ kqp, const int* __restrict__ kqm,
                                                      int nself, int x16, const float* __restrict__ T,
                                                      const double* __restrict__ X, double* __restrict__ part) {
  using TT = float;
  extern __shared__ __attribute__((aligned(16))) unsigned char sbytes[];
  const int k = blockIdx.x, chunk = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = nc * nv, nt2 = nt * nt, nv2 = nv * nv;
  const int tbytes = nt2 * 2 * (int)sizeof(TT);
  const int tstride = (tbytes + 15) & ~15;
  const bool t16 = (tbytes & 15) == 0;
  TT* Ts = reinterpret_cast<TT*>(sbytes);
  TT* Xs = reinterpret_cast<TT*>(sbytes + tstride);  // [nt][nb] complex
  const int CT = (2 * nb + 15) / 16, ntile = ((nt + 15) / 16) * CT;
  const int ksteps = (2 * nt + 3) / 4;
  const int l4 = lane >> 4, l16 = lane & 15;
  double acc[TX_MAXT][4];
#pragma unroll
  for (int s = 0; s < TX_MAXT; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[s][q] = 0.0;
  const int qa = chunk * qlen, qe = min(nq, qa + qlen);
  for (int qi = qa; qi < qe; ++qi) {
    const int j = q0 + qi;
    for (int pass = 0; pass < (j >= nself ? 2 : 1); ++pass) {
      const int kb = pass == 0 ? k : kqm[(long long)k * Nk + j];  // block row of the stored T
      const int kx = pass == 0 ? kqp[(long long)k * Nk + j] : kb;  // k-point of the X slice
      const TT* Tg = T + 2 * ((long long)qi * Nk + kb) * nt2;
      const double* Xg = X + 2 * (long long)kx * nt * nb;
      __syncthreads();  // the previous item's reads are done
      if (t16) {
        for (int i = threadIdx.x; i < tbytes / 16; i += blockDim.x)
          reinterpret_cast<uint4*>(Ts)[i] = reinterpret_cast<const uint4*>(Tg)[i];
      } else {
        for (int i = threadIdx.x; i < tbytes / 8; i += blockDim.x)
          reinterpret_cast<uint2*>(Ts)[i] = reinterpret_cast<const uint2*>(Tg)[i];
      }
      if (x16) {
        for (int i = threadIdx.x; i < nt * nb; i += blockDim.x) {
          const double2 v = reinterpret_cast<const double2*>(Xg)[i];
          Xs[2 * i] = (TT)v.x;
          Xs[2 * i + 1] = (TT)v.y;
        }
      } else {
        for (int i = threadIdx.x; i < 2 * nt * nb; i += blockDim.x) Xs[i] = (TT)Xg[i];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < TX_MAXT; ++s) {
        const int t = wave + 4 * s;
        if (t >= ntile) break;
        const int rt = t / CT, ct = t % CT;
        // A row of this lane: i = (c v); its part of the T' index
        const int i = rt * 16 + l16;
        const bool row_ok = i < nt;
        const int c = row_ok ? i / nv : 0, v = row_ok ? i % nv : 0;
        const int arow = pass == 0 ? c * nv2 + v : c * nc * nv2 + v * nv;
        // B column of this lane: real column cc = 2 b + sb; the lane's K parity r = l4 & 1 is fixed
        const int cc = ct * 16 + l16;
        const bool col_ok = cc < 2 * nb;
        const int b = cc >> 1, sb = cc & 1, r = l4 & 1;
        const int comp = (r != sb) ? 1 : 0;
        const TT bsg = (r == 1 && sb == 0) ? TT(-1) : TT(1);
        const TT asg = (pass == 1 && r == 1) ? TT(-1) : TT(1);  // conj of the partner block
        // complex column j = 2 ks + (l4 >> 1) of T' as (c', v'), advanced by 2 per step
        int jc = l4 >> 1;
        int cp = jc / nv, vp = jc % nv;
        f4v a4 = {0, 0, 0, 0};
        for (int ks = 0; ks < ksteps; ++ks) {
          TT av = TT(0), bv = TT(0);
          if (jc < nt) {
            if (row_ok) {
              const int idx = arow + (pass == 0 ? cp * nc * nv2 + vp * nv : cp * nv2 + vp);
              av = asg * Ts[2 * idx + r];
            }
            if (col_ok) bv = bsg * Xs[2 * (jc * nb + b) + comp];
          }
          a4 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, a4, 0, 0, 0);
          jc += 2;
          vp += 2;
          while (vp >= nv) {
            vp -= nv;
            ++cp;
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[s][q] += (double)a4[q];
      }
    }
  }
  // register q of a lane holds real column l16 of row 4 l4 + q
  const int nout = nt * nb;
#pragma unroll
  for (int s = 0; s < TX_MAXT; ++s) {
    const int t = wave + 4 * s;
    if (t >= ntile) break;
    const int rt = t / CT, ct = t % CT;
    const int cc = ct * 16 + l16;
    if (cc >= 2 * nb) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = rt * 16 + 4 * l4 + q;
      if (i >= nt) continue;
      part[2 * (((long long)chunk * Nk + k) * nout + (long long)i * nb + (cc >> 1)) + (cc & 1)] = acc[s][q];
    }
  }
}

// The same sums for 16-row tiles of T (n_c n_v a multiple of 16, at most 64) and 2 n_b <= 32, laid out so
// that the product loop has no index arithmetic.  Per (q, pass) item the block stages T' as the interleaved
// real matrix [n_t][2 n_t] (row stride 2 n_t + 16 bytes) and X as its expanded transpose [2 n_b][2 n_t]
// (X'[2b][2j] = Re X_jb, [2b][2j+1] = -Im, [2b+1][2j] = Im, [2b+1][2j+1] = Re).  The real contraction index
// kk runs over the lanes' four K groups as kk = (2 n_t / 4) l4 + ks, so a lane reads 16 / sizeof(TT)
// consecutive k steps of A and B with one 16-byte LDS read each.  The next item's T block is loaded into
// registers while the current item is multiplied.  TT = float: c64 T on 16x16x4 FP32 MFMA (FP32 products per
// item, FP64 sums over the items, as in direct_tx_mfma); TT = double: c128 T on 16x16x4 FP64 MFMA.
// NV, NC > 0 fix the band counts at compile time (the index arithmetic of the staging becomes shifts and
// multiplications); 0 takes them from the arguments.
template <typename TT>
struct Tx2 {
  static constexpr int EPC = 16 / sizeof(TT);          // reals per 16-byte LDS read (k steps per read)
  static constexpr int CPC = 8 / sizeof(TT);           // complex elements of T per 16-byte chunk
  static constexpr int TREG = sizeof(TT) == 8 ? 16 : 8;  // 16-byte T chunks per thread (n_t = 64)
  static constexpr int PAD = EPC;                      // row padding: 16 bytes
};

__device__ __forceinline__ f4v tx_mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ d4v tx_mfma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename TT, int NV, int NC>
__global__ __launch_bounds__(256) void direct_tx_mfma2(int Nk, int nq, int q0, int nv_, int nc_, int nb, int qlen,
                                                       const int* __restrict__ kqp, const int* __restrict__ kqm,
                                                       int nself, const TT* __restrict__ T,
                                                       const double* __restrict__ X, double* __restrict__ part) {
  using C = Tx2<TT>;
  using V4 = typename std::conditional<sizeof(TT) == 8, d4v, f4v>::type;
  extern __shared__ __attribute__((aligned(16))) unsigned char sbytes2[];
  TT* const sf = reinterpret_cast<TT*>(sbytes2);
  const int nv = NV > 0 ? NV : nv_, nc = NC > 0 ? NC : nc_;
  const int k = blockIdx.x, chunk = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = nc * nv, nt2 = nt * nt, nv2 = nv * nv, K2 = 2 * nt, RS = K2 + C::PAD, KG = K2 / 4;
  const int CT = (2 * nb + 15) / 16, ntile = (nt / 16) * CT;
  TT* Ta = sf;               // [nt][RS]
  TT* Xs = Ta + nt * RS;     // [16 CT][RS], X' of the current item (rows from 2 nb on stay zero)
  const int l4 = lane >> 4, l16 = lane & 15;
  const int qa = chunk * qlen, qe = min(nq, qa + qlen);
  // X' of the slice at kx into Xd
  auto stage_x = [&](int kx, TT* Xd) {
    const double* Xg = X + 2 * (long long)kx * nt * nb;
    for (int e = tid; e < nt * nb; e += 256) {
      const int j = e / nb, b = e % nb;
      const TT re = (TT)Xg[2 * e], im = (TT)Xg[2 * e + 1];
      Xd[(2 * b) * RS + 2 * j] = re;
      Xd[(2 * b) * RS + 2 * j + 1] = -im;
      Xd[(2 * b + 1) * RS + 2 * j] = im;
      Xd[(2 * b + 1) * RS + 2 * j + 1] = re;
    }
  };
  for (int e = tid; e < 16 * CT * RS; e += 256) Xs[e] = TT(0);
  double acc[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[s][q] = 0.0;
  // items (qi, pass) in order: pass 1 only for q from nself on
  auto tblock = [&](int qi, int pass) -> const TT* {
    const int j = q0 + qi;
    const int kb = pass == 0 ? k : kqm[(long long)k * Nk + j];
    return T + 2 * ((long long)qi * Nk + kb) * nt2;
  };
  const int nchunk16 = nt2 / C::CPC;  // 16-byte chunks of a T block
  uint4 tr[C::TREG];
  auto load_t = [&](const TT* Tg) {
#pragma unroll
    for (int r = 0; r < C::TREG; ++r) {
      const int c = tid + 256 * r;
      if (c < nchunk16) tr[r] = reinterpret_cast<const uint4*>(Tg)[c];
    }
  };
  int qi = qa, pass = 0;
  if (qi < qe) load_t(tblock(qi, 0));
  while (qi < qe) {
    const int j = q0 + qi;
    // next item
    int nqi = qi, npass = pass + 1;
    if (npass > (j >= nself ? 1 : 0)) {
      npass = 0;
      ++nqi;
    }
    __syncthreads();  // the previous item's products are done with Ta and Xs (and the zero fill is done)
    // T' of this item from the registers: T element (c1 c2, v1 v2); first pass T'[(c2 v2)][(c1 v1)] =
    // T[(c1 c2)][(v1 v2)], partner pass T'[(c1 v1)][(c2 v2)] = conj T[(c1 c2)][(v1 v2)]
#pragma unroll
    for (int r = 0; r < C::TREG; ++r) {
      const int c = tid + 256 * r;
      if (c < nchunk16) {
        const TT* v = reinterpret_cast<const TT*>(&tr[r]);
#pragma unroll
        for (int h = 0; h < C::CPC; ++h) {
          const int e = C::CPC * c + h;
          const int r1 = e / nv2, r2 = e % nv2;
          const int c1 = r1 / nc, c2 = r1 % nc, v1 = r2 / nv, v2 = r2 % nv;
          const int row = pass == 0 ? c2 * nv + v2 : c1 * nv + v1;
          const int col = pass == 0 ? c1 * nv + v1 : c2 * nv + v2;
          Ta[row * RS + 2 * col] = v[2 * h];
          Ta[row * RS + 2 * col + 1] = pass == 0 ? v[2 * h + 1] : -v[2 * h + 1];
        }
      }
    }
    // X at k + q for the first pass, at the partner block's row k - q for the second
    stage_x(pass == 0 ? kqp[(long long)k * Nk + j] : kqm[(long long)k * Nk + j], Xs);
    __syncthreads();
    if (nqi < qe) load_t(tblock(nqi, npass));  // in flight during the products below
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int t = wave + 4 * s;
      if (t >= ntile) break;
      const int rt = t / CT, ct = t % CT;
      const TT* pa = Ta + (16 * rt + l16) * RS + KG * l4;
      const TT* pb = Xs + (16 * ct + l16) * RS + KG * l4;
      V4 a4 = {0, 0, 0, 0};
      for (int m = 0; m < KG; m += C::EPC) {
        const uint4 au = *reinterpret_cast<const uint4*>(pa + m);
        const uint4 bu = *reinterpret_cast<const uint4*>(pb + m);
        const TT* av = reinterpret_cast<const TT*>(&au);
        const TT* bv = reinterpret_cast<const TT*>(&bu);
#pragma unroll
        for (int e = 0; e < C::EPC; ++e) a4 = tx_mfma(av[e], bv[e], a4);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[s][q] += (double)a4[q];
    }
    qi = nqi;
    pass = npass;
  }
  // register q of a lane holds real column l16 of tile row 4 l4 + q (FP32 instruction) or l4 + 4 q (FP64)
  const int nout = nt * nb;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int t = wave + 4 * s;
    if (t >= ntile) break;
    const int rt = t / CT, ct = t % CT;
    const int cc = ct * 16 + l16;
    if (cc >= 2 * nb) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = rt * 16 + (sizeof(TT) == 8 ? l4 + 4 * q : 4 * l4 + q);
      part[2 * (((long long)chunk * Nk + k) * nout + (long long)i * nb + (cc >> 1)) + (cc & 1)] = acc[s][q];
    }
  }
}

// LDS bytes of direct_tx_mfma2 for elements of esz bytes, 0 when its shape conditions do not hold
size_t tx2_lds(int nv, int nc, int nb, size_t esz) {
  const int nt = nc * nv;
  const int cpc = esz == 8 ? 1 : 2, treg = esz == 8 ? 16 : 8;  // as Tx2<TT>
  if (nt % 16 != 0 || nt > 64 || 2 * nb > 32 || nt * nt / cpc > 256 * treg) return 0;
  const int RS = 2 * nt + (int)(16 / esz), CT = (2 * nb + 15) / 16;
  return esz * (size_t)RS * (nt + 16 * CT);
}

// Y[i] += scale * sum_chunk part[chunk][i] (complex, n = N * nb), chunks added in order
__global__ void tx_reduce(long long n, int nchunks, double scale, const double* __restrict__ part,
                          double* __restrict__ Y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double sr = 0, si = 0;
    for (int c = 0; c < nchunks; ++c) {
      sr += part[2 * (c * n + i)];
      si += part[2 * (c * n + i) + 1];
    }
    Y[2 * i] += scale * sr;
    Y[2 * i + 1] += scale * si;
  }
}

template <typename TT>
bse_status tx_set_attributes() {
  if (sizeof(TT) == 4)
    BSE_HIP(hipFuncSetAttribute((const void*)direct_tx_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024));
  BSE_HIP(hipFuncSetAttribute((const void*)direct_tx_kernel<TT, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024));
  BSE_HIP(hipFuncSetAttribute((const void*)direct_tx_kernel<TT, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024));
  BSE_HIP(hipFuncSetAttribute((const void*)direct_tx_kernel<TT, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024));
  BSE_HIP(hipFuncSetAttribute((const void*)direct_tx_kernel<TT, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024));
  return BSE_OK;
}

// outputs per thread: the smallest of 1, 2, 4, 8 that covers nt * nb over 256 threads
template <typename TT>
bse_status launch_tx(int slots, dim3 grid, size_t sh, hipStream_t st, int Nk, int nq, int q0, int nv, int nc, int nb,
                     int qlen, const int* kqp, const int* kqm, int nself, int group, const TT* T, const double* X,
                     double* part) {
  const int x16 = (reinterpret_cast<uintptr_t>(X) & 15) == 0 ? 1 : 0;
  if (slots <= 1)
    hipLaunchKernelGGL((direct_tx_kernel<TT, 1>), grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kqp, kqm,
                       nself, group, x16, T, X, part);
  else if (slots <= 2)
    hipLaunchKernelGGL((direct_tx_kernel<TT, 2>), grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kqp, kqm,
                       nself, group, x16, T, X, part);
  else if (slots <= 4)
    hipLaunchKernelGGL((direct_tx_kernel<TT, 4>), grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kqp, kqm,
                       nself, group, x16, T, X, part);
  else
    hipLaunchKernelGGL((direct_tx_kernel<TT, 8>), grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kqp, kqm,
                       nself, group, x16, T, X, part);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

__global__ void diag_kernel(long long N, int nv, int nc, int nb, const double* __restrict__ eps,
                            const double* __restrict__ X, double* __restrict__ Y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nb) return;
  const long long I = t / nb;
  const int v = (int)(I % nv);
  const long long kc = I / nv;
  const int c = (int)(kc % nc);
  const long long k = kc / nc;
  const double d = eps[k * (nv + nc) + nv + c] - eps[k * (nv + nc) + v];
  Y[2 * t] = d * X[2 * t];
  Y[2 * t + 1] = d * X[2 * t + 1];
}

// t[m][b] = sum_s part[s][m][b]
__global__ void splitk_reduce(int nsplit, int n, const double* __restrict__ part, double* __restrict__ out) {
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

// Gm[qi][k][(v' v)][(c' c)] = sum_b Ybar[k][(c v)][b] conj(X[k'][(c' v')][b])
template <typename TT>
__global__ void adj_gm_kernel(int Nk, int nq, int q0, int nv, int nc, int nb, const int* __restrict__ kq,
                              const double* __restrict__ Yb, const double* __restrict__ X, TT* __restrict__ Gm) {
  const int k = blockIdx.x % Nk, qi = blockIdx.x / Nk;
  const int nt = nc * nv, nt2 = nt * nt;
  const int kp = kq[(long long)k * Nk + q0 + qi];
  const double* y = Yb + 2 * (long long)k * nt * nb;
  const double* x = X + 2 * (long long)kp * nt * nb;
  TT* out = Gm + 2 * ((long long)qi * Nk + k) * nt2;
  for (int e = threadIdx.x; e < nt2; e += blockDim.x) {
    const int row = e / (nc * nc), col = e % (nc * nc);
    const int vp = row / nv, v = row % nv, cp = col / nc, c = col % nc;
    const double* yr = y + 2 * (long long)(c * nv + v) * nb;
    const double* xr = x + 2 * (long long)(cp * nv + vp) * nb;
    double sr = 0, si = 0;
    for (int b = 0; b < nb; ++b) {
      const double ar = yr[2 * b], ai = yr[2 * b + 1], br = xr[2 * b], bi = -xr[2 * b + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    out[2 * e] = (TT)sr;
    out[2 * e + 1] = (TT)si;
  }
}

// GmT[qi][k][(c' c)][(v' v)] = sum_b Ybar[k][(c v)][b] conj(X[k'][(c' v')][b]) as four bf16 planes (plane
// stride ps): the k-major operand of Z = Gm conj(Mc) on the BF16x3 path, k' = k + q.  SWAP forms the
// operand of the partner gradient g_W(-q) from the same pairs instead:
//   G'T[qi][k][(c c')][(v v')] = sum_b Ybar[k'][(c v)][b] conj(X[k][(c' v')][b]).
template <bool SWAP>
__global__ void adj_gmT_split_kernel(int Nk, int nq, int q0, int nv, int nc, int nb, const int* __restrict__ kq,
                                     const double* __restrict__ Yb, const double* __restrict__ X,
                                     __bf16* __restrict__ G, long long ps) {
  const int k = blockIdx.x % Nk, qi = blockIdx.x / Nk;
  const int nt = nc * nv, nt2 = nt * nt, nv2 = nv * nv;
  const int kp = kq[(long long)k * Nk + q0 + qi];
  const double* yg = Yb + 2 * (long long)(SWAP ? kp : k) * nt * nb;
  const double* xg = X + 2 * (long long)(SWAP ? k : kp) * nt * nb;
  // both slices in LDS, each row of n_b complex padded by one (row stride 2 n_b + 2 doubles): a wave's outputs
  // read a few distinct rows of each slice at once, which without the padding would all start in one bank
  // when 16 n_b bytes is a multiple of the bank period
  extern __shared__ double gsm[];
  const int rs = 2 * nb + 2;
  double* y = gsm;
  double* x = gsm + (long long)nt * rs;
  for (int i = threadIdx.x; i < 2 * nt * nb; i += blockDim.x) {
    const int r = i / (2 * nb), o = i % (2 * nb);
    y[r * rs + o] = yg[i];
    x[r * rs + o] = xg[i];
  }
  __syncthreads();
  __bf16* out = G + ((long long)qi * Nk + k) * nt2;
  for (int e = threadIdx.x; e < nt2; e += blockDim.x) {
    const int col = e / nv2, row = e % nv2;  // col = (first c, second c), row = (first v, second v)
    const int cp = SWAP ? col % nc : col / nc, c = SWAP ? col / nc : col % nc;
    const int vp = SWAP ? row % nv : row / nv, v = SWAP ? row / nv : row % nv;
    const double* yr = y + (long long)(c * nv + v) * rs;
    const double* xr = x + (long long)(cp * nv + vp) * rs;
    double sr = 0, si = 0;
    for (int b = 0; b < nb; ++b) {
      const double ar = yr[2 * b], ai = yr[2 * b + 1], br = xr[2 * b], bi = -xr[2 * b + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    __bf16 h, l;
    split_bf16((float)sr, h, l);
    out[e] = h;
    out[ps + e] = l;
    split_bf16((float)si, h, l);
    out[2 * ps + e] = h;
    out[3 * ps + e] = l;
  }
}

__global__ void adj_eps_kernel(int nv, int nc, int nb, const double* __restrict__ Yb,
                               const double* __restrict__ X, double* __restrict__ g, int acc) {
  const int k = blockIdx.x;
  const int nt = nc * nv;
  // one thread per band of this k
  for (int n = threadIdx.x; n < nv + nc; n += blockDim.x) {
    double s = 0;
    if (n < nv) {
      for (int c = 0; c < nc; ++c)
        for (int b = 0; b < nb; ++b) {
          const long long o = 2 * (((long long)k * nt + c * nv + n) * nb + b);
          s -= Yb[o] * X[o] + Yb[o + 1] * X[o + 1];
        }
    } else {
      const int c = n - nv;
      for (int v = 0; v < nv; ++v)
        for (int b = 0; b < nb; ++b) {
          const long long o = 2 * (((long long)k * nt + c * nv + v) * nb + b);
          s += Yb[o] * X[o] + Yb[o + 1] * X[o + 1];
        }
    }
    if (acc)
      g[(long long)k * (nv + nc) + n] += s;
    else
      g[(long long)k * (nv + nc) + n] = s;
  }
}

Arith arith_of(bse_prec p) { return p == BSE_F64 ? AR_F64 : (p == BSE_F32 ? AR_F32 : AR_BF16X3); }

char* off_bytes(void* base, long long elems, size_t esz) { return (char*)base + elems * (long long)esz; }

// two-centre pair densities of one q batch, from the one-sided products N (pairs (k, k'), k' = kq[k][q0+qi])
// and N2 (the reversed pairs, N(k', k) stored at slot (qi, k')):
//   M[qi][k][a][b][mu] = N[qi][k][a][b][mu] + conj(N2[qi][k'][b][a][mu]),  a < na_, b < nb_
// written in the plan's storage: four bf16 planes at plane stride ps (SPLIT) or interleaved T
template <typename T, bool SPLIT>
__global__ void tc_combine_kernel(int nq, int Nk, int na_, int nb_, int na, int q0, const int* __restrict__ kq,
                                  const T* __restrict__ N, const T* __restrict__ N2, void* __restrict__ out,
                                  long long ps) {
  const long long n = (long long)nq * Nk * na_ * nb_ * na;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int mu = (int)(e % na);
    long long r = e / na;
    const int b = (int)(r % nb_);
    r /= nb_;
    const int a = (int)(r % na_);
    r /= na_;
    const int k = (int)(r % Nk);
    const int qi = (int)(r / Nk);
    const int kp = kq[(long long)k * Nk + q0 + qi];
    const long long e2 = ((((long long)qi * Nk + kp) * nb_ + b) * na_ + a) * na + mu;
    const T re = N[2 * e] + N2[2 * e2];
    const T im = N[2 * e + 1] - N2[2 * e2 + 1];
    if constexpr (SPLIT) {
      __bf16* o = (__bf16*)out;
      __bf16 hi, lo;
      split_bf16((float)re, hi, lo);
      o[e] = hi;
      o[ps + e] = lo;
      split_bf16((float)im, hi, lo);
      o[2 * ps + e] = hi;
      o[3 * ps + e] = lo;
    } else {
      T* o = (T*)out;
      o[2 * e] = re;
      o[2 * e + 1] = im;
    }
  }
}

// launch of the combine in the plan's storage (f64: c128; split: bf16 planes; else c64)
bse_status tc_combine(Plan* p, int nq, int na_, int nb_, int q0, const int* kq, const void* n1, const void* n2,
                      void* out, bool split_out, long long ps, hipStream_t st) {
  const int Nk = p->Nk, na = p->d.n_aux;
  if (p->prec == BSE_F64)
    hipLaunchKernelGGL((tc_combine_kernel<double, false>), dim3(4096), dim3(256), 0, st, nq, Nk, na_, nb_, na, q0, kq,
                       (const double*)n1, (const double*)n2, out, ps);
  else if (split_out)
    hipLaunchKernelGGL((tc_combine_kernel<float, true>), dim3(4096), dim3(256), 0, st, nq, Nk, na_, nb_, na, q0, kq,
                       (const float*)n1, (const float*)n2, out, ps);
  else
    hipLaunchKernelGGL((tc_combine_kernel<float, false>), dim3(4096), dim3(256), 0, st, nq, Nk, na_, nb_, na, q0, kq,
                       (const float*)n1, (const float*)n2, out, ps);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// S1: pair-density halves -> Gv and Mc for one q batch
//   k-independent C: one GEMM per band set, the half at k times psi(k') from the table
//   two-centre C(R): the same GEMM gives the one-sided product N(k, k') (half psi(k)^H C(-k)^T); it runs
//   again with the reverse table for N(k', k), and the pair density is N(k, k') + conj N(k', k)^T
//   (the second centre's term, C^mu(k') acting on psi(k'), is the first centre's term of the reversed
//   pair because C(R) is real)
bse_status form_pair_densities(Plan* p, int q0, int nq, bool need_c, const int* kq, hipStream_t st,
                                 bool c_split = false) {
  const bse_dims& d = p->d;
  const int Nk = p->Nk, nv = d.nv, nc = d.nc, na = d.n_aux, no = d.n_ao;
  const Arith ar = arith_of(p->prec);
  const bool f64 = p->prec == BSE_F64;
  const bool tc = p->two_centre != 0;
  const size_t gsz = f64 ? 16 : 8;  // bytes per element of a non-split GEMM result
  const long long nt_c = (long long)p->qb * Nk * nv * nv * na;  // offset of the conduction part in Nt / Nt2
  // out == nullptr: the plan's Mv / Mc; otherwise the non-split one-sided product buffer
  auto gemms = [&](const int* ktab, void* out) -> bse_status {
    {
      StageMark sm_(p, BSE_STAGE_TABLES, st);
      hipLaunchKernelGGL(tables_kernel, dim3(Nk), dim3(256), 0, st, Nk, nq, q0, nv, nc, p->nbnd, no, na, ktab,
                         p->tab_psi_v, p->tab_psi_c, p->tab_mv, p->tab_mc);
      BSE_CHECK_LAUNCH();
    }
    {
      StageMark sm_(p, BSE_STAGE_PAIRDENS_V, st);
      GemmArgs g;
      g.batch = Nk;
      g.M = nq * nv;
      g.N = nv * na;
      g.K = no;
      g.A = p->psi;
      g.a_tab = p->tab_psi_v;
      g.a_tab_pb = 1;
      g.a_sk = 1;
      g.B = p->Bv;
      g.b_frag = p->frag_halves;
      g.b_sb = (long long)nv * na * no;
      g.b_sj = no;
      g.b_sk = 1;
      g.C = out ? out : p->Mv;
      g.c_tab = p->tab_mv;
      g.c_tab_pb = 1;
      g.c_sj = 1;
      g.tab_aligned = (no % 8 == 0);
      if (p->split) {
        g.a_ps = p->ps_psi;
        g.b_ps = p->ps_Bv;
        g.c_ps = p->ps_Mv;
        BSE_TRY(cgemm_split(g, true, true, out == nullptr, false, st));
      } else {
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    if (need_c) {
      StageMark sm_(p, BSE_STAGE_PAIRDENS_C, st);
      GemmArgs g;
      g.batch = Nk;
      g.M = nq * nc;
      g.N = nc * na;
      g.K = no;
      g.A = p->psi;
      g.a_tab = p->tab_psi_c;
      g.a_tab_pb = 1;
      g.a_sk = 1;
      g.B = p->Bc;
      g.b_frag = p->frag_halves;
      g.b_sb = (long long)nc * na * no;
      g.b_sj = no;
      g.b_sk = 1;
      g.C = out ? off_bytes(out, nt_c, gsz) : p->Mc;
      g.c_tab = p->tab_mc;
      g.c_tab_pb = 1;
      g.c_sj = 1;
      g.tab_aligned = (no % 8 == 0);
      if (p->split) {
        g.a_ps = p->ps_psi;
        g.b_ps = p->ps_Bc;
        g.c_ps = p->ps_Mc;
        BSE_TRY(cgemm_split(g, true, true, out == nullptr && c_split, false, st));
      } else {
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    return BSE_OK;
  };
  if (!tc) return gemms(kq, nullptr);

  const int* kinv = (kq == p->kqp) ? p->kqm : p->kqinv;
  BSE_TRY(gemms(kq, p->Nt));
  BSE_TRY(gemms(kinv, p->Nt2));
  StageMark sm_(p, BSE_STAGE_PAIRDENS_V, st);
  for (int part = 0; part < (need_c ? 2 : 1); ++part) {
    const int nb = part == 0 ? nv : nc;
    const long long off = part == 0 ? 0 : nt_c;
    void* out = part == 0 ? p->Mv : p->Mc;
    const bool split_out = p->split && (part == 0 || c_split);
    const long long ps = part == 0 ? p->ps_Mv : p->ps_Mc;
    BSE_TRY(tc_combine(p, nq, nb, nb, q0, kq, off_bytes(p->Nt, off, gsz), off_bytes(p->Nt2, off, gsz), out, split_out,
                       ps, st));
  }
  return BSE_OK;
}

// tables of one q batch of the coupling block, per-batch layout [k][nq*nband]:
//   rows (q, c') of psi_c(k') and their Gb slots, rows (q, v') of psi_v(k') and their M2 slots
__global__ void tables_b_kernel(int Nk, int nq, int q0, int nv, int nc, int nbnd, int n_ao, int n_aux,
                                const int* __restrict__ kq, long long* __restrict__ tpc, long long* __restrict__ tg,
                                long long* __restrict__ tpv, long long* __restrict__ tm2) {
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < nq * (nv + nc); t += blockDim.x) {
    if (t < nq * nc) {
      const int qi = t / nc, c = t % nc;
      const int kp = kq[(long long)k * Nk + q0 + qi];
      tpc[(long long)k * nq * nc + t] = ((long long)kp * nbnd + nv + c) * n_ao;
      tg[(long long)k * nq * nc + t] = (((long long)qi * Nk + k) * nc + c) * nv * n_aux;
    } else {
      const int u = t - nq * nc;
      const int qi = u / nv, v = u % nv;
      const int kp = kq[(long long)k * Nk + q0 + qi];
      tpv[(long long)k * nq * nv + u] = ((long long)kp * nbnd + v) * n_ao;
      tm2[(long long)k * nq * nv + u] = (((long long)qi * Nk + k) * nv + v) * nc * n_aux;
    }
  }
}

// part[chunk][k][(c v)][b] = sum_{qi in chunk} sum_{c'v'} Tb[qi][k][(v' c)][(c' v)] X[k'][(c' v')][b],
// k' = kq[k][q0 + qi]; for j = q0 + qi >= nself also the transposed partner block
// D_B(k, k - q_j) = D_B(k - q_j, k)^T:  part += sum_{CV} Tb[qi][k''][(v C)][(c V)] X[k''][(C V)][b],
// k'' = kqm[k][j].  One Tb block and one X slice staged in LDS per (q, pass).
template <typename TT>
__global__ __launch_bounds__(256) void coupling_tx_kernel(int Nk, int nq, int q0, int nv, int nc, int nb, int qlen,
                                                          const int* __restrict__ kq, const int* __restrict__ kqm,
                                                          int nself, const TT* __restrict__ T,
                                                          const double* __restrict__ X, double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sbytes[];
  const int k = blockIdx.x, chunk = blockIdx.y;
  const int nt = nc * nv, nt2 = nt * nt, ne = nt * nb;
  TT* ts = reinterpret_cast<TT*>(sbytes);
  double* xs = reinterpret_cast<double*>(sbytes + (((size_t)nt2 * 2 * sizeof(TT) + 15) & ~(size_t)15));
  const int qa = chunk * qlen, qe = min(nq, qa + qlen);
  double accr[8], acci[8];
  for (int sl = 0; sl < 8; ++sl) accr[sl] = acci[sl] = 0.0;
  for (int qi = qa; qi < qe; ++qi) {
    const int npass = (q0 + qi >= nself) ? 2 : 1;
    for (int pass = 0; pass < npass; ++pass) {
      const int kk = pass == 0 ? kq[(long long)k * Nk + q0 + qi] : kqm[(long long)k * Nk + q0 + qi];
      const TT* tb = T + 2 * (((long long)qi * Nk + (pass == 0 ? k : kk)) * nt2);
      const double* xb = X + 2 * ((long long)kk * ne);
      __syncthreads();
      for (int i = threadIdx.x; i < 2 * nt2; i += blockDim.x) ts[i] = tb[i];
      for (int i = threadIdx.x; i < 2 * ne; i += blockDim.x) xs[i] = xb[i];
      __syncthreads();
      for (int sl = 0; sl < 8; ++sl) {
        const int e = threadIdx.x + 256 * sl;
        if (e >= ne) break;
        const int b = e % nb, cv = e / nb, c = cv / nv, v = cv % nv;
        double sr = 0.0, si = 0.0;
        for (int c2 = 0; c2 < nc; ++c2)
          for (int v2 = 0; v2 < nv; ++v2) {
            const int ti = pass == 0 ? (v2 * nc + c) * nt + c2 * nv + v : (v * nc + c2) * nt + c * nv + v2;
            const double tr = (double)ts[2 * ti], tim = (double)ts[2 * ti + 1];
            const double xr = xs[2 * ((c2 * nv + v2) * nb + b)], xi = xs[2 * ((c2 * nv + v2) * nb + b) + 1];
            sr += tr * xr - tim * xi;
            si += tr * xi + tim * xr;
          }
        accr[sl] += sr;
        acci[sl] += si;
      }
    }
  }
  const long long n = (long long)Nk * ne;
  for (int sl = 0; sl < 8; ++sl) {
    const int e = threadIdx.x + 256 * sl;
    if (e >= ne) break;
    double* o = part + 2 * ((long long)chunk * n + (long long)k * ne + e);
    o[0] = accr[sl];
    o[1] = acci[sl];
  }
}

}  // namespace

// Direct term of the coupling block B of Eq. (Hamiltonian), added to Y:
//   Y[(c v k)] -= (1/N_k) sum_{k'} sum_{c'v'} sum_munu M^mu_{c'v}(k',k) W_munu(k'-k) M^nu_{cv'}(k,k') X[(c'v'k')]
// in q batches: Gb = conj M_{c'v}(k',k) = M_{vc'}(k,k') and M2 = M_{cv'}(k,k') from the halves (Hermitian
// C), Pb = conj(Gb) W(q), Tb = M2 Pb^T, then Tb X(k').  When W(-q) = W(q)^T (checked at plan creation) the
// blocks obey D_B(k', k) = D_B(k, k')^T and only the q of the pair-symmetric order's first half are formed.
bse_status apply_coupling_direct(Plan* p, const double* X, double* Y, int nb, hipStream_t st) {
  const bse_dims& d = p->d;
  const int Nk = p->Nk, nv = d.nv, nc = d.nc, na = d.n_aux, no = d.n_ao, nt = nv * nc;
  const Arith ar = arith_of(p->prec);
  const bool f64 = p->prec == BSE_F64;
  const bool tc = p->two_centre != 0;
  const size_t gsz = f64 ? 16 : 8;  // bytes per element of a non-split GEMM result
  if (!p->qbB) {
    // the same workspace budget as the resonant direct term
    const double per_q_a =
        (double)p->esz * Nk * (nv * nv * na * 2 + (p->mc_direct ? nc * nc * na : 0) + nt * nt) +
        (tc ? 2.0 * gsz * Nk * (nv * nv + nc * nc) * na : 0.0);
    const double per_q_b =
        (double)p->esz * Nk * (3.0 * nc * nv * na + (double)nt * nt) + (tc ? 4.0 * gsz * Nk * nc * nv * na : 0.0);
    const long long qb = std::max(1LL, std::min<long long>(Nk, (long long)((double)p->qb * per_q_a / per_q_b)));
    BSE_HIP(hipFuncSetAttribute((const void*)coupling_tx_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024));
    BSE_HIP(hipFuncSetAttribute((const void*)coupling_tx_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024));
    p->ps_Gb = qb * Nk * nc * nv * na;
    p->qbB = (int)qb;
  }
  {
    // each buffer on its own, so that a call after a failed allocation completes the set
    const long long qb = p->qbB;
    if (!p->Gb) BSE_TRY(plan_alloc(p, &p->Gb, p->esz * (size_t)p->ps_Gb));
    if (!p->Pb) BSE_TRY(plan_alloc(p, &p->Pb, p->esz * (size_t)p->ps_Gb));
    if (!p->M2) BSE_TRY(plan_alloc(p, &p->M2, p->esz * (size_t)p->ps_Gb));
    if (tc)
      for (int i = 0; i < 4; ++i)
        if (!p->Btc[i]) BSE_TRY(plan_alloc(p, &p->Btc[i], gsz * (size_t)p->ps_Gb));
    if (!p->Tb) BSE_TRY(plan_alloc(p, &p->Tb, p->esz * (size_t)(qb * Nk * nt * nt)));
    if (!p->tabB_psi_c) BSE_TRY(plan_alloc(p, (void**)&p->tabB_psi_c, sizeof(long long) * (size_t)(qb * Nk * nc)));
    if (!p->tabB_g) BSE_TRY(plan_alloc(p, (void**)&p->tabB_g, sizeof(long long) * (size_t)(qb * Nk * nc)));
    if (!p->tabB_psi_v) BSE_TRY(plan_alloc(p, (void**)&p->tabB_psi_v, sizeof(long long) * (size_t)(qb * Nk * nv)));
    if (!p->tabB_m2) BSE_TRY(plan_alloc(p, (void**)&p->tabB_m2, sizeof(long long) * (size_t)(qb * Nk * nv)));
  }
  // q in the plan's order (W(q) is stored in that order): the first half only with the transpose relation
  const bool sym = p->herm_half && p->b_pairs;
  const int nqt = sym ? p->nhalf : Nk;
  const int nself = sym ? p->nself : nqt;
  const int* kq = p->herm_half ? p->kqp : p->kq;
  const long long slot = (long long)nc * nv * na;
  for (int q0 = 0; q0 < nqt; q0 += p->qbB) {
    const int nq = std::min(p->qbB, nqt - q0);
    StageMark sm_(p, BSE_STAGE_COUPLING, st);
    // the pair densities Gb and M2 of the batch (into the plan's storage), or with two-centre coefficients
    // the one-sided products (non-split) of the pairs or, with the reverse table, of their reverses
    auto gemms = [&](const int* ktab, void* outG, void* outM2) -> bse_status {
      hipLaunchKernelGGL(tables_b_kernel, dim3(Nk), dim3(256), 0, st, Nk, nq, q0, nv, nc, p->nbnd, no, na, ktab,
                         p->tabB_psi_c, p->tabB_g, p->tabB_psi_v, p->tabB_m2);
      BSE_CHECK_LAUNCH();
      const bool split_out = p->split && !tc;
      {  // Gb[(q c')][(v mu)] = sum_t psi_c'(k')_t B^mu_vt(k)
        GemmArgs g;
        g.batch = Nk;
        g.M = nq * nc;
        g.N = nv * na;
        g.K = no;
        g.A = p->psi;
        g.a_tab = p->tabB_psi_c;
        g.a_tab_pb = 1;
        g.a_sk = 1;
        g.B = p->Bv;
        g.b_frag = p->frag_halves;
        g.b_sb = (long long)nv * na * no;
        g.b_sj = no;
        g.b_sk = 1;
        g.C = outG;
        g.c_tab = p->tabB_g;
        g.c_tab_pb = 1;
        g.c_sj = 1;
        g.tab_aligned = (no % 8 == 0);
        if (p->split) {
          g.a_ps = p->ps_psi;
          g.b_ps = p->ps_Bv;
          g.c_ps = p->ps_Gb;
          BSE_TRY(cgemm_split(g, true, true, split_out, false, st));
        } else {
          BSE_TRY(cgemm(g, ar, f64, f64, st));
        }
      }
      {  // M2[(q v')][(c nu)] = sum_t psi_v'(k')_t B^nu_ct(k)
        GemmArgs g;
        g.batch = Nk;
        g.M = nq * nv;
        g.N = nc * na;
        g.K = no;
        g.A = p->psi;
        g.a_tab = p->tabB_psi_v;
        g.a_tab_pb = 1;
        g.a_sk = 1;
        g.B = p->Bc;
        g.b_frag = p->frag_halves;
        g.b_sb = (long long)nc * na * no;
        g.b_sj = no;
        g.b_sk = 1;
        g.C = outM2;
        g.c_tab = p->tabB_m2;
        g.c_tab_pb = 1;
        g.c_sj = 1;
        g.tab_aligned = (no % 8 == 0);
        if (p->split) {
          g.a_ps = p->ps_psi;
          g.b_ps = p->ps_Bc;
          g.c_ps = p->ps_Gb;
          BSE_TRY(cgemm_split(g, true, true, split_out, false, st));
        } else {
          BSE_TRY(cgemm(g, ar, f64, f64, st));
        }
      }
      return BSE_OK;
    };
    if (!tc) {
      BSE_TRY(gemms(kq, p->Gb, p->M2));
    } else {
      // Gb = N_vc'(k, k') + conj N_c'v(k', k),  M2 = N_cv'(k, k') + conj N_v'c(k', k): the reversed pairs'
      // products come from the other GEMM of the pair with the reverse table
      const int* kinv = (kq == p->kqp) ? p->kqm : p->kqinv;
      BSE_TRY(gemms(kq, p->Btc[0], p->Btc[1]));
      BSE_TRY(gemms(kinv, p->Btc[2], p->Btc[3]));
      BSE_TRY(tc_combine(p, nq, nc, nv, q0, kq, p->Btc[0], p->Btc[3], p->Gb, p->split, p->ps_Gb, st));
      BSE_TRY(tc_combine(p, nq, nv, nc, q0, kq, p->Btc[1], p->Btc[2], p->M2, p->split, p->ps_Gb, st));
    }
    {  // Pb = conj(Gb) W(q)
      GemmArgs g;
      g.batch = nq;
      g.M = Nk * nc * nv;
      g.N = na;
      g.K = na;
      g.A = p->Gb;
      g.a_sb = (long long)Nk * slot;
      g.a_si = na;
      g.a_sk = 1;
      g.conjA = 1;
      g.C = p->Pb;
      g.c_sb = (long long)Nk * slot;
      g.c_si = na;
      g.c_sj = 1;
      if (p->split) {
        g.B = (const __bf16*)p->Wq + (long long)q0 * na * na;
        g.b_sb = (long long)na * na;
        g.b_sk = 1;
        g.b_sj = na;
        g.a_ps = p->ps_Gb;
        g.b_ps = p->ps_W;
        g.c_ps = p->ps_Gb;
        BSE_TRY(cgemm_split(g, true, true, true, false, st));
      } else {
        g.B = off_bytes(p->Wq, (long long)q0 * na * na, p->esz);
        g.b_sb = (long long)na * na;
        g.b_sk = f64 ? na : 1;  // FP32 plans store W(q) transposed
        g.b_sj = f64 ? 1 : na;
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    {  // Tb[(v' c)][(c' v)] = sum_nu M2[(v' c)][nu] Pb[(c' v)][nu]
      GemmArgs g;
      g.batch = nq * Nk;
      g.M = nt;
      g.N = nt;
      g.K = na;
      g.A = p->M2;
      g.a_sb = slot;
      g.a_si = na;
      g.a_sk = 1;
      g.B = p->Pb;
      g.b_sb = slot;
      g.b_sj = na;
      g.b_sk = 1;
      g.C = p->Tb;
      g.c_sb = (long long)nt * nt;
      g.c_si = nt;
      g.c_sj = 1;
      if (p->split) {
        g.a_ps = p->ps_Gb;
        g.b_ps = p->ps_Gb;
        BSE_TRY(cgemm_split(g, true, true, false, false, st));
      } else {
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    {
      const size_t tsz = f64 ? 8 : 4;
      const size_t sh = ((((size_t)nt * nt * 2 * tsz) + 15) & ~(size_t)15) + (size_t)nt * nb * 16;
      const int nch = std::min(TX_CHUNKS, nq);
      const int qlen = (nq + nch - 1) / nch;
      const dim3 grid((unsigned)Nk, (unsigned)nch);
      if (f64)
        hipLaunchKernelGGL(coupling_tx_kernel<double>, grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kq,
                           p->kqm, nself, (const double*)p->Tb, X, p->txp);
      else
        hipLaunchKernelGGL(coupling_tx_kernel<float>, grid, dim3(256), sh, st, Nk, nq, q0, nv, nc, nb, qlen, kq,
                           p->kqm, nself, (const float*)p->Tb, X, p->txp);
      BSE_CHECK_LAUNCH();
      const long long n = p->N * nb;
      hipLaunchKernelGGL(tx_reduce, dim3((unsigned)std::min<long long>((n + 255) / 256, 65536)), dim3(256), 0, st, n,
                         nch, -1.0 / (double)Nk, p->txp, Y);
      BSE_CHECK_LAUNCH();
    }
  }
  return BSE_OK;
}

bse_status apply_diag(Plan* p, const double* X, double* Y, int nb, hipStream_t st) {
  StageMark sm_(p, BSE_STAGE_DIAG, st);
  const long long n = p->N * nb;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p->N, p->d.nv, p->d.nc,
                     nb, p->eps, X, Y);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// resonant exchange (alpha/N_k) rho Vbar rho^H X, or with transpose the exchange part of the coupling
// block, (alpha/N_k) rho Vbar rho^T X
bse_status apply_exchange(Plan* p, const double* X, double* Y, int nb, hipStream_t st, bool transpose) {
  if (p->d.alpha == 0.0) return BSE_OK;
  StageMark sm_(p, BSE_STAGE_EXCHANGE, st);
  const int na = p->d.n_aux;
  const long long Ks = p->N / p->xsplit;
  {  // partial t_s = rho_s^H X_s (rho_s^T X_s)
    GemmArgs g;
    g.batch = p->xsplit;
    g.M = na;
    g.N = nb;
    g.K = (int)Ks;
    g.A = p->rho;
    g.a_sb = Ks * na;
    g.a_si = 1;
    g.a_sk = na;
    g.conjA = transpose ? 0 : 1;
    g.B = X;
    g.b_sb = Ks * nb;
    g.b_sk = nb;
    g.b_sj = 1;
    g.C = p->xt;
    g.c_sb = (long long)na * nb;
    g.c_si = nb;
    g.c_sj = 1;
    BSE_TRY(cgemm(g, AR_F64, true, true, st));
  }
  double* t = p->xt + 2 * (long long)p->xsplit * na * p->max_nb;  // reduced t after the partials
  {
    const int n = na * nb;
    hipLaunchKernelGGL(splitk_reduce, dim3((n + 255) / 256), dim3(256), 0, st, p->xsplit, n, p->xt, t);
    BSE_CHECK_LAUNCH();
  }
  {  // u = Vbar t
    GemmArgs g;
    g.M = na;
    g.N = nb;
    g.K = na;
    g.A = p->vbar;
    g.a_si = na;
    g.a_sk = 1;
    g.B = t;
    g.b_sk = nb;
    g.b_sj = 1;
    g.C = p->xu;
    g.c_si = nb;
    g.c_sj = 1;
    BSE_TRY(cgemm(g, AR_F64, true, true, st));
  }
  {  // Y += (alpha / N_k) rho u
    GemmArgs g;
    g.M = (int)p->N;
    g.N = nb;
    g.K = na;
    g.A = p->rho;
    g.a_si = na;
    g.a_sk = 1;
    g.B = p->xu;
    g.b_sk = nb;
    g.b_sj = 1;
    g.C = Y;
    g.c_si = nb;
    g.c_sj = 1;
    g.alpha = p->d.alpha / (double)p->Nk;
    g.beta = 1;
    BSE_TRY(cgemm(g, AR_F64, true, true, st));
  }
  return BSE_OK;
}

// BSE_FUSED_WSTEP=0 keeps the W step and the direct block as two GEMMs (identical results; read at every
// apply so that one process can time and compare both)
// BSE_TX2=0 in the environment selects direct_tx_mfma over direct_tx_mfma2 (read at every apply)
bool tx2_enabled() {
  const char* e = std::getenv("BSE_TX2");
  return !(e && e[0] == '0');
}

bool fused_wstep_enabled() {
  const char* e = std::getenv("BSE_FUSED_WSTEP");
  return !(e && e[0] == '0');
}

bse_status apply_direct(Plan* p, const double* X, double* Y, int nb, hipStream_t st) {
  const bse_dims& d = p->d;
  const int Nk = p->Nk, nv = d.nv, nc = d.nc, na = d.n_aux;
  const Arith ar = arith_of(p->prec);
  const bool f64 = p->prec == BSE_F64;
  const int nt = nc * nv;
  // with the pair symmetry only the first nhalf q of the plan's order are formed (W(q) is stored in
  // that order); T.X adds the partner blocks D(k, k-q) = D(k-q, k)^dagger
  const int nqt = p->herm_half ? p->nhalf : Nk;
  const int* kq = p->herm_half ? p->kqp : p->kq;
  // n_v = n_c = 8 with N_aux a multiple of 256 on the M_cc' route: the W step and the direct block run as one
  // kernel and P stays on chip (same result as the two GEMMs below)
  const bool fused = p->fused_wt && fused_wstep_enabled();
  for (int q0 = 0; q0 < nqt; q0 += p->qb) {
    const int nq = (nqt - q0) < p->qb ? (nqt - q0) : p->qb;
    BSE_TRY(form_pair_densities(p, q0, nq, p->mc_direct, kq, st, p->split));
    if (fused) {
      StageMark sm_(p, BSE_STAGE_WSTEP, st);
      GemmArgs g;
      g.batch = nq;
      g.M = Nk * nv * nv;
      g.N = na;
      g.K = na;
      g.A = p->Mv;
      g.a_sb = (long long)Nk * nv * nv * na;
      g.a_si = na;
      g.a_sk = 1;
      g.conjA = 1;
      g.B = (const __bf16*)p->Wq + (long long)q0 * na * na;
      g.b_sb = (long long)na * na;
      g.b_sk = 1;
      g.b_sj = na;
      g.a_ps = p->ps_Mv;
      g.b_ps = p->ps_W;
      BSE_TRY(wstep_dblock(g, (const __bf16*)p->Mc, (long long)Nk * nc * nc * na, p->ps_Mc, (float*)p->T,
                           (long long)Nk * nc * nc * nv * nv, st));
    }
    if (!fused) {  // P = conj(Gv) W(q)
    StageMark sm_(p, BSE_STAGE_WSTEP, st);
      GemmArgs g;
      g.batch = nq;
      g.M = Nk * nv * nv;
      g.N = na;
      g.K = na;
      g.A = p->Mv;
      g.a_sb = (long long)Nk * nv * nv * na;
      g.a_si = na;
      g.a_sk = 1;
      g.conjA = 1;
      g.C = p->P;
      g.c_sb = (long long)Nk * nv * nv * na;
      g.c_si = na;
      g.c_sj = 1;
      if (p->split) {
        // W stored transposed per q: B[mu][nu] at q*na^2 + nu*na + mu
        g.B = (const __bf16*)p->Wq + (long long)q0 * na * na;
        g.b_sb = (long long)na * na;
        g.b_sk = 1;
        g.b_sj = na;
        g.a_ps = p->ps_Mv;
        g.b_ps = p->ps_W;
        g.c_ps = p->ps_Mv;  // P is written pre-split for the conduction-side kernel
        BSE_TRY(cgemm_split(g, true, true, true, false, st));
      } else {
        g.B = off_bytes(p->Wq, (long long)q0 * na * na, p->esz);
        g.b_sb = (long long)na * na;
        g.b_sk = f64 ? na : 1;  // FP32 plans store W(q) transposed
        g.b_sj = f64 ? 1 : na;
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    if (fused) {
      // T formed with the W step
    } else if (!p->mc_direct) {  // T from B_c(k) and P without the conduction pair densities (BF16X3)
      StageMark sm_(p, BSE_STAGE_DBLOCK, st);
      BSE_TRY(direct_u_b3(p, q0, nq, kq, st));
    } else {  // T = Mc P^T over nu
      StageMark sm_(p, BSE_STAGE_DBLOCK, st);
      GemmArgs g;
      g.batch = nq * Nk;
      g.M = nc * nc;
      g.N = nv * nv;
      g.K = na;
      g.A = p->Mc;
      g.a_sb = (long long)nc * nc * na;
      g.a_si = na;
      g.a_sk = 1;
      g.B = p->P;
      g.b_sb = (long long)nv * nv * na;
      g.b_sj = na;
      g.b_sk = 1;
      g.C = p->T;
      g.c_sb = (long long)nc * nc * nv * nv;
      g.c_si = nv * nv;
      g.c_sj = 1;
      if (p->split) {  // both operands pre-split, T in c64
        g.a_ps = p->ps_Mc;
        g.b_ps = p->ps_Mv;
        BSE_TRY(cgemm_split(g, true, true, false, false, st));
      } else {
        BSE_TRY(cgemm(g, ar, f64, f64, st));
      }
    }
    {
      StageMark sm_(p, BSE_STAGE_TX, st);
      // LDS per staged (q, pass) item: one T block (16-byte padded) and one X slice; up to 8 items in
      // TX_STAGE_BYTES
      const size_t item = (((size_t)nt * nt * p->esz + 15) & ~(size_t)15) + (size_t)nt * nb * 16;
      const int group = (int)std::max<size_t>(1, std::min<size_t>(8, TX_STAGE_BYTES / item));
      const size_t sh = item * group;
      const int nself = p->herm_half ? p->nself : nqt;  // q from index nself on also give partner blocks
      const double scale = -1.0 / (double)Nk;
      static bool attr_set = false;
      if (!attr_set) {
        BSE_TRY(tx_set_attributes<double>());
        BSE_TRY(tx_set_attributes<float>());
        attr_set = true;
      }
      // q chunks spread the pairs of one k over several blocks (enough for about 16k blocks); partial sums
      // are added in chunk order
      const int nch = std::max(1, std::min(std::min(TX_CHUNKS, nq), (16384 + Nk - 1) / Nk));
      const int qlen = (nq + nch - 1) / nch;
      const dim3 grid((unsigned)Nk, (unsigned)nch);
      const int slots = (nt * nb + 255) / 256;
      const int ntile = ((nt + 15) / 16) * ((2 * nb + 15) / 16);
      const size_t sh2 = tx2_lds(nv, nc, nb, f64 ? 8 : 4);
      if (sh2 > 0 && tx2_enabled()) {  // matrix cores, staged for 16-byte operand reads
        auto go = [&](auto kern, auto tp) -> bse_status {
          BSE_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh2));
          hipLaunchKernelGGL(kern, grid, dim3(256), sh2, st, Nk, nq, q0, nv, nc, nb, qlen, kq, p->kqm, nself,
                             (decltype(tp))p->T, X, p->txp);
          BSE_CHECK_LAUNCH();
          return BSE_OK;
        };
        if (f64) {
          const double* tp = nullptr;
          if (nv == 8 && nc == 8)
            BSE_TRY(go(direct_tx_mfma2<double, 8, 8>, tp));
          else if (nv == 4 && nc == 8)
            BSE_TRY(go(direct_tx_mfma2<double, 4, 8>, tp));
          else
            BSE_TRY(go(direct_tx_mfma2<double, 0, 0>, tp));
        } else {
          const float* tp = nullptr;
          if (nv == 8 && nc == 8)
            BSE_TRY(go(direct_tx_mfma2<float, 8, 8>, tp));
          else if (nv == 4 && nc == 8)
            BSE_TRY(go(direct_tx_mfma2<float, 4, 8>, tp));
          else
            BSE_TRY(go(direct_tx_mfma2<float, 0, 0>, tp));
        }
      } else if (!f64 && ntile <= 4 * TX_MAXT) {  // FP32 matrix cores for c64 T: one item staged at a time
        const size_t tb = ((size_t)nt * nt * p->esz + 15) & ~(size_t)15;
        const size_t shm = tb + (size_t)nt * nb * p->esz;
        const int x16 = (reinterpret_cast<uintptr_t>(X) & 15) == 0 ? 1 : 0;
        hipLaunchKernelGGL(direct_tx_mfma, grid, dim3(256), shm, st, Nk, nq, q0, nv, nc, nb, qlen, kq, p->kqm,
                           nself, x16, (const float*)p->T, X, p->txp);
        BSE_CHECK_LAUNCH();
      } else if (f64) {
        BSE_TRY(launch_tx<double>(slots, grid, sh, st, Nk, nq, q0, nv, nc, nb, qlen, kq, p->kqm, nself, group,
                                  (const double*)p->T, X, p->txp));
      } else {
        BSE_TRY(launch_tx<float>(slots, grid, sh, st, Nk, nq, q0, nv, nc, nb, qlen, kq, p->kqm, nself, group,
                                 (const float*)p->T, X, p->txp));
      }
      const long long n = p->N * nb;
      hipLaunchKernelGGL(tx_reduce, dim3((unsigned)std::min<long long>((n + 255) / 256, 65536)), dim3(256), 0, st, n,
                         nch, scale, p->txp, Y);
      BSE_CHECK_LAUNCH();
    }
  }
  return BSE_OK;
}

// One q batch of the k-major BF16x3 adjoint: Z = Gm conj(Mc) (or, for the partner, Z' = G' Mc) written
// pre-split into P, then g_W of the batch's q = -(1/N_k) sum over pairs of Gv^T Z (conj(Gv)^T Z'), stored
// at the W-gradient index given by dst (plan-order q -> dense-mesh q) or at q0 + i without a table
bse_status adjoint_tn_pass(Plan* p, int q0, int i0, int nq, bool swap, const int* kq, const int* dst,
                           const double* Ybar, const double* X, int nb, double* gWq, bool acc, hipStream_t st) {
  const int Nk = p->Nk, nv = p->d.nv, nc = p->d.nc, na = p->d.n_aux;
  const long long pair_v = (long long)nv * nv * na, pair_c = (long long)nc * nc * na;
  const long long nt2 = (long long)nc * nc * nv * nv;
  __bf16* G = (__bf16*)p->T + (long long)i0 * Nk * nt2;
  // two padded slices: 2 nt (nb + 1) complex, <= 64 KiB + 32 nt bytes since nv nc max_nb <= 2048
  const size_t gsh = 2 * (size_t)nc * nv * (nb + 1) * 16;
  static bool gsh_attr = false;
  if (gsh > 64 * 1024 && !gsh_attr) {
    BSE_HIP(hipFuncSetAttribute((const void*)adj_gmT_split_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024));
    BSE_HIP(hipFuncSetAttribute((const void*)adj_gmT_split_kernel<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    gsh_attr = true;
  }
  if (swap)
    hipLaunchKernelGGL(adj_gmT_split_kernel<true>, dim3(nq * Nk), dim3(256), gsh, st, Nk, nq, q0 + i0, nv, nc, nb, kq,
                       Ybar, X, G, p->ps_T);
  else
    hipLaunchKernelGGL(adj_gmT_split_kernel<false>, dim3(nq * Nk), dim3(256), gsh, st, Nk, nq, q0 + i0, nv, nc, nb,
                       kq, Ybar, X, G, p->ps_T);
  BSE_CHECK_LAUNCH();
  {  // Z[(v'v)][nu] = sum_{c'c} Gm[(v'v)][(c'c)] conj(Mc[(c'c)][nu]); the partner: Z' = sum G'[.][(c c')] Mc[(c c')]
    GemmArgs g;
    g.batch = nq * Nk;
    g.M = nv * nv;
    g.N = na;
    g.K = nc * nc;
    g.A = G;
    g.a_sb = nt2;
    g.a_si = 1;
    g.a_sk = nv * nv;
    g.a_ps = p->ps_T;
    g.B = (const __bf16*)p->Mc + (long long)i0 * Nk * pair_c;
    g.b_sb = pair_c;
    g.b_sk = na;
    g.b_sj = 1;
    g.b_ps = p->ps_Mc;
    g.conjB = swap ? 0 : 1;
    g.C = (__bf16*)p->P + (long long)i0 * Nk * pair_v;
    g.c_sb = pair_v;
    g.c_si = na;
    g.c_sj = 1;
    g.c_ps = p->ps_Mv;
    BSE_TRY(cgemm_split(g, true, true, true, false, st));
  }
  {  // gWq[q][mu][nu] = -(1/N_k) sum_{(k v' v)} Gv[(k v' v)][mu] Z[(k v' v)][nu]   (conj(Gv) for the partner)
    GemmArgs g;
    g.batch = nq;
    g.M = na;
    g.N = na;
    g.K = Nk * nv * nv;
    g.A = (const __bf16*)p->Mv + (long long)i0 * Nk * pair_v;
    g.a_sb = (long long)Nk * pair_v;
    g.a_si = 1;
    g.a_sk = na;
    g.a_ps = p->ps_Mv;
    g.conjA = swap ? 1 : 0;
    g.B = (const __bf16*)p->P + (long long)i0 * Nk * pair_v;
    g.b_sb = (long long)Nk * pair_v;
    g.b_sk = na;
    g.b_sj = 1;
    g.b_ps = p->ps_Mv;
    g.C = dst ? gWq : gWq + 2 * (long long)(q0 + i0) * na * na;
    g.c_bidx = dst ? dst + q0 + i0 : nullptr;
    g.c_sb = (long long)na * na;
    g.c_si = na;
    g.c_sj = 1;
    g.alpha = -1.0 / (double)Nk;
    g.beta = acc ? 1 : 0;
    BSE_TRY(cgemm_split(g, true, true, false, true, st));
  }
  return BSE_OK;
}

bse_status adjoint_direct(Plan* p, const double* Ybar, const double* X, int nb, double* gWq, bool acc,
                          hipStream_t st) {
  const bse_dims& d = p->d;
  const int Nk = p->Nk, nv = d.nv, nc = d.nc, na = d.n_aux;
  const Arith ar = arith_of(p->prec);
  const bool f64 = p->prec == BSE_F64;
  // BF16x3 with 8-aligned n_v^2 and N_aux: every operand pre-split, both reductions on the k-major kernel
  const bool tn = p->split && (nv * nv) % 8 == 0 && na % 8 == 0;
  if (!p->Mc) BSE_TRY(plan_alloc(p, &p->Mc, p->esz * (size_t)p->qb * Nk * nc * nc * na));
  if (tn && p->herm_half) {
    // pair symmetry of the gradient: with Hermitian C^mu the pairs (k, k - q) of g_W(-q) carry the pair
    // densities of (k - q, k), M_vv'(k, k-q) = conj M_v'v(k-q, k) and M_c'c(k-q, k) = conj M_cc'(k, k-q),
    // so the pair densities of one q of each pair {q, -q} serve both gradients:
    //   g_W(-q) = -(1/N_k) sum_{k, k' = k + q} sum conj(Gv[(v v')]) Mc[(c c')] Ybar(k')[(c v)] conj X(k)[(c' v')]
    for (int q0 = 0; q0 < p->nhalf; q0 += p->qb) {
      const int nq = (p->nhalf - q0) < p->qb ? (p->nhalf - q0) : p->qb;
      BSE_TRY(form_pair_densities(p, q0, nq, true, p->kqp, st, true));
      StageMark sm_(p, BSE_STAGE_ADJOINT, st);
      BSE_TRY(adjoint_tn_pass(p, q0, 0, nq, false, p->kqp, p->qord, Ybar, X, nb, gWq, acc, st));
      // partners: plan-order q j >= nself, whose -q sits at j + (nhalf - nself) of the order
      const int i0 = q0 < p->nself ? std::min(nq, p->nself - q0) : 0;
      if (i0 < nq)
        BSE_TRY(adjoint_tn_pass(p, q0, i0, nq - i0, true, p->kqp, p->qord + (p->nhalf - p->nself), Ybar, X, nb,
                                gWq, acc, st));
    }
    return BSE_OK;
  }
  for (int q0 = 0; q0 < Nk; q0 += p->qb) {
    const int nq = (Nk - q0) < p->qb ? (Nk - q0) : p->qb;
    BSE_TRY(form_pair_densities(p, q0, nq, true, p->kq, st, tn));
    StageMark sm_(p, BSE_STAGE_ADJOINT, st);
    if (tn) {
      BSE_TRY(adjoint_tn_pass(p, q0, 0, nq, false, p->kq, nullptr, Ybar, X, nb, gWq, acc, st));
      continue;
    }
    if (f64)
      hipLaunchKernelGGL(adj_gm_kernel<double>, dim3(nq * Nk), dim3(256), 0, st, Nk, nq, q0, nv, nc, nb, p->kq,
                         Ybar, X, (double*)p->T);
    else
      hipLaunchKernelGGL(adj_gm_kernel<float>, dim3(nq * Nk), dim3(256), 0, st, Nk, nq, q0, nv, nc, nb, p->kq,
                         Ybar, X, (float*)p->T);
    BSE_CHECK_LAUNCH();
    {  // Z[(v'v)][nu] = sum_{c'c} Gm[(v'v)][(c'c)] conj(Mc[(c'c)][nu])   (stored in P)
      GemmArgs g;
      g.batch = nq * Nk;
      g.M = nv * nv;
      g.N = na;
      g.K = nc * nc;
      g.A = p->T;
      g.a_sb = (long long)nc * nc * nv * nv;
      g.a_si = nc * nc;
      g.a_sk = 1;
      g.B = p->Mc;
      g.b_sb = (long long)nc * nc * na;
      g.b_sk = na;
      g.b_sj = 1;
      g.conjB = 1;
      g.C = p->P;
      g.c_sb = (long long)nv * nv * na;
      g.c_si = na;
      g.c_sj = 1;
      BSE_TRY(cgemm(g, ar, f64, f64, st));
    }
    {  // gWq[q][mu][nu] = -(1/N_k) sum_{(k v' v)} Gv[(k v' v)][mu] Z[(k v' v)][nu]
      GemmArgs g;
      g.batch = nq;
      g.M = na;
      g.N = na;
      g.K = Nk * nv * nv;
      g.A = p->Mv;
      g.a_sb = (long long)Nk * nv * nv * na;
      g.a_si = 1;
      g.a_sk = na;
      g.B = p->P;
      g.b_sb = (long long)Nk * nv * nv * na;
      g.b_sk = na;
      g.b_sj = 1;
      g.C = gWq + 2 * (long long)q0 * na * na;
      g.c_sb = (long long)na * na;
      g.c_si = na;
      g.c_sj = 1;
      g.alpha = -1.0 / (double)Nk;
      g.beta = acc ? 1 : 0;
      if (p->split) {
        g.a_ps = p->ps_Mv;
        BSE_TRY(cgemm_split(g, true, false, false, true, st));
      } else {
        BSE_TRY(cgemm(g, ar, f64, true, st));
      }
    }
  }
  return BSE_OK;
}

bse_status adjoint_eps(Plan* p, const double* Ybar, const double* X, int nb, double* geps, bool acc,
                       hipStream_t st) {
  hipLaunchKernelGGL(adj_eps_kernel, dim3(p->Nk), dim3(64), 0, st, p->d.nv, p->d.nc, nb, Ybar, X, geps,
                     acc ? 1 : 0);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

}  // namespace bse
