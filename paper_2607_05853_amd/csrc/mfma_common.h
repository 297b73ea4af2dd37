// Device helpers shared by the matrix-core kernels: vector types, the bf16
// hi/lo split and operand-offset lookup.
#pragma once

#include <hip/hip_runtime.h>

#include "bse_internal.h"

namespace bse {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// x = hi + lo + O(2^-16 |x|): hi = bf16_rn(x), lo = bf16_rn(x - hi)
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// flip the sign of 8 packed bf16 values
__device__ __forceinline__ bf8v neg8(bf8v x) {
  u4v u = __builtin_bit_cast(u4v, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf8v, u);
}

__device__ __forceinline__ long long off_of(const long long* tab, int pb, long long sb, long long si, int b, int M,
                                            int i) {
  long long o = (long long)b * sb;
  if (tab) return o + tab[(pb ? (long long)b * M : 0LL) + i];
  return o + (long long)i * si;
}

// XCD-aware block order for a 1-D grid of nbatch * per_batch blocks.  Hardware
// deals consecutive workgroups round-robin to the 8 XCDs (each with its own
// L2); this maps the j-th block landing on XCD x to batch x + 8 (j / per_batch)
// so every block of one batch entry (which share operand panels) runs on the
// same XCD, back to back.  Falls back to the identity when nbatch % 8 != 0.
__device__ __forceinline__ void xcd_map(long long L, long long per_batch, long long nbatch, long long& bt,
                                        long long& t) {
  if ((nbatch & 7) == 0) {
    const long long x = L & 7, j = L >> 3;
    bt = x + 8 * (j / per_batch);
    t = j % per_batch;
  } else {
    bt = L / per_batch;
    t = L % per_batch;
  }
}

// output tile (m0, n0) of the t-th block of one batch entry: the dimension with fewer tiles runs fastest, so
// the blocks that share a panel of the other operand (a B column panel when there are few row tiles, an A row
// panel otherwise) run back to back on the same XCD and fetch it from HBM about once
__device__ __forceinline__ void tile_of(long long t, int gxn, int gyn, int BM, int BN, int& m0, int& n0) {
  if (gyn <= gxn) {
    m0 = (int)(t % gyn) * BM;
    n0 = (int)(t / gyn) * BN;
  } else {
    m0 = (int)(t / gxn) * BM;
    n0 = (int)(t % gxn) * BN;
  }
}

// one complex tile step of the BF16x3 product on 32x32x16 MFMA:
//   cr += ar br - ai bi,  ci += ar bi + ai br   (each as hi*hi + hi*lo + lo*hi)
// a[0..3] = (Re hi, Re lo, Im hi, Im lo) of A, b[0..3] likewise; nih / nil = -Im parts of A
__device__ __forceinline__ void cmma_b3(const bf8v* a, bf8v nih, bf8v nil, const bf8v* b, f16v& cr, f16v& ci) {
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[2], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[3], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nil, b[2], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[3], b[0], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, b[3], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[1], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[2], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, b[2], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[0], ci, 0, 0, 0);
}

// the same products with the roles of the operands exchanged: the fragments b give the rows of the
// 32 x 32 result and a its columns (result transposed, each element summed exactly as by cmma_b3)
__device__ __forceinline__ void cmma_b3_t(const bf8v* a, bf8v nih, bf8v nil, const bf8v* b, f16v& cr, f16v& ci) {
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[0], a[1], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2], a[1], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[1], a[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[3], a[0], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2], nil, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[0], a[3], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[3], nih, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[1], a[2], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[0], a[0], cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2], a[0], ci, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2], nih, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[0], a[2], ci, 0, 0, 0);
}

}  // namespace bse
