// Small streaming kernels: precision conversion and fills.
#include <cstdlib>

#include "bse_internal.h"

namespace bse {
namespace {

__global__ void cvt_kernel(const double* __restrict__ in, float* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 v = reinterpret_cast<const double2*>(in)[i];
    reinterpret_cast<float2*>(out)[i] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void fill_kernel(uint32_t* __restrict__ p, long long n_words) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_words;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void fill_bytes_kernel(unsigned char* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536LL * 4) g = 65536LL * 4;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
__global__ void split_kernel(const T* __restrict__ in, __bf16* __restrict__ out, long long n, long long ps) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float re = (float)in[2 * i], im = (float)in[2 * i + 1];
    const __bf16 rh = (__bf16)re, ih = (__bf16)im;
    out[i] = rh;
    out[ps + i] = (__bf16)(re - (float)rh);
    out[2 * ps + i] = ih;
    out[3 * ps + i] = (__bf16)(im - (float)ih);
  }
}

// out[b][c][r] (planes) = split(in[b][r][c])
template <typename T>
__global__ void split_T_kernel(const T* __restrict__ in, __bf16* __restrict__ out, int batch, int rows, int cols,
                               long long ps) {
  const long long per = (long long)rows * cols, n = per * batch;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / per, rc = i % per;
    const int c = (int)(rc / rows), r = (int)(rc % rows);  // output order: consecutive threads -> consecutive r
    const long long src = b * per + (long long)r * cols + c;
    const float re = (float)in[2 * src], im = (float)in[2 * src + 1];
    const __bf16 rh = (__bf16)re, ih = (__bf16)im;
    out[i] = rh;
    out[ps + i] = (__bf16)(re - (float)rh);
    out[2 * ps + i] = ih;
    out[3 * ps + i] = (__bf16)(im - (float)ih);
  }
}

// fragment order (see split_planes_frag): output element i of batch entry b comes from column
// 32 jb + (l % 32), k = 16 s + 8 (l / 32) + e of in[b], i = ((jb * (K / 16) + s) * 64 + l) * 8 + e
__global__ void split_frag_kernel(const double* __restrict__ in, __bf16* __restrict__ out, int batch, int N, int K,
                                  long long ps) {
  const long long per = (long long)N * K, n = per * batch;
  const int S = K / 16;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / per, r = i % per;
    const int e = (int)(r & 7), l = (int)((r >> 3) & 63);
    const long long f = r >> 9;  // jb * S + s
    const int s = (int)(f % S), jb = (int)(f / S);
    const int col = 32 * jb + (l & 31), kk = 16 * s + 8 * (l >> 5) + e;
    const long long src = b * per + (long long)col * K + kk;
    const float re = (float)in[2 * src], im = (float)in[2 * src + 1];
    const __bf16 rh = (__bf16)re, ih = (__bf16)im;
    out[i] = rh;
    out[ps + i] = (__bf16)(re - (float)rh);
    out[2 * ps + i] = ih;
    out[3 * ps + i] = (__bf16)(im - (float)ih);
  }
}

// out[b][c][r] = (complex64) in[b][r][c]: batch complex128 matrices rows x cols, transposed and rounded
__global__ void cvt_T_kernel(const double* __restrict__ in, float* __restrict__ out, int batch, int rows, int cols) {
  const long long per = (long long)rows * cols, n = per * batch;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / per, rc = i % per;
    const int c = (int)(rc / rows), r = (int)(rc % rows);
    const long long src = b * per + (long long)r * cols + c;
    out[2 * i] = (float)in[2 * src];
    out[2 * i + 1] = (float)in[2 * src + 1];
  }
}

}  // namespace

bse_status convert_c128_to_c64_T(const double* in, float* out, int batch, int rows, int cols, hipStream_t st) {
  const long long n = (long long)batch * rows * cols;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(cvt_T_kernel, dim3(grid_for(n)), dim3(256), 0, st, in, out, batch, rows, cols);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bse_status split_planes(const void* in, bool in_f64, __bf16* out, long long n, long long plane_stride,
                        hipStream_t st) {
  if (n <= 0) return BSE_OK;
  if (in_f64)
    hipLaunchKernelGGL(split_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, (const double*)in, out, n,
                       plane_stride);
  else
    hipLaunchKernelGGL(split_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, (const float*)in, out, n,
                       plane_stride);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bse_status split_planes_frag(const double* in, __bf16* out, int batch, int N, int K, long long plane_stride,
                             hipStream_t st) {
  if (N % 32 != 0 || K % 16 != 0) {
    set_error("split_planes_frag: N must be a multiple of 32 and K of 16");
    return BSE_ESHAPE;
  }
  const long long n = (long long)batch * N * K;
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(split_frag_kernel, dim3(grid_for(n)), dim3(256), 0, st, in, out, batch, N, K, plane_stride);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bool frag_halves_enabled() {
  const char* e = std::getenv("BSE_FRAG_HALVES");
  return !(e && e[0] == '0');
}

bse_status split_planes_T(const void* in, bool in_f64, __bf16* out, int batch, int rows, int cols,
                          long long plane_stride, hipStream_t st) {
  const long long n = (long long)batch * rows * cols;
  if (n <= 0) return BSE_OK;
  if (in_f64)
    hipLaunchKernelGGL(split_T_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, (const double*)in, out, batch,
                       rows, cols, plane_stride);
  else
    hipLaunchKernelGGL(split_T_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, (const float*)in, out, batch,
                       rows, cols, plane_stride);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

// n = number of complex elements
bse_status convert_c128_to_c64(const double* in, float* out, long long n, hipStream_t st) {
  if (n <= 0) return BSE_OK;
  hipLaunchKernelGGL(cvt_kernel, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
  BSE_CHECK_LAUNCH();
  return BSE_OK;
}

bse_status zero_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return BSE_OK;
  const long long words = (long long)(bytes / 4);
  if (words > 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(words)), dim3(256), 0, st, (uint32_t*)p, words);
    BSE_CHECK_LAUNCH();
  }
  const long long rest = (long long)(bytes - 4 * (size_t)words);
  if (rest > 0) {
    hipLaunchKernelGGL(fill_bytes_kernel, dim3(1), dim3(256), 0, st, (unsigned char*)p + 4 * words, rest);
    BSE_CHECK_LAUNCH();
  }
  return BSE_OK;
}

}  // namespace bse
