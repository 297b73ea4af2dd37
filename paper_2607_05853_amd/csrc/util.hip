// Small streaming kernels: precision conversion and fills.
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

}  // namespace

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
