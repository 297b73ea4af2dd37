// Interpolation of the screened interaction (Sec. III.B, phase of Eq. (W_LRI)) without any device
// allocation: the same phase kernel and FP64 GEMM as bse_interpolate_W, with the workspace (the q, R and
// weight tables and the phase table) in a file-scope device array instead of stream-ordered allocations.
//
// The array is one per GPU and lives until the process ends.  Host code never passes its name to a kernel
// or a copy (in host code the name is only a stand-in, not a device address): on the first call on a
// device, with that device current, hipGetSymbolAddress gives the device address, which is kept per device
// and used from then on.  Every call on a GPU shares that GPU's array, so calls that overlap on one GPU
// (different streams, or other host threads) race; calls on one stream are ordered.
#include <limits>
#include <mutex>

#include "bse_internal.h"

namespace bse {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch array, looked up once per device with that device current
bse_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(std::string("bse_interpolate_W_noalloc: no usable current device: ") + hipGetErrorString(e));
    return BSE_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      set_error(std::string("bse_interpolate_W_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                hipGetErrorString(e));
      return BSE_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BSE_OK;
}

}  // namespace
}  // namespace bse

extern "C" {

bse_status bse_interpolate_W_noalloc(int32_t n_aux, int32_t n_R, const void* W_R, const int32_t* R,
                                     const double* w_R, int32_t n_q, const double* q_frac, void* W_q,
                                     bse_prec out_prec, void* hip_stream) {
  using namespace bse;
  set_error("");
  if (n_aux <= 0 || n_R <= 0 || n_q <= 0) {
    set_error("bse_interpolate_W_noalloc: sizes must be positive");
    return BSE_EINVAL;
  }
  if (!W_R || !R || !w_R || !q_frac || !W_q) {
    set_error("bse_interpolate_W_noalloc: NULL pointer");
    return BSE_EINVAL;
  }
  if (out_prec != BSE_F64 && out_prec != BSE_F32 && out_prec != BSE_BF16X3) {
    set_error("bse_interpolate_W_noalloc: unknown precision");
    return BSE_EINVAL;
  }
  if ((long long)n_aux * n_aux > std::numeric_limits<int>::max()) {
    set_error("bse_interpolate_W_noalloc: n_aux too large");
    return BSE_ESHAPE;
  }
  const size_t need = interp_scratch_bytes(n_q, n_R);
  if (need > kScratchBytes) {
    set_error("bse_interpolate_W_noalloc: n_q = " + std::to_string(n_q) + " and n_R = " + std::to_string(n_R) +
              " need " + std::to_string(need) + " bytes of workspace, the static scratch holds " +
              std::to_string(kScratchBytes) + " (use bse_interpolate_W)");
    return BSE_ESHAPE;
  }
  void* ws = nullptr;
  BSE_TRY(scratch_address(&ws));
  return interp_forward_ws(n_aux, n_R, static_cast<const double*>(W_R), R, w_R, n_q, q_frac, W_q,
                           out_prec == BSE_F64, ws, reinterpret_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
