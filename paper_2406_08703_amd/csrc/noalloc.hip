// dlx_loss_grad_noalloc: the loss, residual and flat-field gradient of dlx_loss_grad without a plan
// and without any device allocation, for callers that cannot allocate (HIP graph capture, serving
// loops that forbid hipMalloc). Its FP64 per-block loss partials and its status word live in a
// fixed, file-scope device array held by the library on every device it runs on.
#include <array>
#include <cmath>
#include <mutex>

#include "dlx_internal.h"

namespace {

using namespace dlx;

// Loss partials of at most this many 256-pixel blocks: frames of up to 2048 x 2048 pixels.
constexpr int kMaxBlocks = DLX_NOALLOC_MAX_PIXELS / 256;
// the partials, then one int status word (bit 0: non-finite, bit 1: domain) on its own 256 bytes
constexpr int kScratchDoubles = kMaxBlocks + 32;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
std::array<double*, kMaxDevices> g_ptr{};   // device address of `scratch` on each device

// The device address of `scratch` on the current device, looked up once per device. The array's
// name is only a host-side handle: kernels and copies get this address.
hipError_t scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

// Hand the call's status flags to the caller (if asked) and leave the word zero for the next call.
__global__ void take_status_kernel(int* status, int32_t* out) {
  if (out) out[0] = status[0];
  status[0] = 0;
}

}  // namespace

extern "C" dlx_status dlx_loss_grad_noalloc(int32_t n_frames, int32_t n_det, const float* model, const float* binned,
                                            const float* data, const float* flat, dlx_loss_kind kind,
                                            double prior_mu, double prior_sigma, double* loss_out,
                                            float* dloss_dmodel, double* grad_flat, int32_t* status_out,
                                            void* stream) {
  if (n_frames < 1 || n_det < 1 || !model || !binned || !data || !flat || !loss_out || !dloss_dmodel || !grad_flat)
    return DLX_ERR_INVALID_ARG;
  if (kind != DLX_LOSS_POISSON && kind != DLX_LOSS_CHI2) return DLX_ERR_INVALID_ARG;
  if (!(prior_sigma > 0.0) || !std::isfinite(prior_sigma) || !std::isfinite(prior_mu)) return DLX_ERR_INVALID_ARG;
  const long long npix = (long long)n_det * n_det;
  if (npix > DLX_NOALLOC_MAX_PIXELS) return DLX_ERR_UNSUPPORTED;
  double* blk = nullptr;
  if (scratch_on_current_device(&blk) != hipSuccess) return DLX_ERR_HIP;
  int* status = reinterpret_cast<int*>(blk + kMaxBlocks);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (launch_loss_plain(n_frames, npix, model, binned, data, flat, (int)kind, prior_mu, prior_sigma, dloss_dmodel,
                        grad_flat, blk, status, loss_out, st) != hipSuccess)
    return DLX_ERR_HIP;
  hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(1), 0, st, status, status_out);
  return hipGetLastError() == hipSuccess ? DLX_OK : DLX_ERR_HIP;
}
