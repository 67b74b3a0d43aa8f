// Host-side validation of the C ABI's problem descriptions, and the status strings. Plain C++ with
// no HIP dependency: built into libdlx by hipcc, and on its own under AddressSanitizer for the CPU
// tests of the validation layer.
#include <cmath>
#include <cstdint>

#include "dlx.h"

namespace {
constexpr int kMaxSide = 16384;   // largest pupil or focal grid side
}  // namespace

extern "C" {

const char* dlx_status_string(dlx_status s) {
  switch (s) {
    case DLX_OK: return "DLX_OK";
    case DLX_ERR_INVALID_ARG: return "DLX_ERR_INVALID_ARG: null pointer, non-positive size or bad enum";
    case DLX_ERR_SHAPE: return "DLX_ERR_SHAPE: inconsistent sizes";
    case DLX_ERR_OOM: return "DLX_ERR_OOM: workspace does not fit";
    case DLX_ERR_HIP: return "DLX_ERR_HIP: a HIP runtime call failed";
    case DLX_ERR_NONFINITE: return "DLX_ERR_NONFINITE: non-finite model or data";
    case DLX_ERR_DOMAIN: return "DLX_ERR_DOMAIN: model <= 0 under the Poisson loss (clamped)";
    case DLX_ERR_UNSUPPORTED: return "DLX_ERR_UNSUPPORTED: not implemented by the library";
  }
  return "unknown dlx_status";
}

dlx_status dlx_validate(const dlx_problem_desc* probs, int32_t n_probs) {
  if (!probs || n_probs < 1) return DLX_ERR_INVALID_ARG;
  for (int i = 0; i < n_probs; ++i) {
    const dlx_problem_desc& d = probs[i];
    if (d.n_pupil < 2 || d.n_focal < 1 || d.oversample < 1 || d.n_wavelengths < 1 || d.n_sources < 1 ||
        d.n_frames < 1 || d.n_zernike < 0 || d.n_map < 0)
      return DLX_ERR_INVALID_ARG;
    if (!(d.diameter_m > 0.0) || !(d.focal_pixel_rad > 0.0) || !std::isfinite(d.diameter_m) ||
        !std::isfinite(d.focal_pixel_rad))
      return DLX_ERR_INVALID_ARG;
    if (!d.wavelengths_m || !d.spectral_weights) return DLX_ERR_INVALID_ARG;
    for (int l = 0; l < d.n_wavelengths; ++l) {
      if (!(d.wavelengths_m[l] > 0.0) || !std::isfinite(d.wavelengths_m[l])) return DLX_ERR_INVALID_ARG;
      if (!std::isfinite(d.spectral_weights[l])) return DLX_ERR_INVALID_ARG;
    }
    if (d.n_focal % d.oversample != 0) return DLX_ERR_SHAPE;
    if (d.n_pupil > kMaxSide || d.n_focal > kMaxSide) return DLX_ERR_SHAPE;
    if (d.frame_dithers) {
      if (d.dither_margin < 0) return DLX_ERR_INVALID_ARG;
      if ((long long)d.n_focal + 2LL * d.oversample * d.dither_margin > kMaxSide) return DLX_ERR_SHAPE;
      for (int f = 0; f < d.n_frames; ++f)
        for (int c = 0; c < 2; ++c) {
          const int v = d.frame_dithers[2 * f + c];
          if (v > d.dither_margin || v < -d.dither_margin) return DLX_ERR_INVALID_ARG;
        }
    }
    if ((long long)d.n_frames * d.n_sources * d.n_wavelengths > (1LL << 24)) return DLX_ERR_SHAPE;
  }
  return DLX_OK;
}

}  // extern "C"
