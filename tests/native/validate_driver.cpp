// Drives dlx_validate and dlx_status_string (the library's host validation layer) over good and
// malformed problem descriptions; built with AddressSanitizer and UBSan by tests/test_abi.py, so
// that any out-of-bounds read of the caller's host arrays or undefined arithmetic aborts the run.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "dlx.h"

namespace {

int failures = 0;

void expect(const char* what, dlx_status got, dlx_status want) {
  if (got != want) {
    std::printf("FAIL %s: got %d want %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

struct Desc {
  std::vector<double> lam{5.45e-7, 5.95e-7, 6.45e-7}, w{1.0 / 3, 1.0 / 3, 1.0 / 3};
  std::vector<int32_t> dith{0, 0, 2, -2, -1, 2};
  dlx_problem_desc d{};
  Desc() {
    d.n_pupil = 64;
    d.n_focal = 96;
    d.oversample = 3;
    d.n_wavelengths = 3;
    d.n_sources = 2;
    d.n_frames = 3;
    d.n_zernike = 10;
    d.n_map = 0;
    d.diameter_m = 0.5;
    d.focal_pixel_rad = 2e-7;
    d.wavelengths_m = lam.data();
    d.spectral_weights = w.data();
    d.frame_dithers = nullptr;
    d.dither_margin = 0;
  }
};

}  // namespace

int main() {
  {
    Desc a;
    expect("good", dlx_validate(&a.d, 1), DLX_OK);
    a.d.frame_dithers = a.dith.data();
    a.d.dither_margin = 2;
    expect("good dithers", dlx_validate(&a.d, 1), DLX_OK);
    a.d.dither_margin = 1;
    expect("dither beyond margin", dlx_validate(&a.d, 1), DLX_ERR_INVALID_ARG);
    a.d.dither_margin = -1;
    expect("negative margin", dlx_validate(&a.d, 1), DLX_ERR_INVALID_ARG);
    a.d.dither_margin = 2000000000;
    expect("margin overflowing the grid", dlx_validate(&a.d, 1), DLX_ERR_SHAPE);
  }
  expect("null", dlx_validate(nullptr, 1), DLX_ERR_INVALID_ARG);
  {
    Desc a;
    expect("zero problems", dlx_validate(&a.d, 0), DLX_ERR_INVALID_ARG);
    a.d.wavelengths_m = nullptr;
    expect("null wavelengths", dlx_validate(&a.d, 1), DLX_ERR_INVALID_ARG);
  }
  {
    Desc a;
    a.lam[2] = std::numeric_limits<double>::quiet_NaN();
    expect("nan wavelength", dlx_validate(&a.d, 1), DLX_ERR_INVALID_ARG);
    a.lam[2] = 6e-7;
    a.w[1] = std::numeric_limits<double>::infinity();
    expect("inf weight", dlx_validate(&a.d, 1), DLX_ERR_INVALID_ARG);
  }
  {
    // sizes at and beyond the limits, in every integer field
    const int32_t bad[] = {0, -1, std::numeric_limits<int32_t>::min(), std::numeric_limits<int32_t>::max()};
    for (int32_t v : bad) {
      for (int field = 0; field < 8; ++field) {
        Desc a;
        int32_t* f[8] = {&a.d.n_pupil, &a.d.n_focal, &a.d.oversample, &a.d.n_wavelengths,
                         &a.d.n_sources, &a.d.n_frames, &a.d.n_zernike, &a.d.n_map};
        *f[field] = v;
        // the host arrays hold three wavelengths: a larger count is the caller's error, so only
        // counts the arrays can back are tried
        if (field == 3 && v > 3) continue;
        const dlx_status s = dlx_validate(&a.d, 1);
        if (s == DLX_OK && !(field >= 6 && v >= 0) && !(field == 4 && v > 0) && !(field == 5 && v > 0))
          expect("bad size accepted", s, DLX_ERR_INVALID_ARG);
      }
    }
    Desc a;
    a.d.n_frames = 1 << 20;
    a.d.n_sources = 1 << 10;
    expect("too many PSFs", dlx_validate(&a.d, 1), DLX_ERR_SHAPE);
    Desc b;
    b.d.n_focal = 97;
    expect("focal not a multiple of Q", dlx_validate(&b.d, 1), DLX_ERR_SHAPE);
    Desc c;
    c.d.n_pupil = 16385;
    expect("pupil too large", dlx_validate(&c.d, 1), DLX_ERR_SHAPE);
  }
  {
    // several problems: the second is checked as well
    Desc a, b;
    b.d.diameter_m = -1.0;
    dlx_problem_desc two[2] = {a.d, b.d};
    expect("second problem", dlx_validate(two, 2), DLX_ERR_INVALID_ARG);
  }
  for (int s = -3; s < 12; ++s) {
    const char* t = dlx_status_string((dlx_status)s);
    if (!t || std::strncmp(t, s >= 0 && s <= 7 ? "DLX_" : "unknown", 3) != 0) {
      std::printf("FAIL status string %d\n", s);
      ++failures;
    }
  }
  std::printf(failures ? "validation driver: %d failures\n" : "validation driver ok\n", failures);
  return failures ? 1 : 0;
}
