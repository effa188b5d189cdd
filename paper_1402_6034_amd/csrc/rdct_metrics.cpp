// Host-side metrics of the C-ABI: error-sum units, PSNR and MSE (Section 3),
// the mean universal quality index of the comparison path (Section 3), and the
// decoding of packed run-length pair words.  Plain C++ on host arrays: no GPU
// call, so it also builds alone for the sanitizer tests.
#include <math.h>
#include <stdint.h>

#include "../../include/rdct.h"
#include "rdct_host.h"

using namespace rdct;

namespace {

// Error-sum unit of a selection mode of the main path.
double sse_unit(int32_t mode) { return mode == RDCT_SEL_QUANT ? 1.0 / 1048576.0 : 1.0 / 331776.0; }

// PSNR = 10 log10(255^2 / MSE), MSE = sse * unit / pixels; +inf when exact.
double psnr_of(uint64_t sse, double unit, double pixels) {
  if (sse == 0) return INFINITY;
  const double mse = (double)sse * unit / pixels;
  return 10.0 * log10(255.0 * 255.0 / mse);
}

}  // namespace

extern "C" {

double rdct_sse_unit(int32_t mode) { return sse_unit(mode); }

double rdct_psnr(uint64_t sse, int32_t mode, int32_t width, int32_t height) {
  return psnr_of(sse, sse_unit(mode), (double)width * (double)height);
}

rdct_status_t rdct_psnr_planes(const uint64_t* sse, int32_t n, int32_t r_count, int32_t mode,
                               const int32_t* widths, const int32_t* heights, double* psnr_out,
                               double* mean_out) {
  if (!sse || !widths || !heights || !psnr_out || n < 0 || r_count < 1) return RDCT_ERR_INVALID_ARG;
  if (mode != RDCT_SEL_NONE && mode != RDCT_SEL_ZIGZAG && mode != RDCT_SEL_QUANT)
    return RDCT_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n; ++i)
    if (widths[i] <= 0 || heights[i] <= 0) return RDCT_ERR_INVALID_ARG;
  const double unit = sse_unit(mode);
  for (int32_t i = 0; i < n; ++i) {
    const double px = (double)widths[i] * (double)heights[i];
    for (int32_t j = 0; j < r_count; ++j) {
      const int64_t k = (int64_t)i * r_count + j;
      psnr_out[k] = psnr_of(sse[k], unit, px);
    }
  }
  if (mean_out) {
    // The average PSNR over images is the mean of their dB values (Section 3).
    for (int32_t j = 0; j < r_count; ++j) {
      double s = 0.0;
      for (int32_t i = 0; i < n; ++i) s += psnr_out[(int64_t)i * r_count + j];
      mean_out[j] = n > 0 ? s / (double)n : NAN;
    }
  }
  return RDCT_OK;
}

int64_t rdct_num_blocks(int32_t width, int32_t height) { return blocks_of(width, height); }

double rdct_quality_sse_unit(int32_t transform) {
  switch (transform) {
    case RDCT_T_RDCT: return 1.0 / (576.0 * 576.0);
    case RDCT_T_SDCT: return 1.0 / (64.0 * 64.0);
    case RDCT_T_DCT:
    case RDCT_T_RDCT_CEIL: return 1.0 / 1048576.0;
    default: return 0.0;
  }
}

int64_t rdct_quality_windows(int32_t width, int32_t height) {
  if (width < 8 || height < 8) return 0;
  return (int64_t)(width - 7) * (int64_t)(height - 7);
}

rdct_status_t rdct_quality_metrics(const uint64_t* sse, const int64_t* uqi, int32_t n,
                                   int32_t transform, int32_t width, int32_t height,
                                   double* mse_out, double* uqi_out) {
  if (n < 0 || (n > 0 && (!sse || !uqi || !mse_out || !uqi_out))) return RDCT_ERR_INVALID_ARG;
  const double unit = rdct_quality_sse_unit(transform);
  const int64_t windows = rdct_quality_windows(width, height);
  if (unit == 0.0 || windows <= 0) return RDCT_ERR_INVALID_ARG;
  const double px = (double)width * (double)height;
  for (int32_t i = 0; i < n; ++i) {
    mse_out[i] = (double)sse[i] * unit / px;
    uqi_out[i] = (double)uqi[i] * (1.0 / 4294967296.0) / (double)windows;
  }
  return RDCT_OK;
}

rdct_status_t rdct_codec_unpack_pairs(const int32_t* words, int64_t n, int32_t* run_out,
                                      int32_t* value_out) {
  if (n < 0 || (n > 0 && (!words || !run_out || !value_out))) return RDCT_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t w = (uint32_t)words[i];
    run_out[i] = (int32_t)(w >> 16);
    value_out[i] = (int32_t)(int16_t)(uint16_t)(w & 0xffffu);
  }
  return RDCT_OK;
}

}  // extern "C"
