// PSNR of many planes on the device (Section 3: PSNR per image from its error
// sum; the average PSNR over images is the mean of their dB values), so that a
// caller that reads results back copies decibels, not sums, and does no
// per-value arithmetic on the host.
#include <math.h>

#include "rdct_internal.h"

namespace rdct {

// One thread per (plane i, value j): psnr[i * r_count + j] from sse[i * r_count + j].
__global__ void k_psnr(const uint64_t* __restrict__ sse, int32_t n, int32_t r_count, double unit,
                       const int64_t* __restrict__ pixels, double* __restrict__ psnr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)n * r_count) return;
  const int64_t i = k / r_count;
  const uint64_t s = sse[k];
  psnr[k] = s == 0 ? INFINITY
                   : 10.0 * log10(255.0 * 255.0 * (double)pixels[i] / ((double)s * unit));
}

// One thread per value j: the mean over the n planes.
__global__ void k_psnr_mean(const double* __restrict__ psnr, int32_t n, int32_t r_count,
                            double* __restrict__ mean) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r_count) return;
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += psnr[(int64_t)i * r_count + j];
  mean[j] = n > 0 ? s / (double)n : NAN;
}

}  // namespace rdct

using namespace rdct;

extern "C" rdct_status_t rdct_psnr_device(const uint64_t* sse, int32_t n, int32_t r_count,
                                          int32_t mode, const int64_t* pixels, double* psnr_out,
                                          double* mean_out, void* stream) {
  if (n < 0 || r_count < 1 || (n > 0 && (!sse || !pixels || !psnr_out)) ||
      (mode != RDCT_SEL_NONE && mode != RDCT_SEL_ZIGZAG && mode != RDCT_SEL_QUANT) ||
      !aligned(sse, 8) || !aligned(pixels, 8) || !aligned(psnr_out, 8) ||
      (mean_out && !aligned(mean_out, 8)))
    return RDCT_ERR_INVALID_ARG;
  if ((int64_t)n * r_count > ((int64_t)1 << 31)) return RDCT_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const int64_t total = (int64_t)n * r_count;
  if (total > 0) {
    hipLaunchKernelGGL(k_psnr, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, sse, n,
                       r_count, rdct_sse_unit(mode), pixels, psnr_out);
    if (hipGetLastError() != hipSuccess) return RDCT_ERR_HIP;
  }
  if (mean_out) {
    hipLaunchKernelGGL(k_psnr_mean, dim3((r_count + 63) / 64), dim3(64), 0, s, psnr_out, n, r_count,
                       mean_out);
    if (hipGetLastError() != hipSuccess) return RDCT_ERR_HIP;
  }
  return RDCT_OK;
}
