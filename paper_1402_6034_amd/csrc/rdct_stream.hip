// Streaming calibration kernels: the practical HBM ceilings that the
// transform kernels' rooflines are read against.  They compute nothing of the
// method; they move bytes in the read:write mixes of the library's kernels
// (the frame quantiser reads 64 B and writes 128 B per block, the batch kernel
// with reconstruction 64 B and 384 B) with the same access granularity: a wave
// reads or writes 1 KiB per instruction, 16 bytes per lane.
//
// A unit is RL read instructions followed by WL write instructions of one
// wave (RL KiB in, WL KiB out); stores depend on the loaded data so that none
// can be dropped.  Units go either one per wave (the grid covers the buffer,
// as the frame kernel's chunks do) or to persistent waves striding over them.
#include "rdct_device.h"

namespace rdct {

template <bool NTL, bool NTS, int RL, int WL>
__global__ __launch_bounds__(256) void k_stream(const u32x4* __restrict__ src,
                                                u32x4* __restrict__ dst, int64_t n_units,
                                                int xcd) {
  const int lane = threadIdx.x & 63;
  const int b = xcd ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int64_t wave = (int64_t)b * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  uint32_t acc = 0;
  for (int64_t u = wave; u < n_units; u += n_waves) {
    u32x4 v[RL > 0 ? RL : 1];
    if constexpr (RL > 0) {
      const RDCT_GLOBAL u32x4* s = gptr(src) + u * (RL * 64) + lane;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        if constexpr (NTL) v[i] = __builtin_nontemporal_load(s + i * 64);
        else v[i] = s[i * 64];
      }
    } else {
      v[0] = (u32x4){(uint32_t)u, (uint32_t)lane, 0u, 0u};
    }
    if constexpr (WL > 0) {
      RDCT_GLOBAL u32x4* d = gptr(dst) + u * (WL * 64) + lane;
#pragma unroll
      for (int j = 0; j < WL; ++j) {
        const u32x4 w = v[j % (RL > 0 ? RL : 1)] ^ (uint32_t)j;
        if constexpr (NTS) __builtin_nontemporal_store(w, d + j * 64);
        else d[j * 64] = w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < (RL > 0 ? RL : 1); ++i) acc ^= v[i].x ^ v[i].y ^ v[i].z ^ v[i].w;
    }
  }
  // Reads only: keep the loads alive; the store happens only for one value of
  // the data, which the calibration buffers never hold.
  if constexpr (WL == 0) {
    if (acc == 0x9e3779b9u) gptr(dst)[lane] = (u32x4){acc, acc, acc, acc};
  }
}

template <bool NTL, bool NTS, int RL, int WL>
static hipError_t launch_stream_t(const void* src, void* dst, int64_t units, int grid, int xcd,
                                  hipStream_t s) {
  hipLaunchKernelGGL((k_stream<NTL, NTS, RL, WL>), dim3(grid), dim3(256), 0, s,
                     reinterpret_cast<const u32x4*>(src), reinterpret_cast<u32x4*>(dst), units,
                     xcd);
  return hipGetLastError();
}

template <int RL, int WL>
static hipError_t launch_stream_mix(const void* src, void* dst, int64_t units, int grid,
                                    int flags, hipStream_t s) {
  const int xcd = (flags >> 2) & 1;
  switch (flags & 3) {
    case 0: return launch_stream_t<false, false, RL, WL>(src, dst, units, grid, xcd, s);
    case 1: return launch_stream_t<true, false, RL, WL>(src, dst, units, grid, xcd, s);
    case 2: return launch_stream_t<false, true, RL, WL>(src, dst, units, grid, xcd, s);
    default: return launch_stream_t<true, true, RL, WL>(src, dst, units, grid, xcd, s);
  }
}

// Read and written KiB per unit of each pattern (rdct_stream_pattern_t).
static const int kStreamRL[5] = {8, 0, 8, 8, 4};
static const int kStreamWL[5] = {0, 16, 8, 16, 24};

}  // namespace rdct

using namespace rdct;

extern "C" {

rdct_status_t rdct_stream_unit_bytes(int32_t pattern, int64_t* read_bytes, int64_t* write_bytes) {
  if (pattern < 0 || pattern > 4) return RDCT_ERR_INVALID_ARG;
  if (read_bytes) *read_bytes = (int64_t)kStreamRL[pattern] * 1024;
  if (write_bytes) *write_bytes = (int64_t)kStreamWL[pattern] * 1024;
  return RDCT_OK;
}

rdct_status_t rdct_stream(const void* src, void* dst, int64_t units, int32_t pattern,
                          int32_t flags, int32_t wgs_per_cu, void* stream) {
  if (pattern < 0 || pattern > 4 || units < 0 || flags < 0 || flags > 7 || wgs_per_cu < 0 ||
      wgs_per_cu > 32)
    return RDCT_ERR_INVALID_ARG;
  if ((kStreamRL[pattern] > 0 && (!src || !aligned(src, 16))) || !dst || !aligned(dst, 16))
    return RDCT_ERR_INVALID_ARG;
  if (units == 0) return RDCT_OK;
  if (units > (int64_t)1 << 34) return RDCT_ERR_UNSUPPORTED;
  // Four waves per workgroup; one unit per wave, or persistent workgroups.
  int64_t grid = (units + 3) / 4;
  if (wgs_per_cu > 0) grid = std::min<int64_t>(grid, (int64_t)device_cu_count() * wgs_per_cu);
  if (grid > INT32_MAX) return RDCT_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (pattern) {
    case 0: e = launch_stream_mix<8, 0>(src, dst, units, (int)grid, flags, s); break;
    case 1: e = launch_stream_mix<0, 16>(src, dst, units, (int)grid, flags, s); break;
    case 2: e = launch_stream_mix<8, 8>(src, dst, units, (int)grid, flags, s); break;
    case 3: e = launch_stream_mix<8, 16>(src, dst, units, (int)grid, flags, s); break;
    default: e = launch_stream_mix<4, 24>(src, dst, units, (int)grid, flags, s); break;
  }
  return e == hipSuccess ? RDCT_OK : RDCT_ERR_HIP;
}

}  // extern "C"
