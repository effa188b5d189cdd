// C-ABI of the codec output: zig-zag run-length pairs of the kept coefficients
// and the 8-bit reconstruction (encode), and their concatenation (pack).
#include <mutex>
#include <unordered_map>

#include "rdct_internal.h"

using namespace rdct;

namespace {
constexpr int64_t kMaxCodecBlocks = 1ll << 22;

// Workspace of rdct_codec_pack_noalloc: the chunk prefixes of the largest plane
// the codec accepts (one uint32 per 64-block group: 65,536 entries, 256 KiB),
// in a device array of the library's own.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t kScratchGroups = kMaxCodecBlocks / 64;
static __device__ __align__(256) uint32_t scratch[kScratchGroups];

std::mutex g_scratch_mu;
std::unordered_map<int, uint32_t*> g_scratch_ptr;  // device -> address of its copy

// Device address of the current device's copy, looked up once per device.
rdct_status_t scratch_for_current_device(uint32_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RDCT_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
      return RDCT_ERR_HIP;
    it = g_scratch_ptr.emplace(dev, static_cast<uint32_t*>(ptr)).first;
  }
  *out = it->second;
  return RDCT_OK;
}
}  // namespace


extern "C" {

int64_t rdct_codec_groups(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0) return 0;
  return (rdct_num_blocks(width, height) + 63) / 64;
}

rdct_status_t rdct_codec_encode(const uint8_t* src, int32_t width, int32_t height,
                                int64_t src_pitch, const rdct_select_t* sel, uint16_t* counts,
                                uint32_t* group_pairs, int32_t* slots, uint8_t* recon_u8,
                                int64_t recon_pitch, void* stream) {
  SelInfo si;
  rdct_status_t st = check_sel(sel, &si);
  if (st != RDCT_OK) return st;
  if ((st = check_plane(src, width, height, src_pitch, kMaxCodecBlocks)) != RDCT_OK) return st;
  if (!counts || !group_pairs || !slots || !aligned(counts, 2) || !aligned(group_pairs, 4) ||
      !aligned(slots, 4))
    return RDCT_ERR_INVALID_ARG;
  if (recon_u8 && recon_pitch < width) return RDCT_ERR_INVALID_ARG;
  Plane P = make_plane(src, width, height, src_pitch);
  P.r = si.r;
  P.keep = keep_bits(si.r);
  P.shift = si.shift;
  CodecOutArgs o{counts, group_pairs, slots, recon_u8, recon_pitch};
  return launch_codec_encode(si.sel, P, o, si.qc, (hipStream_t)stream) == hipSuccess
             ? RDCT_OK
             : RDCT_ERR_HIP;
}

rdct_status_t rdct_codec_pack(const uint16_t* counts, const uint32_t* group_pairs,
                              const int32_t* slots, int32_t width, int32_t height,
                              uint32_t* offsets, int32_t* packed, int64_t capacity,
                              uint32_t* workspace, void* stream) {
  if (width <= 0 || height <= 0 || !counts || !group_pairs || !slots || !offsets || !workspace ||
      capacity < 0 || (capacity > 0 && !packed))
    return RDCT_ERR_INVALID_ARG;
  const int64_t nb = rdct_num_blocks(width, height);
  if (nb > kMaxCodecBlocks) return RDCT_ERR_UNSUPPORTED;
  return launch_codec_pack(counts, group_pairs, slots, (int32_t)nb, offsets, packed, capacity,
                           workspace, (hipStream_t)stream) == hipSuccess
             ? RDCT_OK
             : RDCT_ERR_HIP;
}

rdct_status_t rdct_codec_pack_noalloc(const uint16_t* counts, const uint32_t* group_pairs,
                                      const int32_t* slots, int32_t width, int32_t height,
                                      uint32_t* offsets, int32_t* packed, int64_t capacity,
                                      void* stream) {
  if (width <= 0 || height <= 0 || !counts || !group_pairs || !slots || !offsets ||
      capacity < 0 || (capacity > 0 && !packed))
    return RDCT_ERR_INVALID_ARG;
  const int64_t nb = rdct_num_blocks(width, height);
  // The library's workspace holds the prefixes of at most kScratchGroups groups.
  if (nb > kMaxCodecBlocks || (nb + 63) / 64 > kScratchGroups) return RDCT_ERR_UNSUPPORTED;
  uint32_t* ws = nullptr;
  const rdct_status_t st = scratch_for_current_device(&ws);
  if (st != RDCT_OK) return st;
  return launch_codec_pack(counts, group_pairs, slots, (int32_t)nb, offsets, packed, capacity, ws,
                           (hipStream_t)stream) == hipSuccess
             ? RDCT_OK
             : RDCT_ERR_HIP;
}

}  // extern "C"
