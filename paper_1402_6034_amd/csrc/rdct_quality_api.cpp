// C-ABI of the comparison path: keep-r sweep of a plane under one of the
// comparison transforms, scored by SSE and UQI (Section 3), single-plane and
// planned over many planes.
#include <vector>

#include "rdct_internal.h"

using namespace rdct;

namespace {

constexpr int64_t kMaxQualityBlocks = 1ll << 20;

rdct_status_t check_quality_plane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch) {
  rdct_status_t st = check_plane(src, w, h, pitch, kMaxQualityBlocks);
  if (st != RDCT_OK) return st;
  if ((w % 8) != 0 || (h % 8) != 0) return RDCT_ERR_UNSUPPORTED;
  return RDCT_OK;
}

rdct_status_t make_args(int32_t transform, int32_t r_first, int32_t r_count, QualityArgs* a) {
  if (r_first < 1 || r_count < 1 || r_first + r_count - 1 > 64) return RDCT_ERR_INVALID_ARG;
  rdct_status_t st = build_transform(transform, &a->T);
  if (st != RDCT_OK) return st;
  a->r_first = r_first;
  a->r_count = r_count;
  return RDCT_OK;
}

QPlane make_qplane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch) {
  QPlane P{};
  P.src = src;
  P.pitch = pitch;
  P.width = w;
  P.height = h;
  P.tiles_x = quality_tiles_x(w);
  P.tiles_y = quality_tiles_y(h);
  return P;
}

}  // namespace

struct rdct_quality_plan {
  QualityArgs args{};
  QPlane* d_planes = nullptr;
  QTile* d_tiles = nullptr;
  int32_t n_tiles = 0;
  int32_t n_planes = 0;
  uint64_t* sse = nullptr;
  int64_t* uqi = nullptr;
  int64_t n_out = 0;
};

extern "C" {

rdct_status_t rdct_quality_sweep(const uint8_t* src, int32_t width, int32_t height,
                                 int64_t src_pitch, int32_t transform, int32_t r_first,
                                 int32_t r_count, uint64_t* sse_out, int64_t* uqi_out,
                                 void* stream) {
  if (!sse_out || !uqi_out || !aligned(sse_out, 8) || !aligned(uqi_out, 8))
    return RDCT_ERR_INVALID_ARG;
  QualityArgs a;
  rdct_status_t st = make_args(transform, r_first, r_count, &a);
  if (st != RDCT_OK) return st;
  if ((st = check_quality_plane(src, width, height, src_pitch)) != RDCT_OK) return st;
  QPlane P = make_qplane(src, width, height, src_pitch);
  P.sse = sse_out;
  P.uqi = uqi_out;
  hipStream_t s = (hipStream_t)stream;
  if (launch_zero_u64(sse_out, r_count, s) != hipSuccess ||
      launch_zero_u64(reinterpret_cast<uint64_t*>(uqi_out), r_count, s) != hipSuccess)
    return RDCT_ERR_HIP;
  return launch_quality(P, a, s) == hipSuccess ? RDCT_OK : RDCT_ERR_HIP;
}

rdct_status_t rdct_quality_plan_create(const rdct_quality_desc_t* planes, int32_t n,
                                       int32_t transform, int32_t r_first, int32_t r_count,
                                       uint64_t* sse_out, int64_t* uqi_out,
                                       rdct_quality_plan_t** out) {
  if (!out) return RDCT_ERR_INVALID_ARG;
  *out = nullptr;
  if (!planes || n <= 0 || !sse_out || !uqi_out || !aligned(sse_out, 8) || !aligned(uqi_out, 8))
    return RDCT_ERR_INVALID_ARG;
  QualityArgs a;
  rdct_status_t st = make_args(transform, r_first, r_count, &a);
  if (st != RDCT_OK) return st;
  std::vector<QPlane> hp(n);
  std::vector<QTile> tiles;
  for (int32_t i = 0; i < n; ++i) {
    const rdct_quality_desc_t& d = planes[i];
    if ((st = check_quality_plane(d.src, d.width, d.height, d.src_pitch)) != RDCT_OK) return st;
    hp[i] = make_qplane(d.src, d.width, d.height, d.src_pitch);
    hp[i].sse = sse_out + (int64_t)i * r_count;
    hp[i].uqi = uqi_out + (int64_t)i * r_count;
    const int nt = hp[i].tiles_x * hp[i].tiles_y;
    for (int k = 0; k < nt; ++k) tiles.push_back(QTile{i, k});
  }
  if (tiles.size() > (size_t)0x7fffffff) return RDCT_ERR_UNSUPPORTED;
  rdct_quality_plan* p = new rdct_quality_plan();
  p->args = a;
  p->n_tiles = (int32_t)tiles.size();
  p->n_planes = n;
  p->sse = sse_out;
  p->uqi = uqi_out;
  p->n_out = (int64_t)n * r_count;
  if (hipMalloc(&p->d_planes, sizeof(QPlane) * n) != hipSuccess ||
      hipMalloc(&p->d_tiles, sizeof(QTile) * tiles.size()) != hipSuccess) {
    rdct_quality_plan_destroy(p);
    return RDCT_ERR_NO_MEMORY;
  }
  if (hipMemcpy(p->d_planes, hp.data(), sizeof(QPlane) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_tiles, tiles.data(), sizeof(QTile) * tiles.size(), hipMemcpyHostToDevice) !=
          hipSuccess) {
    rdct_quality_plan_destroy(p);
    return RDCT_ERR_HIP;
  }
  *out = p;
  return RDCT_OK;
}

rdct_status_t rdct_quality_plan_run(rdct_quality_plan_t* p, void* stream) {
  if (!p) return RDCT_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (launch_zero_u64(p->sse, p->n_out, s) != hipSuccess ||
      launch_zero_u64(reinterpret_cast<uint64_t*>(p->uqi), p->n_out, s) != hipSuccess)
    return RDCT_ERR_HIP;
  return launch_quality_batch(p->d_planes, p->d_tiles, p->n_tiles, p->args, s) == hipSuccess
             ? RDCT_OK
             : RDCT_ERR_HIP;
}

void rdct_quality_plan_destroy(rdct_quality_plan_t* p) {
  if (!p) return;
  if (p->d_planes) (void)hipFree(p->d_planes);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  delete p;
}

}  // extern "C"
