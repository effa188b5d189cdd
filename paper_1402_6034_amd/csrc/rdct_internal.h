// Internal host/device interface of librdct: argument blocks shared by the C-ABI
// front end, the batch planner and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rdct.h"
#include "rdct_host.h"

namespace rdct {

// One plane as the kernels see it.
struct Plane {
  const uint8_t* src;
  int64_t pitch;        // bytes per source row
  int32_t width, height;
  int32_t nbx, nby;     // blocks per row / column
  int32_t nblocks;      // nbx * nby
  int32_t aligned8;     // src and pitch are multiples of 8 bytes
  void* coef;           // block-major coefficients (nullable)
  float* recon;         // reconstruction (nullable)
  int64_t rpitch;       // floats per reconstruction row
  uint64_t* sse;        // accumulators (nullable)
  int32_t r;            // first retained count (zig-zag), 1..64
  uint64_t keep;        // bit kl set when natural position kl has zig-zag rank < r
  int32_t r_count;      // number of r values scored (sweep)
  int32_t shift;        // level shift
  int32_t table;        // index of the quantisation constants (batch)
};

// Per-table constants of the quantisation path and the scaled-coefficient paths.
//  qm[kl]  rational positions (g_k == g_l): two floats, lo = 1/(c Q), hi =
//          (c Q + 1/2) / (2 c Q), c = g_k; irrational positions: the float64
//          bits of 1 / (Q sqrt(g_k g_l)).
//  dq[kl]  Q sqrt(1/(g_k g_l)) in float64 (dequantise and scale in one factor).
//  qi[kl]  Q itself (integer), for the coefficient-domain error z - q Q.
//  qf[kl]  float64 bits of quant_multiplier (the FMA form of the quantiser).
struct QuantConsts {
  uint64_t qm[64];
  double dq[64];
  int32_t qi[64];
  uint64_t qf[64];
};

// Comparison transforms: forward matrix F (block -> F A F^T) and inverse basis
// G with scale D (keep-r reconstruction G (M . Y) G^T / D); `exact` when F, G
// and D are integers.
struct TransformTables {
  double F[64];
  double G[64];
  double D;
  int32_t exact;
  // Integer copies of F, G and D, valid when int_form is 1: the tables are
  // integral and small enough that the comparison kernel's integer form (int32
  // numerators, 24-bit multiplies) stays in range for every r and 8-bit input.
  int32_t Fi[64], Gi[64];
  int32_t Di;
  int32_t int_form;
};
rdct_status_t build_transform(int id, TransformTables* out);

// Quality sweep: plane descriptor, tile work item and kernel constants.
struct QPlane {
  const uint8_t* src;
  int64_t pitch;
  int32_t width, height;     // multiples of 8
  int32_t tiles_x, tiles_y;  // tiles of 32 x 32 windows
  uint64_t* sse;             // r_count accumulators
  int64_t* uqi;              // r_count accumulators (2^-32 units)
};
struct QTile {
  int32_t plane;
  int32_t tile;              // ty * tiles_x + tx
};
struct QualityArgs {
  TransformTables T;
  int32_t r_first, r_count;
};
int quality_tiles_x(int width);
int quality_tiles_y(int height);
hipError_t launch_quality(const QPlane& P, const QualityArgs& A, hipStream_t stream);
hipError_t launch_quality_batch(const QPlane* planes, const QTile* tiles, int32_t n_tiles,
                                const QualityArgs& A, hipStream_t stream);

// Codec output (zig-zag run-length pairs and 8-bit reconstruction).
struct CodecOutArgs {
  uint16_t* counts;       // pairs per block
  uint32_t* group_pairs;  // pairs per 64-block group
  int32_t* slots;         // 4096 pairs per group
  uint8_t* recon;         // nullable
  int64_t rpitch;         // bytes per reconstruction row
};
hipError_t launch_codec_encode(int sel, const Plane& P, const CodecOutArgs& o,
                               const QuantConsts& qc, hipStream_t stream);
hipError_t launch_codec_pack(const uint16_t* counts, const uint32_t* group_pairs,
                             const int32_t* slots, int32_t nblocks, uint32_t* offsets,
                             int32_t* packed, int64_t capacity, uint32_t* workspace,
                             hipStream_t stream);

enum SelKind { SEL_ZZ = 0, SEL_Q = 1 };
enum CoefKind { CO_NONE = 0, CO_I32 = 1, CO_I16 = 2, CO_F32 = 3 };
// EV_SPATIAL: squared error from the reconstruction, pixel by pixel.
// EV_SWEEP:   retention errors for r .. r + r_count - 1 from coefficient energies.
// EV_COEF:    quantisation error ||Z - q Q||^2 in the coefficient domain (equal to
//             the pixel-domain error because C_orth is orthogonal); planes made of
//             whole blocks only.
enum EvalKind { EV_NONE = 0, EV_SPATIAL = 1, EV_SWEEP = 2, EV_COEF = 3 };
enum InvKind { INV_INT_I32 = 0, INV_INT_I16 = 1, INV_F32 = 2, INV_Q_I32 = 3, INV_Q_I16 = 4 };

// Launch geometry choices (tuned per shape class).
struct Geometry {
  int32_t waves_per_wg;   // 1, 2, 4, 8
  int32_t grid_per_cu;    // persistent kernel: workgroups per CU
};

void fill_quant_consts(const uint16_t q[64], QuantConsts* out);
uint64_t keep_bits(int r);

hipError_t launch_plane(int sel, int co, bool recon, int ev, const Plane& P,
                        const QuantConsts& qc, int waves_per_wg,
                        hipStream_t stream);
hipError_t launch_inverse(int kind, const void* coef, int32_t width, int32_t height,
                          int32_t r, int32_t shift, float* dst, int64_t dpitch,
                          const QuantConsts& qc, hipStream_t stream);
hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t stream);

// Batch launch over a work list.  `planes` and `tables` are device arrays;
// `items` has n_items entries, grouped by plane.  first == nullptr: `grid`
// persistent workgroups stride over the list and add the error sums atomically
// (cleared beforehand).  Otherwise first[b] .. first[b + 1] - 1 are plane b's
// items, grid is the plane count, and each workgroup stores its plane's sums.
hipError_t launch_batch(int sel, int co, bool recon, int ev, const Plane* planes,
                        const QuantConsts* tables,
                        const WorkItem* items, int32_t n_items, int32_t grid,
                        int32_t waves_per_wg, hipStream_t stream,
                        const int32_t* first = nullptr, int xcd = 0,  // xcd: see xcd_remap
                        int strip = 1);  // strided layout: consecutive items per wave

// Compute units of the current device (looked up on every call).
int device_cu_count();
// Waves per workgroup of the single-plane kernels (measured best: one).
constexpr int kPlaneWavesPerWg = 1;

constexpr int64_t kMaxBlocks = 1ll << 26;   // transform calls
constexpr int64_t kMaxEvalBlocks = 6000000;  // evaluation: the uint64 SSE sums cannot wrap

// Validated selection: effective mode, r and the quantisation constants.
struct SelInfo {
  int sel;        // SEL_ZZ or SEL_Q
  int r;          // ZZ: 1..64 (NONE -> 64)
  int shift;
  uint16_t q[64]; // SEL_Q: the quantisation table
  QuantConsts qc;
};
rdct_status_t check_sel(const rdct_select_t* s, SelInfo* out);
rdct_status_t check_plane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch,
                          int64_t max_blocks);
Plane make_plane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch);
bool aligned(const void* p, uintptr_t a);


}  // namespace rdct
