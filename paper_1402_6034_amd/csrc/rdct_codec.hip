// Codec output of the keep-r and quantisation paths (Section 3 keeps the r
// initial zig-zag coefficients of every block; a codec stores exactly those and
// shows 8-bit pixels).
//
// Encode: one block per lane, 64 blocks (a group) per wave.  Each lane
// transforms its block (22-addition flow graphs), selects (keep r, or the
// exact quantiser), codes the kept coefficients in zig-zag order as
// (run, value) pairs -- a count pass, a wave prefix sum, an emit pass into the
// wave's LDS area at the lane's offset -- and the wave copies the group's
// pairs contiguously into the group's slot.  The lane then inverts its block
// and writes clamp(round(A'), 0, 255).  Pack: the group totals are scanned in
// chunks of 256 groups; every group then adds the chunk totals before it, writes
// its block offsets and copies its pairs into the packed stream.
#include "rdct_device.h"

namespace rdct {

constexpr int kGroup = 64;                 // blocks per group (one wave)
constexpr int kSlot = kGroup * 64;         // pairs a group can hold
// At most this many nonzero positions across a wave: reconstruct basis image by
// basis image (about 40 additions each) instead of the full inverse.
constexpr int kSparseRanks = 10;

using CodecOut = CodecOutArgs;

struct CodecKArgs {
  Plane P;
  CodecOut out;
  QuantConsts qc;
};

__device__ __forceinline__ QCPtr codec_table() {
  const RDCT_CONST char* seg = (const RDCT_CONST char*)__builtin_amdgcn_kernarg_segment_ptr();
  return (QCPtr)(seg + offsetof(CodecKArgs, qc));
}

// Pair word: run in the high 16 bits, the value as int16 in the low 16 bits.
__device__ __forceinline__ int32_t pair_word(int run, int v) {
  return (int32_t)(((uint32_t)run << 16) | ((uint32_t)v & 0xffffu));
}

// clamp(round(v), 0, 255) with halves away from zero, given t = v + 1/2: for
// v >= 0 the rounding is floor(t) = trunc(t); every v < 0 clamps to 0, and so
// does trunc(t) for t < 1.
__device__ __forceinline__ uint32_t to_u8(double t) {
  return (uint32_t)min(max((int)t, 0), 255);
}

// Store one reconstructed 8-pixel row (bytes b[0..7]), clipped to the plane.
__device__ __forceinline__ void store_u8_row(const Plane& P, const CodecOut& o, int x0, int y,
                                             const uint32_t (&b)[8], bool al8) {
  if (y >= P.height) return;
  uint8_t* row = o.recon + (int64_t)y * o.rpitch + x0;
  if (al8 && x0 + 8 <= P.width) {
    const uint32_t lo = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
    const uint32_t hi = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
    *reinterpret_cast<RDCT_GLOBAL u32x2*>(gptr(row)) = (u32x2){lo, hi};
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (x0 + j < P.width) row[j] = (uint8_t)b[j];
  }
}

template <int SEL>
__global__ __launch_bounds__(256) void k_codec(Plane P, CodecOut o, QuantConsts /*qc*/) {
  extern __shared__ int32_t lds_pairs[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int group = blockIdx.x * (blockDim.x >> 6) + wave;
  const int t0 = group * kGroup;
  if (t0 >= P.nblocks) return;
  const int t = t0 + lane;
  const bool valid = t < P.nblocks;
  int32_t* wpairs = lds_pairs + wave * kSlot;

  uint32_t px[16];
  int x0, y0;
  load_block(P, t, valid, px, x0, y0);
  int v[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) v[i][j] = pixel(px, i, j);
  pass2d<int, true>(v);
  // The level shift only moves the DC term: row 0 of C0 is all ones and rows
  // 1..7 sum to zero, so C0 (A - s) C0^T = C0 A C0^T - 64 s e_00.
  if constexpr (SEL == SEL_Q) v[0][0] -= 64 * P.shift;

  // Selection: keep the first r zig-zag positions, or quantise all 64.
  const int n_kept = SEL == SEL_Q ? 64 : P.r;
  if constexpr (SEL == SEL_Q) {
    const QCPtr qc = codec_table();
    static_for<0, 64>([&](auto c) {
      constexpr int kl = decltype(c)::value;
      v[kl >> 3][kl & 7] = quantize<kl>(v[kl >> 3][kl & 7], qc->qm[kl]);
    });
  }

  // Nonzero kept values by zig-zag rank (bit rank of nz_lo / nz_hi), the count,
  // a wave prefix, and the emit pass.  The emit walks the ranks in chunks of 8
  // and skips a chunk that is zero in every lane of the wave (its 8 zeros only
  // lengthen the run), which at ordinary qualities is most of them.
  uint32_t nz_lo = 0, nz_hi = 0;
#pragma unroll
  for (int rank = 0; rank < 64; ++rank) {
    const int kl = kZigZag.order[rank];
    const uint32_t nz = (rank < n_kept) ? min((uint32_t)v[kl >> 3][kl & 7], 1u) : 0u;
    if (rank < 32) nz_lo |= nz << rank;
    else nz_hi |= nz << (rank - 32);
  }
  if (!valid) nz_lo = nz_hi = 0;
  const int cnt = __builtin_popcount(nz_lo) + __builtin_popcount(nz_hi);
  // Ranks that are nonzero anywhere in the wave (wave-uniform).
  uint32_t any_lo = nz_lo, any_hi = nz_hi;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    any_lo |= __shfl_xor(any_lo, d, 64);
    any_hi |= __shfl_xor(any_hi, d, 64);
  }
  any_lo = __builtin_amdgcn_readfirstlane(any_lo);
  any_hi = __builtin_amdgcn_readfirstlane(any_hi);
  int off = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(off, d, 64);
    if (lane >= d) off += u;
  }
  const int total = __shfl(off, 63, 64);
  off -= cnt;                                  // exclusive
  {
    int run = 0, k = off;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {
      const uint32_t bits = ((c8 < 4 ? nz_lo : nz_hi) >> (8 * (c8 & 3))) & 0xffu;
      if (__ballot(bits != 0) == 0) {
        run += 8;
        continue;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int rank = 8 * c8 + i;
        const int kl = kZigZag.order[rank];
        if ((bits >> i) & 1u) {
          wpairs[k++] = pair_word(run, v[kl >> 3][kl & 7]);
          run = 0;
        } else {
          ++run;
        }
      }
    }
    if (valid) o.counts[t] = (uint16_t)cnt;
  }
  wave_sync();
  int32_t* slot = o.slots + (int64_t)group * kSlot;
  for (int i = lane; i < total; i += 64) slot[i] = wpairs[i];
  if (lane == 0) o.group_pairs[group] = (uint32_t)total;

  // 8-bit reconstruction.
  if (o.recon == nullptr || !valid) return;
  const bool al8 = ((reinterpret_cast<uintptr_t>(o.recon) | (uintptr_t)o.rpitch) & 7u) == 0;
  if constexpr (SEL == SEL_Q) {
    const QCPtr qc = codec_table();
    const double sh = (double)P.shift + 0.5;
    double w[8][8];
    if (__builtin_popcount(any_lo) + __builtin_popcount(any_hi) <= kSparseRanks) {
      // Few positions are nonzero anywhere in the wave (the common case at
      // ordinary qualities): add their basis images one by one.  Basis (k, l) is
      // z C0[k][i] C0[l][j] with z = q Q s_k s_l and entries 0 or +-1, so each
      // costs at most 64 additions, against ~450 operations for the full inverse.
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) w[i][j] = sh;
      static_for<0, 64>([&](auto rc) {
        constexpr int rank = decltype(rc)::value;
        constexpr int kl = kZigZag.order[rank], k = kl >> 3, l = kl & 7;
        if ((((rank < 32) ? any_lo : any_hi) >> (rank & 31)) & 1u) {
          const double z = (double)v[k][l] * qc->dq[kl];
          static_for<0, 64>([&](auto pc) {
            constexpr int i = decltype(pc)::value >> 3, j = decltype(pc)::value & 7;
            constexpr int sgn = kC0[k][i] * kC0[l][j];
            if constexpr (sgn > 0) w[i][j] += z;
            else if constexpr (sgn < 0) w[i][j] -= z;
          });
        }
      });
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) w[k][l] = (double)v[k][l] * qc->dq[k * 8 + l];
      pass2d<double, false>(w);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) w[i][j] += sh;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint32_t b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = to_u8(w[i][j]);
      store_u8_row(P, o, x0, y0 + i, b, al8);
    }
  } else {
    // R = C0^T D' (M . Y) D' C0 exactly; pixel = clamp(floor((R + 288) / 576), 0, 255).
    const uint64_t keep = P.keep;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int l = 0; l < 8; ++l)
        v[k][l] = ((keep >> (k * 8 + l)) & 1) ? v[k][l] * (kDp[k] * kDp[l]) : 0;
    pass2d<int, false>(v);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint32_t b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rr = v[i][j] + 288;
        b[j] = rr <= 0 ? 0u : min(255u, (uint32_t)rr / 576u);
      }
      store_u8_row(P, o, x0, y0 + i, b, al8);
    }
  }
}

// Offsets of the groups' pairs, in two steps with no single-workgroup stage
// (one workgroup scanning every total is bound by its own memory latency).
// k_codec_scan: workgroup c takes the chunk of kScanChunk consecutive groups
// and writes each group's exclusive prefix within its chunk to local[].
// k_codec_pack: the wave of group g adds the totals of the chunks before its
// own (chunk total = last group's local prefix + its pair count) to local[g].
constexpr int kScanChunk = 256;

__global__ __launch_bounds__(kScanChunk) void k_codec_scan(
    const uint32_t* __restrict__ group_pairs, int32_t n_groups, uint32_t* __restrict__ local) {
  __shared__ uint32_t wave_tot[kScanChunk / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = blockIdx.x * kScanChunk + t;
  const uint32_t v = g < n_groups ? group_pairs[g] : 0u;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) wave_tot[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int w = 0; w < kScanChunk / 64; ++w) before += w < wave ? wave_tot[w] : 0u;
  if (g < n_groups) local[g] = before + inc - v;
}

// One wave per group, kPackWaves groups per workgroup (64-thread workgroups
// leave the run bound by workgroup dispatch): the group's offset, its blocks'
// offsets and the copy of its pairs.
constexpr int kPackWaves = 4;

__global__ __launch_bounds__(64 * kPackWaves) void k_codec_pack(const uint16_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ group_pairs,
                                                   const int32_t* __restrict__ slots,
                                                   const uint32_t* __restrict__ local,
                                                   int32_t n_groups, int32_t nblocks,
                                                   uint32_t* __restrict__ offsets,
                                                   int32_t* __restrict__ packed, int64_t capacity) {
  const int g = blockIdx.x * kPackWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (g >= n_groups) return;
  // Every load that does not depend on the group's offset is issued first, so
  // the wave waits on memory about twice (these loads, then its stores) rather
  // than once per dependent step.  The first 128 words of the slot are loaded
  // whatever the pair count (a group averages about 66 pairs at Q50); the slot
  // always holds 4096 words.
  const int t = g * kGroup + lane;
  const int cnt = t < nblocks ? (int)counts[t] : 0;
  const uint32_t n = group_pairs[g];
  const uint32_t loc = local[g];
  const int32_t* src = slots + (int64_t)g * kSlot;
  const int32_t w0 = src[lane], w1 = src[lane + 64];
  // Totals of the chunks before this group's (all of them full chunks).
  const int chunk = g / kScanChunk;
  uint32_t prev = 0;
  for (int c = lane; c < chunk; c += 64) {
    const int last = c * kScanChunk + kScanChunk - 1;
    prev += local[last] + group_pairs[last];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) prev += __shfl_xor(prev, d, 64);
  const uint32_t b = prev + loc;
  if (g == n_groups - 1 && lane == 0) offsets[nblocks] = b + n;

  int off = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(off, d, 64);
    if (lane >= d) off += u;
  }
  if (t < nblocks) offsets[t] = b + (uint32_t)(off - cnt);
  if ((uint32_t)lane < n && (int64_t)b + lane < capacity) packed[b + lane] = w0;
  if ((uint32_t)lane + 64 < n && (int64_t)b + lane + 64 < capacity) packed[b + lane + 64] = w1;
  for (uint32_t i = lane + 128; i < n; i += 64)
    if ((int64_t)b + i < capacity) packed[b + i] = src[i];
}

hipError_t launch_codec_encode(int sel, const Plane& P, const CodecOut& o, const QuantConsts& qc,
                               hipStream_t s) {
  const int groups = (P.nblocks + kGroup - 1) / kGroup;
  if (groups <= 0) return hipSuccess;
  const int wpg = 2;   // 16 KB of LDS per wave
  const dim3 grid((groups + wpg - 1) / wpg), block(64 * wpg);
  const size_t lds = (size_t)wpg * kSlot * sizeof(int32_t);
  if (sel == SEL_Q)
    hipLaunchKernelGGL(k_codec<SEL_Q>, grid, block, lds, s, P, o, qc);
  else
    hipLaunchKernelGGL(k_codec<SEL_ZZ>, grid, block, lds, s, P, o, qc);
  return hipGetLastError();
}

hipError_t launch_codec_pack(const uint16_t* counts, const uint32_t* group_pairs,
                             const int32_t* slots, int32_t nblocks, uint32_t* offsets,
                             int32_t* packed, int64_t capacity, uint32_t* workspace,
                             hipStream_t s) {
  const int groups = (nblocks + kGroup - 1) / kGroup;
  if (groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_codec_scan, dim3((groups + kScanChunk - 1) / kScanChunk),
                     dim3(kScanChunk), 0, s, group_pairs, groups, workspace);
  hipLaunchKernelGGL(k_codec_pack, dim3((groups + kPackWaves - 1) / kPackWaves),
                     dim3(64 * kPackWaves), 0, s, counts, group_pairs, slots,
                     workspace, groups, nblocks, offsets, packed, capacity);
  return hipGetLastError();
}

}  // namespace rdct
