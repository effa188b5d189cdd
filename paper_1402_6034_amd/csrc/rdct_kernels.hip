// HIP kernels of the round-off DCT hot path for gfx950 (CDNA4, wave64).
//
// Method (Cintra & Bayer): every 8x8 block A of a plane is mapped to
// Y = C0 A C0^T with C0 = [2 C] (entries 0, +-1), using an addition-only flow
// graph of 22 additions per 8-point pass (Section 2, Fig. 1, Table 1); the
// diagonal orthogonaliser S is folded into the zig-zag retention or the
// quantisation that follows (Sections 2-3); the inverse runs through C0^T since
// C_orth = S C0 is orthogonal (Section 2); the error is scored by SSE (Section 3).
//
// Mapping to the hardware.  The transform has no dense contraction (an 8-point
// pass is 22 integer additions), so nothing here uses MFMA.  The kernels are
// streaming and HBM-bound: each wave owns a chunk of 128 consecutive blocks in
// raster order; lane j transforms blocks t0 + j and t0 + 64 + j at once, packed
// as the low and high halves of 16-bit pairs (v_pk_add/sub_u16), which is exact
// because |Y| <= 16320.  Row loads are 8 bytes per lane and consecutive lanes
// read consecutive blocks, so one load instruction covers 512 contiguous bytes
// of an image row.  Both passes stay in registers (the transpose between the
// row and the column pass is free: a lane holds whole blocks).
#include "rdct_device.h"

namespace rdct {

__constant__ ZigZag c_zz = make_zigzag();

__device__ __forceinline__ s16x2 as_pair(uint32_t u) { return __builtin_bit_cast(s16x2, u); }

// Pack byte j of two row dwords into a (lo block, hi block) 16-bit pair.
template <int J>
__device__ __forceinline__ s16x2 unpack_pair(uint32_t lo, uint32_t hi) {
  constexpr uint32_t sel = 0x0c000c00u | ((uint32_t)(4 + J) << 16) | (uint32_t)J;
  return as_pair(__builtin_amdgcn_perm(hi, lo, sel));
}

__device__ __forceinline__ void forward_pair(const uint32_t (&al)[16], const uint32_t (&ah)[16],
                                             int shift, s16x2 (&v)[8][8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    v[i][0] = unpack_pair<0>(al[2 * i], ah[2 * i]);
    v[i][1] = unpack_pair<1>(al[2 * i], ah[2 * i]);
    v[i][2] = unpack_pair<2>(al[2 * i], ah[2 * i]);
    v[i][3] = unpack_pair<3>(al[2 * i], ah[2 * i]);
    v[i][4] = unpack_pair<0>(al[2 * i + 1], ah[2 * i + 1]);
    v[i][5] = unpack_pair<1>(al[2 * i + 1], ah[2 * i + 1]);
    v[i][6] = unpack_pair<2>(al[2 * i + 1], ah[2 * i + 1]);
    v[i][7] = unpack_pair<3>(al[2 * i + 1], ah[2 * i + 1]);
  }
  pass2d<s16x2, true>(v);
  // A level shift only moves the DC term: rows 1..7 of C0 sum to zero and the
  // DC gain of C0 (x) C0 is 64.
  const short dc = (short)(64 * shift);
  v[0][0] -= (s16x2){dc, dc};
}

// Signed 16-bit half h (0 = low block, 1 = high block) of a packed pair.
__device__ __forceinline__ int half(s16x2 v, int h) {
  return __builtin_amdgcn_sbfe((int)__builtin_bit_cast(uint32_t, v), 16 * h, 16);
}

// ---------------------------------------------------------------------------
// Stores of one block's coefficients (64 values, 16-byte vector stores).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_i32(int32_t* out, const s16x2 (&v)[8][8], uint64_t keep,
                                          int h) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int e[8];
#pragma unroll
    for (int l = 0; l < 8; ++l) e[l] = ((keep >> (k * 8 + l)) & 1) ? half(v[k][l], h) : 0;
    reinterpret_cast<int4*>(out)[2 * k] = make_int4(e[0], e[1], e[2], e[3]);
    reinterpret_cast<int4*>(out)[2 * k + 1] = make_int4(e[4], e[5], e[6], e[7]);
  }
}

__device__ __forceinline__ void store_i16(int16_t* out, const s16x2 (&v)[8][8], uint64_t keep,
                                          int h) {
  // Byte selectors of v_perm_b32 that gather the 16-bit half h of two pairs.
  const uint32_t sel = h ? 0x07060302u : 0x05040100u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uint32_t d[4];
#pragma unroll
    for (int l = 0; l < 8; l += 2) {
      const uint32_t m0 = ((keep >> (k * 8 + l)) & 1) ? 0xffffffffu : 0u;
      const uint32_t m1 = ((keep >> (k * 8 + l + 1)) & 1) ? 0xffffffffu : 0u;
      const uint32_t u0 = __builtin_bit_cast(uint32_t, v[k][l]) & m0;
      const uint32_t u1 = __builtin_bit_cast(uint32_t, v[k][l + 1]) & m1;
      d[l >> 1] = __builtin_amdgcn_perm(u1, u0, sel);
    }
    reinterpret_cast<uint4*>(out)[k] = make_uint4(d[0], d[1], d[2], d[3]);
  }
}

__device__ __forceinline__ void store_f32(float* out, const s16x2 (&v)[8][8], uint64_t keep,
                                          int h) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float e[8];
#pragma unroll
    for (int l = 0; l < 8; ++l)
      e[l] = ((keep >> (k * 8 + l)) & 1) ? (float)((double)half(v[k][l], h) * scale_kl(k, l))
                                         : 0.0f;
    reinterpret_cast<float4*>(out)[2 * k] = make_float4(e[0], e[1], e[2], e[3]);
    reinterpret_cast<float4*>(out)[2 * k + 1] = make_float4(e[4], e[5], e[6], e[7]);
  }
}

// Store one reconstructed row of 8 pixels (clipped to the plane).
__device__ __forceinline__ void store_row(const Plane& P, int x0, int y, const float (&px)[8]) {
  if (y >= P.height) return;
  RDCT_GLOBAL float* row = gptr(P.recon) + (int64_t)y * P.rpitch + x0;
  if (x0 + 8 <= P.width && ((reinterpret_cast<uintptr_t>(row) & 15u) == 0)) {
    reinterpret_cast<RDCT_GLOBAL f32x4*>(row)[0] = (f32x4){px[0], px[1], px[2], px[3]};
    reinterpret_cast<RDCT_GLOBAL f32x4*>(row)[1] = (f32x4){px[4], px[5], px[6], px[7]};
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (x0 + j < P.width) row[j] = px[j];
  }
}

// ---------------------------------------------------------------------------
// Coefficient output through LDS.  A lane produces its block's 64 values in
// natural order; written straight to HBM that is 16-byte pieces 128-256 bytes
// apart across the wave, which splits every cache line between many requests.
// Instead each lane writes its block into a per-wave LDS stage (block stride
// padded by 16 bytes, so the eight lanes of one 128-byte LDS pass hit distinct
// banks), and the wave then copies the stage out in order: every store
// instruction covers 1 KB of contiguous output.
// ---------------------------------------------------------------------------
template <int CO>
struct Stage {
  static constexpr int bytes = (CO == CO_I16) ? 128 : 256;  // one block's coefficients
  static constexpr int stride = bytes + 16;                   // padded LDS block stride
  static constexpr int wave_bytes = (CO == CO_NONE) ? 0 : 64 * stride;
};


// Copy the stage of 64 consecutive blocks (first block t_first, `nvalid` of them
// inside the plane) to the block-major output.
template <int CO>
__device__ __forceinline__ void flush_stage(const uint8_t* stage, void* coef, int64_t t_first,
                                            int nvalid, int lane) {
  constexpr int per_block = Stage<CO>::bytes / 16;   // 16-byte pieces per block
  constexpr int pieces = 64 * per_block;
  RDCT_GLOBAL uint8_t* out = gptr(reinterpret_cast<uint8_t*>(coef)) + t_first * Stage<CO>::bytes;
  const int limit = nvalid * per_block;
#pragma unroll
  for (int m = 0; m < pieces / 64; ++m) {
    const int c = lane + 64 * m;
    const int b = c / per_block, o = c - b * per_block;
    if (c < limit) {
      const u32x4 val = *reinterpret_cast<const u32x4*>(stage + b * Stage<CO>::stride + o * 16);
      __builtin_nontemporal_store(val, reinterpret_cast<RDCT_GLOBAL u32x4*>(out + (int64_t)c * 16));
    }
  }
}

// ---------------------------------------------------------------------------
// Quantisation path.  Both blocks of a lane's pair are quantised together, so
// every table constant is read once per chunk; q of the high block waits in
// registers (16-bit pairs) while the low block's stage is written out.
// ---------------------------------------------------------------------------
// Per-block error of the quantisation path in the coefficient domain,
// ||Z - q Q||^2 (the orthogonal C_orth preserves it, Section 2).  At rational
// positions (s_k s_l = 1/c, c = g_k) Z - qQ = (Y - c qQ) / c exactly, so the
// squares are summed in integers per c; irrational positions use float64.
struct QErr {
  double irr = 0.0;
  int r8 = 0, r6 = 0, r4 = 0;
};

__device__ __forceinline__ uint64_t qerr_units(const QErr& e) {
  // |Y - c qQ| <= c Q / 2 + 1, so each sum stays far below 2^31.
  const double rat = (double)e.r8 * (1.0 / 64.0) + (double)e.r6 / 36.0 + (double)e.r4 * (1.0 / 16.0);
  return (uint64_t)__builtin_fma(e.irr + rat, 1048576.0, 0.5);
}

// Quantise one coefficient y at position KL; z = q Q (|z| < 2^15) for the inverse.
template <int KL, bool ERR, bool FQ>
__device__ __forceinline__ int quant_one(int y, QCPtr qc, QErr& e, int& z) {
  constexpr int k = KL >> 3, l = KL & 7;
  const int Q = qc->qi[KL];
  const int q = FQ ? quantize_fma(y, qc->qf[KL]) : quantize<KL>(y, qc->qm[KL]);
  z = __mul24(q, Q);
  if constexpr (ERR) {
    if constexpr (rational_pos(k, l)) {
      const int en = y - kGram[k] * z;
      if constexpr (kGram[k] == 8) e.r8 += __mul24(en, en);
      else if constexpr (kGram[k] == 6) e.r6 += __mul24(en, en);
      else e.r4 += __mul24(en, en);
    } else {
      // z_kl - q Q with z_kl = s_k s_l Y: one rounding (FMA) per coefficient.
      const double d = __builtin_fma((double)y, scale_kl(k, l), -(double)z);
      e.irr = __builtin_fma(d, d, e.irr);
    }
  }
  return q;
}

// Row K of block h of the pair: q goes to the lane's stage; with WB, q Q
// replaces half h of the row's pairs (|q Q| < 2^15) for the inverse.  FQ picks
// the FMA form of the quantiser.  Returns a value of the row's result, used to
// gate the table reads of a later row.
template <int K, int CO, bool ERR, bool WB, bool FQ, int... L>
__device__ __forceinline__ uint32_t quant_row(s16x2 (&row)[8], int h, QCPtr qc, uint8_t* stage,
                                              QErr& e, std::integer_sequence<int, L...>) {
  int q[8];
  // v_perm_b32 selectors that replace half h of a pair by the low half of z.
  const uint32_t put = h ? 0x01000504u : 0x07060100u;
  auto one = [&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int kl = K * 8 + l;
    int z;
    q[l] = quant_one<kl, ERR, FQ>(half(row[l], h), qc, e, z);
    if constexpr (WB)
      row[l] = as_pair(__builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, row[l]), (uint32_t)z, put));
  };
  (one(std::integral_constant<int, L>{}), ...);
  if constexpr (CO == CO_I32) {
    int4* out = reinterpret_cast<int4*>(stage + K * 32);
    out[0] = make_int4(q[0], q[1], q[2], q[3]);
    out[1] = make_int4(q[4], q[5], q[6], q[7]);
  } else if constexpr (CO == CO_I16) {
    uint32_t d[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if constexpr (FQ)  // low halves of q[2m] (bits 0-15) and q[2m+1] (16-31)
        d[m] = __builtin_amdgcn_perm((uint32_t)q[2 * m + 1], (uint32_t)q[2 * m], 0x05040100u);
      else
        d[m] = ((uint32_t)q[2 * m] & 0xffffu) | ((uint32_t)q[2 * m + 1] << 16);
    }
    *reinterpret_cast<uint4*>(stage + K * 16) = make_uint4(d[0], d[1], d[2], d[3]);
  }
  return (uint32_t)q[7];
}

template <int CO, bool ERR, bool WB, bool FQ>
__device__ __forceinline__ void quant_rows(s16x2 (&v)[8][8], int h, QCPtr qc, uint8_t* stage,
                                           QErr& e) {
  QCPtr row_qc[8];
  row_qc[0] = qc;
  row_qc[1] = qc;
  static_for<0, 8>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const uint32_t dep = quant_row<K, CO, ERR, WB, FQ>(v[K], h, row_qc[K], stage, e,
                                                   std::make_integer_sequence<int, 8>{});
    if constexpr (K + 2 < 8) row_qc[K + 2] = qc_after(qc, dep);
    // Finish the row (including its error terms) before the next one starts.
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Inverse of the quantisation path, A' = C0^T S (q . Q) S C0 + shift.
// Column pass (over k), exact, on the (low, high) 16-bit pairs of q Q: grouped
// by the three values of s_k, column l gives p = Z0 + Z4 and m = Z0 - Z4
// (s = 1/sqrt8), Z2 and Z6 (s = 1/2) and the odd combinations b0..b3 of Z1, Z3,
// Z5, Z7 (s = 1/sqrt6) -- the transposed flow graph without its last stage.
// Every partial sum is below 2^15 in magnitude.  The level shift enters as
// 8 * shift on Z_00 (the DC basis function of C_orth is 1/8 everywhere).
// Results replace the rows of v: 0 = p, 1 = m, 2 = Z2, 3 = Z6, 4..7 = b0..b3.
__device__ __forceinline__ void quant_columns_pair(s16x2 (&v)[8][8], int shift) {
  const short s8 = (short)(8 * shift);
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    s16x2 z[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) z[k] = v[k][l];
    if (l == 0) z[0] += (s16x2){s8, s8};
    v[0][l] = z[0] + z[4];
    v[1][l] = z[0] - z[4];
    v[2][l] = z[2];
    v[3][l] = z[6];
    v[4][l] = z[1] + (z[3] + z[5]);
    v[5][l] = z[1] - (z[5] + z[7]);
    v[6][l] = (z[1] + z[7]) - z[3];
    v[7][l] = z[5] - (z[3] + z[7]);
  }
}

// Reconstruction through LDS.  Written straight from the lanes, a row of a
// block is 32 bytes and lanes are 32 bytes apart, so every 16-byte store
// instruction leaves gaps that the next one fills; HBM writes that way run far
// below contiguous ones.  For planes made of whole blocks the row pass instead
// writes four rows of the 64 blocks of one half into the wave's stage (one
// padded 2 KB slot per row) and the wave stores each slot as two contiguous
// 1 KB pieces.
constexpr int kReconSlot = 64 * 32 + 16;
constexpr int kReconStageBytes = 4 * kReconSlot;

// LDS bytes of a wave's stage: the coefficient stage, or the reconstruction
// staging (whole-block quantisation planes; keep-r planes whose blocks are
// whole) if that is larger.
template <int SEL, int CO, bool RECON, int EV>
constexpr int wave_stage_bytes() {
  constexpr int coef = Stage<CO>::wave_bytes;
  constexpr bool staged = RECON && ((SEL == SEL_Q && EV == EV_COEF) || SEL == SEL_ZZ);
  return (staged && kReconStageBytes > coef) ? kReconStageBytes : coef;
}

// Reconstruction rows go through the stage when the plane is made of whole
// blocks (every staged piece lies inside the plane); planes with partial
// blocks store row pieces clipped to the plane.
__device__ __forceinline__ bool recon_stageable(const Plane& P) {
  return ((P.width | P.height) & 7) == 0;
}

__device__ __forceinline__ void recon_stage_row(uint8_t* stage_wave, int slot, int lane,
                                                const float (&px)[8]) {
  f32x4* p = reinterpret_cast<f32x4*>(stage_wave + slot * kReconSlot + lane * 32);
  p[0] = (f32x4){px[0], px[1], px[2], px[3]};
  p[1] = (f32x4){px[4], px[5], px[6], px[7]};
}

// Where the lanes store: lane j writes piece (j & 1) of blocks j / 2 and
// 32 + j / 2 of the half.
struct ReconFlush {
  int64_t off0, off1;  // float offsets of those pieces' row 0 in the plane
  bool ok0, ok1;       // block inside the plane (the last chunk may be short)
};

__device__ __forceinline__ ReconFlush recon_flush_setup(const Plane& P, int x0, int y0,
                                                        int nvalid, int lane) {
  const int b0 = lane >> 1, b1 = 32 + (lane >> 1);
  const int piece = (lane & 1) * 4;
  ReconFlush f;
  const int xa = __shfl(x0, b0, 64), ya = __shfl(y0, b0, 64);
  const int xb = __shfl(x0, b1, 64), yb = __shfl(y0, b1, 64);
  f.off0 = (int64_t)ya * P.rpitch + xa + piece;
  f.off1 = (int64_t)yb * P.rpitch + xb + piece;
  f.ok0 = b0 < nvalid;
  f.ok1 = b1 < nvalid;
  return f;
}

__device__ __forceinline__ void recon_flush_rows(const Plane& P, const uint8_t* stage_wave,
                                                 const ReconFlush& f, const int (&rows)[4],
                                                 int lane) {
  RDCT_GLOBAL float* out = gptr(P.recon);
  // Rows are 16-byte aligned unless the caller's pointer or pitch is not.
  const bool al16 = ((reinterpret_cast<uintptr_t>(P.recon) & 15u) | (P.rpitch & 3)) == 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint8_t* slot = stage_wave + s * kReconSlot;
    const int64_t ro = (int64_t)rows[s] * P.rpitch;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m ? f.ok1 : f.ok0) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(slot + 1024 * m + lane * 16);
        RDCT_GLOBAL float* dst = out + (m ? f.off1 : f.off0) + ro;
        if (al16) {
          __builtin_nontemporal_store(v, reinterpret_cast<RDCT_GLOBAL f32x4*>(dst));
        } else {
          dst[0] = v.x;
          dst[1] = v.y;
          dst[2] = v.z;
          dst[3] = v.w;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse of one block of the pair + reconstruction + squared error.
// Retention: R = C0^T (D' (M . Y) D') C0 in int32 (|R| <= 576 * 2040), A' = R/576.
// Returns the block's exact sum of (576 (A - shift) - R)^2 over its own pixels.
// With STAGE (wave-uniform; whole-block planes) every lane of the wave takes
// part -- lanes without a block compute on zeros and are masked at the store
// and by the caller -- and rows leave through the stage four at a time.
// ---------------------------------------------------------------------------
template <bool RECON, bool SSE>
__device__ __forceinline__ uint64_t retention_inverse(const Plane& P, const s16x2 (&v)[8][8],
                                                      uint64_t keep, const uint32_t (&a)[16],
                                                      int x0, int y0, int h, bool stage,
                                                      uint8_t* stage_wave, int lane, int nvalid) {
  int w[8][8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int l = 0; l < 8; ++l)
      w[k][l] = ((keep >> (k * 8 + l)) & 1) ? half(v[k][l], h) * (kDp[k] * kDp[l]) : 0;
  pass2d<int, false>(w);
  ReconFlush fl;
  if constexpr (RECON) {
    if (stage) fl = recon_flush_setup(P, x0, y0, nvalid, lane);
  }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if constexpr (RECON) {
      float px[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        px[j] = (float)__builtin_fma((double)w[i][j], 1.0 / 576.0, (double)P.shift);
      if (stage) {
        recon_stage_row(stage_wave, i & 3, lane, px);
        if ((i & 3) == 3) {
          const int rows[4] = {i - 3, i - 2, i - 1, i};
          wave_sync();
          recon_flush_rows(P, stage_wave, fl, rows, lane);
          wave_sync();
        }
      } else {
        store_row(P, x0, y0 + i, px);
      }
    }
    if constexpr (SSE) {
      const bool row_ok = y0 + i < P.height;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = 576 * (pixel(a, i, j) - P.shift) - w[i][j];
        const double ed = (row_ok && x0 + j < P.width) ? (double)e : 0.0;
        acc = __builtin_fma(ed, ed, acc);
      }
    }
  }
  return (uint64_t)acc;  // exact: < 2^53 per block
}

// Row pass (over l) in float64 for block h of the pair.  Rows i and 7 - i of
// C0^T S Z are a_i +- b_i with a_i = {p or m}/sqrt8 +- {Z2 or Z6}/2 and
// b_i = b_i/sqrt6; scaled by s_l they feed the transposed flow graph.  With SP,
// accumulates the pixel-domain squared error over the block's own pixels.
template <bool RECON, bool SP, bool STAGED>
__device__ __forceinline__ void quant_row_pass(const Plane& P, const s16x2 (&c)[8][8], int h,
                                               const uint32_t (&a)[16], int x0, int y0,
                                               double& err, uint8_t* stage_wave, int lane,
                                               int nvalid) {
  ReconFlush fl;
  if constexpr (RECON && STAGED) fl = recon_flush_setup(P, x0, y0, nvalid, lane);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double up[8], um[8];
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      const int e8 = half(c[(i == 0 || i == 3) ? 0 : 1][l], h);
      const int e4 = half(c[(i == 0 || i == 3) ? 2 : 3][l], h);
      const int eb = half(c[4 + i][l], h);
      const double s4 = (i == 0 || i == 2) ? scale_kl(2, l) : -scale_kl(2, l);
      const double al = __builtin_fma((double)e4, s4, (double)e8 * scale_kl(0, l));
      const double be = (double)eb * scale_kl(1, l);
      up[l] = al + be;
      um[l] = al - be;
    }
    c0_transpose(up);
    c0_transpose(um);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int row = side ? 7 - i : i;
      const double (&o)[8] = side ? um : up;
      if constexpr (RECON) {
        float px[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) px[j] = (float)o[j];
        if constexpr (STAGED)
          recon_stage_row(stage_wave, (i & 1) * 2 + side, lane, px);
        else
          store_row(P, x0, y0 + row, px);
      }
      if constexpr (SP) {
        const bool row_ok = y0 + row < P.height;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double e = (double)pixel(a, row, j) - o[j];
          const double ed = (row_ok && x0 + j < P.width) ? e : 0.0;
          err = __builtin_fma(ed, ed, err);
        }
      }
    }
    if constexpr (RECON && STAGED) {
      if (i & 1) {
        // Slots hold rows i - 1, 8 - i, i, 7 - i.
        const int rows[4] = {i - 1, 8 - i, i, 7 - i};
        wave_sync();
        recon_flush_rows(P, stage_wave, fl, rows, lane);
        wave_sync();
      }
    }
  }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t s) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// ---------------------------------------------------------------------------
// One wave, one chunk of 128 blocks.
// ---------------------------------------------------------------------------
// Pixels of one chunk as loaded by a lane: blocks t0 + lane (lo) and
// t0 + 64 + lane (hi).
// With `half`, the chunk is blocks t0 .. t0 + 63 only (the high blocks of the
// pairs stay empty; see half_chunks).  nv0 / nv1 count the blocks of each half
// inside the plane (wave-uniform).
struct Pixels {
  uint32_t al[16], ah[16];
  int xl, yl, xh, yh;
  int t0;
  int nv0, nv1;
  bool vl, vh;
};

__device__ __forceinline__ void chunk_load(const Plane& P, int t0, int lane, Pixels& px,
                                           bool half = false) {
  px.t0 = t0;
  px.nv0 = min(64, max(0, P.nblocks - t0));
  px.nv1 = half ? 0 : min(64, max(0, P.nblocks - t0 - 64));
  px.vl = lane < px.nv0;
  px.vh = lane < px.nv1;
  load_block(P, t0 + lane, px.vl, px.al, px.xl, px.yl);
  load_block(P, t0 + 64 + lane, px.vh, px.ah, px.xh, px.yh);
}

// Error sums of one wave: a lane's part, added to others and written by
// flush_sums.  EV_SPATIAL / EV_COEF: every lane holds a partial of the plane's
// one sum.  EV_SWEEP: lane rho holds the dropped energy at rank rho, the sum for
// r = rho (lanes outside r .. r + r_count - 1 hold nothing that is written).
template <int EV>
__device__ __forceinline__ void flush_sums(const Plane& P, uint64_t part, int lane) {
  if constexpr (EV == EV_SPATIAL || EV == EV_COEF) {
    const uint64_t s = wave_sum_u64(part);
    if (lane == 0 && s != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(P.sse), (unsigned long long)s);
  } else if constexpr (EV == EV_SWEEP) {
    if (lane >= P.r && lane < P.r + P.r_count && part != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(P.sse + (lane - P.r)),
                (unsigned long long)part);
  }
}

// One chunk: outputs written, the lane's part of the error sums returned.
template <int SEL, int CO, bool RECON, int EV>
__device__ __forceinline__ uint64_t plane_chunk(const Plane& P, QCPtr qc, const Pixels& px,
                                                int lane, uint32_t* lds_wave,
                                                uint8_t* stage_wave) {
  const int t0 = px.t0;
  const bool vl = px.vl, vh = px.vh;
  const int xl = px.xl, yl = px.yl, xh = px.xh, yh = px.yh;
  const uint32_t (&al)[16] = px.al;
  const uint32_t (&ah)[16] = px.ah;

  s16x2 v[8][8];
  forward_pair(al, ah, P.shift, v);

  if constexpr (SEL == SEL_Q) {
    constexpr bool ERR = (EV == EV_COEF);
    constexpr bool SP = (EV == EV_SPATIAL);
    constexpr bool WB = RECON || SP;
    // The FMA form of the quantiser everywhere but in the kernels that keep the
    // pixels for a pixel-domain error.  Those keep the split form: with the FMA
    // form, the strided batch kernel of that kind wrote wrong reconstructions
    // of planes with partial blocks, and no cause was found in the source.
    constexpr bool FQ = !SP;
    uint64_t s = 0;
    uint8_t* my_stage = stage_wave + lane * Stage<CO>::stride;
    // Quantise one block of the pair at a time through the lane's stage slot.
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      if ((h ? px.nv1 : px.nv0) == 0) continue;  // an empty half (64-block chunks)
      QErr e;
      quant_rows<CO, ERR, WB, FQ>(v, h, qc_after_s(qc, h), my_stage, e);
      if constexpr (ERR) {
        const uint64_t valid = (uint64_t)0 - (uint64_t)(h ? vh : vl);
        s += qerr_units(e) & valid;
        // Materialise the sum here: otherwise the compiler sinks the whole error
        // computation past the stage flush and keeps its inputs live through it.
        asm volatile("" : "+v"(s));
      }
      if constexpr (CO != CO_NONE) {
        const int first = t0 + 64 * h;
        // Recompute the flush addresses in every iteration rather than keeping
        // them live (and spilled) across the loop.
        int ln = lane;
        asm volatile("" : "+v"(ln) : "s"(h));
        wave_sync();
        flush_stage<CO>(stage_wave, P.coef, first, h ? px.nv1 : px.nv0, ln);
        wave_sync();
      }
    }
    if constexpr (WB) {
      quant_columns_pair(v, P.shift);
      // One block of the pair at a time keeps a single float64 row pass live.
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        if ((h ? px.nv1 : px.nv0) == 0) continue;
        // The staged store is a wave-wide operation: every lane takes part, and
        // lanes past the end of the plane are masked at the store.
        if constexpr (!(RECON && EV == EV_COEF)) {
          if (!(h ? vh : vl)) continue;
        }
        uint32_t a[16];
        if constexpr (SP) {
#pragma unroll
          for (int i = 0; i < 16; ++i) a[i] = h ? ah[i] : al[i];
        }
        double err = 0.0;
        // EV_COEF is only used for planes made of whole blocks; those stage the
        // reconstruction.
        quant_row_pass<RECON, SP, EV == EV_COEF>(P, v, h, a, h ? xh : xl, h ? yh : yl, err,
                                                 stage_wave, lane, h ? px.nv1 : px.nv0);
        if constexpr (SP) s += (uint64_t)__builtin_fma(err, 1048576.0, 0.5);
      }
    }
    return s;
  } else {
  const uint64_t keep = P.keep;
  if constexpr (CO != CO_NONE) {
    uint8_t* my_stage = stage_wave + lane * Stage<CO>::stride;
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      if ((h ? px.nv1 : px.nv0) == 0) continue;
      if (h ? vh : vl) {
        if constexpr (CO == CO_I32)
          store_i32(reinterpret_cast<int32_t*>(my_stage), v, keep, h);
        else if constexpr (CO == CO_I16)
          store_i16(reinterpret_cast<int16_t*>(my_stage), v, keep, h);
        else
          store_f32(reinterpret_cast<float*>(my_stage), v, keep, h);
      }
      const int first = t0 + 64 * h;
      wave_sync();
      flush_stage<CO>(stage_wave, P.coef, first, h ? px.nv1 : px.nv0, lane);
      wave_sync();
    }
  }

  constexpr bool SP = (EV == EV_SPATIAL);
  if constexpr (RECON || SP) {
    uint64_t s = 0;
    const bool stage = RECON && recon_stageable(P);
    // One block at a time keeps a single 8x8 inverse live in registers.
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      const bool valid = h ? vh : vl;
      if ((h ? px.nv1 : px.nv0) == 0) continue;
      // A staged store is a wave-wide operation: every lane takes part.
      if (!valid && !stage) continue;
      uint32_t a[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = h ? ah[i] : al[i];
      const uint64_t e = retention_inverse<RECON, SP>(P, v, keep, a, h ? xh : xl, h ? yh : yl, h,
                                                      stage, stage_wave, lane,
                                                      h ? px.nv1 : px.nv0);
      s += valid ? e : 0;
    }
    if constexpr (SP) return s;
  }

  if constexpr (EV == EV_SWEEP) {
    // Per-position energies of the pair, transposed through LDS so that lane rho
    // sums the position of zig-zag rank rho over the chunk.
#pragma unroll
    for (int kl = 0; kl < 64; ++kl) {
      const int y0v = vl ? (int)v[kl >> 3][kl & 7].x : 0;
      const int y1v = vh ? (int)v[kl >> 3][kl & 7].y : 0;
      lds_wave[lane * 65 + kl] = (uint32_t)(y0v * y0v) + (uint32_t)(y1v * y1v);
    }
    wave_sync();
    const int pos = c_zz.order[lane];
    uint64_t e = 0;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) e += lds_wave[j * 65 + pos];
    wave_sync();
    // Weighted energy d'_k d'_l sum Y^2 at rank `lane`, then suffix sums over rank:
    // the dropped energy when the first rho coefficients are kept.
    uint64_t x = e * (uint64_t)(kDp[pos >> 3] * kDp[pos & 7]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t o = __shfl_down(x, off, 64);
      if (lane + off < 64) x += o;
    }
    return 576ull * x;
  }
  return 0;
  }
}

// Register budget: two waves per SIMD, except the variants that would spill
// heavily at that budget and get a full wave-per-SIMD budget instead:
// quantisation keeping pixels live for a pixel-domain error (planes with
// partial blocks) or staging int32 coefficients beside the reconstruction, and
// retention writing 32-bit coefficients beside the reconstruction (8192^2,
// r = 10: 154 -> 141 us with int32, 159 -> 142 us with float32; with the
// 45-value sweep 198 -> 147 and 209 -> 150 us).  Retention variants spilling
// less (32-bit coefficients without reconstruction, 16-bit with it) measured
// the same either way and keep two waves per SIMD.
template <int SEL, int CO, bool RECON, int EV>
struct WideRegs {
  static constexpr bool value =
      ((SEL == SEL_Q) && (EV == EV_SPATIAL || (RECON && CO == CO_I32))) ||
      ((SEL == SEL_ZZ) && RECON && (CO == CO_I32 || CO == CO_F32) &&
       (EV == EV_SPATIAL || EV == EV_SWEEP));
};

// Persistent batch kernels: prefetching the next work item costs ~40 registers;
// it is used where the kernel is a pure stream (transform, quantise, store).
// Kernels that also invert keep a float64 or int32 block live and run without it.
template <int SEL, bool RECON, int EV>
struct Prefetch {
  static constexpr bool value = !RECON && (EV == EV_NONE || EV == EV_COEF || EV == EV_SWEEP);
};

// Chunks of 64 blocks, one per lane (the high halves of the pairs empty):
//  * for the pure streams (forward, selection or quantisation, coefficient
//    stores; no error sums) at every size: twice the waves, each with half the
//    stores, keep more of the plane in flight (8192^2 quantised to int16,
//    input and output rotating past the last-level cache: 37.6 -> 36.4 us);
//  * for the other kernels on a plane of at most 128 blocks per CU (on 256
//    CUs): its waves are few and each one's latency decides the launch.  On
//    larger planes the doubled forward work per block costs more than it gains.
template <int EV>
__host__ __device__ constexpr bool half_chunks(int nblocks) {
  return EV == EV_NONE || nblocks <= 128 * 256;
}

template <int SEL, int CO, bool RECON, int EV>
__device__ __forceinline__ void plane_kernel_body(const Plane& P, QCPtr qc) {
  // Chunks of 128 blocks (64 where half_chunks says so): wave w takes
  // chunks w, w + W, ... (W waves in the grid).  Without error sums the grid
  // covers the plane, one chunk per wave; with them the grid is capped, so a
  // large plane's sums take one atomic per wave instead of one per chunk, all on
  // the same address.
  extern __shared__ uint32_t lds[];
  const int wpg = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n_waves = gridDim.x * wpg;
  const bool half = half_chunks<EV>(P.nblocks);
  const int cs = half ? 64 : 128;
  int c = blockIdx.x * wpg + wave;
  if (c * cs >= P.nblocks) return;
  uint8_t* stage = reinterpret_cast<uint8_t*>(lds + (EV == EV_SWEEP ? wpg * 64 * 65 : 0)) +
                   wave * wave_stage_bytes<SEL, CO, RECON, EV>();
  uint64_t acc = 0;
  for (; c * cs < P.nblocks; c += n_waves) {
    Pixels cur;
    chunk_load(P, c * cs, lane, cur, half);
    acc += plane_chunk<SEL, CO, RECON, EV>(P, qc, cur, lane, lds + wave * (64 * 65), stage);
    if constexpr (EV == EV_NONE) break;
  }
  flush_sums<EV>(P, acc, lane);
}

// The single-plane kernels take the quantisation table by value, so a call needs
// no device allocation; it is read in place from the kernel-argument segment,
// whose layout is that of PlaneArgs.
struct PlaneArgs {
  Plane P;
  QuantConsts qc;
};

__device__ __forceinline__ QCPtr kernarg_table() {
  const RDCT_CONST char* seg = (const RDCT_CONST char*)__builtin_amdgcn_kernarg_segment_ptr();
  return (QCPtr)(seg + offsetof(PlaneArgs, qc));
}

template <int SEL, int CO, bool RECON, int EV>
__global__ __launch_bounds__(256, 2) void k_plane(Plane P, QuantConsts /*qc*/) {
  plane_kernel_body<SEL, CO, RECON, EV>(P, kernarg_table());
}

template <int SEL, int CO, bool RECON, int EV>
__global__ __launch_bounds__(256, 1) void k_plane_w(Plane P, QuantConsts /*qc*/) {
  plane_kernel_body<SEL, CO, RECON, EV>(P, kernarg_table());
}

// Plain stores of one plane's error sums (the wave's lanes each hold a part;
// see flush_sums): every sum of the plane is written, so no clearing is needed.
template <int EV>
__device__ __forceinline__ void store_sums(const Plane& P, uint64_t part, int lane) {
  if constexpr (EV == EV_SPATIAL || EV == EV_COEF) {
    const uint64_t s = wave_sum_u64(part);
    if (lane == 0) *P.sse = s;
  } else if constexpr (EV == EV_SWEEP) {
    if (lane >= P.r && lane < P.r + P.r_count) P.sse[lane - P.r] = part;
    // r = 64 keeps every coefficient: no lane holds it and its sum is zero.
    if (lane == 0 && P.r + P.r_count > 64) P.sse[64 - P.r] = 0;
  }
}

// Batch kernel over a device work list, in one of two forms.
//  * Strided (first == nullptr): persistent workgroups; each wave takes items
//    wave_id, wave_id + n_waves, ...  and every wave runs to the end of the
//    list, so the grid drains without any device-side queue.  Error sums are
//    added with atomics (the caller clears them first).
//  * One workgroup per plane (first != nullptr; plane b's items are
//    first[b] .. first[b + 1] - 1): the workgroup's waves stride over the
//    plane's items, their sums meet in LDS, and one wave stores the plane's
//    totals -- no atomics and no clearing launch.  Suits batches of many
//    planes of similar size.
template <int SEL, int CO, bool RECON, int EV>
__device__ __forceinline__ void batch_kernel_body(const Plane* __restrict__ planes,
                                                  const QuantConsts* __restrict__ tables,
                                                  const WorkItem* __restrict__ items,
                                                  int n_items, const int* __restrict__ first,
                                                  int xcd, int strip) {
  extern __shared__ uint32_t lds[];
  const int wpg = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n_waves = gridDim.x * wpg;
  uint8_t* stage = reinterpret_cast<uint8_t*>(lds + (EV == EV_SWEEP ? wpg * 64 * 65 : 0)) +
                   wave * wave_stage_bytes<SEL, CO, RECON, EV>();
  uint32_t* sweep = lds + wave * (64 * 65);

  // Items it, it + stride, ... below end; part(plane, lane part) after each.
  auto run_items = [&](int it, int stride, int end, auto&& part) {
    if (it >= end) return;
    if constexpr (Prefetch<SEL, RECON, EV>::value) {
      WorkItem w = items[it];
      Pixels cur;
      chunk_load(planes[w.plane], w.t0, lane, cur);
      for (;;) {
        const int itn = it + stride;
        const bool more = itn < end;
        WorkItem wn = w;
        Pixels nxt;
        if (more) {
          wn = items[itn];
          chunk_load(planes[wn.plane], wn.t0, lane, nxt);
        }
        const Plane& P = planes[w.plane];
        part(w.plane, plane_chunk<SEL, CO, RECON, EV>(P, (QCPtr)(tables + P.table), cur, lane,
                                                      sweep, stage));
        if (!more) break;
        cur = nxt;
        w = wn;
        it = itn;
      }
    } else {
      for (; it < end; it += stride) {
        const WorkItem w = items[it];
        const Plane& P = planes[w.plane];
        Pixels cur;
        chunk_load(P, w.t0, lane, cur);
        part(w.plane, plane_chunk<SEL, CO, RECON, EV>(P, (QCPtr)(tables + P.table), cur, lane,
                                                      sweep, stage));
      }
    }
  };

  if (first != nullptr) {
    const int b = blockIdx.x;
    uint64_t acc = 0;
    run_items(first[b] + wave, wpg, first[b + 1], [&](int, uint64_t part) { acc += part; });
    if constexpr (EV != EV_NONE) {
      // After the stages: wpg x 64 lane parts.
      uint64_t* red = reinterpret_cast<uint64_t*>(
          lds + (EV == EV_SWEEP ? wpg * 64 * 65 : 0) + wpg * wave_stage_bytes<SEL, CO, RECON, EV>() / 4);
      red[wave * 64 + lane] = acc;
      __syncthreads();
      if (wave == 0) {
        uint64_t v = 0;
        for (int w = 0; w < wpg; ++w) v += red[w * 64 + lane];
        store_sums<EV>(planes[b], v, lane);
      }
    }
    return;
  }

  // Wave w takes the strip of `strip` consecutive items starting at item
  // w * strip, then strides by the grid's waves x strip.
  const int b = xcd ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int it = (b * wpg + wave) * strip;
  if (it >= n_items) return;
  // The wave's error parts accumulate while its items stay in one plane and are
  // written when the plane changes: a large plane gets one atomic per wave
  // rather than one per item, all on the same address.
  uint64_t acc = 0;
  int acc_plane = items[it].plane;
  auto add_part = [&](int plane, uint64_t part) {
    if constexpr (EV != EV_NONE) {
      if (plane != acc_plane) {
        flush_sums<EV>(planes[acc_plane], acc, lane);
        acc = 0;
        acc_plane = plane;
      }
      acc += part;
    }
  };
  if (strip == 1) {
    run_items(it, n_waves, n_items, add_part);
  } else {
    for (int s0 = it; s0 < n_items; s0 += n_waves * strip)
      run_items(s0, 1, min(s0 + strip, n_items), add_part);
  }
  if constexpr (EV != EV_NONE) flush_sums<EV>(planes[acc_plane], acc, lane);
}

template <int SEL, int CO, bool RECON, int EV>
__global__ __launch_bounds__(256, 2) void k_batch(const Plane* __restrict__ planes,
                                                  const QuantConsts* __restrict__ tables,
                                                  const WorkItem* __restrict__ items, int n_items,
                                                  const int* __restrict__ first, int xcd,
                                                  int strip) {
  batch_kernel_body<SEL, CO, RECON, EV>(planes, tables, items, n_items, first, xcd, strip);
}

template <int SEL, int CO, bool RECON, int EV>
__global__ __launch_bounds__(256, 1) void k_batch_w(const Plane* __restrict__ planes,
                                                    const QuantConsts* __restrict__ tables,
                                                    const WorkItem* __restrict__ items,
                                                    int n_items, const int* __restrict__ first,
                                                    int xcd, int strip) {
  batch_kernel_body<SEL, CO, RECON, EV>(planes, tables, items, n_items, first, xcd, strip);
}

// ---------------------------------------------------------------------------
// Inverse from coefficients: one block per lane, 64 consecutive blocks per
// wave.  For planes of whole blocks the rows leave through the wave's LDS
// stage, four at a time, as 1 KB contiguous pieces (see recon_flush_rows);
// lanes past the plane's end then recompute the wave's first block and are
// masked at the store.  Planes with partial blocks store clipped row pieces.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void k_inverse(const void* __restrict__ coef, Plane P,
                                                 QuantConsts qc) {
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int t0 = blockIdx.x * blockDim.x + wave * 64;
  if (t0 >= P.nblocks) return;  // the whole wave
  const int t = t0 + lane;
  const bool valid = t < P.nblocks;
  const int tb = valid ? t : t0;
  const int by = tb / P.nbx, bx = tb - by * P.nbx;
  const int x0 = bx * 8, y0 = by * 8;
  const bool stage = recon_stageable(P);
  uint8_t* stage_wave = reinterpret_cast<uint8_t*>(lds) + wave * kReconStageBytes;
  ReconFlush fl;
  if (stage) fl = recon_flush_setup(P, x0, y0, min(64, P.nblocks - t0), lane);
  auto emit = [&](int i, const float (&px)[8]) {
    if (stage) {
      recon_stage_row(stage_wave, i & 3, lane, px);
      if ((i & 3) == 3) {
        const int rows[4] = {i - 3, i - 2, i - 1, i};
        wave_sync();
        recon_flush_rows(P, stage_wave, fl, rows, lane);
        wave_sync();
      }
    } else if (valid) {
      store_row(P, x0, y0 + i, px);
    }
  };
  if constexpr (KIND == INV_INT_I32 || KIND == INV_INT_I16) {
    const uint64_t keep = P.keep;
    int w[8][8];
    if constexpr (KIND == INV_INT_I32) {
      const int4* p = reinterpret_cast<const int4*>(coef) + (int64_t)tb * 16;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int4 u = p[2 * k], s = p[2 * k + 1];
        w[k][0] = u.x; w[k][1] = u.y; w[k][2] = u.z; w[k][3] = u.w;
        w[k][4] = s.x; w[k][5] = s.y; w[k][6] = s.z; w[k][7] = s.w;
      }
    } else {
      const uint4* p = reinterpret_cast<const uint4*>(coef) + (int64_t)tb * 8;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint4 u = p[k];
        const uint32_t d[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          w[k][2 * m] = (int)(short)(d[m] & 0xffffu);
          w[k][2 * m + 1] = (int)(short)(d[m] >> 16);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int l = 0; l < 8; ++l)
        w[k][l] = ((keep >> (k * 8 + l)) & 1) ? w[k][l] * (kDp[k] * kDp[l]) : 0;
    pass2d<int, false>(w);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float px[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        px[j] = (float)__builtin_fma((double)w[i][j], 1.0 / 576.0, (double)P.shift);
      emit(i, px);
    }
  } else {
    double w[8][8];
    if constexpr (KIND == INV_F32) {
      const uint64_t keep = P.keep;
      const float4* p = reinterpret_cast<const float4*>(coef) + (int64_t)tb * 16;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float4 u = p[2 * k], s = p[2 * k + 1];
        const float z[8] = {u.x, u.y, u.z, u.w, s.x, s.y, s.z, s.w};
#pragma unroll
        for (int l = 0; l < 8; ++l)
          w[k][l] = ((keep >> (k * 8 + l)) & 1) ? (double)z[l] * scale_kl(k, l) : 0.0;
      }
    } else if constexpr (KIND == INV_Q_I32) {
      const int4* p = reinterpret_cast<const int4*>(coef) + (int64_t)tb * 16;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int4 u = p[2 * k], s = p[2 * k + 1];
        const int q[8] = {u.x, u.y, u.z, u.w, s.x, s.y, s.z, s.w};
#pragma unroll
        for (int l = 0; l < 8; ++l) w[k][l] = (double)q[l] * qc.dq[k * 8 + l];
      }
    } else {
      const uint4* p = reinterpret_cast<const uint4*>(coef) + (int64_t)tb * 8;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint4 u = p[k];
        const uint32_t d[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          w[k][2 * m] = (double)(int)(short)(d[m] & 0xffffu) * qc.dq[k * 8 + 2 * m];
          w[k][2 * m + 1] = (double)(int)(short)(d[m] >> 16) * qc.dq[k * 8 + 2 * m + 1];
        }
      }
    }
    pass2d<double, false>(w);
    const double sh = (double)P.shift;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float px[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) px[j] = (float)(w[i][j] + sh);
      emit(i, px);
    }
  }
}

__global__ void k_zero_u64(uint64_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
// Waves per CU that the single-plane kernels keep resident (two per SIMD).
constexpr int kPlaneWavesPerCU = 8;

template <int SEL, int CO, bool RECON, int EV>
static hipError_t launch_plane_t(const Plane& P, const QuantConsts& qc, int wpg, hipStream_t s) {
  const int n_cu = device_cu_count();
  const int chunks = half_chunks<EV>(P.nblocks) ? (P.nblocks + 63) / 64 : (P.nblocks + 127) / 128;
  int grid = (chunks + wpg - 1) / wpg;
  if constexpr (EV != EV_NONE) {
    const int cap = n_cu * kPlaneWavesPerCU / wpg;
    if (grid > cap) grid = cap;
  }
  const size_t lds = (EV == EV_SWEEP ? (size_t)wpg * 64 * 65 * 4 : 0) +
                     (size_t)wpg * wave_stage_bytes<SEL, CO, RECON, EV>();
  if constexpr (WideRegs<SEL, CO, RECON, EV>::value)
    hipLaunchKernelGGL((k_plane_w<SEL, CO, RECON, EV>), dim3(grid), dim3(64 * wpg), lds, s, P, qc);
  else
    hipLaunchKernelGGL((k_plane<SEL, CO, RECON, EV>), dim3(grid), dim3(64 * wpg), lds, s, P, qc);
  return hipGetLastError();
}

template <int SEL, int CO, bool RECON, int EV>
static hipError_t launch_batch_t(const Plane* planes, const QuantConsts* tables,
                                 const WorkItem* items, int n_items, const int* first,
                                 int grid, int wpg, int xcd, int strip, hipStream_t s) {
  static_assert(Stage<CO>::wave_bytes % 8 == 0 && kReconStageBytes % 8 == 0,
                "stages keep the per-plane sums area 8-byte aligned");
  const size_t lds = (EV == EV_SWEEP ? (size_t)wpg * 64 * 65 * 4 : 0) +
                     (size_t)wpg * wave_stage_bytes<SEL, CO, RECON, EV>() +
                     (first != nullptr && EV != EV_NONE ? (size_t)wpg * 64 * 8 : 0);
  if constexpr (WideRegs<SEL, CO, RECON, EV>::value)
    hipLaunchKernelGGL((k_batch_w<SEL, CO, RECON, EV>), dim3(grid), dim3(64 * wpg), lds, s, planes,
                       tables, items, n_items, first, xcd, strip);
  else
    hipLaunchKernelGGL((k_batch<SEL, CO, RECON, EV>), dim3(grid), dim3(64 * wpg), lds, s, planes,
                       tables, items, n_items, first, xcd, strip);
  return hipGetLastError();
}

// Dispatch table over the supported (selection, output, reconstruction, eval)
// combinations.
#define RDCT_DISPATCH(FN, ...)                                                           \
  switch (sel * 1000 + co * 100 + (recon ? 10 : 0) + ev) {                               \
    case SEL_ZZ * 1000 + CO_I32 * 100 + 0 + EV_NONE: return FN<SEL_ZZ, CO_I32, false, EV_NONE>(__VA_ARGS__); \
    case SEL_ZZ * 1000 + CO_I16 * 100 + 0 + EV_NONE: return FN<SEL_ZZ, CO_I16, false, EV_NONE>(__VA_ARGS__); \
    case SEL_ZZ * 1000 + CO_F32 * 100 + 0 + EV_NONE: return FN<SEL_ZZ, CO_F32, false, EV_NONE>(__VA_ARGS__); \
    case SEL_Q * 1000 + CO_I32 * 100 + 0 + EV_NONE: return FN<SEL_Q, CO_I32, false, EV_NONE>(__VA_ARGS__);   \
    case SEL_Q * 1000 + CO_I16 * 100 + 0 + EV_NONE: return FN<SEL_Q, CO_I16, false, EV_NONE>(__VA_ARGS__);   \
    RDCT_EVAL_CASES(FN, EV_SPATIAL, __VA_ARGS__)                                         \
    RDCT_EVAL_CASES(FN, EV_SWEEP, __VA_ARGS__)                                           \
    RDCT_QEVAL_CASES(FN, __VA_ARGS__)                                                    \
    default: return hipErrorInvalidValue;                                                \
  }
#define RDCT_EVAL_CASE(FN, CO, R, EV, ...) \
  case SEL_ZZ * 1000 + CO * 100 + (R ? 10 : 0) + EV: return FN<SEL_ZZ, CO, R, EV>(__VA_ARGS__);
#define RDCT_EVAL_CASES(FN, EV, ...)                                              \
  RDCT_EVAL_CASE(FN, CO_NONE, false, EV, __VA_ARGS__) RDCT_EVAL_CASE(FN, CO_NONE, true, EV, __VA_ARGS__) \
  RDCT_EVAL_CASE(FN, CO_I32, false, EV, __VA_ARGS__) RDCT_EVAL_CASE(FN, CO_I32, true, EV, __VA_ARGS__)   \
  RDCT_EVAL_CASE(FN, CO_I16, false, EV, __VA_ARGS__) RDCT_EVAL_CASE(FN, CO_I16, true, EV, __VA_ARGS__)   \
  RDCT_EVAL_CASE(FN, CO_F32, false, EV, __VA_ARGS__) RDCT_EVAL_CASE(FN, CO_F32, true, EV, __VA_ARGS__)
#define RDCT_QEVAL_CASE(FN, CO, R, ...) \
  case SEL_Q * 1000 + CO * 100 + (R ? 10 : 0) + EV_SPATIAL: return FN<SEL_Q, CO, R, EV_SPATIAL>(__VA_ARGS__);
#define RDCT_QEVAL_CASE2(FN, CO, R, EV, ...) \
  case SEL_Q * 1000 + CO * 100 + (R ? 10 : 0) + EV: return FN<SEL_Q, CO, R, EV>(__VA_ARGS__);
#define RDCT_QEVAL_CASES(FN, ...)                                                      \
  RDCT_QEVAL_CASE(FN, CO_NONE, false, __VA_ARGS__) RDCT_QEVAL_CASE(FN, CO_NONE, true, __VA_ARGS__) \
  RDCT_QEVAL_CASE(FN, CO_I32, false, __VA_ARGS__) RDCT_QEVAL_CASE(FN, CO_I32, true, __VA_ARGS__)   \
  RDCT_QEVAL_CASE(FN, CO_I16, false, __VA_ARGS__) RDCT_QEVAL_CASE(FN, CO_I16, true, __VA_ARGS__)   \
  RDCT_QEVAL_CASE2(FN, CO_NONE, false, EV_COEF, __VA_ARGS__)                                        \
  RDCT_QEVAL_CASE2(FN, CO_NONE, true, EV_COEF, __VA_ARGS__)                                         \
  RDCT_QEVAL_CASE2(FN, CO_I32, false, EV_COEF, __VA_ARGS__)                                         \
  RDCT_QEVAL_CASE2(FN, CO_I32, true, EV_COEF, __VA_ARGS__)                                          \
  RDCT_QEVAL_CASE2(FN, CO_I16, false, EV_COEF, __VA_ARGS__)                                         \
  RDCT_QEVAL_CASE2(FN, CO_I16, true, EV_COEF, __VA_ARGS__)

hipError_t launch_plane(int sel, int co, bool recon, int ev, const Plane& P,
                        const QuantConsts& qc, int wpg, hipStream_t s) {
  if (P.nblocks <= 0) return hipSuccess;
  RDCT_DISPATCH(launch_plane_t, P, qc, wpg, s)
}

hipError_t launch_batch(int sel, int co, bool recon, int ev, const Plane* planes,
                        const QuantConsts* tables, const WorkItem* items,
                        int32_t n_items, int32_t grid, int32_t wpg, hipStream_t s,
                        const int32_t* first, int xcd, int strip) {
  if (n_items <= 0) return hipSuccess;
  if (strip < 1) strip = 1;
  RDCT_DISPATCH(launch_batch_t, planes, tables, items, n_items, first, grid, wpg, xcd, strip, s)
}

hipError_t launch_inverse(int kind, const void* coef, int32_t width, int32_t height, int32_t r,
                          int32_t shift, float* dst, int64_t dpitch, const QuantConsts& qc,
                          hipStream_t s) {
  Plane P{};
  P.width = width;
  P.height = height;
  P.nbx = (width + 7) / 8;
  P.nby = (height + 7) / 8;
  P.nblocks = P.nbx * P.nby;
  P.recon = dst;
  P.rpitch = dpitch;
  P.r = r;
  P.keep = keep_bits(r);
  P.shift = shift;
  if (P.nblocks <= 0) return hipSuccess;
  const dim3 grid((P.nblocks + 255) / 256), block(256);
  const size_t lds = 4 * (size_t)kReconStageBytes;  // one stage per wave
  switch (kind) {
    case INV_INT_I32: hipLaunchKernelGGL(k_inverse<INV_INT_I32>, grid, block, lds, s, coef, P, qc); break;
    case INV_INT_I16: hipLaunchKernelGGL(k_inverse<INV_INT_I16>, grid, block, lds, s, coef, P, qc); break;
    case INV_F32: hipLaunchKernelGGL(k_inverse<INV_F32>, grid, block, lds, s, coef, P, qc); break;
    case INV_Q_I32: hipLaunchKernelGGL(k_inverse<INV_Q_I32>, grid, block, lds, s, coef, P, qc); break;
    case INV_Q_I16: hipLaunchKernelGGL(k_inverse<INV_Q_I16>, grid, block, lds, s, coef, P, qc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace rdct
