// Keep-r sweep with image-quality metrics for any 8x8 transform (the comparison
// of Section 3: the approximation against the exact DCT and the signed DCT,
// scored by SSE and by the universal quality index, UQI).
//
// A workgroup owns a tile of 32 x 32 window positions (8x8 windows at stride 1);
// the windows reach 7 pixels further, so the tile transforms the 5 x 5 blocks
// covering 40 x 40 pixels.  For r = 1, 2, ... it forms coefficient (k, l) of
// zig-zag rank r - 1 of every block (Y = F A F^T, eight lanes per block) and
// adds its basis image, scaled by that coefficient, to the reconstruction it
// keeps in LDS -- the keep-r reconstruction is linear in the kept
// coefficients -- and, for the requested r, scores:
//   UQI  over its 32 x 32 windows, from separable box sums: one thread per
//        (pixel row, 8 window columns) slides an 8-pixel window along the row
//        and stores the row sums of y, y^2 and x y in LDS; then one thread per
//        (window column, 4 window rows) sums 8 of those down the column;
//   SSE  over the 32 x 32 pixels the tile owns (its 4 x 4 blocks), as
//        D^2 x^2 - 2 D x y + y^2 summed, from the row sums of the owned rows'
//        8-pixel segments at window columns 0, 8, 16 and 24.
// For the round-off and signed transforms the reconstruction is kept as an
// integer numerator (A' = numerator / D) and every window or error sum is an
// exact integer in float64.  No MFMA: per r the work is a rank-1 update and
// sliding sums, not a dense contraction.
#include "rdct_internal.h"
#include "rdct_tables.h"

namespace rdct {

#define RDCT_CONST __attribute__((address_space(4)))

constexpr int kWinRows = 32, kWinCols = 32;             // windows per tile
constexpr int kPixRows = kWinRows + 8, kPixCols = kWinCols + 8;  // 40 x 40
constexpr int kBlkRows = kPixRows / 8, kBlkCols = kPixCols / 8;  // 5 x 5
constexpr int kTileBlocks = kBlkRows * kBlkCols;        // 25
constexpr int kThreads = 256;
// Row strides (elements): odd numbers of doubles put consecutive rows on
// different LDS banks.
constexpr int kYStride = kPixCols + 1;                  // 41
constexpr int kHStride = kWinCols + 1;                  // 33
constexpr int kSeg = 8;                                 // window columns per row task
constexpr int kRowTasks = kPixRows * (kWinCols / kSeg); // 160
constexpr int kColGroups = kThreads / kWinCols;         // 8
constexpr int kWinPerThread = kWinRows / kColGroups;    // 4 window rows per thread
constexpr int kSumRows = kWinPerThread + 7;             // 11 row sums per thread
static_assert(kTileBlocks * 8 <= kThreads, "eight lanes per block");
static_assert(kRowTasks <= kThreads, "one row task per thread");

__constant__ ZigZag c_zz_quality = make_zigzag();

struct QualityKArgs1 {
  QPlane P;
  QualityArgs A;
};
struct QualityKArgsN {
  const QPlane* planes;
  const QTile* tiles;
  int32_t n_tiles;
  QualityArgs A;
};

template <typename KA>
__device__ __forceinline__ const RDCT_CONST QualityArgs* quality_args() {
  const RDCT_CONST char* seg = (const RDCT_CONST char*)__builtin_amdgcn_kernarg_segment_ptr();
  return (const RDCT_CONST QualityArgs*)(seg + offsetof(KA, A));
}

// A float64 moved between lanes by a DPP control (two 32-bit halves); lanes the
// control does not write, or whose source is out of range, get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, true);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the wave, complete in lane 63: shifts by 1, 2, 4, 8 within each row
// of 16 lanes leave every row's total in its lane 15; row 15's lane then adds
// into rows 1 and 3, and lane 31 into rows 2 and 3.  No LDS round trips.
__device__ __forceinline__ double wave_sum_to_63(double v) {
  v += dpp_f64<0x111, 0xf>(v);   // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);   // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);   // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);   // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
  return v;
}

// Sum over each aligned group of 8 lanes, in all 8: pairs and quads by quad
// permutations, then the two quads of the group by the half-row mirror.
__device__ __forceinline__ double block_sum8(double v) {
  v += dpp_f64<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141, 0xf>(v);   // row_half_mirror
  return v;
}

// num / den for den > 0 in the range of window terms: reciprocal estimate, two
// Newton steps and a residual correction (within an ulp of the rounded quotient).
__device__ __forceinline__ double quotient(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = __builtin_fma(r, __builtin_fma(-den, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-den, r, 1.0), r);
  const double q = num * r;
  return __builtin_fma(__builtin_fma(-den, q, num), r, q);
}

// n_m / d_m for four windows (d_m > 0, their product far from overflow) with
// one reciprocal: that of the product, refined by two Newton steps, times the
// other three denominators (a few roundings each, ~1e-15 relative).
__device__ __forceinline__ double quotient_sum4(const double (&n)[4], const double (&d)[4]) {
  const double d01 = d[0] * d[1], d23 = d[2] * d[3];
  const double p = d01 * d23;
  double r = __builtin_amdgcn_rcp(p);
  r = __builtin_fma(r, __builtin_fma(-p, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-p, r, 1.0), r);
  const double r01 = r * d23, r23 = r * d01;   // 1 / (d0 d1), 1 / (d2 d3)
  return (n[0] * d[1] + n[1] * d[0]) * r01 + (n[2] * d[3] + n[3] * d[2]) * r23;
}

// Terms of one window's index that depend on the original pixels only
// (sx = sum x, sxx = sum x^2 over the window; N = 64; D the numerator scale).
struct WinX {
  double vx;     // N^2 var_x
  double dvx;    // D^2 N^2 var_x
  double dsx2;   // 2 D sx
  double dsxx;   // D^2 sx^2
};

__device__ __forceinline__ WinX window_x(double sx, double sxx, double d) {
  WinX w;
  w.vx = __builtin_fma(64.0, sxx, -sx * sx);
  w.dvx = d * d * w.vx;
  w.dsx2 = 2.0 * d * sx;
  w.dsxx = d * d * sx * sx;
  return w;
}

// Q of one window from its sums (numerators of y = numerator / D; N = 64):
// Q = [2 cov / (var_x + var_y)] [2 mx my / (mx^2 + my^2)], each factor 1 when
// its denominator is 0.  Float64 noise must not decide the index: a constant
// block keeps only its DC term and is exact in real arithmetic, but the float64
// transforms leave ~1e-13 of noise in it.  So, in grey levels, a
// reconstruction window with variance <= 2^-32 counts as flat (no variance, no
// covariance), a window mean of magnitude <= 2^-32 counts as 0, and a flat
// pixel window has no covariance.  With integer numerators every quantity here
// is an exact integer and the rules are decided exactly.  The two factors
// share one division.
__device__ __forceinline__ double window_uqi(const WinX& w, double sx, double sy, double syy,
                                             double sxy, double d) {
  constexpr double N = 64.0, EPS = 0x1p-32;
  const double vy_raw = __builtin_fma(N, syy, -sy * sy);              // N^2 D^2 var_y
  const bool flat_y = vy_raw <= (N * N) * (d * d) * EPS;
  const double vy = flat_y ? 0.0 : vy_raw;
  const double cov = (w.vx == 0.0 || flat_y) ? 0.0 : __builtin_fma(N, sxy, -sx * sy);
  const double sym = __builtin_fabs(sy) <= N * d * EPS ? 0.0 : sy;
  const double ds = w.dvx + vy;                                       // D^2 N^2 (var_x + var_y)
  const double dm = __builtin_fma(sym, sym, w.dsxx);                  // N^2 D^2 (mx^2 + my^2)
  const bool zs = ds == 0.0, zm = dm == 0.0;
  const double ns = zs ? 1.0 : 2.0 * d * cov;
  const double nm = zm ? 1.0 : w.dsx2 * sym;
  return quotient(ns * nm, (zs ? 1.0 : ds) * (zm ? 1.0 : dm));
}

// Byte u of pixels packed four to a word.
__device__ __forceinline__ int packed_pixel(const uint32_t* w, int u) {
  return (int)((w[u >> 2] >> (8 * (u & 3))) & 0xffu);
}

__device__ void quality_tile(const QPlane& P, int tile, const RDCT_CONST QualityArgs* A) {
  __shared__ double s_y[kPixRows][kYStride];
  __shared__ double s_h[3][kPixRows][kHStride];     // row sums of y, y^2, x y
  __shared__ double s_F[64], s_G[64];
  __shared__ double s_red[2][2][kThreads / 64];    // (UQI, SSE) x (r & 1) x wave
  // The tile's pixels are staged only until every thread holds its own in
  // registers; they share storage with the row sums, first written later.
  static_assert(sizeof(s_h[1]) >= kPixRows * kPixCols, "pixel stage fits");
  uint8_t* s_x8 = reinterpret_cast<uint8_t*>(&s_h[1][0][0]);
  auto xat = [&](int row, int col) { return (double)s_x8[row * kPixCols + col]; };

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int ty = tile / P.tiles_x, tx = tile - ty * P.tiles_x;
  const int y0 = ty * kWinRows, x0 = tx * kWinCols;   // tile origin in pixels
  const int by0 = y0 / 8, bx0 = x0 / 8;
  const int nby = P.height / 8, nbx = P.width / 8;
  const double D = A->T.D;
  const bool exact = A->T.exact != 0;

  // Pixels (0 outside the plane: no valid window or owned pixel reads them),
  // tables, and a zero reconstruction.
  for (int p = t; p < kPixRows * kPixCols; p += kThreads) {
    const int row = p / kPixCols, col = p - row * kPixCols;
    const int gy = y0 + row, gx = x0 + col;
    uint8_t v = 0;
    if (gy < P.height && gx < P.width) v = P.src[(int64_t)gy * P.pitch + gx];
    s_x8[p] = v;
    s_y[row][col] = 0.0;
  }
  if (t < 64) s_F[t] = A->T.F[t];
  else if (t < 128) s_G[t - 64] = A->T.G[t - 64];
  __syncthreads();

  // Thread (block ub, index ui): the eight lanes of a block hold its pixel
  // columns; coefficient (k, l) of Y_b = F A_b F^T is formed when it is needed,
  // as sum_n (sum_m F[k][m] A[m][n]) F[l][n], lane n taking column n.
  const int ub = t >> 3, ui = t & 7;
  const int ubr = ub / kBlkCols, ubc = ub - ubr * kBlkCols;
  const bool u_on = ub < kTileBlocks && by0 + ubr < nby && bx0 + ubc < nbx;
  double xcol[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) xcol[m] = u_on ? xat(ubr * 8 + m, ubc * 8 + ui) : 0.0;

  // This thread's windows: column c, rows 4 g .. 4 g + 3.  Their sums of x and
  // x^2 (exact integers) and the terms built from them.
  const int c = t & (kWinCols - 1), g = t / kWinCols;
  WinX wx[kWinPerThread];
  double sxw[kWinPerThread], kq[kWinPerThread];
  bool w_ok[kWinPerThread], x_special[kWinPerThread];
  // D^2 x^2 over the thread's owned pixels if c is a multiple of 8: rows
  // 4 g .. 4 g + 3, columns c .. c + 7 (0 off the plane); these segments cover
  // the tile's 32 x 32 owned pixels once.
  double own_x2v = 0.0;
  {
    double hx[kSumRows], hxx[kSumRows];
#pragma unroll
    for (int rr = 0; rr < kSumRows; ++rr) {
      double a = 0.0, a2 = 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double xv = xat(kWinPerThread * g + rr, c + u);
        a += xv;
        a2 = __builtin_fma(xv, xv, a2);
      }
      hx[rr] = a;
      hxx[rr] = a2;
    }
    const bool col_ok = x0 + c + 8 <= P.width;
#pragma unroll
    for (int m = 0; m < kWinPerThread; ++m) {
      double a = 0.0, a2 = 0.0;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        a += hx[m + rr];
        a2 += hxx[m + rr];
      }
      sxw[m] = a;
      if (m == 0 && (c & 7) == 0) own_x2v = D * D * (hxx[0] + hxx[1] + hxx[2] + hxx[3]);
      wx[m] = window_x(a, a2, D);
      w_ok[m] = col_ok && (y0 + kWinPerThread * g + m + 8 <= P.height);
      x_special[m] = wx[m].vx == 0.0 || a == 0.0;
      kq[m] = w_ok[m] ? 2.0 * D * wx[m].dsx2 : 0.0;   // 4 D^2 sx, 0 off the plane
    }
  }
  // Thresholds of the flat and zero-mean rules in numerator units.
  const double flat_lim = (64.0 * 64.0) * (D * D) * 0x1p-32, mean_lim = 64.0 * D * 0x1p-32;
  // Row task: pixel row hr, window columns 8 hs .. 8 hs + 7; its 15 pixels
  // (rows 0 .. 38 feed windows).
  const int hr = t % kPixRows, hs = t / kPixRows;
  const bool row_task = t < kRowTasks && hr < kWinRows + 7;
  uint32_t xr[4] = {0u, 0u, 0u, 0u};
  if (row_task) {
#pragma unroll
    for (int u = 0; u < kSeg + 7; ++u)
      xr[u >> 2] |= (uint32_t)xat(hr, kSeg * hs + u) << (8 * (u & 3));
  }
  __syncthreads();   // the pixel stage is reused from here on

  const int r_first = A->r_first, r_last = A->r_first + A->r_count - 1;
  // Add coefficient (k, l) of rank r - 1 of every block times its basis image
  // G[:, k] G[:, l]^T.
  auto add_basis = [&](int r) {
    if (!u_on) return;
    const int kl = c_zz_quality.order[r - 1];
    const int k = kl >> 3, l = kl & 7;
    double u = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) u = __builtin_fma(A->T.F[k * 8 + m], xcol[m], u);
    const double coef = block_sum8(u * s_F[l * 8 + ui]);
    const double ci = coef * s_G[ui * 8 + k];
    double* row = &s_y[ubr * 8 + ui][ubc * 8];
#pragma unroll
    for (int j = 0; j < 8; ++j) row[j] = __builtin_fma(ci, A->T.G[j * 8 + l], row[j]);
  };
  // The tile's sums for r (the waves' totals, in LDS slot r & 1) to the outputs.
  auto flush = [&](int r) {
    double q = 0.0, e = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      q += s_red[0][r & 1][w];
      e += s_red[1][r & 1][w];
    }
    const int o = r - r_first;
    atomicAdd(reinterpret_cast<unsigned long long*>(P.uqi + o),
              (unsigned long long)(long long)__builtin_rint(q * 4294967296.0));
    // Exact families: e is an integer below 2^53; otherwise 2^-20 units.
    const double eu = exact ? e : __builtin_rint(e * 1048576.0);
    atomicAdd(reinterpret_cast<unsigned long long*>(P.sse + o), (unsigned long long)eu);
  };

  // Two barriers per r: row sums of r | window sums and SSE of r, and the
  // basis update for r + 1 (which only the next row sums read).
  add_basis(1);
  __syncthreads();
  for (int r = 1; r <= r_last; ++r) {
    const bool scored = r >= r_first;
    if (scored) {
      // Row sums over 8 pixels, sliding along the row.
      if (row_task) {
        // The empty asm keeps the pixels packed across iterations of r.
#pragma unroll
        for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(xr[i]));
        const double* yr = &s_y[hr][kSeg * hs];
        double yv[kSeg + 7], xv[kSeg + 7];
#pragma unroll
        for (int u = 0; u < kSeg + 7; ++u) {
          yv[u] = yr[u];
          xv[u] = (double)packed_pixel(xr, u);
        }
        double a = 0.0, a2 = 0.0, ax = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a += yv[u];
          a2 = __builtin_fma(yv[u], yv[u], a2);
          ax = __builtin_fma(xv[u], yv[u], ax);
        }
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
          if (j > 0) {
            a += yv[j + 7] - yv[j - 1];
            a2 = __builtin_fma(-yv[j - 1], yv[j - 1], __builtin_fma(yv[j + 7], yv[j + 7], a2));
            ax = __builtin_fma(-xv[j - 1], yv[j - 1], __builtin_fma(xv[j + 7], yv[j + 7], ax));
          }
          s_h[0][hr][kSeg * hs + j] = a;
          s_h[1][hr][kSeg * hs + j] = a2;
          s_h[2][hr][kSeg * hs + j] = ax;
        }
      }
    }
    if (t == 0 && r - 1 >= r_first) flush(r - 1);
    __syncthreads();

    if (scored) {
      // Window sums down the column, and the index of each window.
      double hy[kSumRows], hyy[kSumRows], hxy[kSumRows];
#pragma unroll
      for (int rr = 0; rr < kSumRows; ++rr) {
        hy[rr] = s_h[0][kWinPerThread * g + rr][c];
        hyy[rr] = s_h[1][kWinPerThread * g + rr][c];
        hxy[rr] = s_h[2][kWinPerThread * g + rr][c];
      }
      // Squared error of the owned pixels, sum of (D x - y)^2 = D^2 x^2 -
      // 2 D x y + y^2, from the row sums of the 8-pixel segments at columns 0,
      // 8, 16, 24 of the owned rows (pixels off the plane have x = y = 0).
      {
        const double oyy = (hyy[0] + hyy[1]) + (hyy[2] + hyy[3]);
        const double oxy = (hxy[0] + hxy[1]) + (hxy[2] + hxy[3]);
        double e_acc = (c & 7) == 0 ? __builtin_fma(-2.0 * D, oxy, oyy) + own_x2v : 0.0;
        e_acc = wave_sum_to_63(e_acc);
        if (lane == 63) s_red[1][r & 1][wave] = e_acc;
      }
      double sy = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        sy += hy[rr];
        syy += hyy[rr];
        sxy += hxy[rr];
      }
      double wy[kWinPerThread], wyy[kWinPerThread], wxy[kWinPerThread];
      bool special = false;
#pragma unroll
      for (int m = 0; m < kWinPerThread; ++m) {
        if (m > 0) {
          sy += hy[m + 7] - hy[m - 1];
          syy += hyy[m + 7] - hyy[m - 1];
          sxy += hxy[m + 7] - hxy[m - 1];
        }
        wy[m] = sy;
        wyy[m] = syy;
        wxy[m] = sxy;
        // Windows that need one of the rules of window_uqi: a flat or zero-mean
        // reconstruction, or a flat or zero pixel window.
        special |= (__builtin_fma(64.0, syy, -sy * sy) <= flat_lim) |
                   (__builtin_fabs(sy) <= mean_lim) | x_special[m];
      }
      double q_acc = 0.0;
      if (__ballot(special) == 0) {
        // No rule applies anywhere in the wave: both factors have nonzero
        // denominators, Q = 4 D^2 sx cov sy / ((D^2 vx + vy)(sy^2 + D^2 sx^2)).
        double num[kWinPerThread], den[kWinPerThread];
#pragma unroll
        for (int m = 0; m < kWinPerThread; ++m) {
          const double vy = __builtin_fma(64.0, wyy[m], -wy[m] * wy[m]);
          const double cov = __builtin_fma(64.0, wxy[m], -sxw[m] * wy[m]);
          den[m] = (wx[m].dvx + vy) * __builtin_fma(wy[m], wy[m], wx[m].dsxx);
          num[m] = kq[m] * cov * wy[m];
        }
        q_acc = quotient_sum4(num, den);
      } else {
#pragma unroll
        for (int m = 0; m < kWinPerThread; ++m) {
          const double q = window_uqi(wx[m], sxw[m], wy[m], wyy[m], wxy[m], D);
          q_acc += w_ok[m] ? q : 0.0;
        }
      }
      q_acc = wave_sum_to_63(q_acc);
      if (lane == 63) s_red[0][r & 1][wave] = q_acc;
    }
    if (r < r_last) add_basis(r + 1);
    __syncthreads();
  }
  if (t == 0) flush(r_last);
}

// ---------------------------------------------------------------------------
// Integer form, for transforms with integer tables (the round-off and signed
// transforms; TransformTables::int_form).  Same tile, phases and barriers as
// above, but the reconstruction numerators and their 8-pixel row sums are
// int32, each coefficient comes from 24-bit multiplies and 32-bit lane sums,
// and only what leaves 32 bits (squares, products with x, errors) is float64:
// every quantity is still exact.  With 32-bit numerators and row sums a
// workgroup holds about 33 KB of LDS (the float64 form 46 KB), so four
// workgroups share a CU.
// ---------------------------------------------------------------------------
constexpr int kSumPixRows = kWinRows + 7;                    // 39 rows feed windows
constexpr int kRowTasksI = kSumPixRows * (kWinCols / kSeg);  // 156
static_assert(kRowTasksI <= kThreads, "one row task per thread");

// Sum over each aligned group of 8 lanes, in all 8 (32-bit lanes).
__device__ __forceinline__ int block_sum8_i32(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, true);   // quad_perm [1, 0, 3, 2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, true);   // quad_perm [2, 3, 0, 1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, true);  // row_half_mirror
  return v;
}


__device__ void quality_tile_int(const QPlane& P, int tile, const RDCT_CONST QualityArgs* A) {
  __shared__ int32_t s_y[kPixRows][kYStride];        // reconstruction numerators
  __shared__ int32_t s_h0[kSumPixRows][kHStride];    // row sums of y
  __shared__ double s_h1[kSumPixRows][kHStride];     // row sums of y^2
  __shared__ double s_h2[kSumPixRows][kHStride];     // row sums of x y
  __shared__ int8_t s_F[64], s_G[64];
  __shared__ double s_red[2][2][kThreads / 64];     // (UQI, SSE) x (r & 1) x wave
  // The tile's pixels are staged only until every thread holds its own in
  // registers; they share storage with the y^2 row sums, first written later.
  static_assert(sizeof(s_h1) >= kPixRows * kPixCols, "pixel stage fits");
  uint8_t* s_x = reinterpret_cast<uint8_t*>(&s_h1[0][0]);

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int ty = tile / P.tiles_x, tx = tile - ty * P.tiles_x;
  const int y0 = ty * kWinRows, x0 = tx * kWinCols;   // tile origin in pixels
  const int by0 = y0 / 8, bx0 = x0 / 8;
  const int nby = P.height / 8, nbx = P.width / 8;
  const int Di = A->T.Di;
  const double D = (double)Di;

  // Pixels (0 outside the plane: no valid window or owned pixel reads them),
  // integer tables, and a zero reconstruction.
  for (int p = t; p < kPixRows * kPixCols; p += kThreads) {
    const int row = p / kPixCols, col = p - row * kPixCols;
    const int gy = y0 + row, gx = x0 + col;
    uint8_t v = 0;
    if (gy < P.height && gx < P.width) v = P.src[(int64_t)gy * P.pitch + gx];
    s_x[p] = v;
    s_y[row][col] = 0;
  }
  if (t < 64) s_F[t] = A->T.Fi[t];
  else if (t < 128) s_G[t - 64] = A->T.Gi[t - 64];
  __syncthreads();
  auto xat = [&](int row, int col) { return (int)s_x[row * kPixCols + col]; };

  // Thread (block ub, index ui): the eight lanes of a block hold its pixel
  // columns (see quality_tile).
  const int ub = t >> 3, ui = t & 7;
  const int ubr = ub / kBlkCols, ubc = ub - ubr * kBlkCols;
  const bool u_on = ub < kTileBlocks && by0 + ubr < nby && bx0 + ubc < nbx;
  uint32_t xcol[2] = {0u, 0u};   // the column's 8 pixels, packed
  if (u_on) {
#pragma unroll
    for (int m = 0; m < 8; ++m) xcol[m >> 2] |= (uint32_t)xat(ubr * 8 + m, ubc * 8 + ui) << (8 * (m & 3));
  }

  // This thread's windows: column c, rows 4 g .. 4 g + 3; their sums of x and
  // x^2 (integers below 2^23).
  const int c = t & (kWinCols - 1), g = t / kWinCols;
  int sxw[kWinPerThread], sxxw[kWinPerThread];
  double dvx[kWinPerThread], dsxx[kWinPerThread];   // D^2 N^2 var_x, D^2 sx^2
  bool w_ok[kWinPerThread], x_special[kWinPerThread];
  // D^2 x^2 over the thread's owned pixels if c is a multiple of 8: rows
  // 4 g .. 4 g + 3, columns c .. c + 7 (0 off the plane); these segments cover
  // the tile's 32 x 32 owned pixels once.
  double own_x2 = 0.0;
  {
    int hx[kSumRows], hxx[kSumRows];
#pragma unroll
    for (int rr = 0; rr < kSumRows; ++rr) {
      int a = 0, a2 = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int xv = xat(kWinPerThread * g + rr, c + u);
        a += xv;
        a2 += __mul24(xv, xv);
      }
      hx[rr] = a;
      hxx[rr] = a2;
    }
    const bool col_ok = x0 + c + 8 <= P.width;
#pragma unroll
    for (int m = 0; m < kWinPerThread; ++m) {
      int a = 0, a2 = 0;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        a += hx[m + rr];
        a2 += hxx[m + rr];
      }
      sxw[m] = a;
      sxxw[m] = a2;
      dvx[m] = D * D * (double)(__mul24(64, a2) - __mul24(a, a));
      dsxx[m] = D * D * (double)a * (double)a;
      if (m == 0 && (c & 7) == 0)
        own_x2 = D * D * (double)(hxx[0] + hxx[1] + hxx[2] + hxx[3]);
      w_ok[m] = col_ok && (y0 + kWinPerThread * g + m + 8 <= P.height);
      x_special[m] = __mul24(64, a2) == __mul24(a, a) || a == 0;   // both below 2^29
    }
  }
  const double flat_lim = (64.0 * 64.0) * (D * D) * 0x1p-32, mean_lim = 64.0 * D * 0x1p-32;
  // Row task: pixel row hr, window columns 8 hs .. 8 hs + 7; its 15 pixels.
  const int hr = t % kSumPixRows, hs = t / kSumPixRows;
  uint32_t xr[4] = {0u, 0u, 0u, 0u};
  if (t < kRowTasksI) {
#pragma unroll
    for (int u = 0; u < kSeg + 7; ++u)
      xr[u >> 2] |= (uint32_t)xat(hr, kSeg * hs + u) << (8 * (u & 3));
  }
  __syncthreads();   // the pixel stage is reused from here on

  const int r_first = A->r_first, r_last = A->r_first + A->r_count - 1;
  // Add coefficient (k, l) of rank r - 1 of every block times its basis image
  // G[:, k] G[:, l]^T, in numerator units.
  auto add_basis = [&](int r) {
    if (!u_on) return;
    const int kl = c_zz_quality.order[r - 1];
    const int k = kl >> 3, l = kl & 7;
    int u = 0;
    // Table entries fit 8 bits and every product operand 24 bits (checked on
    // the host); the explicit sign extensions tell the compiler so, which keeps
    // it on 24-bit multiplies (a full 32-bit multiply issues at a quarter of
    // the rate).
    auto i8 = [](int v) { return __builtin_amdgcn_sbfe(v, 0, 8); };
    auto i24 = [](int v) { return __builtin_amdgcn_sbfe(v, 0, 24); };
#pragma unroll
    for (int m = 0; m < 8; ++m) u = __mul24(i8(A->T.Fi[k * 8 + m]), packed_pixel(xcol, m)) + u;
    const int coef = block_sum8_i32(__mul24(i24(u), (int)s_F[l * 8 + ui]));
    const int ci = __mul24(i24(coef), (int)s_G[ui * 8 + k]);
    int* row = &s_y[ubr * 8 + ui][ubc * 8];
#pragma unroll
    for (int j = 0; j < 8; ++j) row[j] = __mul24(i24(ci), i8(A->T.Gi[j * 8 + l])) + row[j];
  };
  auto flush = [&](int r) {
    double q = 0.0, e = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      q += s_red[0][r & 1][w];
      e += s_red[1][r & 1][w];
    }
    const int o = r - r_first;
    atomicAdd(reinterpret_cast<unsigned long long*>(P.uqi + o),
              (unsigned long long)(long long)__builtin_rint(q * 4294967296.0));
    atomicAdd(reinterpret_cast<unsigned long long*>(P.sse + o), (unsigned long long)e);
  };

  add_basis(1);
  __syncthreads();
  for (int r = 1; r <= r_last; ++r) {
    const bool scored = r >= r_first;
    if (scored) {
      if (t < kRowTasksI) {
        // One sliding sum at a time, so that only one row of operands is live.
        // The empty asm keeps the pixels packed across iterations of r (hoisted
        // out of the loop, their 15 float64 conversions would hold 30 VGPRs).
#pragma unroll
        for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(xr[i]));
        const int32_t* yr = &s_y[hr][kSeg * hs];
        int yv[kSeg + 7];
#pragma unroll
        for (int u = 0; u < kSeg + 7; ++u) yv[u] = yr[u];
        int a = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) a += yv[u];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
          if (j > 0) a += yv[j + 7] - yv[j - 1];
          s_h0[hr][kSeg * hs + j] = a;
        }
        double v[kSeg + 7];   // y^2, then x y (exact: below 2^53)
#pragma unroll
        for (int u = 0; u < kSeg + 7; ++u) v[u] = (double)yv[u] * (double)yv[u];
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
          if (j > 0) s += v[j + 7] - v[j - 1];
          s_h1[hr][kSeg * hs + j] = s;
        }
#pragma unroll
        for (int u = 0; u < kSeg + 7; ++u) v[u] = (double)packed_pixel(xr, u) * (double)yv[u];
        s = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
          if (j > 0) s += v[j + 7] - v[j - 1];
          s_h2[hr][kSeg * hs + j] = s;
        }
      }
    }
    if (t == 0 && r - 1 >= r_first) flush(r - 1);
    __syncthreads();

    if (scored) {
      // Window m sums rows m .. m + 7 of the thread's 11; rows 3 .. 7 are
      // common to all four, the others enter one by one.
      const int rb = kWinPerThread * g;
      // Rows 0 .. 3 of the 11 are also the thread's owned pixel rows (their
      // sum is returned: the error of the 8 owned pixels at column c, for c a
      // multiple of 8).
      auto windows = [&](auto at, auto (&w)[kWinPerThread]) {
        const auto h3 = at(rb + 3);
        auto rest = at(rb + 4);
#pragma unroll
        for (int rr = 5; rr < 8; ++rr) rest += at(rb + rr);
        const auto h0 = at(rb), h1 = at(rb + 1), h2 = at(rb + 2);
        const auto h8 = at(rb + 8), h9 = at(rb + 9), h10 = at(rb + 10);
        const auto core = h3 + rest, head = h0 + (h1 + h2);
        w[0] = core + head;
        w[1] = core + ((h1 + h2) + h8);
        w[2] = core + ((h2 + h8) + h9);
        w[3] = core + ((h8 + h9) + h10);
        return head + h3;
      };
      // As for the pixels: the window sums of x are converted where they are
      // used rather than held in float64 across iterations (the two terms
      // that cost most to rebuild are held).
#pragma unroll
      for (int m = 0; m < kWinPerThread; ++m) asm volatile("" : "+v"(sxw[m]), "+v"(sxxw[m]));
      int iy[kWinPerThread];
      double wy[kWinPerThread], wyy[kWinPerThread], wxy[kWinPerThread];
      windows([&](int row) { return s_h0[row][c]; }, iy);
      const double own_yy = windows([&](int row) { return s_h1[row][c]; }, wyy);
      const double own_xy = windows([&](int row) { return s_h2[row][c]; }, wxy);
      // Squared error of the owned pixels, sum of (D x - y)^2 = D^2 x^2 -
      // 2 D x y + y^2, from the row sums of the 8-pixel segments at columns 0,
      // 8, 16, 24 of the owned rows (pixels off the plane have x = y = 0).
      double e_acc = (c & 7) == 0 ? __builtin_fma(-2.0 * D, own_xy, own_yy) + own_x2 : 0.0;
      e_acc = wave_sum_to_63(e_acc);
      if (lane == 63) s_red[1][r & 1][wave] = e_acc;
      bool special = false;
#pragma unroll
      for (int m = 0; m < kWinPerThread; ++m) {
        wy[m] = (double)iy[m];
        special |= (__builtin_fma(64.0, wyy[m], -wy[m] * wy[m]) <= flat_lim) |
                   (__builtin_fabs(wy[m]) <= mean_lim) | x_special[m];
      }
      double q_acc = 0.0;
      if (__ballot(special) == 0) {
        double num[kWinPerThread], den[kWinPerThread];
#pragma unroll
        for (int m = 0; m < kWinPerThread; ++m) {
          const double sx = (double)sxw[m];
          const double vy = __builtin_fma(64.0, wyy[m], -wy[m] * wy[m]);
          const double cov = __builtin_fma(64.0, wxy[m], -sx * wy[m]);
          den[m] = (dvx[m] + vy) * __builtin_fma(wy[m], wy[m], dsxx[m]);
          const double kq = w_ok[m] ? 4.0 * D * D * sx : 0.0;
          num[m] = kq * cov * wy[m];
        }
        q_acc = quotient_sum4(num, den);
      } else {
#pragma unroll
        for (int m = 0; m < kWinPerThread; ++m) {
          const WinX wx = window_x((double)sxw[m], (double)sxxw[m], D);
          const double q = window_uqi(wx, (double)sxw[m], wy[m], wyy[m], wxy[m], D);
          q_acc += w_ok[m] ? q : 0.0;
        }
      }
      q_acc = wave_sum_to_63(q_acc);
      if (lane == 63) s_red[0][r & 1][wave] = q_acc;
    }
    if (r < r_last) add_basis(r + 1);
    __syncthreads();
  }
  if (t == 0) flush(r_last);
}

// Four workgroups of the integer form fit a CU's LDS; the register budget is
// set to match (at most 128 VGPRs, four waves per SIMD).
template <bool INT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(INT ? 4 : 1)))
void k_quality(QPlane P, QualityArgs /*A*/) {
  if constexpr (INT) quality_tile_int(P, blockIdx.x, quality_args<QualityKArgs1>());
  else quality_tile(P, blockIdx.x, quality_args<QualityKArgs1>());
}

template <bool INT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(INT ? 4 : 1)))
void k_quality_batch(const QPlane* __restrict__ planes, const QTile* __restrict__ tiles,
                     int32_t n_tiles, QualityArgs /*A*/) {
  if ((int)blockIdx.x >= n_tiles) return;
  const QTile w = tiles[blockIdx.x];
  if constexpr (INT) quality_tile_int(planes[w.plane], w.tile, quality_args<QualityKArgsN>());
  else quality_tile(planes[w.plane], w.tile, quality_args<QualityKArgsN>());
}

int quality_tiles_x(int width) { return (width + kWinCols - 1) / kWinCols; }
int quality_tiles_y(int height) { return (height + kWinRows - 1) / kWinRows; }

hipError_t launch_quality(const QPlane& P, const QualityArgs& A, hipStream_t s) {
  const int n = P.tiles_x * P.tiles_y;
  if (n <= 0) return hipSuccess;
  if (A.T.int_form)
    hipLaunchKernelGGL(k_quality<true>, dim3(n), dim3(kThreads), 0, s, P, A);
  else
    hipLaunchKernelGGL(k_quality<false>, dim3(n), dim3(kThreads), 0, s, P, A);
  return hipGetLastError();
}

hipError_t launch_quality_batch(const QPlane* planes, const QTile* tiles, int32_t n_tiles,
                                const QualityArgs& A, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (A.T.int_form)
    hipLaunchKernelGGL(k_quality_batch<true>, dim3(n_tiles), dim3(kThreads), 0, s, planes, tiles,
                       n_tiles, A);
  else
    hipLaunchKernelGGL(k_quality_batch<false>, dim3(n_tiles), dim3(kThreads), 0, s, planes,
                       tiles, n_tiles, A);
  return hipGetLastError();
}

}  // namespace rdct
