// Keep-r sweep with image-quality metrics for any 8x8 transform (the comparison
// of Section 3: the approximation against the exact DCT and the signed DCT,
// scored by SSE and by the universal quality index, UQI).
//
// A workgroup owns a tile of 32 x 64 window positions (8x8 windows at stride 1);
// the windows reach 7 pixels further, so the tile transforms the 5 x 9 blocks
// covering 40 x 72 pixels.  It computes every block's coefficients once
// (Y = F A F^T), then for r = 1, 2, ... adds the basis image of the zig-zag
// position of rank r - 1, scaled by that coefficient, to the reconstruction it
// keeps in LDS -- the keep-r reconstruction is linear in the kept
// coefficients -- and, for the requested r, scores:
//   SSE  over the 32 x 64 pixels the tile owns (its 4 x 8 blocks);
//   UQI  over its 32 x 64 windows: each thread owns one window column and eight
//        window rows, forms 8-pixel row sums of y, y^2 and x y, and slides a
//        window of eight of them down the column.
// For the round-off and signed transforms the reconstruction is kept as an
// integer numerator (A' = numerator / D) and every window or error sum is an
// exact integer in float64.  No MFMA: per r the work is a rank-1 update and
// sliding sums, not a dense contraction.
#include "rdct_internal.h"
#include "rdct_tables.h"

namespace rdct {

#define RDCT_CONST __attribute__((address_space(4)))

constexpr int kWinRows = 32, kWinCols = 64;             // windows per tile
constexpr int kPixRows = kWinRows + 8, kPixCols = kWinCols + 8;  // 40 x 72
constexpr int kBlkRows = kPixRows / 8, kBlkCols = kPixCols / 8;  // 5 x 9
constexpr int kTileBlocks = kBlkRows * kBlkCols;        // 45
constexpr int kThreads = 256;

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

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Q of one window from its sums (numerators of y = numerator / D; N = 64).
// Float64 noise must not decide the index: a constant block keeps only its DC
// term and is exact in real arithmetic, but the float64 transforms leave ~1e-13
// of noise in it.  So, in grey levels, a reconstruction window with variance
// <= 2^-24 counts as flat (no variance, no covariance), a window mean of
// magnitude <= 2^-24 counts as 0, and a flat pixel window has no covariance.
// With integer numerators every quantity here is an exact integer and the
// rules are decided exactly.
__device__ __forceinline__ double window_uqi(double sx, double sxx, double sy, double syy,
                                             double sxy, double d) {
  constexpr double N = 64.0, EPS = 0x1p-24;
  const double vx = __builtin_fma(N, sxx, -sx * sx);                  // N^2 var_x
  const double vy_raw = __builtin_fma(N, syy, -sy * sy);              // N^2 D^2 var_y
  const bool flat_y = vy_raw <= (N * N) * (d * d) * EPS;
  const double vy = flat_y ? 0.0 : vy_raw;
  const double cov = (vx == 0.0 || flat_y) ? 0.0 : __builtin_fma(N, sxy, -sx * sy);  // N^2 D cov
  const double sym = __builtin_fabs(sy) <= N * d * EPS ? 0.0 : sy;
  const double ns = 2.0 * d * cov;
  const double ds = __builtin_fma(d * d, vx, vy);
  const double nm = 2.0 * d * sx * sym;
  const double dm = __builtin_fma(d * d, sx * sx, sym * sym);
  const double fs = ds == 0.0 ? 1.0 : ns / ds;
  const double fm = dm == 0.0 ? 1.0 : nm / dm;
  return fs * fm;
}

__device__ void quality_tile(const QPlane& P, int tile, const RDCT_CONST QualityArgs* A) {
  __shared__ double s_coef[kTileBlocks][64];
  __shared__ double s_y[kPixRows][kPixCols];
  __shared__ float s_x[kPixRows][kPixCols];
  __shared__ double s_F[64], s_G[64];
  __shared__ double s_red[2][kThreads / 64];

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
    float v = 0.0f;
    if (gy < P.height && gx < P.width) v = (float)P.src[(int64_t)gy * P.pitch + gx];
    s_x[row][col] = v;
    s_y[row][col] = 0.0;
  }
  if (t < 64) s_F[t] = A->T.F[t];
  else if (t < 128) s_G[t - 64] = A->T.G[t - 64];
  __syncthreads();

  // Forward: Y_b = F A_b F^T, one (block, row k) task per thread.
  for (int task = t; task < kTileBlocks * 8; task += kThreads) {
    const int b = task >> 3, k = task & 7;
    const int br = b / kBlkCols, bc = b - br * kBlkCols;
    double u[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m) acc = __builtin_fma(s_F[k * 8 + m], (double)s_x[br * 8 + m][bc * 8 + n], acc);
      u[n] = acc;
    }
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      double acc = 0.0;
#pragma unroll
      for (int n = 0; n < 8; ++n) acc = __builtin_fma(u[n], s_F[l * 8 + n], acc);
      s_coef[b][k * 8 + l] = acc;
    }
  }

  // Window sums of x (exact integers), for this thread's window column c and
  // window rows 8 g .. 8 g + 7.
  const int c = lane, g = wave;
  double sx[8], sxx[8];
  {
    double hx[15], hxx[15];
#pragma unroll
    for (int rr = 0; rr < 15; ++rr) {
      double a = 0.0, a2 = 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double xv = (double)s_x[8 * g + rr][c + u];
        a += xv;
        a2 = __builtin_fma(xv, xv, a2);
      }
      hx[rr] = a;
      hxx[rr] = a2;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      double a = 0.0, a2 = 0.0;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        a += hx[m + rr];
        a2 += hxx[m + rr];
      }
      sx[m] = a;
      sxx[m] = a2;
    }
  }
  const bool col_ok = x0 + c + 8 <= P.width;
  // Owned pixels for the SSE: row t / 8, columns 8 (t % 8) .. + 7 of the tile.
  const int orow = t >> 3, ocol = (t & 7) * 8;
  const bool own_ok = (y0 + orow < P.height) && (x0 + ocol < P.width);
  __syncthreads();

  const int r_first = A->r_first, r_last = A->r_first + A->r_count - 1;
  for (int r = 1; r <= r_last; ++r) {
    const int kl = c_zz_quality.order[r - 1];
    const int k = kl >> 3, l = kl & 7;
    // Add coefficient (k, l) of every block times its basis image
    // G[:, k] G[:, l]^T.
    double gl[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) gl[j] = A->T.G[j * 8 + l];
    for (int task = t; task < kTileBlocks * 8; task += kThreads) {
      const int b = task >> 3, i = task & 7;
      const int br = b / kBlkCols, bc = b - br * kBlkCols;
      if (by0 + br >= nby || bx0 + bc >= nbx) continue;   // block outside the plane
      const double ci = s_coef[b][kl] * s_G[i * 8 + k];
      double* row = &s_y[br * 8 + i][bc * 8];
#pragma unroll
      for (int j = 0; j < 8; ++j) row[j] = __builtin_fma(ci, gl[j], row[j]);
    }
    __syncthreads();
    if (r >= r_first) {
      // UQI of the eight windows of this thread.
      double q_acc = 0.0;
      {
        double hy[15], hyy[15], hxy[15];
        double sy = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
        for (int rr = 0; rr < 15; ++rr) {
          double a = 0.0, a2 = 0.0, ax = 0.0;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double yv = s_y[8 * g + rr][c + u];
            const double xv = (double)s_x[8 * g + rr][c + u];
            a += yv;
            a2 = __builtin_fma(yv, yv, a2);
            ax = __builtin_fma(xv, yv, ax);
          }
          hy[rr] = a;
          hyy[rr] = a2;
          hxy[rr] = ax;
          sy += a;
          syy += a2;
          sxy += ax;
          if (rr >= 7) {
            const int m = rr - 7;
            const bool ok = col_ok && (y0 + 8 * g + m + 8 <= P.height);
            const double q = window_uqi(sx[m], sxx[m], sy, syy, sxy, D);
            q_acc += ok ? q : 0.0;
            sy -= hy[m];
            syy -= hyy[m];
            sxy -= hxy[m];
          }
        }
      }
      // Squared error over the owned pixels: (D x - numerator)^2.
      double e_acc = 0.0;
      if (own_ok) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double e = __builtin_fma(D, (double)s_x[orow][ocol + j], -s_y[orow][ocol + j]);
          e_acc = __builtin_fma(e, e, e_acc);
        }
      }
      q_acc = wave_sum_f64(q_acc);
      e_acc = wave_sum_f64(e_acc);
      if (lane == 0) {
        s_red[0][wave] = q_acc;
        s_red[1][wave] = e_acc;
      }
      __syncthreads();
      if (t == 0) {
        double q = 0.0, e = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
          q += s_red[0][w];
          e += s_red[1][w];
        }
        const int o = r - r_first;
        atomicAdd(reinterpret_cast<unsigned long long*>(P.uqi + o),
                  (unsigned long long)(long long)__builtin_rint(q * 4294967296.0));
        // Exact families: e is an integer below 2^53; otherwise 2^-20 units.
        const double eu = exact ? e : __builtin_rint(e * 1048576.0);
        atomicAdd(reinterpret_cast<unsigned long long*>(P.sse + o), (unsigned long long)eu);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_quality(QPlane P, QualityArgs /*A*/) {
  quality_tile(P, blockIdx.x, quality_args<QualityKArgs1>());
}

__global__ __launch_bounds__(kThreads) void k_quality_batch(const QPlane* __restrict__ planes,
                                                            const QTile* __restrict__ tiles,
                                                            int32_t n_tiles, QualityArgs /*A*/) {
  if ((int)blockIdx.x >= n_tiles) return;
  const QTile w = tiles[blockIdx.x];
  quality_tile(planes[w.plane], w.tile, quality_args<QualityKArgsN>());
}

int quality_tiles_x(int width) { return (width + kWinCols - 1) / kWinCols; }
int quality_tiles_y(int height) { return (height + kWinRows - 1) / kWinRows; }

hipError_t launch_quality(const QPlane& P, const QualityArgs& A, hipStream_t s) {
  const int n = P.tiles_x * P.tiles_y;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quality, dim3(n), dim3(kThreads), 0, s, P, A);
  return hipGetLastError();
}

hipError_t launch_quality_batch(const QPlane* planes, const QTile* tiles, int32_t n_tiles,
                                const QualityArgs& A, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quality_batch, dim3(n_tiles), dim3(kThreads), 0, s, planes, tiles,
                     n_tiles, A);
  return hipGetLastError();
}

}  // namespace rdct
