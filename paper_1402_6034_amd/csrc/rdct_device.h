// Device helpers shared by the HIP kernels of the library: address-space casts,
// gated table pointers, the addition-only flow graphs of C0 and C0^T, the exact
// quantiser and block loads.
#pragma once
#include "rdct_internal.h"
#include "rdct_tables.h"

#include <utility>

namespace rdct {

typedef short s16x2 __attribute__((ext_vector_type(2)));

// Pointers read from descriptors are generic; casting them to the global
// address space lets the compiler emit global (not flat) memory instructions.
#define RDCT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RDCT_GLOBAL T* gptr(T* p) {
  return (RDCT_GLOBAL T*)p;
}
// Quantisation tables are read through constant-address-space pointers, which
// become scalar loads.
#define RDCT_CONST __attribute__((address_space(4)))
typedef const RDCT_CONST QuantConsts* QCPtr;

// Returns p once `dep` has been computed.  A table is 192 dwords, more than the
// scalar register file: without this the compiler loads all of it up front and
// spills it.  Gating the pointer of row K + 2 on a result of row K keeps one row
// of look-ahead.
__device__ __forceinline__ QCPtr qc_after(QCPtr p, uint32_t dep) {
  asm volatile("" : "+s"(p) : "v"(dep));
  return p;
}
__device__ __forceinline__ QCPtr qc_after_s(QCPtr p, int dep) {
  asm volatile("" : "+s"(p) : "s"(dep));
  return p;
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));



// ---------------------------------------------------------------------------
// Addition-only flow graphs for C0 and C0^T (22 additions each).
// Forward: mirrored sums a_i = x_i + x_{7-i} feed the even outputs, mirrored
// differences b_i = x_i - x_{7-i} feed the odd outputs.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void c0_forward(T (&x)[8]) {
  const T a0 = x[0] + x[7], a1 = x[1] + x[6], a2 = x[2] + x[5], a3 = x[3] + x[4];
  const T b0 = x[0] - x[7], b1 = x[1] - x[6], b2 = x[2] - x[5], b3 = x[3] - x[4];
  const T p = a0 + a3, q = a1 + a2;
  x[0] = p + q;
  x[4] = p - q;
  x[2] = a0 - a3;
  x[6] = a2 - a1;
  x[1] = b0 + (b1 + b2);
  x[3] = b0 - (b2 + b3);
  x[5] = (b0 + b3) - b1;
  x[7] = b2 - (b1 + b3);
}

// Transposed graph: x = C0^T X.
template <typename T>
__device__ __forceinline__ void c0_transpose(T (&X)[8]) {
  const T p = X[0] + X[4], m = X[0] - X[4];
  const T a0 = p + X[2], a3 = p - X[2], a1 = m - X[6], a2 = m + X[6];
  const T b0 = X[1] + (X[3] + X[5]);
  const T b1 = X[1] - (X[5] + X[7]);
  const T b2 = (X[1] + X[7]) - X[3];
  const T b3 = X[5] - (X[3] + X[7]);
  X[0] = a0 + b0;
  X[7] = a0 - b0;
  X[1] = a1 + b1;
  X[6] = a1 - b1;
  X[2] = a2 + b2;
  X[5] = a2 - b2;
  X[3] = a3 + b3;
  X[4] = a3 - b3;
}

// Separable 2-D pass on an 8x8 register array: rows first, then columns.
template <typename T, bool FWD>
__device__ __forceinline__ void pass2d(T (&v)[8][8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if constexpr (FWD) c0_forward(v[i]); else c0_transpose(v[i]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    T c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = v[i][j];
    if constexpr (FWD) c0_forward(c); else c0_transpose(c);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i][j] = c[i];
  }
}

// ---------------------------------------------------------------------------
// Exact quantiser: q = round(s_k s_l Y / Q), halves away from zero.
// Rational positions (s_k s_l = 1/c): |q| = floor((2|Y| + cQ + 1/2) / (2cQ)),
// one float FMA whose rounding error stays below the half-step margin 1/(4cQ).
// Irrational positions (no exact ties): float64 FMA Y * m +- 1/2, whose error is
// far below the distance of any Y / (Q sqrt(g_k g_l)) from a half-integer.
// ---------------------------------------------------------------------------
template <int KL>
__device__ __forceinline__ int quantize(int y, uint64_t qm) {
  constexpr int k = KL >> 3, l = KL & 7;
  if constexpr (rational_pos(k, l)) {
    const float a = __uint_as_float((uint32_t)qm);
    const float b = __uint_as_float((uint32_t)(qm >> 32));
    const float yf = (float)y;
    const float t = __builtin_fmaf(__builtin_fabsf(yf), a, b);
    return (int)__builtin_copysignf(t, yf);
  } else {
    const double m = __longlong_as_double((long long)qm);
    const double yd = (double)y;
    const double t = __builtin_fma(__builtin_fabs(yd), m, 0.5);
    return (int)__builtin_copysign(t, yd);
  }
}

// The same q from the low word of one float64 FMA, Y * qf + 1.5 * 2^52, with
// qf from quant_multiplier: the addend pins the exponent, so the FMA's single
// rounding is to the nearest integer and leaves q (two's complement) in the low
// 32 bits.  Three instructions per coefficient (extract, convert, FMA) against
// five or six above.
__device__ __forceinline__ int quantize_fma(int y, uint64_t qf) {
  const double t = __builtin_fma((double)y, __longlong_as_double((long long)qf), 0x1.8p52);
  return (int)(uint32_t)__double_as_longlong(t);
}

// ---------------------------------------------------------------------------
// Block loads (8 rows x 8 bytes), edge-replicating partial blocks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_block(const Plane& P, int t, bool valid, uint32_t (&w)[16],
                                           int& x0, int& y0) {
  if (!valid) {
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = 0;
    x0 = 0;
    y0 = 0;
    return;
  }
  const int by = t / P.nbx;
  const int bx = t - by * P.nbx;
  x0 = bx * 8;
  y0 = by * 8;
  if (P.aligned8 && x0 + 8 <= P.width && y0 + 8 <= P.height) {
    const RDCT_GLOBAL uint8_t* base = gptr(P.src) + (int64_t)y0 * P.pitch + x0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const u32x2 r = __builtin_nontemporal_load(
          reinterpret_cast<const RDCT_GLOBAL u32x2*>(base + (int64_t)i * P.pitch));
      w[2 * i] = r.x;
      w[2 * i + 1] = r.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int y = min(y0 + i, P.height - 1);
      const RDCT_GLOBAL uint8_t* row = gptr(P.src) + (int64_t)y * P.pitch;
      uint32_t d0 = 0, d1 = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        d0 |= (uint32_t)row[min(x0 + j, P.width - 1)] << (8 * j);
        d1 |= (uint32_t)row[min(x0 + 4 + j, P.width - 1)] << (8 * j);
      }
      w[2 * i] = d0;
      w[2 * i + 1] = d1;
    }
  }
}

__device__ __forceinline__ int pixel(const uint32_t (&w)[16], int i, int j) {
  return (int)((w[2 * i + (j >> 2)] >> (8 * (j & 3))) & 0xffu);
}


// Workgroups are dealt to the eight XCDs round-robin (workgroup b runs on XCD
// b % 8), and each XCD has its own L2.  The remap gives each XCD a contiguous
// range of logical workgroup indices, so neighbouring work lands in one L2:
// bijective on [0, 8 * (G / 8)), the identity on the last G % 8 workgroups.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int per = G >> 3;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace rdct
