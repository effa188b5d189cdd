// Compile-time tables of the round-off DCT approximation (Cintra & Bayer, Section 2-3).
//
// C0 = [2 C] has entries in {0, +1, -1}; its Gram matrix C0 C0^T is diagonal with
// g = (8, 6, 4, 6, 8, 6, 4, 6).  The orthogonaliser S is diag(1/sqrt(g_k)), and the
// orthogonal approximation is C_orth = S C0 (Section 2).  S never multiplies pixels
// here: it is folded into the retention / quantisation step (Section 2).
//
// Natural coefficient order: index k * 8 + l with k the vertical and l the
// horizontal frequency.  Zig-zag order: the JPEG scan (Section 3 keeps the
// coefficients in the usual zig-zag order), generated here by walking the block
// with bounces.
#pragma once
#include <stdint.h>

namespace rdct {

// Diagonal of C0 C0^T.
constexpr int kGram[8] = {8, 6, 4, 6, 8, 6, 4, 6};

// C0 itself (Section 2), for code that needs single basis images rather than the
// 22-addition flow graph.  Checked below: its rows are orthogonal with the Gram
// diagonal above.
constexpr int kC0[8][8] = {
    {1, 1, 1, 1, 1, 1, 1, 1},      {1, 1, 1, 0, 0, -1, -1, -1},  {1, 0, 0, -1, -1, 0, 0, 1},
    {1, 0, -1, -1, 1, 1, 0, -1},   {1, -1, -1, 1, 1, -1, -1, 1}, {1, -1, 0, 1, -1, 0, 1, -1},
    {0, -1, 1, 0, 0, 1, -1, 0},    {0, -1, 1, -1, 1, -1, 1, 0}};

constexpr bool c0_gram_ok() {
  for (int k = 0; k < 8; ++k)
    for (int l = 0; l < 8; ++l) {
      int d = 0;
      for (int j = 0; j < 8; ++j) d += kC0[k][j] * kC0[l][j];
      if (d != (k == l ? kGram[k] : 0)) return false;
    }
  return true;
}
static_assert(c0_gram_ok(), "C0 rows must be orthogonal with norms g");
// 24 / g_k: S^2 = diag(kDp) / 24, so the exact reconstruction numerator is
// R = C0^T D' Y D' C0 with A' = R / 576.
constexpr int kDp[8] = {3, 4, 6, 4, 3, 4, 6, 4};

// Position classes of s_k s_l = 1 / sqrt(g_k g_l): rational (g_k == g_l, the
// square root is g_k) or irrational.
constexpr bool rational_pos(int k, int l) { return kGram[k] == kGram[l]; }

// s_k s_l = 1 / sqrt(g_k g_l) in float64, as 1.0 / sqrt(double(g_k g_l)) rounds
// it; g_k g_l takes six values (64, 48, 32, 36, 24, 16).  Hexadecimal literals
// keep the values exact at compile time.
constexpr double scale_kl(int k, int l) {
  switch (kGram[k] * kGram[l]) {
    case 64: return 0x1.0000000000000p-3;
    case 48: return 0x1.279a74590331dp-3;
    case 32: return 0x1.6a09e667f3bccp-3;
    case 36: return 0x1.5555555555555p-3;
    case 24: return 0x1.a20bd700c2c3fp-3;
    default: return 0x1.0000000000000p-2;  // 16
  }
}

struct ZigZag {
  int order[64];  // rank -> natural index
  int rank[64];   // natural index -> rank
};

// Walk the 8x8 grid from (0,0): moving "up-right" means row - 1, column + 1;
// "down-left" the opposite; bounce off the borders.  The first move goes to
// (row 0, column 1).
constexpr ZigZag make_zigzag() {
  ZigZag z{};
  int k = 0, l = 0;
  bool up = true;  // up-right
  for (int i = 0; i < 64; ++i) {
    z.order[i] = k * 8 + l;
    z.rank[k * 8 + l] = i;
    if (up) {
      if (l == 7) { ++k; up = false; }
      else if (k == 0) { ++l; up = false; }
      else { --k; ++l; }
    } else {
      if (k == 7) { ++l; up = true; }
      else if (l == 0) { ++k; up = true; }
      else { ++k; --l; }
    }
  }
  return z;
}
constexpr ZigZag kZigZag = make_zigzag();

// JPEG luminance quantisation table at quality 50 (ITU-T T.81 Annex K), natural
// order, rows = vertical frequency.  The paper names no table.
constexpr uint16_t kLumaQ50[64] = {
    16, 11, 10, 16, 24,  40,  51,  61,
    12, 12, 14, 19, 26,  58,  60,  55,
    14, 13, 16, 24, 40,  57,  69,  56,
    14, 17, 22, 29, 51,  87,  80,  62,
    18, 22, 37, 56, 68,  109, 103, 77,
    24, 35, 55, 64, 81,  104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101,
    72, 92, 95, 98, 112, 100, 103, 99};

// IJG quality scaling: factor 5000/q below 50, 200 - 2q from 50 up; entries
// (Q50 * f + 50) / 100 clamped to 1..255.
inline void ijg_table(int quality, uint16_t out[64]) {
  const int f = quality < 50 ? 5000 / quality : 200 - 2 * quality;
  for (int i = 0; i < 64; ++i) {
    int v = (kLumaQ50[i] * f + 50) / 100;
    out[i] = (uint16_t)(v < 1 ? 1 : (v > 255 ? 255 : v));
  }
}

}  // namespace rdct
