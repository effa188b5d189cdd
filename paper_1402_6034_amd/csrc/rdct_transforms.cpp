// 8x8 transform tables for the comparison path: the exact DCT, the round-off
// approximation, the signed DCT and the ceiling variant of the round-off
// construction (Sections 2-4).  Each transform is given as a forward matrix F
// applied to a block as F A F^T, and an inverse basis G with scale D such that
// the keep-r reconstruction is A' = G (M_r . (F A F^T)) G^T / D.  For the
// round-off and signed transforms F, G and D are integers, so numerators stay
// exact.
#include <cmath>
#include <cstring>

#include "rdct_internal.h"
#include "rdct_tables.h"

namespace rdct {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Orthonormal type-II DCT: C[k][n] = a_k cos(pi (2n + 1) k / 16).
void dct_matrix(double c[8][8]) {
  for (int k = 0; k < 8; ++k)
    for (int n = 0; n < 8; ++n)
      c[k][n] = (k == 0 ? std::sqrt(1.0 / 8.0) : 0.5) * std::cos(kPi * (2 * n + 1) * k / 16.0);
}

// Round half away from zero, the round-off operator of Section 2.
double round_away(double x) { return x < 0 ? -std::floor(-x + 0.5) : std::floor(x + 0.5); }

// Inverse of an 8x8 matrix by Gauss-Jordan elimination with partial pivoting;
// false if singular.
bool invert(const double a_in[8][8], double inv[8][8]) {
  double a[8][16];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 16; ++j) a[i][j] = j < 8 ? a_in[i][j] : (j - 8 == i ? 1.0 : 0.0);
  for (int c = 0; c < 8; ++c) {
    int p = c;
    for (int r = c + 1; r < 8; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
    if (std::fabs(a[p][c]) < 1e-9) return false;
    if (p != c)
      for (int j = 0; j < 16; ++j) std::swap(a[p][j], a[c][j]);
    const double d = a[c][c];
    for (int j = 0; j < 16; ++j) a[c][j] /= d;
    for (int r = 0; r < 8; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      for (int j = 0; j < 16; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) inv[i][j] = a[i][j + 8];
  return true;
}

// Eigen-decomposition of a symmetric 8x8 matrix by cyclic Jacobi rotations:
// a = V diag(w) V^T.
void jacobi_eigen(const double a_in[8][8], double w[8], double v[8][8]) {
  double a[8][8];
  std::memcpy(a, a_in, sizeof(a));
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < 8; ++i)
      for (int j = i + 1; j < 8; ++j) off += a[i][j] * a[i][j];
    if (off < 1e-30) break;
    for (int p = 0; p < 8; ++p)
      for (int q = p + 1; q < 8; ++q) {
        if (std::fabs(a[p][q]) < 1e-300) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 8; ++k) {  // columns p, q of a
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 8; ++k) {  // rows p, q of a
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 8; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 8; ++i) w[i] = a[i][i];
}

// Polar-decomposition orthogonalisation of Section 2: T = (C0 C0^T)^(-1/2) C0.
// False if C0 C0^T is singular.
bool polar_orthogonal(const double c0[8][8], double t[8][8]) {
  double g[8][8], w[8], v[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double s = 0;
      for (int n = 0; n < 8; ++n) s += c0[i][n] * c0[j][n];
      g[i][j] = s;
    }
  jacobi_eigen(g, w, v);
  for (int i = 0; i < 8; ++i)
    if (w[i] < 1e-9) return false;
  double s[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double acc = 0;
      for (int k = 0; k < 8; ++k) acc += v[i][k] * v[j][k] / std::sqrt(w[k]);
      s[i][j] = acc;
    }
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double acc = 0;
      for (int k = 0; k < 8; ++k) acc += s[i][k] * c0[k][j];
      t[i][j] = acc;
    }
  return true;
}

// Integer form of exact tables.  With 8-bit pixels x, |Y_kl| <= 255 a_k a_l for
// a_k = sum_m |F_km|, and any keep-r numerator is at most
// sum_kl |Y_kl| |G_ik| |G_jl| <= 255 (max_i sum_k a_k |G_ik|)^2 = N.  The
// integer kernel needs |Y| max|G| < 2^23 (24-bit multiply operands),
// 8 N < 2^31 (8-pixel row sums of numerators) and 255 D + N < 2^31 (errors).
void set_integer_form(TransformTables* t) {
  t->int_form = 0;
  if (!t->exact) return;
  for (int i = 0; i < 64; ++i) {
    if (t->F[i] != std::nearbyint(t->F[i]) || std::fabs(t->F[i]) > 127.0) return;
    if (t->G[i] != std::nearbyint(t->G[i]) || std::fabs(t->G[i]) > 127.0) return;
    t->Fi[i] = (int32_t)t->F[i];
    t->Gi[i] = (int32_t)t->G[i];
  }
  if (t->D != std::nearbyint(t->D) || t->D < 1.0 || t->D > 4096.0) return;
  t->Di = (int32_t)t->D;
  double a[8], a_max = 0.0, g_max = 0.0, row_max = 0.0;
  for (int k = 0; k < 8; ++k) {
    a[k] = 0.0;
    for (int m = 0; m < 8; ++m) a[k] += std::fabs(t->F[k * 8 + m]);
    a_max = std::fmax(a_max, a[k]);
  }
  for (int i = 0; i < 8; ++i) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) {
      s += a[k] * std::fabs(t->G[i * 8 + k]);
      g_max = std::fmax(g_max, std::fabs(t->G[i * 8 + k]));
    }
    row_max = std::fmax(row_max, s);
  }
  const double y_max = 255.0 * a_max * a_max, n_max = 255.0 * row_max * row_max;
  if (y_max * g_max >= 0x1p23 || 8.0 * n_max >= 0x1p31 || 255.0 * t->D + n_max >= 0x1p31) return;
  t->int_form = 1;
}

void set_orthogonal(const double t[8][8], TransformTables* out) {
  for (int k = 0; k < 8; ++k)
    for (int n = 0; n < 8; ++n) {
      out->F[k * 8 + n] = t[k][n];
      out->G[n * 8 + k] = t[k][n];  // G = T^T
    }
  out->D = 1.0;
  out->exact = 0;
  out->int_form = 0;
}

}  // namespace

rdct_status_t build_transform(int id, TransformTables* out) {
  *out = TransformTables{};
  double c[8][8];
  dct_matrix(c);
  switch (id) {
    case RDCT_T_DCT:
      set_orthogonal(c, out);
      return RDCT_OK;
    case RDCT_T_RDCT: {
      // F = C0, G = C0^T diag(d'), D = 576 (S^2 = diag(d') / 24).
      for (int k = 0; k < 8; ++k)
        for (int n = 0; n < 8; ++n) {
          const double e = round_away(2.0 * c[k][n]);
          out->F[k * 8 + n] = e;
          out->G[n * 8 + k] = e * kDp[k];
        }
      out->D = 576.0;
      out->exact = 1;
      set_integer_form(out);
      return RDCT_OK;
    }
    case RDCT_T_SDCT: {
      // T = sign(C) / sqrt8: F = sign(C), G = 8 sign(C)^-1 (integral), D = 64.
      double sg[8][8], inv[8][8];
      for (int k = 0; k < 8; ++k)
        for (int n = 0; n < 8; ++n) sg[k][n] = c[k][n] < 0 ? -1.0 : 1.0;
      if (!invert(sg, inv)) return RDCT_ERR_UNSUPPORTED;
      for (int i = 0; i < 8; ++i)
        for (int k = 0; k < 8; ++k) {
          const double m = std::nearbyint(8.0 * inv[i][k]);
          if (std::fabs(m - 8.0 * inv[i][k]) > 1e-9) return RDCT_ERR_UNSUPPORTED;
          out->G[i * 8 + k] = m;
          out->F[i * 8 + k] = sg[i][k];
        }
      out->D = 64.0;
      out->exact = 1;
      set_integer_form(out);
      return RDCT_OK;
    }
    case RDCT_T_RDCT_CEIL:
    case RDCT_T_RDCT_FLOOR: {
      double c0[8][8], t[8][8];
      for (int k = 0; k < 8; ++k)
        for (int n = 0; n < 8; ++n)
          c0[k][n] = id == RDCT_T_RDCT_CEIL ? std::ceil(2.0 * c[k][n]) : std::floor(2.0 * c[k][n]);
      // floor(2C) has a zero first row: C0 C0^T is singular.
      if (!polar_orthogonal(c0, t)) return RDCT_ERR_UNSUPPORTED;
      set_orthogonal(t, out);
      return RDCT_OK;
    }
    default:
      return RDCT_ERR_INVALID_ARG;
  }
}

}  // namespace rdct
