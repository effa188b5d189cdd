// C-ABI front end of librdct: argument validation, constant tables, dispatch.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/rdct.h"
#include "rdct_internal.h"
#include "rdct_tables.h"

namespace rdct {

void fill_quant_consts(const uint16_t q[64], QuantConsts* out) {
  for (int kl = 0; kl < 64; ++kl) {
    const int k = kl >> 3, l = kl & 7;
    const double Q = (double)q[kl];
    const double gg = (double)kGram[k] * (double)kGram[l];
    if (rational_pos(k, l)) {
      const double cq = (double)kGram[k] * Q;  // sqrt(g_k g_l) = g_k
      const float a = (float)(1.0 / cq);
      const float b = (float)((cq + 0.5) / (2.0 * cq));
      uint32_t ua, ub;
      memcpy(&ua, &a, 4);
      memcpy(&ub, &b, 4);
      out->qm[kl] = (uint64_t)ua | ((uint64_t)ub << 32);
    } else {
      const double m = 1.0 / (Q * sqrt(gg));
      memcpy(&out->qm[kl], &m, 8);
    }
    out->dq[kl] = Q * scale_kl(k, l);
    out->qi[kl] = (int32_t)q[kl];
    const double f = quant_multiplier(kGram[k], kGram[l], q[kl]);
    memcpy(&out->qf[kl], &f, 8);
  }
}

uint64_t keep_bits(int r) {
  uint64_t m = 0;
  for (int kl = 0; kl < 64; ++kl)
    if (kZigZag.rank[kl] < r) m |= 1ull << kl;
  return m;
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    return 256;
  return n;
}

rdct_status_t check_sel(const rdct_select_t* s, SelInfo* out) {
  if (!s) return RDCT_ERR_INVALID_ARG;
  if (s->level_shift < 0 || s->level_shift > 255) return RDCT_ERR_INVALID_ARG;
  out->shift = s->level_shift;
  memset(&out->qc, 0, sizeof(out->qc));
  switch (s->mode) {
    case RDCT_SEL_NONE:
      out->sel = SEL_ZZ;
      out->r = 64;
      return RDCT_OK;
    case RDCT_SEL_ZIGZAG:
      if (s->r < 1 || s->r > 64) return RDCT_ERR_INVALID_ARG;
      out->sel = SEL_ZZ;
      out->r = s->r;
      return RDCT_OK;
    case RDCT_SEL_QUANT: {
      uint16_t q[64];
      if (s->qtable) {
        for (int i = 0; i < 64; ++i) {
          if (s->qtable[i] < 1 || s->qtable[i] > 255) return RDCT_ERR_INVALID_ARG;
          q[i] = s->qtable[i];
        }
      } else {
        if (s->quality < 1 || s->quality > 100) return RDCT_ERR_INVALID_ARG;
        ijg_table(s->quality, q);
      }
      fill_quant_consts(q, &out->qc);
      memcpy(out->q, q, sizeof(q));
      out->sel = SEL_Q;
      out->r = 64;
      return RDCT_OK;
    }
    default:
      return RDCT_ERR_INVALID_ARG;
  }
}

static int coef_kind(rdct_coef_t t) {
  switch (t) {
    case RDCT_COEF_I32: return CO_I32;
    case RDCT_COEF_I16: return CO_I16;
    case RDCT_COEF_F32: return CO_F32;
    default: return -1;
  }
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }


rdct_status_t check_plane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch,
                          int64_t max_blocks) {
  return check_plane_dims(src, w, h, pitch, max_blocks);
}

Plane make_plane(const uint8_t* src, int32_t w, int32_t h, int64_t pitch) {
  Plane P;
  memset(&P, 0, sizeof(P));
  P.src = src;
  P.pitch = pitch;
  P.width = w;
  P.height = h;
  P.nbx = (w + 7) / 8;
  P.nby = (h + 7) / 8;
  P.nblocks = P.nbx * P.nby;
  P.aligned8 = (aligned(src, 8) && (pitch % 8) == 0) ? 1 : 0;
  return P;
}

static rdct_status_t hip_status(hipError_t e) { return e == hipSuccess ? RDCT_OK : RDCT_ERR_HIP; }

}  // namespace rdct

using namespace rdct;

extern "C" {

rdct_status_t rdct_forward(const uint8_t* src, int32_t width, int32_t height, int64_t src_pitch,
                           const rdct_select_t* sel, void* coef, rdct_coef_t coef_type,
                           void* stream) {
  rdct_status_t st = check_plane(src, width, height, src_pitch, kMaxBlocks);
  if (st != RDCT_OK) return st;
  SelInfo si;
  if ((st = check_sel(sel, &si)) != RDCT_OK) return st;
  const int co = coef_kind(coef_type);
  if (co < 0 || !coef || !aligned(coef, 16)) return RDCT_ERR_INVALID_ARG;
  if (si.sel == SEL_Q && co == CO_F32) return RDCT_ERR_INVALID_ARG;
  Plane P = make_plane(src, width, height, src_pitch);
  P.coef = coef;
  P.r = si.r;
  P.keep = keep_bits(si.r);
  P.r_count = 1;
  P.shift = si.shift;
  return hip_status(launch_plane(si.sel, co, false, EV_NONE, P, si.qc,
                                 kPlaneWavesPerWg, (hipStream_t)stream));
}

rdct_status_t rdct_inverse(const void* coef, rdct_coef_t coef_type, int32_t width, int32_t height,
                           const rdct_select_t* sel, float* dst, int64_t dst_pitch, void* stream) {
  if (!coef || !dst || width <= 0 || height <= 0 || dst_pitch < width) return RDCT_ERR_INVALID_ARG;
  if (blocks_of(width, height) > kMaxBlocks) return RDCT_ERR_UNSUPPORTED;
  if (!aligned(coef, 16) || !aligned(dst, 4)) return RDCT_ERR_INVALID_ARG;
  SelInfo si;
  rdct_status_t st = check_sel(sel, &si);
  if (st != RDCT_OK) return st;
  int kind;
  if (si.sel == SEL_Q) {
    if (coef_type == RDCT_COEF_I32) kind = INV_Q_I32;
    else if (coef_type == RDCT_COEF_I16) kind = INV_Q_I16;
    else return RDCT_ERR_INVALID_ARG;
  } else {
    if (coef_type == RDCT_COEF_I32) kind = INV_INT_I32;
    else if (coef_type == RDCT_COEF_I16) kind = INV_INT_I16;
    else if (coef_type == RDCT_COEF_F32) kind = INV_F32;
    else return RDCT_ERR_INVALID_ARG;
  }
  return hip_status(launch_inverse(kind, coef, width, height, si.r, si.shift, dst, dst_pitch,
                                   si.qc, (hipStream_t)stream));
}

rdct_status_t rdct_compress_eval(const uint8_t* src, int32_t width, int32_t height,
                                 int64_t src_pitch, const rdct_select_t* sel, int32_t r_count,
                                 void* coef_out, rdct_coef_t coef_type, float* recon_out,
                                 int64_t recon_pitch, uint64_t* sse_out, void* stream) {
  rdct_status_t st = check_plane(src, width, height, src_pitch, kMaxEvalBlocks);
  if (st != RDCT_OK) return st;
  SelInfo si;
  if ((st = check_sel(sel, &si)) != RDCT_OK) return st;
  if (!sse_out || !aligned(sse_out, 8) || r_count < 1) return RDCT_ERR_INVALID_ARG;
  int co = CO_NONE;
  if (coef_out) {
    co = coef_kind(coef_type);
    if (co < 0 || !aligned(coef_out, 16)) return RDCT_ERR_INVALID_ARG;
    if (si.sel == SEL_Q && co == CO_F32) return RDCT_ERR_INVALID_ARG;
  }
  if (recon_out && (recon_pitch < width || !aligned(recon_out, 4))) return RDCT_ERR_INVALID_ARG;
  int ev = EV_SPATIAL;
  if (si.sel == SEL_Q) {
    if (r_count != 1) return RDCT_ERR_INVALID_ARG;
    if ((width % 8) == 0 && (height % 8) == 0) ev = EV_COEF;
  } else {
    if (sel->mode == RDCT_SEL_NONE && r_count != 1) return RDCT_ERR_INVALID_ARG;
    if (si.r + r_count - 1 > 64) return RDCT_ERR_INVALID_ARG;
    if (r_count > 1) {
      if ((width % 8) != 0 || (height % 8) != 0) return RDCT_ERR_UNSUPPORTED;
      ev = EV_SWEEP;
    }
  }
  Plane P = make_plane(src, width, height, src_pitch);
  P.coef = coef_out;
  P.recon = recon_out;
  P.rpitch = recon_pitch;
  P.sse = sse_out;
  P.r = si.r;
  P.keep = keep_bits(si.r);
  P.r_count = r_count;
  P.shift = si.shift;
  hipError_t e = launch_zero_u64(sse_out, r_count, (hipStream_t)stream);
  if (e != hipSuccess) return RDCT_ERR_HIP;
  return hip_status(launch_plane(si.sel, co, recon_out != nullptr, ev, P, si.qc,
                                 kPlaneWavesPerWg, (hipStream_t)stream));
}

const char* rdct_status_string(rdct_status_t s) {
  switch (s) {
    case RDCT_OK: return "ok";
    case RDCT_ERR_INVALID_ARG: return "invalid argument";
    case RDCT_ERR_UNSUPPORTED: return "unsupported";
    case RDCT_ERR_HIP: return "HIP runtime error";
    case RDCT_ERR_NO_MEMORY: return "out of device memory";
    case RDCT_ERR_BUDGET: return "request exceeds the device-memory budget";
    case RDCT_ERR_NOT_FOUND: return "unknown ticket";
    case RDCT_ERR_BUSY: return "busy: queue or staging full";
    case RDCT_ERR_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

const char* rdct_version(void) { return "rdct 0.1 gfx950"; }

}  // extern "C"
