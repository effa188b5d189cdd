// Host-only logic of librdct that needs no GPU: the server's first-fit arena
// and its batch admission, the work lists of batch plans, and the argument
// checks on plane sizes and launch geometries.  Plain C++ (no HIP headers), so
// it also builds on its own, with the address and undefined-behaviour
// sanitizers, for tests on a machine without a GPU.
#pragma once
#include <math.h>
#include <stdint.h>

#include <iterator>
#include <map>
#include <vector>

#include "../../include/rdct.h"

namespace rdct {

// Blocks per work item of the batch kernels.
constexpr int kItemBlocks = 128;

// Work item of the persistent batch kernel: `kItemBlocks` (or fewer, at a
// plane's end) consecutive blocks of plane `plane` starting at block `t0`.
struct WorkItem {
  int32_t plane;
  int32_t t0;
};

// Multiplier m of the exact quantiser q = round(Y / (Q sqrt(g_k g_l))), halves
// away from zero (Section 3 quantises the orthogonal coefficients S Y S with the
// JPEG tables; g_k, g_l are diagonal entries of C0 C0^T, Section 2).  The
// kernels take q from the low word of the float64 FMA Y * m + 1.5 * 2^52, whose
// one rounding is to the nearest integer.  Where g_k == g_l the quotient
// Y / (g_k Q) is rational and can be a tie: m = 1 / (g_k Q) is then raised by a
// relative 2^-32, so a tie lies beyond the half-integer away from zero while
// every other value (at least 1 / (2 g_k Q) from a half-integer, |Y| < 2^15)
// keeps its side.  Elsewhere the quotient is irrational and at least ~4e-9 from
// any half-integer (Q <= 255), far above the float64 error of m.
inline double quant_multiplier(int gk, int gl, int Q) {
  if (gk == gl) return (1.0 / ((double)gk * (double)Q)) * (1.0 + 0x1p-32);
  return 1.0 / ((double)Q * sqrt((double)gk * (double)gl));
}

// Number of 8x8 blocks of a w x h plane (partial blocks included).
inline int64_t blocks_of(int32_t w, int32_t h) {
  if (w <= 0 || h <= 0) return 0;
  return (((int64_t)w + 7) / 8) * (((int64_t)h + 7) / 8);
}

inline int64_t items_of(int64_t nblocks) { return (nblocks + kItemBlocks - 1) / kItemBlocks; }

inline bool whole_blocks(int32_t w, int32_t h) { return (w % 8) == 0 && (h % 8) == 0; }

// Plane arguments that can be checked without touching memory: a non-null
// source, positive sides, a pitch of at least the width, and at most
// `max_blocks` blocks (UNSUPPORTED beyond).
inline rdct_status_t check_plane_dims(const void* src, int32_t w, int32_t h, int64_t pitch,
                                      int64_t max_blocks) {
  if (!src || w <= 0 || h <= 0 || pitch < w) return RDCT_ERR_INVALID_ARG;
  if (blocks_of(w, h) > max_blocks) return RDCT_ERR_UNSUPPORTED;
  return RDCT_OK;
}

// A batch geometry the kernels accept.
inline bool valid_tuning(const rdct_tuning_t& t) {
  return (t.waves_per_wg == 1 || t.waves_per_wg == 2 || t.waves_per_wg == 4) &&
         t.wgs_per_cu >= 1 && t.wgs_per_cu <= 16 &&
         (t.layout == RDCT_LAYOUT_STRIDED || t.layout == RDCT_LAYOUT_PER_PLANE) &&
         (t.xcd_ranges == 0 || t.xcd_ranges == 1) &&
         (t.strip == 1 || t.strip == 2 || t.strip == 4 || t.strip == 8);
}

// Work list of planes 0 .. n-1 (nblocks[i] blocks each): plane i's items are
// first[i] .. first[i + 1] - 1, in block order.  False (and nothing built) when
// the list would exceed INT32_MAX items or a count is negative.
inline bool build_work_list(const int64_t* nblocks, int n, std::vector<WorkItem>* items,
                            std::vector<int32_t>* first) {
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (nblocks[i] < 0 || nblocks[i] > INT32_MAX) return false;
    total += items_of(nblocks[i]);
    if (total > INT32_MAX) return false;
  }
  items->clear();
  items->reserve((size_t)total);
  first->assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) {
    (*first)[i] = (int32_t)items->size();
    for (int64_t t0 = 0; t0 < nblocks[i]; t0 += kItemBlocks) items->push_back(WorkItem{i, (int32_t)t0});
  }
  (*first)[n] = (int32_t)items->size();
  return true;
}

// Stable order of n planes with the flagged ones first; returns how many are
// flagged.  (Quantisation batches score whole-block planes in the coefficient
// domain and the others pixel by pixel, as the single-plane call does, in one
// launch each.)
inline int flagged_first(const std::vector<bool>& flag, std::vector<int>* order) {
  order->clear();
  for (size_t i = 0; i < flag.size(); ++i)
    if (flag[i]) order->push_back((int)i);
  const int n_flagged = (int)order->size();
  for (size_t i = 0; i < flag.size(); ++i)
    if (!flag[i]) order->push_back((int)i);
  return n_flagged;
}

// First-fit allocator over [0, size) with a coalescing free list; sizes are
// rounded up to `align`.  Offsets only: the caller owns the memory.
class Arena {
 public:
  void reset(int64_t size, int64_t align) {
    size_ = size;
    align_ = align > 0 ? align : 1;
    used_ = 0;
    free_.clear();
    if (size > 0) free_[0] = size;
  }
  // Offset of a block of `bytes` (> 0), or -1 when no free range is large enough.
  int64_t alloc(int64_t bytes) {
    if (bytes <= 0) return -1;
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return -1;
  }
  // Return a block obtained from alloc with the same byte count.
  void release(int64_t off, int64_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t size() const { return size_; }
  int64_t in_use() const { return used_; }
  int64_t round(int64_t b) const { return (b + align_ - 1) / align_ * align_; }
  // Largest free range (for checks).
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  // Free ranges are disjoint, ordered, coalesced, inside [0, size), and they
  // add up with the blocks in use to the whole arena.
  bool consistent() const {
    int64_t end = -1, sum = 0;
    for (const auto& kv : free_) {
      if (kv.first < 0 || kv.second <= 0 || kv.first + kv.second > size_) return false;
      if (kv.first <= end) return false;  // overlapping or touching (not coalesced)
      end = kv.first + kv.second;
      sum += kv.second;
    }
    return sum + used_ == size_;
  }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t size_ = 0, align_ = 256, used_ = 0;
};

// Sizes of the records a batch uploads with its planes.
struct MetaSizes {
  int64_t plane;  // one plane descriptor
  int64_t table;  // one quantisation table's constants
  int64_t item;   // one work item
};

// Bytes of a batch's metadata block: descriptors, tables, work items and one
// uint64 error sum per plane, each section starting on a 256-byte boundary.
inline int64_t batch_meta_bytes(const MetaSizes& s, int64_t n_planes, int64_t n_tables,
                                int64_t n_items) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  return up(s.plane * n_planes) + up(s.table * (n_tables > 0 ? n_tables : 1)) +
         up(s.item * n_items) + up(8 * n_planes);
}

// A pending request as admission sees it.
struct AdmitRequest {
  int kind;           // selection kind: requests of one batch share it
  int n;              // planes, 1..3
  int64_t bytes[3];   // device bytes of each plane
  int64_t items;      // work items of all its planes
};

struct AdmitLimits {
  int64_t max_planes;    // planes per batch
  int64_t max_requests;  // requests this batch may still take (in-flight cap)
  int64_t meta_cap;      // bytes of the batch's metadata region
  MetaSizes sizes;
};

// Metadata bytes of one request alone (a batch of its own).
inline int64_t request_meta_bytes(const AdmitRequest& r, const MetaSizes& s) {
  return batch_meta_bytes(s, r.n, 1, r.items);
}

// Admit pending requests, front first, into one batch: a request joins while
// it has the first request's kind, the plane and request caps hold, the
// batch's metadata (one table counted per request) stays within meta_cap and
// its planes fit in `dev`.  Admission stops at the first request that does
// not join.  offs[i][p] receives the device offset of admitted request i's
// plane p; nothing else is allocated, and a request that does not join leaves
// `dev` as it was.  Returns the number admitted.
inline int admit_batch(const AdmitRequest* pending, int n_pending, Arena* dev,
                       const AdmitLimits& lim, int64_t (*offs)[3]) {
  int64_t planes = 0, items = 0;
  int k = 0;
  for (; k < n_pending; ++k) {
    const AdmitRequest& r = pending[k];
    if (r.kind != pending[0].kind) break;
    if (r.n < 1 || r.n > 3) break;
    if (planes + r.n > lim.max_planes || k + 1 > lim.max_requests) break;
    if (batch_meta_bytes(lim.sizes, planes + r.n, k + 1, items + r.items) > lim.meta_cap) break;
    bool ok = true;
    int p = 0;
    for (; p < r.n; ++p) {
      offs[k][p] = dev->alloc(r.bytes[p]);
      if (offs[k][p] < 0) {
        ok = false;
        break;
      }
    }
    if (!ok) {
      for (int q = 0; q < p; ++q) dev->release(offs[k][q], r.bytes[q]);
      break;
    }
    planes += r.n;
    items += r.items;
  }
  return k;
}

}  // namespace rdct
