"""Host-only logic of the library built with g++ under the address and
undefined-behaviour sanitizers and exercised without a GPU: the server's
first-fit arena (random alloc/release against a byte-map model), its batch
admission (metadata and plane budgets, including a budget that leaves less
than one request's metadata), the work lists and plane ordering of batch plans,
the plane and geometry checks, the host-side metrics (PSNR of many planes,
quality metrics, pair decoding) and the tuning-cache parser on malformed files.
Any sanitizer report aborts the test program and fails the test.  A second
program checks the quantiser's rule (multiplier and FMA) exhaustively."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1402_6034_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include <math.h>

#include "rdct_host.h"
#include "rdct_tune.h"

using namespace rdct;

static int failures = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

// Random allocations and releases against a model that marks every byte.
static void arena_random(uint32_t seed, int64_t size, int64_t align) {
  Arena a;
  a.reset(size, align);
  std::vector<unsigned char> used((size_t)size, 0);
  struct Blk { int64_t off, bytes; };
  std::vector<Blk> live;
  std::mt19937 rng(seed);
  for (int step = 0; step < 4000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const int64_t bytes = 1 + (int64_t)(rng() % (uint32_t)(size / 8));
      const int64_t largest = a.largest_free();
      const int64_t off = a.alloc(bytes);
      const int64_t rounded = a.round(bytes);
      if (off < 0) {
        CHECK(largest < rounded);   // first fit fails only when nothing is large enough
        continue;
      }
      CHECK(off % align == 0);
      CHECK(off + rounded <= size);
      for (int64_t i = off; i < off + rounded; ++i) {
        CHECK(!used[(size_t)i]);
        used[(size_t)i] = 1;
      }
      live.push_back({off, bytes});
    } else {
      const size_t k = rng() % live.size();
      const Blk b = live[k];
      live.erase(live.begin() + (long)k);
      a.release(b.off, b.bytes);
      for (int64_t i = b.off; i < b.off + a.round(b.bytes); ++i) used[(size_t)i] = 0;
    }
    CHECK(a.consistent());
    int64_t in_use = 0;
    for (unsigned char u : used) in_use += u;
    CHECK(in_use == a.in_use());
  }
  for (const Blk& b : live) a.release(b.off, b.bytes);
  CHECK(a.in_use() == 0 && a.largest_free() == size && a.consistent());
  CHECK(a.alloc(0) == -1 && a.alloc(-5) == -1);
}

static const MetaSizes kSizes = {112, 1280, 8};

static AdmitRequest req(int kind, int n, int64_t bytes, int64_t items) {
  AdmitRequest r;
  r.kind = kind;
  r.n = n;
  for (int i = 0; i < 3; ++i) r.bytes[i] = i < n ? bytes : 0;
  r.items = items;
  return r;
}

static void admission() {
  int64_t offs[64][3];
  // A metadata region smaller than one request's metadata admits nothing and
  // leaves the plane arena untouched.
  {
    Arena dev;
    dev.reset(1 << 20, 256);
    AdmitRequest r = req(0, 3, 4096, 3);
    AdmitLimits lim{4096, 100, request_meta_bytes(r, kSizes) - 1, kSizes};
    CHECK(admit_batch(&r, 1, &dev, lim, offs) == 0);
    CHECK(dev.in_use() == 0 && dev.consistent());
    lim.meta_cap += 1;
    CHECK(admit_batch(&r, 1, &dev, lim, offs) == 1);
    CHECK(dev.in_use() == 3 * 4096);
  }
  // The metadata cap decides how many requests join: k such that the batch's
  // metadata fits and one more would not.
  {
    Arena dev;
    dev.reset(64 << 20, 256);
    std::vector<AdmitRequest> rs(64, req(1, 2, 1000, 40));
    const int64_t cap = 64 << 10;
    AdmitLimits lim{4096, 1000, cap, kSizes};
    const int k = admit_batch(rs.data(), (int)rs.size(), &dev, lim, offs);
    CHECK(k > 0 && k < 64);
    CHECK(batch_meta_bytes(kSizes, 2 * k, k, 40 * k) <= cap);
    CHECK(batch_meta_bytes(kSizes, 2 * (k + 1), k + 1, 40 * (k + 1)) > cap);
    CHECK(dev.in_use() == dev.round(1000) * 2 * k);
  }
  // Planes that do not fit stop admission and leave no partial allocation.
  {
    Arena dev;
    dev.reset(9 * 4096 + 256, 256);
    std::vector<AdmitRequest> rs = {req(0, 3, 4096, 1), req(0, 3, 4096, 1), req(0, 3, 4096, 1),
                                    req(0, 1, 4096, 1)};
    AdmitLimits lim{4096, 100, 1 << 20, kSizes};
    CHECK(admit_batch(rs.data(), (int)rs.size(), &dev, lim, offs) == 3);
    CHECK(dev.in_use() == 9 * 4096 && dev.consistent());
    Arena dev2;
    dev2.reset(8 * 4096, 256);
    CHECK(admit_batch(rs.data(), (int)rs.size(), &dev2, lim, offs) == 2);
    CHECK(dev2.in_use() == 6 * 4096 && dev2.consistent());
    // Distinct offsets inside the arena.
    CHECK(offs[0][0] != offs[0][1] && offs[1][2] + 4096 <= 8 * 4096);
  }
  // Kind change, plane cap and request cap.
  {
    Arena dev;
    dev.reset(1 << 24, 256);
    std::vector<AdmitRequest> rs = {req(0, 1, 64, 1), req(0, 3, 64, 1), req(1, 1, 64, 1),
                                    req(0, 1, 64, 1)};
    AdmitLimits lim{4096, 100, 1 << 20, kSizes};
    CHECK(admit_batch(rs.data(), 4, &dev, lim, offs) == 2);
    lim.max_planes = 3;
    dev.reset(1 << 24, 256);
    CHECK(admit_batch(rs.data(), 4, &dev, lim, offs) == 1);
    lim.max_planes = 4096;
    lim.max_requests = 0;
    dev.reset(1 << 24, 256);
    CHECK(admit_batch(rs.data(), 4, &dev, lim, offs) == 0 && dev.in_use() == 0);
    AdmitRequest bad = req(0, 4, 64, 1);
    lim.max_requests = 10;
    CHECK(admit_batch(&bad, 1, &dev, lim, offs) == 0);
  }
}

static void work_lists() {
  const int64_t nb[] = {1, 127, 128, 129, 1000, 0, 4096 * 64 + 5};
  const int n = (int)(sizeof(nb) / sizeof(nb[0]));
  std::vector<WorkItem> items;
  std::vector<int32_t> first;
  CHECK(build_work_list(nb, n, &items, &first));
  CHECK((int)first.size() == n + 1 && first[0] == 0 && first[n] == (int32_t)items.size());
  for (int i = 0; i < n; ++i) {
    CHECK(first[i + 1] - first[i] == items_of(nb[i]));
    int64_t covered = 0;
    for (int32_t j = first[i]; j < first[i + 1]; ++j) {
      CHECK(items[(size_t)j].plane == i);
      CHECK(items[(size_t)j].t0 == covered);
      covered += kItemBlocks;
    }
    CHECK(covered >= nb[i] && covered - nb[i] < kItemBlocks);
  }
  const int64_t too_many[] = {(int64_t)INT32_MAX + 1};
  CHECK(!build_work_list(too_many, 1, &items, &first));
  const int64_t negative[] = {5, -1};
  CHECK(!build_work_list(negative, 2, &items, &first));
  std::vector<int64_t> many(20000, (int64_t)INT32_MAX / 8);
  CHECK(!build_work_list(many.data(), (int)many.size(), &items, &first));

  std::vector<bool> flag = {false, true, false, true, true, false};
  std::vector<int> order;
  CHECK(flagged_first(flag, &order) == 3);
  const int want[] = {1, 3, 4, 0, 2, 5};
  for (int i = 0; i < 6; ++i) CHECK(order[(size_t)i] == want[i]);
  flag.assign(0, false);
  CHECK(flagged_first(flag, &order) == 0 && order.empty());
}

static void checks() {
  const char* p = "x";
  CHECK(check_plane_dims(p, 8, 8, 8, 1) == RDCT_OK);
  CHECK(check_plane_dims(nullptr, 8, 8, 8, 1) == RDCT_ERR_INVALID_ARG);
  CHECK(check_plane_dims(p, 0, 8, 8, 1) == RDCT_ERR_INVALID_ARG);
  CHECK(check_plane_dims(p, 8, -1, 8, 1) == RDCT_ERR_INVALID_ARG);
  CHECK(check_plane_dims(p, 9, 8, 8, 4) == RDCT_ERR_INVALID_ARG);
  CHECK(check_plane_dims(p, 9, 8, 9, 1) == RDCT_ERR_UNSUPPORTED);
  CHECK(check_plane_dims(p, INT32_MAX, INT32_MAX, INT32_MAX, 1ll << 26) == RDCT_ERR_UNSUPPORTED);
  CHECK(blocks_of(INT32_MAX, INT32_MAX) == (int64_t)((INT32_MAX / 8) + 1) * ((INT32_MAX / 8) + 1));
  CHECK(blocks_of(0, 5) == 0 && blocks_of(1, 1) == 1 && blocks_of(9, 17) == 6);
  CHECK(whole_blocks(16, 8) && !whole_blocks(16, 9));
  rdct_tuning_t t{};
  t.waves_per_wg = 4;
  t.wgs_per_cu = 16;
  t.layout = RDCT_LAYOUT_PER_PLANE;
  CHECK(!valid_tuning(t));   // strip 0 is not a geometry
  t.strip = 8;
  CHECK(valid_tuning(t));
  t.strip = 3;
  CHECK(!valid_tuning(t));
  t.strip = 1;
  t.waves_per_wg = 3;
  CHECK(!valid_tuning(t));
  t.waves_per_wg = 1;
  t.wgs_per_cu = 17;
  CHECK(!valid_tuning(t));
  t.wgs_per_cu = 1;
  t.layout = 0;
  CHECK(!valid_tuning(t));
}

static void tune_cache(const char* path) {
  // Lines the scanner must survive: a key without its closing quote, fields
  // without values, a line far longer than the reader's buffer, numbers that
  // overflow, and a valid entry at the end.
  FILE* f = fopen(path, "w");
  fprintf(f, "{\"rdct_tuning\": 1, \"entries\": [\n");
  fprintf(f, "  {\"key\": \"unterminated\n");
  fprintf(f, "  {\"key\": \"gfx950/nofields\", \"waves_per_wg\": , \"wgs_per_cu\": }\n");
  std::string longkey(5000, 'k');
  fprintf(f, "  {\"key\": \"%s\", \"waves_per_wg\": 2, \"wgs_per_cu\": 4},\n", longkey.c_str());
  fprintf(f, "  {\"key\": \"gfx950/big\", \"waves_per_wg\": 99999999999999999999, \"wgs_per_cu\": 1},\n");
  fprintf(f, "  {\"key\": \"\", \"waves_per_wg\": 1, \"wgs_per_cu\": 2},\n");
  fprintf(f, "  {\"key\": \"gfx950/ok\", \"waves_per_wg\": 2, \"wgs_per_cu\": 8, \"layout\": 2, \"us\": 5.0}\n");
  fprintf(f, "]}\n");
  fclose(f);
  rdct_tuning_t t{};
  CHECK(tune_cache_lookup("gfx950/ok", &t));
  CHECK(t.waves_per_wg == 2 && t.wgs_per_cu == 8 && t.layout == 2 && t.use_graph == 0);
  CHECK(t.strip == 1);   // entries written before the strip existed
  CHECK(!tune_cache_lookup("unterminated", &t));
  rdct_tuning_t u{};
  u.waves_per_wg = 4;
  u.wgs_per_cu = 3;
  u.layout = 1;
  u.strip = 4;
  tune_cache_store("gfx950/new", u, 12.5f);
  CHECK(tune_cache_lookup("gfx950/new", &t) && t.wgs_per_cu == 3 && t.strip == 4);
  CHECK(tune_cache_lookup("gfx950/ok", &t) && t.wgs_per_cu == 8);
}

static void metrics() {
  // PSNR of planes and its mean over planes; +inf for an exact reconstruction.
  const uint64_t sse[6] = {0, 331776ull * 64 * 65025, 331776ull * 64, 5, 6, 7};
  const int32_t w[2] = {8, 16}, h[2] = {8, 4};
  double ps[6], mean[3];
  CHECK(rdct_psnr_planes(sse, 2, 3, RDCT_SEL_ZIGZAG, w, h, ps, mean) == RDCT_OK);
  CHECK(isinf(ps[0]) && fabs(ps[1]) < 1e-12 && fabs(ps[2] - 10 * log10(65025.0)) < 1e-12);
  CHECK(isinf(mean[0]) && fabs(mean[1] - 0.5 * (ps[1] + ps[4])) < 1e-12);
  CHECK(rdct_psnr_planes(sse, 2, 3, RDCT_SEL_ZIGZAG, w, h, ps, nullptr) == RDCT_OK);
  const int32_t bad_w[2] = {8, 0};
  CHECK(rdct_psnr_planes(sse, 2, 3, RDCT_SEL_ZIGZAG, bad_w, h, ps, mean) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_psnr_planes(sse, 2, 0, RDCT_SEL_ZIGZAG, w, h, ps, mean) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_psnr_planes(sse, 2, 3, 9, w, h, ps, mean) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_psnr_planes(sse, 0, 3, RDCT_SEL_QUANT, w, h, ps, mean) == RDCT_OK && isnan(mean[0]));
  // Quality metrics: units and window counts.
  const uint64_t qs[2] = {4096ull * 64, 0};
  const int64_t qu[2] = {(int64_t)1 << 32, -((int64_t)1 << 31)};
  double mse[2], uqi[2];
  CHECK(rdct_quality_metrics(qs, qu, 2, RDCT_T_SDCT, 8, 8, mse, uqi) == RDCT_OK);
  CHECK(mse[0] == 1.0 && mse[1] == 0.0 && uqi[0] == 1.0 && uqi[1] == -0.5);
  CHECK(rdct_quality_metrics(qs, qu, 2, RDCT_T_RDCT_FLOOR, 8, 8, mse, uqi) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_quality_metrics(qs, qu, 2, RDCT_T_DCT, 7, 8, mse, uqi) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_quality_metrics(nullptr, nullptr, 0, RDCT_T_DCT, 8, 8, nullptr, nullptr) == RDCT_OK);
  // Pair words.
  const int32_t words[3] = {(int32_t)((5u << 16) | 0xfffeu), (int32_t)(63u << 16 | 0x7fffu),
                            (int32_t)0x8000};
  int32_t runs[3], vals[3];
  CHECK(rdct_codec_unpack_pairs(words, 3, runs, vals) == RDCT_OK);
  CHECK(runs[0] == 5 && vals[0] == -2 && runs[1] == 63 && vals[1] == 32767 && runs[2] == 0 &&
        vals[2] == -32768);
  CHECK(rdct_codec_unpack_pairs(words, -1, runs, vals) == RDCT_ERR_INVALID_ARG);
  CHECK(rdct_num_blocks(INT32_MAX, 9) == (int64_t)(INT32_MAX / 8 + 1) * 2);
}

int main(int argc, char** argv) {
  arena_random(1, 1 << 16, 256);
  arena_random(2, 100000, 1);
  arena_random(3, 1 << 20, 4096);
  admission();
  work_lists();
  checks();
  metrics();
  if (argc > 1) tune_cache(argv[1]);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("host logic ok\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("host")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    res = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                          "-Wall", "-I", CSRC, str(src), os.path.join(CSRC, "rdct_tune.cpp"),
                          os.path.join(CSRC, "rdct_metrics.cpp"),
                          "-o", str(exe), "-lpthread"], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return str(exe)


def test_host_logic_under_sanitizers(driver, tmp_path):
    env = dict(os.environ, RDCT_TUNING_CACHE=str(tmp_path / "tune.json"),
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([driver, str(tmp_path / "tune.json")], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
    assert out.stdout.strip() == "host logic ok"


QUANT_RULE = r"""
#include <stdio.h>
#include <string.h>

#include "rdct_host.h"

// The kernels' quantiser: the low word of the float64 FMA y * m + 1.5 * 2^52.
static int fma_quant(int y, double m) {
  const double t = fma((double)y, m, 0x1.8p52);
  uint64_t b;
  memcpy(&b, &t, 8);
  return (int)(uint32_t)b;
}

// q = round(y / (Q sqrt(gk gl))), halves away from zero, in integers: for a
// rational quotient (gk == gl) from the remainder; otherwise j is the one value
// with (2j - 1)^2 Q^2 gk gl < 4 y^2 < (2j + 1)^2 Q^2 gk gl.
static long exact_quant(int y, int gk, int gl, int Q, long* ties) {
  const long ay = y < 0 ? -(long)y : (long)y;
  long j;
  if (gk == gl) {
    const long cq = (long)gk * Q;
    j = (2 * ay + cq) / (2 * cq);
    if ((2 * ay + cq) % (2 * cq) == 0) ++*ties;
  } else {
    const __int128 p = (__int128)Q * Q * gk * gl, v = (__int128)4 * ay * ay;
    j = 0;
    for (long step = 1L << 16; step; step >>= 1)
      if ((__int128)(2 * (j + step) - 1) * (2 * (j + step) - 1) * p < v) j += step;
    if ((__int128)(2 * j + 1) * (2 * j + 1) * p == v) return -1000000;  // a tie: impossible
  }
  return y < 0 ? -j : j;
}

int main() {
  static const int g[3] = {8, 6, 4};
  long checked = 0, ties = 0, bad = 0;
  for (int Q = 1; Q <= 255; ++Q)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double m = rdct::quant_multiplier(g[a], g[b], Q);
        for (int y = -16384; y <= 16384; ++y, ++checked)
          if (fma_quant(y, m) != exact_quant(y, g[a], g[b], Q, &ties)) {
            if (bad++ < 5) fprintf(stderr, "Q=%d g=(%d,%d) y=%d\n", Q, g[a], g[b], y);
          }
      }
  printf("%ld %ld %ld\n", checked, ties, bad);
  return bad != 0;
}
"""


def test_quantiser_rule_exhaustive(tmp_path):
    """The kernels' quantiser (one float64 FMA with the multiplier the library
    stores) against exact integer rounding, halves away from zero, of
    Y / (Q sqrt(g_k g_l)) (Section 3's quantisation of the orthogonal
    coefficients): every |Y| <= 2^14, every table entry 1..255, every pair of
    diagonal entries of C0 C0^T, ties included."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "quant.cpp"
    src.write_text(QUANT_RULE)
    exe = tmp_path / "quant"
    res = subprocess.run([gxx, "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-I", CSRC,
                          str(src), "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    checked, ties, bad = map(int, out.stdout.split())
    assert checked == 255 * 9 * 32769
    assert ties > 100000      # the rational positions' exact ties are exercised
    assert bad == 0
