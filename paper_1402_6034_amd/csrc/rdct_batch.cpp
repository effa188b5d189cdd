// Batch planner: many planes of uneven sizes in one persistent launch.
//
// A plan uploads, once, a device work list of 128-block items (plane, first
// block) grouped by plane, each plane's first item, the per-plane descriptors
// and the distinct quantisation tables.  Two layouts run the list:
//  * strided: a run zeroes the per-plane error sums with a small kernel and
//    launches the persistent kernel, whose waves stride over the whole list
//    and add their sums atomically;
//  * per plane: one workgroup per plane strides over that plane's items and
//    stores its sums -- one launch, no atomics, but the largest plane bounds
//    the run, so it suits batches of many similar planes.
// On request a run's launches are captured into a hipGraph and replayed.  Per-block arithmetic is the same
// device code as the single-plane calls, so every plane's outputs are identical
// whether it is processed alone or inside a batch.
//
// (Finishing the sums inside the persistent kernel instead -- a per-plane
// counter of finished items, the last wave copying the totals out -- needs an
// agent-scope release fence per wave, which writes back the XCD's L2; measured
// slower than the clearing launch: 124 us against 79 us for the 256-plane
// sweep, 1.42 ms against 1.31 ms for the ragged batch.)
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "rdct_internal.h"
#include "rdct_tables.h"
#include "rdct_tune.h"

using namespace rdct;

// A plan runs one or two groups of planes: quantisation plans score
// whole-block planes in the coefficient domain and planes with partial blocks
// pixel by pixel (the error kind rdct_compress_eval takes for each), so each
// plane's sum has the same bits alone and in any batch.  The device arrays
// hold group 0's planes, then group 1's; a work item's plane index counts from
// its group's first plane.
struct PlanGroup {
  int ev = EV_SPATIAL;
  int32_t plane0 = 0, n_planes = 0;  // descriptors plane0 .. plane0 + n_planes - 1
  int32_t item0 = 0, n_items = 0;    // work items item0 .. item0 + n_items - 1
};

struct rdct_batch_plan {
  int sel = SEL_ZZ, co = CO_NONE;
  bool recon = false;
  int32_t n_planes = 0, n_items = 0;
  int32_t r_count = 1;   // error sums per plane (a retention sweep when > 1)
  int64_t n_blocks = 0;
  int n_groups = 1;
  PlanGroup group[2];
  uint64_t* sse = nullptr;
  Plane* d_planes = nullptr;
  QuantConsts* d_tables = nullptr;
  WorkItem* d_items = nullptr;
  int32_t* d_first = nullptr;  // descriptor b's items: d_first[b] .. d_first[b + 1] - 1
  rdct_tuning_t tuning{};
  int device = 0;
  int n_cu = 256;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_ready = false;
  std::string key;
};

namespace {

void free_plan(rdct_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) {
    (void)hipStreamSynchronize(p->cap_stream);
    (void)hipStreamDestroy(p->cap_stream);
  }
  if (p->d_planes) (void)hipFree(p->d_planes);
  if (p->d_tables) (void)hipFree(p->d_tables);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_first) (void)hipFree(p->d_first);
  delete p;
}

int grid_of(const rdct_batch_plan* p, const PlanGroup& g, const rdct_tuning_t& t) {
  const int wpg = t.waves_per_wg;
  const int max_grid = (g.n_items + wpg - 1) / wpg;
  return std::max(1, std::min(p->n_cu * t.wgs_per_cu, max_grid));
}

hipError_t launch_direct(rdct_batch_plan* p, const rdct_tuning_t& t, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (t.layout != RDCT_LAYOUT_PER_PLANE) {
    e = launch_zero_u64(p->sse, (int64_t)p->n_planes * p->r_count, s);
    if (e != hipSuccess) return e;
  }
  for (int gi = 0; gi < p->n_groups; ++gi) {
    const PlanGroup& g = p->group[gi];
    if (t.layout == RDCT_LAYOUT_PER_PLANE) {
      // Each workgroup stores its plane's sums; items are indexed from the
      // whole list through the group's first-item entries.
      e = launch_batch(p->sel, p->co, p->recon, g.ev, p->d_planes + g.plane0, p->d_tables,
                       p->d_items, g.n_items, g.n_planes, t.waves_per_wg, s,
                       p->d_first + g.plane0);
    } else {
      e = launch_batch(p->sel, p->co, p->recon, g.ev, p->d_planes + g.plane0, p->d_tables,
                       p->d_items + g.item0, g.n_items, grid_of(p, g, t), t.waves_per_wg, s,
                       nullptr, t.xcd_ranges, t.strip);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

rdct_status_t capture(rdct_batch_plan* p) {
  if (p->exec) {
    (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  p->graph_ready = false;
  if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
    return RDCT_ERR_HIP;
  const hipError_t le = launch_direct(p, p->tuning, p->cap_stream);
  const hipError_t ce = hipStreamEndCapture(p->cap_stream, &p->graph);
  if (le != hipSuccess || ce != hipSuccess || !p->graph) return RDCT_ERR_HIP;
  if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
    return RDCT_ERR_HIP;
  p->graph_ready = true;
  return RDCT_OK;
}

std::string plan_key(const rdct_batch_plan* p) {
  // Size classes: log2 of the block count and of the plane count.
  int cls = 0, pcls = 0;
  for (int64_t b = p->n_blocks; b > 1; b >>= 1) ++cls;
  for (int64_t b = p->n_planes; b > 1; b >>= 1) ++pcls;
  char buf[128];
  const int ev = p->n_groups == 2 ? 10 * p->group[0].ev + p->group[1].ev : p->group[0].ev;
  snprintf(buf, sizeof(buf), "gfx950/batch/sel%d/co%d/recon%d/ev%d/log2blocks%d/log2planes%d",
           p->sel, p->co, p->recon ? 1 : 0, ev, cls, pcls);
  return buf;
}

rdct_status_t create_plan(const rdct_plane_desc_t* planes, int32_t n, rdct_coef_t coef_type,
                          uint64_t* sse_out, int32_t r_count, const rdct_tuning_t* tuning,
                          rdct_batch_plan_t** out) {
  if (!out) return RDCT_ERR_INVALID_ARG;
  *out = nullptr;
  if (!planes || n <= 0 || !sse_out || !aligned(sse_out, 8) || r_count < 1)
    return RDCT_ERR_INVALID_ARG;
  const bool want_coef = planes[0].coef_out != nullptr;
  const bool want_recon = planes[0].recon_out != nullptr;
  int co = CO_NONE;
  if (want_coef) {
    switch (coef_type) {
      case RDCT_COEF_I32: co = CO_I32; break;
      case RDCT_COEF_I16: co = CO_I16; break;
      case RDCT_COEF_F32: co = CO_F32; break;
      default: return RDCT_ERR_INVALID_ARG;
    }
  }
  // Validate every plane and collect descriptors.
  std::vector<Plane> hp(n);
  std::vector<QuantConsts> tables;
  std::map<std::vector<uint16_t>, int> table_index;
  int sel_kind = -1;
  std::vector<bool> coef_err(n, false);
  int64_t n_blocks = 0;
  for (int i = 0; i < n; ++i) {
    const rdct_plane_desc_t& d = planes[i];
    rdct_status_t st = check_plane(d.src, d.width, d.height, d.src_pitch, kMaxEvalBlocks);
    if (st != RDCT_OK) return st;
    SelInfo si;
    if ((st = check_sel(&d.sel, &si)) != RDCT_OK) return st;
    if (sel_kind < 0) sel_kind = si.sel;
    if (si.sel != sel_kind) return RDCT_ERR_INVALID_ARG;
    if ((d.coef_out != nullptr) != want_coef || (d.recon_out != nullptr) != want_recon)
      return RDCT_ERR_INVALID_ARG;
    if (want_coef && !aligned(d.coef_out, 16)) return RDCT_ERR_INVALID_ARG;
    if (want_recon && (d.recon_pitch < d.width || !aligned(d.recon_out, 4)))
      return RDCT_ERR_INVALID_ARG;
    if (si.sel == SEL_Q && co == CO_F32) return RDCT_ERR_INVALID_ARG;
    if (r_count > 1) {
      // A sweep scores r = sel.r .. sel.r + r_count - 1 of the zig-zag selection
      // from coefficient energies, which needs planes made of whole blocks.
      if (si.sel != SEL_ZZ || d.sel.mode != RDCT_SEL_ZIGZAG || si.r + r_count - 1 > 64)
        return RDCT_ERR_INVALID_ARG;
      if ((d.width % 8) != 0 || (d.height % 8) != 0) return RDCT_ERR_UNSUPPORTED;
    }
    Plane P = make_plane(d.src, d.width, d.height, d.src_pitch);
    P.coef = d.coef_out;
    P.recon = d.recon_out;
    P.rpitch = d.recon_pitch;
    P.sse = sse_out + (int64_t)i * r_count;
    P.r = si.r;
    P.keep = keep_bits(si.r);
    P.r_count = r_count;
    P.shift = si.shift;
    P.table = 0;
    if (si.sel == SEL_Q) {
      std::vector<uint16_t> key(si.q, si.q + 64);
      auto it = table_index.find(key);
      if (it == table_index.end()) {
        it = table_index.emplace(key, (int)tables.size()).first;
        tables.push_back(si.qc);
      }
      P.table = it->second;
    }
    coef_err[i] = si.sel == SEL_Q && r_count == 1 && whole_blocks(d.width, d.height);
    hp[i] = P;
    n_blocks += P.nblocks;
  }
  if (tables.empty()) {
    tables.emplace_back();
    memset(&tables[0], 0, sizeof(QuantConsts));
  }

  // Groups (see PlanGroup) and the device order of the descriptors.
  std::vector<int> order;
  const int n_coef = flagged_first(coef_err, &order);
  PlanGroup groups[2];
  int n_groups = 0;
  if (n_coef > 0) {
    groups[n_groups].ev = EV_COEF;
    groups[n_groups].plane0 = 0;
    groups[n_groups].n_planes = n_coef;
    ++n_groups;
  }
  if (n_coef < n) {
    groups[n_groups].ev = r_count > 1 ? EV_SWEEP : EV_SPATIAL;
    groups[n_groups].plane0 = n_coef;
    groups[n_groups].n_planes = n - n_coef;
    ++n_groups;
  }
  std::vector<Plane> dev_planes(n);
  std::vector<WorkItem> items;
  std::vector<int32_t> first(n + 1, 0);
  for (int gi = 0; gi < n_groups; ++gi) {
    PlanGroup& g = groups[gi];
    std::vector<int64_t> nb(g.n_planes);
    for (int j = 0; j < g.n_planes; ++j) {
      dev_planes[g.plane0 + j] = hp[order[g.plane0 + j]];
      nb[j] = dev_planes[g.plane0 + j].nblocks;
    }
    std::vector<WorkItem> gitems;
    std::vector<int32_t> gfirst;
    if (!build_work_list(nb.data(), g.n_planes, &gitems, &gfirst) ||
        items.size() + gitems.size() > (size_t)INT32_MAX)
      return RDCT_ERR_UNSUPPORTED;
    g.item0 = (int32_t)items.size();
    g.n_items = (int32_t)gitems.size();
    for (int j = 0; j <= g.n_planes; ++j) first[g.plane0 + j] = g.item0 + gfirst[j];
    items.insert(items.end(), gitems.begin(), gitems.end());
  }

  rdct_batch_plan* p = new rdct_batch_plan();
  p->sel = sel_kind;
  p->co = co;
  p->recon = want_recon;
  p->n_groups = n_groups;
  for (int gi = 0; gi < n_groups; ++gi) p->group[gi] = groups[gi];
  p->r_count = r_count;
  p->n_planes = n;
  p->n_items = (int32_t)items.size();
  p->n_blocks = n_blocks;
  p->sse = sse_out;
  p->n_cu = device_cu_count();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return RDCT_ERR_HIP;
  }
  p->key = plan_key(p);

  // Geometry, decided before anything is allocated: explicit fields > tuning
  // cache > default.  A cache entry that is not a valid geometry is ignored.
  rdct_tuning_t t{};
  t.waves_per_wg = 1;
  t.wgs_per_cu = 8;
  // Plain launches by default: replaying a graph measured slower here (70.4 against
  // 64.7 us per run of the 256-plane sweep), and a replay followed by a copy to
  // the host on the same stream stalled (537 against 81 us per run and copy).
  t.use_graph = 0;
  t.layout = RDCT_LAYOUT_STRIDED;
  // Each XCD takes a contiguous range of items: neighbouring items share an L2,
  // so boundary lines are read once (the ragged batch reads 1.05x its planes
  // this way against 1.18x in the hardware's order, at the same or better speed).
  t.xcd_ranges = 1;
  t.strip = 1;
  rdct_tuning_t cached;
  if (tune_cache_lookup(p->key, &cached)) {
    rdct_tuning_t c = t;
    c.waves_per_wg = cached.waves_per_wg;
    c.wgs_per_cu = cached.wgs_per_cu;
    c.layout = cached.layout;
    c.xcd_ranges = cached.xcd_ranges;
    c.strip = cached.strip;
    if (valid_tuning(c)) t = c;
  }
  if (tuning) {
    if (tuning->waves_per_wg) t.waves_per_wg = tuning->waves_per_wg;
    if (tuning->wgs_per_cu) t.wgs_per_cu = tuning->wgs_per_cu;
    if (tuning->layout) t.layout = tuning->layout;
    t.use_graph = tuning->use_graph ? 1 : 0;
    t.xcd_ranges = tuning->xcd_ranges;
    if (tuning->strip) t.strip = tuning->strip;
  }
  if (!valid_tuning(t)) {
    delete p;
    return RDCT_ERR_INVALID_ARG;
  }

  bool ok = hipMalloc(&p->d_planes, sizeof(Plane) * n) == hipSuccess &&
            hipMalloc(&p->d_tables, sizeof(QuantConsts) * tables.size()) == hipSuccess &&
            hipMalloc(&p->d_items, sizeof(WorkItem) * std::max<size_t>(items.size(), 1)) ==
                hipSuccess &&
            hipMalloc(&p->d_first, sizeof(int32_t) * (n + 1)) == hipSuccess;
  if (!ok) {
    free_plan(p);
    return RDCT_ERR_NO_MEMORY;
  }
  ok = hipMemcpy(p->d_planes, dev_planes.data(), sizeof(Plane) * n, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_tables, tables.data(), sizeof(QuantConsts) * tables.size(),
                 hipMemcpyHostToDevice) == hipSuccess &&
       (items.empty() || hipMemcpy(p->d_items, items.data(), sizeof(WorkItem) * items.size(),
                                   hipMemcpyHostToDevice) == hipSuccess) &&
       hipMemcpy(p->d_first, first.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    free_plan(p);
    return RDCT_ERR_HIP;
  }

  p->tuning = t;
  *out = p;
  return RDCT_OK;
}

}  // namespace

// Median time (us per run) of each candidate geometry on this plan.  Each
// candidate gets one untimed launch, then kRounds rounds; a round queues `reps`
// launches of every candidate in turn, back to back with no synchronisation in
// between (as runs follow each other in use), an event before and after each
// candidate's launches, and waits once at its end.  A drift of the clock or
// temperature during the search thus weighs on every candidate alike, the GPU
// never idles between candidates, and a candidate's median round decides.
// Timing single launches between synchronisations ranked the ragged batch's
// geometries differently from back-to-back runs (1.35 against 1.31 ms for the
// pick), and so did short rounds that each began after a synchronisation.
// Invalid candidates are dropped from `cands` first.
static rdct_status_t time_candidates(rdct_batch_plan* plan, std::vector<rdct_tuning_t>& cands,
                                     int reps, hipStream_t s, std::vector<float>* med) {
  cands.erase(std::remove_if(cands.begin(), cands.end(),
                             [](const rdct_tuning_t& t) { return !valid_tuning(t); }),
              cands.end());
  if (cands.empty()) return RDCT_ERR_INVALID_ARG;
  constexpr int kRounds = 5;
  const size_t nc = cands.size();
  std::vector<hipEvent_t> ev(nc + 1, nullptr);
  std::vector<std::vector<float>> us(nc);
  rdct_status_t st = RDCT_OK;
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = RDCT_ERR_HIP;
  for (size_t c = 0; c < nc && st == RDCT_OK; ++c)
    if (launch_direct(plan, cands[c], s) != hipSuccess) st = RDCT_ERR_HIP;
  for (int round = 0; round < kRounds && st == RDCT_OK; ++round) {
    bool ok = hipEventRecord(ev[0], s) == hipSuccess;
    for (size_t c = 0; c < nc && ok; ++c) {
      for (int r = 0; r < reps && ok; ++r) ok = launch_direct(plan, cands[c], s) == hipSuccess;
      ok = ok && hipEventRecord(ev[c + 1], s) == hipSuccess;
    }
    ok = ok && hipEventSynchronize(ev[nc]) == hipSuccess;
    for (size_t c = 0; c < nc && ok; ++c) {
      float ms = 0.f;
      ok = hipEventElapsedTime(&ms, ev[c], ev[c + 1]) == hipSuccess;
      us[c].push_back(ms * 1000.f / reps);
    }
    if (!ok) st = RDCT_ERR_HIP;
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != RDCT_OK) return st;
  med->assign(nc, 0.f);
  for (size_t c = 0; c < nc; ++c) {
    std::sort(us[c].begin(), us[c].end());
    (*med)[c] = us[c][us[c].size() / 2];
  }
  return RDCT_OK;
}

extern "C" {

rdct_status_t rdct_batch_plan_create(const rdct_plane_desc_t* planes, int32_t n,
                                     rdct_coef_t coef_type, uint64_t* sse_out,
                                     const rdct_tuning_t* tuning, rdct_batch_plan_t** out) {
  return create_plan(planes, n, coef_type, sse_out, 1, tuning, out);
}

rdct_status_t rdct_batch_plan_create_sweep(const rdct_plane_desc_t* planes, int32_t n,
                                           int32_t r_count, rdct_coef_t coef_type,
                                           uint64_t* sse_out, const rdct_tuning_t* tuning,
                                           rdct_batch_plan_t** out) {
  return create_plan(planes, n, coef_type, sse_out, r_count, tuning, out);
}

rdct_status_t rdct_batch_run(rdct_batch_plan_t* plan, void* stream) {
  if (!plan) return RDCT_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!plan->tuning.use_graph)
    return launch_direct(plan, plan->tuning, s) == hipSuccess ? RDCT_OK : RDCT_ERR_HIP;
  if (!plan->graph_ready) {
    const rdct_status_t st = capture(plan);
    if (st != RDCT_OK) return st;
  }
  return hipGraphLaunch(plan->exec, s) == hipSuccess ? RDCT_OK : RDCT_ERR_HIP;
}

rdct_status_t rdct_batch_plan_set_tuning(rdct_batch_plan_t* plan, const rdct_tuning_t* tuning) {
  if (!plan || !tuning) return RDCT_ERR_INVALID_ARG;
  rdct_tuning_t t = *tuning;
  if (t.strip == 0) t.strip = 1;   // the field added last: 0 reads as one item
  if (!valid_tuning(t)) return RDCT_ERR_INVALID_ARG;
  t.use_graph = t.use_graph ? 1 : 0;
  plan->tuning = t;
  plan->graph_ready = false;  // re-captured on the next run when use_graph
  return RDCT_OK;
}

rdct_status_t rdct_batch_plan_info(const rdct_batch_plan_t* plan, int64_t* n_blocks,
                                   int32_t* n_items, rdct_tuning_t* used) {
  if (!plan) return RDCT_ERR_INVALID_ARG;
  if (n_blocks) *n_blocks = plan->n_blocks;
  if (n_items) *n_items = plan->n_items;
  if (used) *used = plan->tuning;
  return RDCT_OK;
}

rdct_status_t rdct_batch_autotune(rdct_batch_plan_t* plan, int32_t reps, void* stream,
                                  rdct_tuning_t* best) {
  if (!plan || reps < 1 || reps > 1000) return RDCT_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  // Stage 1, the geometry: the strided layout (in the XCD-range order, which
  // reads fewer bytes and measured as fast or faster at every geometry from 4
  // resident waves per CU up; one item per strip) over waves per workgroup x
  // resident waves per CU, and the per-plane layout over waves per workgroup.
  std::vector<rdct_tuning_t> cands;
  for (int wpg : {1, 2, 4}) {
    for (int waves : {2, 4, 8, 12, 16}) {
      if (waves % wpg) continue;
      rdct_tuning_t t = plan->tuning;
      t.layout = RDCT_LAYOUT_STRIDED;
      t.waves_per_wg = wpg;
      t.wgs_per_cu = waves / wpg;
      t.xcd_ranges = 1;
      t.strip = 1;
      cands.push_back(t);
    }
    rdct_tuning_t t = plan->tuning;
    t.layout = RDCT_LAYOUT_PER_PLANE;
    t.waves_per_wg = wpg;
    t.wgs_per_cu = 1;
    t.xcd_ranges = 0;
    t.strip = 1;
    cands.push_back(t);
  }
  std::vector<float> med;
  rdct_status_t st = time_candidates(plan, cands, reps, s, &med);
  if (st != RDCT_OK) return st;
  const float fastest = *std::min_element(med.begin(), med.end());
  // Among the candidates within 2% of the fastest, the fewest resident waves
  // per CU (then the faster).  On the ragged batch the geometries from 4 to 16
  // resident waves land within 2-3% of each other in such short rounds, in an
  // order that changed from run to run, while runs of hundreds of plans at a
  // time measured 1 x 4 at 1.30-1.31 ms against 1.33-1.35 ms for 4 x 3 or
  // 1 x 12.
  float best_us = 1e30f;
  int best_waves = 1 << 30;
  rdct_tuning_t best_t = plan->tuning;
  for (size_t c = 0; c < cands.size(); ++c) {
    if (med[c] > fastest * 1.02f) continue;
    // Resident waves per CU: the strided grid holds wgs_per_cu workgroups per
    // CU; the per-plane grid one workgroup per plane.
    const int64_t cus = std::max(plan->n_cu, 1);
    const int waves =
        cands[c].layout == RDCT_LAYOUT_PER_PLANE
            ? (int)std::min<int64_t>((plan->n_planes * cands[c].waves_per_wg + cus - 1) / cus, 1 << 20)
            : cands[c].waves_per_wg * cands[c].wgs_per_cu;
    if (waves < best_waves || (waves == best_waves && med[c] < best_us)) {
      best_waves = waves;
      best_us = med[c];
      best_t = cands[c];
    }
  }
  // Stage 2, the strip of the strided pick: consecutive items per wave.  Two
  // took the ragged batch from 1.305 to 1.260 ms (a wave writes longer runs of
  // neighbouring output), although its reads rose from 1.05x to 1.14x the
  // planes.
  if (best_t.layout == RDCT_LAYOUT_STRIDED) {
    std::vector<rdct_tuning_t> strips;
    for (int strip : {1, 2, 4, 8}) {
      rdct_tuning_t t = best_t;
      t.strip = strip;
      strips.push_back(t);
    }
    if ((st = time_candidates(plan, strips, reps, s, &med)) != RDCT_OK) return st;
    const size_t k = std::min_element(med.begin(), med.end()) - med.begin();
    best_t = strips[k];
    best_us = med[k];
  }
  plan->tuning = best_t;
  plan->graph_ready = false;  // re-captured on the next run
  tune_cache_store(plan->key, best_t, best_us);
  if (best) *best = best_t;
  return RDCT_OK;
}

void rdct_batch_plan_destroy(rdct_batch_plan_t* plan) { free_plan(plan); }

}  // extern "C"
