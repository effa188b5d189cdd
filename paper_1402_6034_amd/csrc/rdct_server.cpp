// Compression server: requests of mixed resolutions are admitted against a
// device-memory budget and scored in batches that run while new requests keep
// arriving (continuous batching).
//
// Submit copies a request's planes into pinned host staging and queues it.  One
// scheduler thread (a) retires launched batches whose event has fired, turning
// their error sums into completions and freeing their memory, and (b) whenever a
// stream is free, forms the next batch from the oldest pending requests that fit
// in the device budget, and launches it: plane uploads, the descriptor upload,
// the zeroing kernel, the persistent batch kernel(s) and the read-back of the
// error sums, all asynchronous on that stream, followed by the stream's event.
// Batches on different streams overlap on the device.  The per-block arithmetic
// is the same device code as the single-plane calls, and every plane is scored
// with the error kind the single-plane call takes for it, so results do not
// depend on what a request was batched with.
//
// Device memory: the budget holds 256 bytes for the plain path's error sum,
// one fixed metadata region per stream (descriptors, tables, work items and
// sums of the batch in flight on that stream) and the plane arena.  Pinned host
// memory: the staging arena for submitted planes and one metadata mirror per
// stream.  A request is refused at submit if it could not run alone (its planes
// larger than the plane arena or the staging, or its metadata larger than a
// region), so the oldest pending request can always start once nothing else is
// in flight.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rdct_internal.h"
#include "rdct_tables.h"

using namespace rdct;

namespace {

struct PlaneSlot {
  int32_t w = 0, h = 0;
  int64_t host_off = -1;  // staging (tightly packed rows)
  int64_t dev_off = -1;   // device copy
  int64_t bytes = 0;
};

struct Request {
  uint64_t ticket = 0, tag = 0;
  int n = 0;
  PlaneSlot p[3];
  int sel = SEL_ZZ, mode = RDCT_SEL_ZIGZAG, r = 64, shift = 0;
  uint16_t q[64];
  double t_submit = 0, t_launch = 0;
};

struct Batch {
  std::vector<Request> reqs;
  int stream = 0;                         // its metadata region is the stream's
  int n_planes = 0;
  int64_t n_blocks = 0;
  double t_launch = 0;
};

int64_t plane_dev_bytes(int w, int h) { return (int64_t)w * h; }

}  // namespace

struct rdct_server {
  rdct_server_cfg_t cfg{};
  int device = 0;
  int n_cu = 256;
  uint8_t* dev_base = nullptr;    // budget_bytes of device memory
  uint8_t* host_base = nullptr;   // staging_bytes of pinned host memory
  uint8_t* host_meta = nullptr;   // n_streams metadata mirrors, pinned
  int64_t meta_cap = 0;           // bytes of one stream's metadata region
  int64_t plane_base = 0;         // offset of the plane arena in dev_base
  Arena dev, host;                // plane arena (offsets from plane_base), staging
  hipStream_t streams[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t events[4] = {nullptr, nullptr, nullptr, nullptr};
  bool stream_busy[4] = {false, false, false, false};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> pending;
  std::deque<Batch> inflight;
  std::deque<rdct_completion_t> done;
  std::atomic<bool> stop{false};
  std::thread worker;
  uint64_t next_ticket = 1;
  rdct_server_stats_t st{};
  int64_t inflight_reqs = 0;
  std::chrono::steady_clock::time_point t0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }
  uint8_t* dev_meta(int stream) const { return dev_base + 256 + (int64_t)stream * meta_cap; }
  uint8_t* host_meta_of(int stream) const { return host_meta + (int64_t)stream * meta_cap; }
  uint8_t* plane_ptr(const PlaneSlot& p) const { return dev_base + plane_base + p.dev_off; }
};

namespace {

const MetaSizes kMetaSizes = {(int64_t)sizeof(Plane), (int64_t)sizeof(QuantConsts),
                              (int64_t)sizeof(WorkItem)};

// Bytes of one stream's metadata region: a sixteenth of the budget, between
// 64 KiB and 4 MiB (4 MiB holds half a million work items, or 64 M blocks).
int64_t meta_region_bytes(int64_t budget) {
  const int64_t m = std::min<int64_t>(4 << 20, std::max<int64_t>(64 << 10, budget / 16));
  return m / 256 * 256;
}

AdmitRequest admit_view(const Request& r) {
  AdmitRequest a;
  a.kind = r.sel;
  a.n = r.n;
  a.items = 0;
  for (int i = 0; i < 3; ++i) a.bytes[i] = i < r.n ? r.p[i].bytes : 0;
  for (int i = 0; i < r.n; ++i) a.items += items_of(blocks_of(r.p[i].w, r.p[i].h));
  return a;
}

void complete(rdct_server* s, const Request& r, int status, const uint64_t* sse, double t_done,
              int batch_planes) {
  rdct_completion_t c;
  memset(&c, 0, sizeof(c));
  c.ticket = r.ticket;
  c.user_tag = r.tag;
  c.status = status;
  c.n_planes = r.n;
  for (int i = 0; i < r.n; ++i) {
    c.sse[i] = sse ? sse[i] : 0;
    c.psnr[i] = sse ? rdct_psnr(sse[i], r.mode, r.p[i].w, r.p[i].h) : 0.0;
  }
  c.t_submit_us = r.t_submit;
  c.t_launch_us = r.t_launch;
  c.t_done_us = t_done;
  c.batch_planes = batch_planes;
  s->done.push_back(c);
}

void release_request(rdct_server* s, const Request& r) {
  for (int i = 0; i < r.n; ++i) {
    if (r.p[i].host_off >= 0) s->host.release(r.p[i].host_off, r.p[i].bytes);
    if (r.p[i].dev_off >= 0) s->dev.release(r.p[i].dev_off, r.p[i].bytes);
  }
}

// Offsets of the sections of a batch's metadata block (same on host and device).
struct MetaLayout {
  int64_t planes, tables, items, sse, end;
};

MetaLayout meta_layout(int64_t n_planes, int64_t n_tables, int64_t n_items) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  MetaLayout m;
  m.planes = 0;
  m.tables = up(m.planes + (int64_t)sizeof(Plane) * n_planes);
  m.items = up(m.tables + (int64_t)sizeof(QuantConsts) * std::max<int64_t>(1, n_tables));
  m.sse = up(m.items + (int64_t)sizeof(WorkItem) * n_items);
  m.end = up(m.sse + 8 * n_planes);
  return m;
}

// Offset of the error sums in the metadata block of a batch (kept for retiring it).
int64_t batch_sse_offset(const Batch& b) {
  int64_t items = 0;
  for (const Request& r : b.reqs) items += admit_view(r).items;
  return meta_layout(b.n_planes, (int64_t)b.reqs.size(), items).sse;
}

// Launch one batch on stream b.stream.  Called with the lock held.
hipError_t launch(rdct_server* s, Batch& b) {
  hipStream_t st = s->streams[b.stream];
  // Distinct quantisation tables of the batch.
  std::vector<std::vector<uint16_t>> tables;
  std::vector<int> table_of;
  for (const Request& r : b.reqs) {
    int t = 0;
    if (r.sel == SEL_Q) {
      std::vector<uint16_t> key(r.q, r.q + 64);
      auto it = std::find(tables.begin(), tables.end(), key);
      t = (int)(it - tables.begin());
      if (it == tables.end()) tables.push_back(key);
    }
    table_of.push_back(t);
  }
  int64_t n_items = 0;
  for (const Request& r : b.reqs) n_items += admit_view(r).items;
  // Admission counted one table per request, so the block fits the region.
  const MetaLayout ml = meta_layout(b.n_planes, (int64_t)b.reqs.size(), n_items);
  uint8_t* hb = s->host_meta_of(b.stream);
  uint8_t* db = s->dev_meta(b.stream);
  Plane* hp = reinterpret_cast<Plane*>(hb + ml.planes);
  QuantConsts* ht = reinterpret_cast<QuantConsts*>(hb + ml.tables);
  WorkItem* hi = reinterpret_cast<WorkItem*>(hb + ml.items);
  uint64_t* dsse = reinterpret_cast<uint64_t*>(db + ml.sse);
  for (size_t t = 0; t < tables.size(); ++t) fill_quant_consts(tables[t].data(), &ht[t]);
  if (tables.empty()) memset(ht, 0, sizeof(QuantConsts));

  // Descriptors in request order; quantisation scores whole-block planes in the
  // coefficient domain (as rdct_compress_eval does), the others pixel by pixel.
  std::vector<Plane> planes;
  std::vector<bool> coef_err;
  for (size_t ri = 0; ri < b.reqs.size(); ++ri) {
    const Request& r = b.reqs[ri];
    for (int i = 0; i < r.n; ++i) {
      const PlaneSlot& p = r.p[i];
      hipError_t e = hipMemcpyAsync(s->plane_ptr(p), s->host_base + p.host_off, (size_t)p.bytes,
                                    hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return e;
      Plane P = make_plane(s->plane_ptr(p), p.w, p.h, p.w);
      P.sse = dsse + planes.size();
      P.r = r.r;
      P.keep = keep_bits(r.r);
      P.r_count = 1;
      P.shift = r.shift;
      P.table = table_of[ri];
      planes.push_back(P);
      coef_err.push_back(r.sel == SEL_Q && whole_blocks(p.w, p.h));
      b.n_blocks += P.nblocks;
    }
  }
  std::vector<int> order;
  const int n_coef = flagged_first(coef_err, &order);
  const int n = (int)planes.size();
  int64_t it = 0;
  int64_t item0[2] = {0, 0}, count[2] = {0, 0};
  for (int j = 0; j < n; ++j) {
    const int g = j < n_coef ? 0 : 1;
    const int rel = g == 0 ? j : j - n_coef;
    if (j == n_coef) item0[1] = it;
    hp[j] = planes[order[j]];
    for (int t0 = 0; t0 < hp[j].nblocks; t0 += kItemBlocks) {
      hi[it++] = WorkItem{rel, t0};
      ++count[g];
    }
  }
  if (n_coef == n) item0[1] = it;
  hipError_t e = hipMemcpyAsync(db, hb, (size_t)ml.sse, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  if ((e = launch_zero_u64(dsse, b.n_planes, st)) != hipSuccess) return e;
  const int sel = b.reqs[0].sel;
  const int wpg = 4;
  const int evs[2] = {EV_COEF, EV_SPATIAL};
  const int p0[2] = {0, n_coef};
  for (int g = 0; g < 2; ++g) {
    if (count[g] == 0) continue;
    const int grid = (int)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)s->n_cu * 2, (count[g] + wpg - 1) / wpg));
    e = launch_batch(sel, CO_NONE, false, evs[g], reinterpret_cast<Plane*>(db + ml.planes) + p0[g],
                     reinterpret_cast<QuantConsts*>(db + ml.tables),
                     reinterpret_cast<WorkItem*>(db + ml.items) + item0[g], (int32_t)count[g], grid,
                     wpg, st);
    if (e != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(hb + ml.sse, dsse, 8 * (size_t)b.n_planes, hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return e;
  return hipEventRecord(s->events[b.stream], st);
}

// Plain path: one plane at a time, synchronously (upload, single-plane launch,
// read back).  Called without the lock.
void run_plain(rdct_server* s, Request& r) {
  hipStream_t st = s->streams[0];
  uint64_t sse[3] = {0, 0, 0};
  int status = RDCT_OK;
  uint64_t* dsse = reinterpret_cast<uint64_t*>(s->dev_base);  // first 256 bytes are reserved
  for (int i = 0; i < r.n && status == RDCT_OK; ++i) {
    const PlaneSlot& p = r.p[i];
    uint8_t* dp = s->plane_ptr(p);
    if (hipMemcpyAsync(dp, s->host_base + p.host_off, (size_t)p.bytes, hipMemcpyHostToDevice, st) !=
        hipSuccess) {
      status = RDCT_ERR_HIP;
      break;
    }
    rdct_select_t sel{};
    sel.mode = r.mode;
    sel.r = r.r;
    sel.quality = 50;
    sel.level_shift = r.shift;
    sel.qtable = r.q;
    if (rdct_compress_eval(dp, p.w, p.h, p.w, &sel, 1, nullptr, RDCT_COEF_I32, nullptr, 0, dsse, st) !=
            RDCT_OK ||
        hipMemcpyAsync(&sse[i], dsse, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      status = RDCT_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  const double t = s->now_us();
  complete(s, r, status, status == RDCT_OK ? sse : nullptr, t, 1);
  release_request(s, r);
  s->st.completed++;
  s->st.planes += r.n;
  s->st.batches += r.n;
  s->inflight_reqs--;
  s->cv_done.notify_all();
}

// Form and launch the next batch on a free stream.  Returns true if the
// pending queue changed (a batch launched or a request failed).
bool form_batch(rdct_server* s, int free_stream) {
  const int n_view = (int)std::min<size_t>(s->pending.size(), (size_t)s->cfg.max_batch_planes);
  std::vector<AdmitRequest> view(n_view);
  for (int i = 0; i < n_view; ++i) view[i] = admit_view(s->pending[i]);
  AdmitLimits lim;
  lim.max_planes = s->cfg.max_batch_planes;
  lim.max_requests = std::max<int64_t>(0, s->cfg.max_inflight - s->inflight_reqs);
  lim.meta_cap = s->meta_cap;
  lim.sizes = kMetaSizes;
  std::vector<int64_t[3]> offs(std::max(1, n_view));
  const int k = admit_batch(view.data(), n_view, &s->dev, lim, offs.data());
  if (k == 0) {
    if (!s->inflight.empty() || lim.max_requests == 0) return false;  // wait for room
    // Nothing in flight and still no room: the submit checks make this
    // unreachable; fail the request rather than retry it forever.
    Request r = s->pending.front();
    s->pending.pop_front();
    release_request(s, r);
    complete(s, r, RDCT_ERR_BUDGET, nullptr, s->now_us(), 0);
    s->st.completed++;
    s->cv_done.notify_all();
    return true;
  }
  Batch b;
  b.stream = free_stream;
  for (int i = 0; i < k; ++i) {
    Request r = s->pending.front();
    s->pending.pop_front();
    for (int p = 0; p < r.n; ++p) r.p[p].dev_off = offs[i][p];
    b.n_planes += r.n;
    b.reqs.push_back(r);
  }
  b.t_launch = s->now_us();
  for (Request& r : b.reqs) r.t_launch = b.t_launch;
  const hipError_t e = launch(s, b);
  s->st.batches++;
  s->st.planes += b.n_planes;
  s->st.blocks += b.n_blocks;
  if (e != hipSuccess) {
    // The event was not recorded: complete with an error now.  Work already
    // queued on the stream is waited for before the planes are reused.
    (void)hipStreamSynchronize(s->streams[b.stream]);
    for (Request& r : b.reqs) {
      complete(s, r, RDCT_ERR_HIP, nullptr, s->now_us(), b.n_planes);
      release_request(s, r);
      s->st.completed++;
    }
    s->cv_done.notify_all();
  } else {
    s->stream_busy[b.stream] = true;
    s->inflight_reqs += (int64_t)b.reqs.size();
    s->inflight.push_back(std::move(b));
  }
  return true;
}

void worker_main(rdct_server* s) {
  const bool device_ok = hipSetDevice(s->device) == hipSuccess;
  std::unique_lock<std::mutex> lk(s->mu);
  if (!device_ok) {
    // This thread cannot reach the device: every request completes with an error.
    for (;;) {
      while (!s->pending.empty()) {
        Request r = s->pending.front();
        s->pending.pop_front();
        release_request(s, r);
        complete(s, r, RDCT_ERR_HIP, nullptr, s->now_us(), 0);
        s->st.completed++;
      }
      s->cv_done.notify_all();
      if (s->stop) return;
      s->cv_work.wait(lk, [&] { return s->stop.load() || !s->pending.empty(); });
    }
  }
  for (;;) {
    // Retire finished batches.
    for (auto bi = s->inflight.begin(); bi != s->inflight.end();) {
      const hipError_t q = hipEventQuery(s->events[bi->stream]);
      if (q == hipErrorNotReady) {
        ++bi;
        continue;
      }
      const double t = s->now_us();
      const int status = q == hipSuccess ? RDCT_OK : RDCT_ERR_HIP;
      const uint64_t* sums =
          status == RDCT_OK
              ? reinterpret_cast<const uint64_t*>(s->host_meta_of(bi->stream) + batch_sse_offset(*bi))
              : nullptr;
      int k = 0;
      for (Request& r : bi->reqs) {
        complete(s, r, status, sums ? sums + k : nullptr, t, bi->n_planes);
        k += r.n;
        release_request(s, r);
        s->inflight_reqs--;
        s->st.completed++;
      }
      s->stream_busy[bi->stream] = false;
      bi = s->inflight.erase(bi);
      s->cv_done.notify_all();
    }
    if (s->stop && s->inflight.empty()) break;

    bool progressed = false;
    if (!s->stop && !s->pending.empty()) {
      if (s->cfg.plain) {
        Request r = s->pending.front();
        s->pending.pop_front();
        // Device copy of the planes: nothing else holds the arena in this mode
        // and submit checked that the planes fit it.
        bool ok = true;
        for (int i = 0; i < r.n && ok; ++i) {
          r.p[i].dev_off = s->dev.alloc(r.p[i].bytes);
          ok = r.p[i].dev_off >= 0;
        }
        if (!ok) {
          release_request(s, r);
          complete(s, r, RDCT_ERR_BUDGET, nullptr, s->now_us(), 0);
          s->st.completed++;
          s->cv_done.notify_all();
          continue;
        }
        r.t_launch = s->now_us();
        s->inflight_reqs++;
        lk.unlock();
        run_plain(s, r);
        lk.lock();
        continue;
      }
      int free_stream = -1;
      for (int i = 0; i < s->cfg.n_streams; ++i)
        if (!s->stream_busy[i]) {
          free_stream = i;
          break;
        }
      if (free_stream >= 0) progressed = form_batch(s, free_stream);
    }
    s->st.peak_device_bytes = std::max(s->st.peak_device_bytes, s->dev.in_use());
    if (progressed) continue;
    if (s->inflight.empty()) {
      s->cv_work.wait(lk, [&] { return s->stop.load() || !s->pending.empty(); });
    } else {
      // Batches in flight: poll their events again at once.  A timed wait
      // sleeps for at least the kernel's timer slack (tens of microseconds),
      // which every request in flight would wait on; yielding only gives the
      // core to other runnable threads (submitters, pollers).
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

void destroy(rdct_server* s) {
  if (!s) return;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      for (const Request& r : s->pending) release_request(s, r);
      s->pending.clear();
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  for (int i = 0; i < 4; ++i) {
    if (s->streams[i]) {
      (void)hipStreamSynchronize(s->streams[i]);
      (void)hipStreamDestroy(s->streams[i]);
    }
    if (s->events[i]) (void)hipEventDestroy(s->events[i]);
  }
  if (s->dev_base) (void)hipFree(s->dev_base);
  if (s->host_base) (void)hipHostFree(s->host_base);
  if (s->host_meta) (void)hipHostFree(s->host_meta);
  delete s;
}

}  // namespace

extern "C" {

rdct_status_t rdct_server_create(const rdct_server_cfg_t* cfg, rdct_server_t** out) {
  if (!cfg || !out || cfg->budget_bytes < (1 << 20)) return RDCT_ERR_INVALID_ARG;
  if (cfg->n_streams < 0 || cfg->n_streams > 4 || cfg->max_inflight < 0 || cfg->max_batch_planes < 0 ||
      cfg->staging_bytes < 0)
    return RDCT_ERR_INVALID_ARG;
  *out = nullptr;
  rdct_server* s = new rdct_server();
  s->cfg = *cfg;
  if (!s->cfg.n_streams) s->cfg.n_streams = 2;
  if (!s->cfg.max_inflight) s->cfg.max_inflight = 4096;
  if (!s->cfg.max_batch_planes) s->cfg.max_batch_planes = 4096;
  if (!s->cfg.staging_bytes) s->cfg.staging_bytes = std::min<int64_t>(cfg->budget_bytes / 4, 2ll << 30);
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return RDCT_ERR_HIP;
  }
  s->n_cu = device_cu_count();
  s->meta_cap = meta_region_bytes(s->cfg.budget_bytes);
  s->plane_base = 256 + (int64_t)s->cfg.n_streams * s->meta_cap;
  // The first 256 bytes of the device budget hold the plain path's error sum.
  if (hipMalloc(&s->dev_base, (size_t)s->cfg.budget_bytes) != hipSuccess ||
      hipHostMalloc(&s->host_base, (size_t)s->cfg.staging_bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&s->host_meta, (size_t)(s->cfg.n_streams * s->meta_cap), hipHostMallocDefault) !=
          hipSuccess) {
    destroy(s);
    return RDCT_ERR_NO_MEMORY;
  }
  s->dev.reset(s->cfg.budget_bytes - s->plane_base, 256);
  s->host.reset(s->cfg.staging_bytes, 256);
  for (int i = 0; i < s->cfg.n_streams; ++i)
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) != hipSuccess) {
      destroy(s);
      return RDCT_ERR_HIP;
    }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return RDCT_OK;
}

rdct_status_t rdct_server_submit(rdct_server_t* s, const rdct_request_t* req, uint64_t* ticket) {
  if (!s || !req || req->n_planes < 1 || req->n_planes > 3) return RDCT_ERR_INVALID_ARG;
  SelInfo si;
  rdct_status_t st = check_sel(&req->sel, &si);
  if (st != RDCT_OK) return st;
  Request r;
  r.n = req->n_planes;
  r.tag = req->user_tag;
  r.sel = si.sel;
  r.mode = req->sel.mode == RDCT_SEL_QUANT ? RDCT_SEL_QUANT : RDCT_SEL_ZIGZAG;
  r.r = si.r;
  r.shift = si.shift;
  memcpy(r.q, si.q, sizeof(r.q));
  int64_t dev_need = 0, host_need = 0;
  for (int i = 0; i < r.n; ++i) {
    if ((st = check_plane(req->planes[i], req->width[i], req->height[i], req->pitch[i],
                          kMaxEvalBlocks)) != RDCT_OK)
      return st;
    r.p[i].w = req->width[i];
    r.p[i].h = req->height[i];
    r.p[i].bytes = plane_dev_bytes(r.p[i].w, r.p[i].h);
    dev_need += s->dev.round(r.p[i].bytes);
    host_need += s->host.round(r.p[i].bytes);
  }
  // A request that could not run alone is refused now rather than queued forever.
  if (dev_need > s->dev.size() || host_need > s->host.size() ||
      request_meta_bytes(admit_view(r), kMetaSizes) > s->meta_cap) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected++;
    return RDCT_ERR_BUDGET;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 0; i < r.n; ++i) {
      r.p[i].host_off = s->host.alloc(r.p[i].bytes);
      if (r.p[i].host_off < 0) {
        for (int j = 0; j < i; ++j) s->host.release(r.p[j].host_off, r.p[j].bytes);
        s->st.rejected++;
        return RDCT_ERR_BUSY;
      }
    }
  }
  // Copy into the reserved staging outside the lock (rows packed to width).
  for (int i = 0; i < r.n; ++i) {
    uint8_t* dst = s->host_base + r.p[i].host_off;
    const uint8_t* src = req->planes[i];
    const int w = r.p[i].w, h = r.p[i].h;
    if (req->pitch[i] == w) {
      memcpy(dst, src, (size_t)w * h);
    } else {
      for (int y = 0; y < h; ++y) memcpy(dst + (int64_t)y * w, src + (int64_t)y * req->pitch[i], w);
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r.ticket = s->next_ticket++;
    r.t_submit = s->now_us();
    s->pending.push_back(r);
    s->st.submitted++;
  }
  s->cv_work.notify_one();
  if (ticket) *ticket = r.ticket;
  return RDCT_OK;
}

rdct_status_t rdct_server_poll(rdct_server_t* s, rdct_completion_t* out, int32_t max, int32_t* n,
                               int32_t wait_us) {
  if (!s || !n || max < 0 || (max > 0 && !out)) return RDCT_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done.empty(); });
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return RDCT_OK;
}

rdct_status_t rdct_server_cancel(rdct_server_t* s, uint64_t ticket) {
  if (!s) return RDCT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
    if (it->ticket == ticket) {
      complete(s, *it, RDCT_ERR_CANCELLED, nullptr, s->now_us(), 0);
      release_request(s, *it);
      s->pending.erase(it);
      s->st.cancelled++;
      s->st.completed++;
      s->cv_done.notify_all();
      return RDCT_OK;
    }
  }
  return ticket > 0 && ticket < s->next_ticket ? RDCT_ERR_BUSY : RDCT_ERR_NOT_FOUND;
}

rdct_status_t rdct_server_drain(rdct_server_t* s, int32_t timeout_ms) {
  if (!s) return RDCT_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                      [&] { return s->st.completed == s->st.submitted; });
  return ok ? RDCT_OK : RDCT_ERR_BUSY;
}

rdct_status_t rdct_server_stats(rdct_server_t* s, rdct_server_stats_t* out) {
  if (!s || !out) return RDCT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->device_bytes_in_use = s->dev.in_use();
  out->pending = (int32_t)s->pending.size();
  out->inflight = (int32_t)s->inflight_reqs;
  return RDCT_OK;
}

void rdct_server_destroy(rdct_server_t* s) { destroy(s); }

}  // extern "C"
