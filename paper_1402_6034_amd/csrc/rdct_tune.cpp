// Tuning cache of librdct: one JSON object per line inside an "entries" array,
// keyed by architecture / path variant / size class, written atomically
// (temporary file + rename) and read back with a small line scanner that only
// understands the format written here.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <map>
#include <mutex>
#include <string>

#include "rdct_tune.h"

namespace rdct {

namespace {

struct Entry {
  int waves_per_wg = 0;
  int wgs_per_cu = 0;
  int layout = 0;
  int xcd_ranges = 0;
  int strip = 1;
  float us = 0.f;
};

std::mutex g_mu;

bool scan_int(const std::string& line, const char* field, int* out) {
  const std::string pat = std::string("\"") + field + "\": ";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  *out = atoi(line.c_str() + p + pat.size());
  return true;
}

std::map<std::string, Entry> load(const std::string& path) {
  std::map<std::string, Entry> m;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return m;
  char buf[1024];
  while (fgets(buf, sizeof(buf), f)) {
    const std::string line(buf);
    const size_t k = line.find("\"key\": \"");
    if (k == std::string::npos) continue;
    const size_t b = k + 8, e = line.find('"', b);
    if (e == std::string::npos) continue;
    Entry en;
    if (!scan_int(line, "waves_per_wg", &en.waves_per_wg) ||
        !scan_int(line, "wgs_per_cu", &en.wgs_per_cu))
      continue;
    if (!scan_int(line, "layout", &en.layout)) en.layout = RDCT_LAYOUT_STRIDED;
    if (!scan_int(line, "xcd_ranges", &en.xcd_ranges)) en.xcd_ranges = 0;
    if (!scan_int(line, "strip", &en.strip)) en.strip = 1;
    const size_t u = line.find("\"us\": ");
    if (u != std::string::npos) en.us = (float)atof(line.c_str() + u + 6);
    m[line.substr(b, e - b)] = en;
  }
  fclose(f);
  return m;
}

void mkdirs_for(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
}

}  // namespace

std::string tune_cache_path() {
  const char* e = getenv("RDCT_TUNING_CACHE");
  if (e && *e) return e;
  const char* home = getenv("HOME");
  return std::string(home && *home ? home : "/tmp") + "/.cache/rdct_tuning.json";
}

bool tune_cache_lookup(const std::string& key, rdct_tuning_t* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  const auto m = load(tune_cache_path());
  const auto it = m.find(key);
  if (it == m.end()) return false;
  out->waves_per_wg = it->second.waves_per_wg;
  out->wgs_per_cu = it->second.wgs_per_cu;
  out->use_graph = 0;
  out->layout = it->second.layout;
  out->xcd_ranges = it->second.xcd_ranges;
  out->strip = it->second.strip;
  return true;
}

void tune_cache_store(const std::string& key, const rdct_tuning_t& t, float us) {
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string path = tune_cache_path();
  auto m = load(path);
  m[key] = Entry{t.waves_per_wg, t.wgs_per_cu, t.layout, t.xcd_ranges, t.strip, us};
  mkdirs_for(path);
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\"rdct_tuning\": 1, \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f,
            "  {\"key\": \"%s\", \"waves_per_wg\": %d, \"wgs_per_cu\": %d, \"layout\": %d, "
            "\"xcd_ranges\": %d, \"strip\": %d, \"us\": %.3f}%s\n",
            kv.first.c_str(), kv.second.waves_per_wg, kv.second.wgs_per_cu, kv.second.layout,
            kv.second.xcd_ranges, kv.second.strip, kv.second.us, ++i < m.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  rename(tmp.c_str(), path.c_str());
}

}  // namespace rdct
