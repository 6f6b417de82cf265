// Persisted work schedules of batches (the autotuner's table).
//
// The table is a small JSON document:
//   {"device": "gfx950", "entries": [
//     {"k": 5, "npad_min": 4, "dense": 1, "npad": 4, "unit_cost": 1024, "ms": 0.41, "systems": 412},
//     ...]}
// one entry per bucket (k, smallest lane-group width as log2); "dense" is the
// kernel (1 lane-dense, 0 lanes as points; absent: lane-dense when certified).  The reader
// accepts exactly what the writer produces (flat objects of numbers and
// strings inside "entries"); anything else is an error and leaves the table
// empty, so a damaged file never changes a schedule silently.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>

#include "runtime.hpp"

namespace bdeg {

namespace {

// numbers of one flat JSON object {"key": value, ...}; false on a syntax error
bool parse_object(const char *&p, const char *end, ScheduleTable &t) {
  long long k = -1, npad_min = -1, npad = 0, systems = 0, dense = -1;
  unsigned long long cost = 0;
  double ms = 0;
  ++p; // '{'
  for (;;) {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t' || *p == ',')) ++p;
    if (p >= end) return false;
    if (*p == '}') {
      ++p;
      break;
    }
    if (*p != '"') return false;
    const char *ks = ++p;
    while (p < end && *p != '"') ++p;
    if (p >= end) return false;
    const std::string key(ks, p - ks);
    ++p;
    while (p < end && (*p == ' ' || *p == ':')) ++p;
    if (p >= end) return false;
    if (*p == '"') { // a string value (ignored)
      ++p;
      while (p < end && *p != '"') ++p;
      if (p >= end) return false;
      ++p;
      continue;
    }
    char *q = nullptr;
    const double v = strtod(p, &q);
    if (q == p) return false;
    p = q;
    if (key == "k") k = (long long)v;
    else if (key == "npad_min") npad_min = (long long)v;
    else if (key == "npad") npad = (long long)v;
    else if (key == "unit_cost") cost = (unsigned long long)v;
    else if (key == "ms") ms = v;
    else if (key == "systems") systems = (long long)v;
    else if (key == "dense") dense = (long long)v;
  }
  if (k < 1 || k > BDEG_MAX_K || npad_min < 3 || npad_min > 6 || npad < npad_min || npad > 6 || cost > (1ull << 26) ||
      dense < -1 || dense > 1)
    return false;
  BucketSchedule &b = t.e[k][npad_min];
  b.dense = (int)dense;
  b.npad_log2 = (int)npad;
  b.unit_cost = cost;
  b.ms = (float)ms;
  b.systems = (int)systems;
  t.any = true;
  return true;
}

std::string library_dir() {
  Dl_info info;
  if (dladdr((void *)&schedule_read, &info) && info.dli_fname) {
    std::string f = info.dli_fname;
    const size_t slash = f.rfind('/');
    if (slash != std::string::npos) return f.substr(0, slash);
  }
  return ".";
}

} // namespace

int schedule_read(const char *path, ScheduleTable &t) {
  t = ScheduleTable{};
  FILE *f = fopen(path, "rb");
  if (!f) return BDEG_E_ARG;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  const char *p = strstr(s.c_str(), "\"entries\"");
  if (!p) return BDEG_E_ARG;
  p = strchr(p, '[');
  if (!p) return BDEG_E_ARG;
  const char *end = s.c_str() + s.size();
  ++p;
  for (;;) {
    while (p < end && *p != '{' && *p != ']') ++p;
    if (p >= end) break;
    if (*p == ']') return BDEG_OK;
    if (!parse_object(p, end, t)) {
      t = ScheduleTable{};
      return BDEG_E_ARG;
    }
  }
  t = ScheduleTable{};
  return BDEG_E_ARG;
}

int schedule_write(const char *path, const ScheduleTable &t) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) return BDEG_E_ARG;
  fprintf(f, "{\"device\": \"gfx950\", \"entries\": [");
  bool first = true;
  for (int k = 1; k <= BDEG_MAX_K; k++)
    for (int g = 3; g <= 6; g++) {
      const BucketSchedule &b = t.e[k][g];
      if (b.npad_log2 == 0 && b.unit_cost == 0) continue;
      fprintf(f,
              "%s\n  {\"k\": %d, \"npad_min\": %d, \"dense\": %d, \"npad\": %d, \"unit_cost\": %llu, \"ms\": %.4f, "
              "\"systems\": %d}",
              first ? "" : ",", k, g, b.dense, b.npad_log2, (unsigned long long)b.unit_cost, (double)b.ms, b.systems);
      first = false;
    }
  fprintf(f, "\n]}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) return BDEG_E_ARG;
  return BDEG_OK;
}

const ScheduleTable &schedule_table() {
  static ScheduleTable table;
  static std::once_flag once;
  std::call_once(once, [] {
    const char *env = getenv("BDEG_TUNE_TABLE");
    const std::string path = env ? std::string(env) : library_dir() + "/tuning/gfx950.json";
    if (schedule_read(path.c_str(), table) != BDEG_OK) table = ScheduleTable{};
  });
  return table;
}

} // namespace bdeg
