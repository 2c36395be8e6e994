// Launch-shape table of the library: choices that change no result (sort
// block size, compaction variant, PR short-row variant on batch unions,
// the split between the two smaller long-row classes, the long-row emission
// variant), one entry per size bucket (arcs of the level being processed).
// The library reads the table at load time from the file named by the
// environment variable VIECUT_TUNING, else from viecut_tuning.txt beside
// libviecut.so; without a file it uses the hand-measured defaults. The
// project's tuner (paper_1708_06127_amd/autotune.py) measures candidates on
// the GPU through viecut_tuning_set and writes the file.
#include <dlfcn.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/viecut.h"
#include "vc_internal.h"

namespace vc {
namespace {

struct Bucket {
  int64_t max_arcs;  // < 0: no bound (the last bucket)
  Tuning t;
};

struct Table {
  std::mutex mu;
  bool loaded = false;
  std::vector<Bucket> b;  // ascending bounds, the unbounded one last
  std::string source = "defaults";
};

Table &table() {
  static Table t;
  return t;
}

int64_t *field(Tuning &t, const char *key) {
  if (!std::strcmp(key, "radix_large_from")) return &t.radix_large_from;
  if (!std::strcmp(key, "compact_direct_max")) return &t.compact_direct_max;
  if (!std::strcmp(key, "pr_merge_tiles")) return &t.pr_merge_tiles;
  if (!std::strcmp(key, "long_split")) return &t.long_split;
  if (!std::strcmp(key, "emit_wave")) return &t.emit_wave;
  if (!std::strcmp(key, "lp_group")) return &t.lp_group;
  if (!std::strcmp(key, "emit_group")) return &t.emit_group;
  if (!std::strcmp(key, "first_group")) return &t.first_group;
  if (!std::strcmp(key, "huge_part")) return &t.huge_part;
  return nullptr;
}
const char *kKeys[] = {"radix_large_from", "compact_direct_max", "pr_merge_tiles", "long_split", "emit_wave",
                       "lp_group", "emit_group", "first_group", "huge_part"};

bool valid(const char *key, int64_t v) {
  // the 1024-slot class holds rows of d < long_split arcs: at most 3/4 full
  if (!std::strcmp(key, "long_split")) return v >= kTile && v <= 768;
  if (!std::strcmp(key, "emit_wave")) return v == 0 || v == 1;
  if (!std::strcmp(key, "lp_group")) return v >= 1 && v <= 4;
  if (!std::strcmp(key, "emit_group")) return v == 1 || v == 2;
  if (!std::strcmp(key, "first_group")) return v == 1 || v == 2;
  if (!std::strcmp(key, "huge_part")) return v == 0 || v == 1;
  return v >= 0;
}

Bucket &bucket_for_bound(Table &T, int64_t max_arcs) {
  for (auto &x : T.b)
    if (x.max_arcs == max_arcs) return x;
  Bucket nb{max_arcs, Tuning{}};
  T.b.push_back(nb);
  std::sort(T.b.begin(), T.b.end(), [](const Bucket &a, const Bucket &c) {
    if ((a.max_arcs < 0) != (c.max_arcs < 0)) return c.max_arcs < 0;
    return a.max_arcs < c.max_arcs;
  });
  for (auto &x : T.b)
    if (x.max_arcs == max_arcs) return x;
  return T.b.back();
}

void load_file(Table &T) {
  std::string path;
  if (const char *e = getenv("VIECUT_TUNING")) {
    path = e;
  } else {
    Dl_info info;
    if (dladdr((void *)&load_file, &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.rfind('/');
      path = (slash == std::string::npos ? std::string() : path.substr(0, slash + 1)) + "viecut_tuning.txt";
    }
  }
  if (path.empty()) return;
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char *p = line;
    while (*p == ' ' || *p == '\t') p++;
    if (*p == '#' || *p == '\n' || !*p) continue;
    char word[32];
    long long bound = 0;
    int used = 0;
    if (sscanf(p, "%31s %lld%n", word, &bound, &used) < 2 || std::strcmp(word, "bucket")) continue;
    Bucket &bk = bucket_for_bound(T, bound < 0 ? -1 : bound);
    p += used;
    char kv[128];
    while (sscanf(p, " %127s%n", kv, &used) == 1) {
      p += used;
      char *eq = std::strchr(kv, '=');
      if (!eq) continue;
      *eq = 0;
      const long long v = atoll(eq + 1);
      int64_t *fp = field(bk.t, kv);
      if (fp && valid(kv, v)) *fp = v;
    }
  }
  fclose(f);
  T.source = path;
}

void ensure_loaded(Table &T) {
  if (T.loaded) return;
  T.loaded = true;
  load_file(T);
}

}  // namespace

Tuning tuning_for(int64_t arcs) {
  Table &T = table();
  std::lock_guard<std::mutex> lk(T.mu);
  ensure_loaded(T);
  for (const auto &x : T.b)
    if (x.max_arcs < 0 || arcs <= x.max_arcs) return x.t;
  return Tuning{};
}

}  // namespace vc

extern "C" {

int viecut_tuning_set(int64_t max_arcs, const char *key, int64_t value) {
  if (!key) return VIECUT_EINVAL;
  vc::Tuning probe;
  if (!vc::field(probe, key) || !vc::valid(key, value)) return VIECUT_EINVAL;
  vc::Table &T = vc::table();
  std::lock_guard<std::mutex> lk(T.mu);
  vc::ensure_loaded(T);
  vc::Bucket &bk = vc::bucket_for_bound(T, max_arcs < 0 ? -1 : max_arcs);
  *vc::field(bk.t, key) = value;
  T.source = "set";
  return VIECUT_OK;
}

int viecut_tuning_clear(void) {
  vc::Table &T = vc::table();
  std::lock_guard<std::mutex> lk(T.mu);
  T.loaded = true;  // the file is not read again
  T.b.clear();
  T.source = "defaults";
  return VIECUT_OK;
}

int viecut_tuning_get(char *buf, size_t len) {
  vc::Table &T = vc::table();
  std::lock_guard<std::mutex> lk(T.mu);
  vc::ensure_loaded(T);
  std::string s = "# source: " + T.source + "\n";
  std::vector<vc::Bucket> rows = T.b;
  if (rows.empty() || rows.back().max_arcs >= 0) rows.push_back(vc::Bucket{-1, vc::Tuning{}});
  for (auto &x : rows) {
    char tmp[64];
    snprintf(tmp, sizeof tmp, "bucket %lld", (long long)x.max_arcs);
    s += tmp;
    for (const char *k : vc::kKeys) {
      snprintf(tmp, sizeof tmp, " %s=%lld", k, (long long)*vc::field(x.t, k));
      s += tmp;
    }
    s += "\n";
  }
  if (!buf) return (int)s.size() + 1;
  if (len == 0) return VIECUT_EINVAL;
  std::strncpy(buf, s.c_str(), len - 1);
  buf[len - 1] = 0;
  return (int)std::min(s.size() + 1, len);
}

}  // extern "C"
