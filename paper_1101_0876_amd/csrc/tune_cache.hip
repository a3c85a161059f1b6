// tune_cache.hip -- the launch shapes the tuner chose, persisted as JSON.
//
// A cache file holds the kernel hash it was measured on (a digest of the
// tuned kernels' sources, fixed at build time) and two tables:
//   "rows":   "<kernel>/<q class>/<L>" -> strip height of that lattice size
//   "shapes": "<kernel>/<q class>"     -> [lanes per workgroup, waves per SIMD]
// A file written for other kernel sources is ignored, so an edit of a kernel
// never reuses shapes timed on its predecessor.
#include "tune_cache.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef POTTS_KERNEL_HASH
#define POTTS_KERNEL_HASH "unversioned"
#endif

namespace potts {

const char *kernel_hash() { return POTTS_KERNEL_HASH; }

}  // namespace potts

extern "C" const char *potts_kernel_digest(void) { return potts::kernel_hash(); }

namespace potts {

namespace {

// Position just after the closing quote of the string starting at s[i] == '"'.
size_t skip_string(const std::string &s, size_t i, std::string *out) {
  size_t j = i + 1;
  while (j < s.size() && s[j] != '"') ++j;
  if (out) *out = s.substr(i + 1, j - i - 1);
  return j + 1;
}

size_t skip_space(const std::string &s, size_t i) {
  while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r' || s[i] == ':' || s[i] == ','))
    ++i;
  return i;
}

// The text of the object that follows "name": {...}, or "" when absent.
std::string object_of(const std::string &s, const char *name) {
  const std::string key = std::string("\"") + name + "\"";
  size_t i = s.find(key);
  if (i == std::string::npos) return "";
  i = s.find('{', i + key.size());
  if (i == std::string::npos) return "";
  const size_t j = s.find('}', i);
  return j == std::string::npos ? "" : s.substr(i + 1, j - i - 1);
}

}  // namespace

void TuneCache::load(const char *file) {
  path = file ? file : "";
  rows.clear();
  shapes.clear();
  dirty = false;
  if (path.empty()) return;
  FILE *f = fopen(path.c_str(), "rb");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  fclose(f);
  const size_t h = text.find("\"kernel_hash\"");
  if (h == std::string::npos) return;
  const size_t q0 = text.find('"', h + 13);
  if (q0 == std::string::npos) return;
  std::string hash;
  skip_string(text, q0, &hash);
  if (hash != kernel_hash()) return;  // measured on other kernels
  const std::string r = object_of(text, "rows");
  for (size_t i = r.find('"'); i != std::string::npos && i < r.size(); i = r.find('"', i)) {
    std::string key;
    i = skip_space(r, skip_string(r, i, &key));
    const long v = strtol(r.c_str() + i, nullptr, 10);
    if (v >= 2 && v <= 32 && v % 2 == 0) rows[key] = (uint32_t)v;
  }
  const std::string sh = object_of(text, "shapes");
  for (size_t i = sh.find('"'); i != std::string::npos && i < sh.size(); i = sh.find('"', i)) {
    std::string key;
    i = skip_space(sh, skip_string(sh, i, &key));
    unsigned block = 0, wpe = 0;
    if (i < sh.size() && sscanf(sh.c_str() + i, "[%u ,%u]", &block, &wpe) == 2) {
      TileShape t;
      t.block = block;
      t.wpe = wpe;
      if (shape_ok(t, 16)) shapes[key] = t;
    }
  }
}

bool TuneCache::save() const {
  if (path.empty() || !dirty) return true;
  const std::string tmp = path + ".tmp";
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fprintf(f, "{\n  \"kernel_hash\": \"%s\",\n  \"rows\": {", kernel_hash());
  const char *sep = "";
  for (const auto &kv : rows) {
    fprintf(f, "%s\n    \"%s\": %u", sep, kv.first.c_str(), kv.second);
    sep = ",";
  }
  fprintf(f, "\n  },\n  \"shapes\": {");
  sep = "";
  for (const auto &kv : shapes) {
    fprintf(f, "%s\n    \"%s\": [%u, %u]", sep, kv.first.c_str(), kv.second.block, kv.second.wpe);
    sep = ",";
  }
  fprintf(f, "\n  }\n}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

std::string TuneCache::rows_key(bool packed, int qc, uint32_t L) {
  return std::string(packed ? "packed/" : "strip/") + std::to_string(qc) + "/" + std::to_string(L);
}

std::string TuneCache::shape_key(bool packed, int qc) {
  return std::string(packed ? "packed/" : "strip/") + std::to_string(qc);
}

}  // namespace potts
