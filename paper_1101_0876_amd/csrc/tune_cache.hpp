// tune_cache.hpp -- persisted launch shapes of the tiled sweep launches.
#pragma once

#include <stdint.h>

#include <map>
#include <string>

#include "kernels.hpp"

namespace potts {

// digest of the tuned kernels' sources, fixed at build time
const char *kernel_hash();

struct TuneCache {
  std::string path;                        // "" = nothing persisted
  std::map<std::string, uint32_t> rows;    // rows_key -> strip height
  std::map<std::string, TileShape> shapes; // shape_key -> launch shape
  bool dirty = false;

  // Reads `file` (NULL or missing: empty; another kernel hash: ignored).
  void load(const char *file);
  // Writes the tables back (atomically) when something changed.
  bool save() const;
  static std::string rows_key(bool packed, int qc, uint32_t L);
  static std::string shape_key(bool packed, int qc);
};

}  // namespace potts
