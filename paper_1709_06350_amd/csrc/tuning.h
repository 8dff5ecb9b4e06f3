// Persistent record of the tuners' choices (host code).
//
// Every tuner of the library (the FP64 sweep and defect schedules, the FP32 sweep of the mixed
// form, the batched FP32 sweep tiles, the adjoint sweep) times candidate launches once per device
// and mesh size. The choice is kept in memory for the process and in a text file, so that later
// processes on the same kind of device skip the timing and make the same choice. A record is a
// list of integers under a key of the tuner's name (with a format version), the device's
// architecture name, memory size and compute-unit count, and the mesh size. A tuner checks a
// recorded choice against its current candidate list before using it, and times again when the
// choice is not among them (another build, another kernel set).
#pragma once

#include <string>
#include <vector>

#include "mr_kernels.h"

namespace mr {

// The integers of a tile configuration, in a fixed order.
inline std::vector<int> tile_code(const TileCfg& t) {
  return {t.tm, t.tj, t.ci, t.tiles_j, t.tiles_m, t.cpt, t.pipe ? 1 : 0};
}

// The recorded choice of tuner `kind` for mesh size n on device dev, if there is one.
bool tuning_lookup(const char* kind, int dev, int n, std::vector<int>& vals);
// Records (and writes to the file, when one is in use) the choice of tuner `kind`.
void tuning_record(const char* kind, int dev, int n, const std::vector<int>& vals);
// Changes whenever the file in use is set again (mr_tuning_file): the tuners then drop the
// choices they keep in memory. Call with the tuner's lock held.
int tuning_generation();
template <class Map>
void tuning_sync(int& gen, Map& m) {
  const int g = tuning_generation();
  if (gen != g) {
    m.clear();
    gen = g;
  }
}

}  // namespace mr
