// Autotuning of the solve-time choices that do not change what a hierarchy
// is: the SAP block shape of every smoothed coarse level (among the shapes
// valid for that level: blocks tile it with an even count per direction,
// Sec. 2) and the batch size for a given number of right-hand sides.  The
// search times whole solves; the choices are cached in a small JSON file
// keyed by device architecture, lattice, precisions, hierarchy shape and
// number of right-hand sides.
#pragma once

#include <array>
#include <string>
#include <vector>

#include "solver.h"

namespace ddamg {

struct TuneChoice {
  int sap[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  int batch = 0;
  double seconds = 0;
};

std::string tune_key(const Hierarchy& H, int nrhs);
// candidate block shapes of coarse level l: equal extents in x, y, z and a
// free extent in t, each dividing the level with an even block count
std::vector<std::array<int, 4>> sap_candidates(const Hierarchy& H, int l);
bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice& c);
void tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c);

}  // namespace ddamg
