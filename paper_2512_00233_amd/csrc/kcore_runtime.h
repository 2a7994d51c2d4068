// Internal host-side declarations shared by the runtime translation units.
#pragma once

#include <string>

#include "../../include/kcore.h"

namespace kcore {

// Resolved launch parameters (library defaults overridden by kcore_tuning).
struct Tuning {
  int t0;         // class 0 (one lane): degree <= t0
  int t1;         // class 1 (16-lane group): degree <= t1
  int t2;         // class 2 (wavefront): degree <= t2; above: class 3 (workgroup)
  int tail;       // frontier work that hands the run to one workgroup
  int grid;       // workgroups per small-class round launch
  int big_grid;   // workgroups per class-3 round launch
  int poll;       // rounds in the first chunk between host checks
  int one_sided;  // activation rule
  int timing;     // HIP events around every round launch
  int list_cap;   // sparse list capacity per class
  int prune;      // pruned adjacency on/off
  int use_graph;  // capture chunks of round launches as hipGraphs
};

Tuning resolve_tuning(const kcore_tuning* t, int num_cus);
kcore_status fail(kcore_status s, const std::string& msg);

}  // namespace kcore
