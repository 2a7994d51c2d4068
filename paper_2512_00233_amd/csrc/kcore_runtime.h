// Internal host-side declarations shared by the runtime translation units.
#pragma once

#include <string>

#include "../../include/kcore.h"

namespace kcore {

// Resolved launch parameters (library defaults overridden by kcore_tuning).
struct Tuning {
  int t1;         // lane class: degree <= t1
  int t2;         // wavefront class: degree <= t2
  int t3;         // workgroup keeps values in registers up to t3 neighbours
  int tail;       // frontier size that hands the run to one workgroup
  int grid;       // workgroups per round launch
  int poll;       // rounds in the first chunk between host checks
  int one_sided;  // activation rule
  int timing;     // HIP events around every round launch
  int list_cap;   // sparse list capacity per class
  int prune;      // pruned adjacency on/off
};

Tuning resolve_tuning(const kcore_tuning* t, int num_cus);
kcore_status fail(kcore_status s, const std::string& msg);

}  // namespace kcore
