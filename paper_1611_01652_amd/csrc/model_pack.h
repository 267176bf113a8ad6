// Host-side packing of a model description (see model_pack.cpp).
#pragma once
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "step_core.h"

namespace sim {

struct PackedModel {
  std::vector<int> hdr, topo, lam_off, team_of, fwd_of, adj_of, ccap_of;
  std::vector<float> cst, target;
  long long seg_total = 0;
  long long tape_rows = 0;   // env-steps of the controller tape (sum of T_e)
  int dump = 0;              // segment buffer holds saved step working sets (no replay)
};

// Largest segment buffer (floats) for which the reverse sweep saves each
// step's working set instead of replaying the step: 2^30 floats (4 GiB).
constexpr long long kDumpBudgetFloats = 1LL << 30;

// Validates the per-env parts of the description and builds, per env, the
// header, topology ints (parents, children, ground bodies, pair codes, colour
// starts, colour-major candidate list) and constants.  Global checks
// (offsets, scalars) are done by the caller.
sim_status pack_model(const sim_model_desc* d, PackedModel& P, std::string& err);

}  // namespace sim
