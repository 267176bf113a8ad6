// Host-side packing of a model description (see model_pack.cpp).
#pragma once
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "step_core.h"

namespace sim {

struct PackedModel {
  std::vector<int> hdr, topo, lam_off, team_of, fwd_of, adj_of, ccap_of;
  std::vector<int> adj_ring_of;   // adjoint LDS floats with a ring of the impulse history (saved working sets)
  std::vector<float> cst, target;
  long long seg_total = 0;   // floats of the reverse sweep's buffer (all envs)
  long long tape_rows = 0;   // env-steps of the controller tape (sum of T_e)
  int dump = 0;              // reverse sweep buffer: DUMP_REPLAY, DUMP_SEGMENT or DUMP_TRAJECTORY
};

// Default memory limit of the automatic choice of reverse sweep mode: 32 GiB.
constexpr long long kGradMemDefault = 32LL << 30;

// Validates the per-env parts of the description and builds, per env, the
// header, topology ints (parents, children, ground bodies, pair codes, colour
// starts, colour-major candidate list) and constants.  Global checks
// (offsets, scalars) are done by the caller.
sim_status pack_model(const sim_model_desc* d, PackedModel& P, std::string& err);

// Some env has a restitution coefficient > 0: the steps then keep the
// predicted velocities in LDS for the restitution adjoint.
inline bool desc_has_rest(const sim_model_desc* d) {
  if (!d->restitution) return false;
  for (int e = 0; e < d->n_envs; ++e)
    if (d->restitution[e] > 0.f) return true;
  return false;
}

}  // namespace sim
