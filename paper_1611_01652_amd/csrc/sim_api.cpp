// C ABI of the batched rigid-body step (declared in include/sim.h): model
// validation, per-env topology (contact candidates and the colour-major sweep
// order), size buckets and env tiles, device upload, and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "model_pack.h"
#include "sim_internal.h"

using namespace sim;

// Device memory of rollout_grad_noalloc: the reverse sweep's workspace for
// callers that cannot allocate.  Each device holds its own copy for the life
// of the process; in host code this name is only a stand-in for the symbol,
// so kernels and copies use the device address looked up at set-up.
static __device__ __align__(256) float scratch[SIM_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

thread_local std::string g_err;

// Device address of `scratch` per device ordinal, looked up once per device
// (with that device current) by sim_init.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[dev] = p;
  return hipSuccess;
}
void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[dev];
}

sim_status fail(sim_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct Bucket {
  int team = 1;
  int team_min = 1;             // narrowest team the bucket's envs allow
  std::vector<int> envs_host;   // tiles * (64/team)
  int n_tiles = 0;
  int floats_fwd = 0, floats_adj = 0;
  int ccap_max = 0;             // largest contact capacity of its envs
  int* envs_dev = nullptr;
};

}  // namespace

struct sim_model {
  DevModel M{};
  sim_info info{};
  std::vector<int> lam_off;     // [E+1]
  std::vector<Bucket> buckets;
  int* d_hdr = nullptr;
  int* d_topo = nullptr;
  float* d_cst = nullptr;
  float* d_target = nullptr;
  int* d_queue = nullptr;       // one counter per bucket
  int n_cu = 256;
  int max_lds = 65536;
  int device = 0;
  std::vector<hipStream_t> streams;  // one per bucket when there are several
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  // controller
  float* d_clock = nullptr;
  WgradTile* d_tiles = nullptr;
  int* d_map = nullptr;
  int n_wtiles = 0, n_params = 0, chunk = 2048;
  long long tape_rows = 0, seg_floats = 0, tape_floats = 0;
  int lds_allowed = 65536;      // dynamic LDS limit set on the kernels
  int n_graphs = 0;             // live step graphs (they hold the tile lists)
  uint16_t* d_wsn = nullptr;    // warm-start network, bfloat16
  hipEvent_t tev[4] = {};       // rollout_grad phase events (sim_time_grad), owned by the caller
  std::vector<hipEvent_t> bev;  // per-bucket reverse launch events (sim_time_buckets), owned by the caller
  float* d_wt = nullptr;        // controller weights transposed for the forward products
  // the camera's scene: spheres per env, their bodies, offsets and radii
  int* d_env_sph = nullptr;
  int* d_env_body = nullptr;
  int* d_sph_body = nullptr;
  float4* d_sph = nullptr;
  int max_env_spheres = 0;
};

struct sim_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  sim_model* h = nullptr;
};

namespace {

template <class T>
sim_status upload(T** dst, const std::vector<T>& src) {
  const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
  if (hipMalloc((void**)dst, n) != hipSuccess) return fail(SIM_E_NOMEM, "hipMalloc failed");
  if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(SIM_E_DEVICE, "hipMemcpy failed");
  return SIM_OK;
}

void release(sim_model* h) {
  if (!h) return;
  for (auto& b : h->buckets)
    if (b.envs_dev) (void)hipFree(b.envs_dev);
  if (h->d_hdr) (void)hipFree(h->d_hdr);
  if (h->d_topo) (void)hipFree(h->d_topo);
  if (h->d_cst) (void)hipFree(h->d_cst);
  if (h->d_target) (void)hipFree(h->d_target);
  if (h->d_queue) (void)hipFree(h->d_queue);
  if (h->d_clock) (void)hipFree(h->d_clock);
  if (h->d_tiles) (void)hipFree(h->d_tiles);
  if (h->d_map) (void)hipFree(h->d_map);
  if (h->d_wsn) (void)hipFree(h->d_wsn);
  if (h->d_wt) (void)hipFree(h->d_wt);
  if (h->d_env_sph) (void)hipFree(h->d_env_sph);
  if (h->d_env_body) (void)hipFree(h->d_env_body);
  if (h->d_sph_body) (void)hipFree(h->d_sph_body);
  if (h->d_sph) (void)hipFree(h->d_sph);
  for (auto sx : h->streams) (void)hipStreamDestroy(sx);
  for (auto ex : h->joins) (void)hipEventDestroy(ex);
  if (h->fork) (void)hipEventDestroy(h->fork);
  delete h;
}

sim_status check_device(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SIM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SIM_OK;
}

// Launch every bucket: directly on the caller's stream when there is one,
// else forked onto the bucket streams and joined back.
template <class F>
sim_status run_buckets(sim_model* h, hipStream_t st, F launch, const char* what) {
  if (h->buckets.size() == 1) {
    if (!launch(0, st)) return check_device(what);
    return SIM_OK;
  }
  if (hipEventRecord(h->fork, st) != hipSuccess) return check_device(what);
  for (size_t i = 0; i < h->buckets.size(); ++i) {
    if (hipStreamWaitEvent(h->streams[i], h->fork, 0) != hipSuccess) return check_device(what);
    if (!launch(i, h->streams[i])) return check_device(what);
    if (hipEventRecord(h->joins[i], h->streams[i]) != hipSuccess) return check_device(what);
  }
  for (size_t i = 0; i < h->buckets.size(); ++i)
    if (hipStreamWaitEvent(st, h->joins[i], 0) != hipSuccess) return check_device(what);
  return SIM_OK;
}

// The CU's LDS and its SIMDs (gfx950): the reverse kernel runs one wave per SIMD.
constexpr long long kLdsPerCu = 160 * 1024;
constexpr long long kSimdsPerCu = 4;

// LDS bytes of a workgroup: the env tiles and, for the forward kernels of a
// learned warm start, the shared network region.
long long fwd_bytes(const DevModel& M, int team, int floats_fwd, int ccap_max) {
  const int epw = 64 / team;
  return 4LL * ((long long)epw * floats_fwd + (M.ctrl ? CTRL_SHARED : 0) +
                (M.ws_kind ? wsn_shared_floats(epw * ccap_max) : 0));
}
long long adj_bytes(const DevModel& M, int team, int floats_adj) {
  return 4LL * ((long long)(64 / team) * floats_adj + (M.ctrl ? CTRL_SHARED : 0));
}
long long fwd_bytes(const sim_model* h, const Bucket& b) { return fwd_bytes(h->M, b.team, b.floats_fwd, b.ccap_max); }

int grid_for(const sim_model* h, long long units, long long bytes) {
  int per_cu = bytes > 0 ? (int)(kLdsPerCu / bytes) : 8;
  per_cu = std::max(1, std::min(per_cu, 8));
  return (int)std::max(1LL, std::min(units, (long long)h->n_cu * per_cu));
}
int grid_for(const sim_model* h, const Bucket& b, long long bytes) { return grid_for(h, b.n_tiles, bytes); }

// One bucket's kernels (queue reset + launch) on stream sx.
bool bucket_step(sim_model* h, size_t i, const DevModel& M, const StepArgs& a, hipStream_t sx) {
  const Bucket& b = h->buckets[i];
  TileSet ts{b.envs_dev, b.n_tiles, b.floats_fwd, h->d_queue + i, 1};
  if (launch_zero(ts.queue, 1, sx) != hipSuccess) return false;
  const long long lds = fwd_bytes(h, b);
  return launch_step(M, ts, b.team, grid_for(h, b, lds), (size_t)lds, a, sx) == hipSuccess;
}
bool bucket_rollout(sim_model* h, size_t i, const DevModel& M, const RolloutArgs& a, hipStream_t sx) {
  const Bucket& b = h->buckets[i];
  TileSet ts{b.envs_dev, b.n_tiles, b.floats_fwd, h->d_queue + i, 1};
  if (launch_zero(ts.queue, 1, sx) != hipSuccess) return false;
  const long long lds = fwd_bytes(h, b);
  if (a.seg) return launch_rollout_keep(M, ts, b.team, grid_for(h, b, lds), (size_t)lds, a, sx) == hipSuccess;
  return launch_rollout(M, ts, b.team, grid_for(h, b, lds), (size_t)lds, a, sx) == hipSuccess;
}
// Trajectory mode: the recompute of every segment of one bucket's envs into
// the workspace (a no-op in the other modes).
bool bucket_recompute(sim_model* h, size_t i, const DevModel& M, const GradArgs& a, hipStream_t sx) {
  const Bucket& b = h->buckets[i];
  const int n_seg = M.T_max > 0 ? (M.T_max + M.ckpt_every - 1) / M.ckpt_every : 0;
  if (M.dump != DUMP_TRAJECTORY || n_seg == 0) return true;
  TileSet tr{b.envs_dev, b.n_tiles, b.floats_fwd, h->d_queue + i, n_seg};
  if (launch_zero(tr.queue, 1, sx) != hipSuccess) return false;
  const long long lf = fwd_bytes(M, b.team, b.floats_fwd, 0);
  return launch_recompute(M, tr, b.team, grid_for(h, (long long)b.n_tiles * n_seg, lf), (size_t)lf, a, sx) ==
         hipSuccess;
}
// The reverse sweep of one bucket (after its recompute in trajectory mode).
bool bucket_reverse(sim_model* h, size_t i, const DevModel& M, const GradArgs& a, hipStream_t sx) {
  const Bucket& b = h->buckets[i];
  TileSet ts{b.envs_dev, b.n_tiles, b.floats_adj, h->d_queue + i, 1};
  if (launch_zero(ts.queue, 1, sx) != hipSuccess) return false;
  const long long lds = adj_bytes(M, b.team, b.floats_adj);
  const bool timed = h->bev.size() == 2 * h->buckets.size();
  if (timed && hipEventRecord(h->bev[2 * i], sx) != hipSuccess) return false;
  if (launch_rollout_grad(M, ts, b.team, grid_for(h, b, lds), (size_t)lds, a, sx) != hipSuccess) return false;
  return !timed || hipEventRecord(h->bev[2 * i + 1], sx) == hipSuccess;
}
bool bucket_grad(sim_model* h, size_t i, const DevModel& M, const GradArgs& a, hipStream_t sx) {
  return bucket_recompute(h, i, M, a, sx) && bucket_reverse(h, i, M, a, sx);
}

// The call's controls: the tape or, with a controller, its weights u, of
// which the forward products read a transposed copy made here on stream st
// (calls on one handle run one at a time).
bool prep_controls(sim_model* h, DevModel& M, const float* u, hipStream_t st) {
  M.W = u;
  if (!M.ctrl) return true;
  M.Wt = h->d_wt;
  return launch_ctrl_transpose(u, h->d_wt, M.mlp_in, M.mlp_h1, M.mlp_h2, M.mlp_out, st) == hipSuccess;
}

sim_status launch_steps(sim_model* h, const float* x_in, float* x_out, const float* u, const float* lam_in,
                        float* lam_out, int32_t t, uint32_t* env_flags, hipStream_t st) {
  StepArgs a{x_in, x_out, h->M.ctrl ? nullptr : u, lam_in, lam_out, env_flags, t};
  DevModel M = h->M;
  if (!prep_controls(h, M, u, st)) return check_device("sim_step controls");
  return run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_step(h, i, M, a, sx); },
                     "sim_step launch");
}

// Team widths a bucket may use: powers of two from its narrowest whose tile
// fits the device's LDS.
std::vector<int> admissible_teams(const sim_model* h, const Bucket& b) {
  std::vector<int> out;
  for (int t = b.team_min; t <= 64; t *= 2)
    if (std::max(adj_bytes(h->M, t, b.floats_adj), fwd_bytes(h->M, t, b.floats_fwd, b.ccap_max)) <= h->max_lds)
      out.push_back(t);
  return out;
}

// Re-tile a bucket for another team width, keeping its env order.
sim_status retile(sim_model* h, Bucket& b, int team) {
  if (team == b.team) return SIM_OK;
  std::vector<int> ids;
  for (int e : b.envs_host)
    if (e >= 0) ids.push_back(e);
  const int epw = 64 / team;
  const int n_tiles = ((int)ids.size() + epw - 1) / epw;
  std::vector<int> host((size_t)n_tiles * epw, -1);
  std::copy(ids.begin(), ids.end(), host.begin());
  const int bytes = (int)std::max(adj_bytes(h->M, team, b.floats_adj), fwd_bytes(h->M, team, b.floats_fwd, b.ccap_max));
  if (bytes > h->lds_allowed) {
    if (allow_large_lds(std::min(bytes, h->max_lds)) != hipSuccess)
      return fail(SIM_E_DEVICE, "cannot raise the dynamic LDS limit");
    h->lds_allowed = bytes;
  }
  int* dev = nullptr;
  const sim_status st = upload(&dev, host);
  if (st != SIM_OK) return st;
  if (b.envs_dev) (void)hipFree(b.envs_dev);
  b.envs_dev = dev;
  b.envs_host.swap(host);
  b.n_tiles = n_tiles;
  b.team = team;
  h->info.n_tiles = 0;
  h->info.max_lds_bytes = 0;
  for (const auto& x : h->buckets) {
    h->info.n_tiles += x.n_tiles;
    h->info.max_lds_bytes = std::max(h->info.max_lds_bytes, (int)std::max(adj_bytes(h->M, x.team, x.floats_adj),
                                                                           fwd_bytes(h, x)));
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_abi_version(void) { return SIM_ABI_VERSION; }

const char* sim_last_error(void) { return g_err.c_str(); }

sim_status sim_init(const sim_model_desc* d, sim_handle* out) {
  g_err.clear();
  if (!d || !out) return fail(SIM_E_ARG, "sim_init: null argument");
  *out = nullptr;
  const int E = d->n_envs;
  if (E < 0) return fail(SIM_E_ARG, "n_envs < 0");
  if (d->ctrl_kind == 1 && d->T_max > 0 && !(d->clock_hz == d->clock_hz)) return fail(SIM_E_ARG, "clock_hz is NaN");
  if (!d->env_body_off || !d->env_joint_off || !d->env_sphere_off)
    return fail(SIM_E_ARG, "null CSR offsets");
  if (d->env_body_off[0] != 0 || d->env_joint_off[0] != 0 || d->env_sphere_off[0] != 0)
    return fail(SIM_E_SHAPE, "CSR offsets must start at 0");
  for (int e = 0; e < E; ++e)
    if (d->env_body_off[e + 1] < d->env_body_off[e] || d->env_joint_off[e + 1] < d->env_joint_off[e] ||
        d->env_sphere_off[e + 1] < d->env_sphere_off[e])
      return fail(SIM_E_SHAPE, "CSR offsets must be non-decreasing (env " + std::to_string(e) + ")");
  const int B = d->env_body_off[E], J = d->env_joint_off[E], S = d->env_sphere_off[E];
  if ((B > 0 && (!d->inv_mass || !d->inv_inertia)) || (J > 0 && (!d->joint_parent || !d->joint_child ||
      !d->anchor_p || !d->anchor_c || !d->axis_p || !d->axis_c || !d->perp_p || !d->perp_c || !d->damping)) ||
      (S > 0 && (!d->sphere_body || !d->sphere_offset || !d->sphere_radius || !d->sphere_flags)) ||
      (E > 0 && (!d->mu || !d->loss_body || !d->target || !d->T_env)))
    return fail(SIM_E_ARG, "null model array");
  if (!(d->dt > 0.f) || !std::isfinite(d->dt)) return fail(SIM_E_ARG, "dt must be > 0");
  if (d->n_iters < 0) return fail(SIM_E_ARG, "n_iters < 0");
  if (d->ckpt_every < 1) return fail(SIM_E_ARG, "ckpt_every < 1");
  if (d->T_max < 0) return fail(SIM_E_ARG, "T_max < 0");
  if (d->loss_kind < 0 || d->loss_kind > 3) return fail(SIM_E_ARG, "unknown loss_kind");
  if (!(d->rest_threshold >= 0.f) || !std::isfinite(d->rest_threshold))
    return fail(SIM_E_ARG, "rest_threshold must be finite and >= 0");
  if (!(d->gamma >= 0.f)) return fail(SIM_E_ARG, "gamma < 0");
  if (d->min_team < 0 || d->min_team > 64 || (d->min_team & (d->min_team - 1)) != 0)
    return fail(SIM_E_ARG, "min_team must be 0 or a power of two <= 64");
  if (d->solve_mode != SIM_SOLVE_FIXED && d->solve_mode != SIM_SOLVE_TOL) return fail(SIM_E_ARG, "unknown solve_mode");
  if (d->solve_mode == SIM_SOLVE_TOL && (!(d->tol >= 0.f) || !std::isfinite(d->tol) || d->max_iters < 1))
    return fail(SIM_E_ARG, "tolerance mode needs tol >= 0 and max_iters >= 1");
  if (d->ws_kind != SIM_WS_PLAIN && d->ws_kind != SIM_WS_LEARNED) return fail(SIM_E_ARG, "unknown ws_kind");
  if (d->ws_kind == SIM_WS_LEARNED && (d->solve_mode != SIM_SOLVE_TOL || !d->ws_net || d->fb_iters < 0 ||
                                       !(d->fb_tol == d->fb_tol)))
    return fail(SIM_E_ARG, "the learned warm start needs tolerance mode, ws_net, fb_iters >= 0 and a fb_tol");
  if (d->use_grad_decay && !(d->grad_decay >= 0.f && d->grad_decay <= 1.f))
    return fail(SIM_E_ARG, "grad_decay must lie in [0, 1]");
  if (d->grad_store < SIM_GRAD_AUTO || d->grad_store > SIM_GRAD_TRAJECTORY || d->grad_mem_limit < 0)
    return fail(SIM_E_ARG, "grad_store must be one of SIM_GRAD_* and grad_mem_limit >= 0");
  for (int e = 0; e < E; ++e) {
    if (d->T_env[e] < 0 || d->T_env[e] > d->T_max) return fail(SIM_E_SHAPE, "T_env outside [0, T_max]");
    if (d->loss_body[e] < d->env_body_off[e] || d->loss_body[e] >= d->env_body_off[e + 1])
      return fail(SIM_E_SHAPE, "loss_body outside its env (env " + std::to_string(e) + ")");
  }
  for (int j = 0; j < J; ++j)
    if (!(d->damping[j] >= 0.f) || !std::isfinite(d->damping[j])) return fail(SIM_E_ARG, "damping < 0");
  if (d->servo != 0 && d->servo != 1) return fail(SIM_E_ARG, "servo must be 0 or 1");
  if (d->servo && J > 0 && (!d->servo_gain || !d->servo_torque || !d->servo_vmax))
    return fail(SIM_E_ARG, "servo motors need servo_gain, servo_torque and servo_vmax");
  if (d->restitution)
    for (int e = 0; e < E; ++e)
      if (!(d->restitution[e] >= 0.f && d->restitution[e] <= 1.f))
        return fail(SIM_E_ARG, "restitution outside [0, 1] (env " + std::to_string(e) + ")");

  // per-env validation and packing happen on the host before any device call
  PackedModel P;
  {
    std::string perr;
    const sim_status st = pack_model(d, P, perr);
    if (st != SIM_OK) return fail(st, perr);
  }
  sim_model* h = new sim_model();
  if (hipGetDevice(&h->device) != hipSuccess) { release(h); return fail(SIM_E_DEVICE, "no HIP device"); }
  {
    const hipError_t e = scratch_lookup(h->device);
    if (e != hipSuccess) {
      release(h);
      return fail(SIM_E_DEVICE, std::string("sim_init: cannot look up the allocation-free scratch: ") +
                                    hipGetErrorString(e));
    }
  }
  (void)hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
  (void)hipDeviceGetAttribute(&h->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
  DevModel& M = h->M;
  M.n_envs = E; M.B = B; M.J = J; M.T_max = d->T_max; M.n_iters = d->n_iters; M.ground = d->ground;
  M.loss_kind = d->loss_kind; M.loss_mask = d->loss_mask; M.ckpt_every = d->ckpt_every;
  M.dt = d->dt; M.gx = d->gravity[0]; M.gy = d->gravity[1]; M.gz = d->gravity[2];
  M.beta = d->beta; M.gamma = d->gamma; M.spec = d->spec_margin; M.warm = d->warm;
  M.solve_mode = d->solve_mode; M.tol = d->tol; M.max_iters = d->max_iters;
  M.ws_kind = d->ws_kind; M.fb_iters = d->fb_iters; M.fb_tol = d->fb_tol;
  M.decay = d->use_grad_decay ? d->grad_decay : 1.f;
  M.has_rest = desc_has_rest(d) ? 1 : 0;
  M.servo = d->servo;
  M.rest_th = d->rest_threshold;
  M.ctrl = d->ctrl_kind == 1 ? 1 : 0;   // (before the LDS sizes: the controller adds a shared region)

  h->lam_off = P.lam_off;
  std::vector<int>& team_of = P.team_of;
  // Per-env LDS strides: an odd number of float4.  The envs of a wave then
  // start on distinct LDS bank groups, so the same field of up to 16 envs is
  // read in one pass (an even stride, e.g. a multiple of 64 floats, makes
  // them collide on the same banks).
  auto lds_stride = [](int f) {
    f = (f + 3) & ~3;
    return (f / 4) % 2 == 0 ? f + 4 : f;
  };
  std::vector<int> fwd_of(E), adj_of(E), adj_ring_of(E);
  for (int e = 0; e < E; ++e) {
    fwd_of[e] = lds_stride(P.fwd_of[e]);
    adj_of[e] = lds_stride(P.adj_of[e]);
    adj_ring_of[e] = lds_stride(P.adj_ring_of[e]);
  }
  const long long seg_total = P.seg_total;
  int max_lds = 0;
  for (int e = 0; e < E; ++e) {
    // The team width: a wave's step time is set by its env's latency chain,
    // not by how many envs share the wave, so what counts is how many envs a
    // CU holds at once in the reverse sweep, the costlier pass: envs per wave
    // times the waves whose tiles fit the CU's LDS, at most one per SIMD (the
    // reverse kernel's registers allow no more).  More envs per CU pay only
    // while the model's envs do not all fit on the device at once: the
    // choice minimises the rounds ceil(E / (CUs x envs per CU)), then takes
    // no ring over a ring and the narrowest width (the ring costs a read per
    // sweep and a wider team longer steps).
    // The reverse of saved working sets may keep only a ring of the impulse
    // history in LDS (the rest is read from the working set sweep by sweep).
    const int team0 = std::min(64, std::max(team_of[e], d->min_team));
    int team = -1, ring = 0;
    long long best = 0;
    for (int r = 0; r < (P.dump != DUMP_REPLAY ? 2 : 1); ++r) {
      const int fa = r ? adj_ring_of[e] : adj_of[e];
      for (int t = team0; t <= 64; t *= 2) {
        if (std::max(adj_bytes(M, t, fa), fwd_bytes(M, t, fwd_of[e], P.ccap_of[e])) > h->max_lds) continue;
        const long long waves =
            std::min<long long>(kSimdsPerCu, kLdsPerCu / std::max<long long>(1, adj_bytes(M, t, fa)));
        const long long envs_cu = (64 / t) * std::max<long long>(1, waves);
        const long long rounds = ((long long)E + (long long)h->n_cu * envs_cu - 1) / ((long long)h->n_cu * envs_cu);
        // (equal rounds, more than one: the smaller tile, which packs among
        // the other buckets' workgroups)
        if (team < 0 || rounds < best || (rounds == best && rounds > 1 && r == ring && t > team)) {
          best = rounds; team = t; ring = r;
        }
      }
    }
    if (ring) {
      adj_of[e] = adj_ring_of[e];
      P.hdr[(size_t)e * H_COUNT + H_RING] = 1;
    }
    if (team < 0) {
      release(h);
      return fail(SIM_E_UNSUPPORTED, "env " + std::to_string(e) + " needs " + std::to_string(adj_of[e] * 4) +
                                         " bytes of LDS, more than the device's " + std::to_string(h->max_lds));
    }
    team_of[e] = team;
  }
  M.lam_tot = h->lam_off[E];
  // buckets by team size and LDS size class (a quarter octave), so a tile
  // reserves about what its envs need; tiles sorted longest episode first
  auto lds_class = [&](int e) { return (int)std::floor(4.0 * std::log2((double)std::max(adj_of[e], 1))); };
  std::vector<std::pair<int, int>> keys;
  for (int e = 0; e < E; ++e) keys.push_back({team_of[e], lds_class(e)});
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  for (const auto& key : keys) {
    const int team = key.first;
    std::vector<int> ids;
    for (int e = 0; e < E; ++e)
      if (team_of[e] == team && lds_class(e) == key.second) ids.push_back(e);
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
      if (d->T_env[a] != d->T_env[b]) return d->T_env[a] > d->T_env[b];
      return adj_of[a] > adj_of[b];
    });
    Bucket bk;
    bk.team = team;
    bk.team_min = team;
    const int epw = 64 / team;
    bk.n_tiles = ((int)ids.size() + epw - 1) / epw;
    bk.envs_host.assign((size_t)bk.n_tiles * epw, -1);
    for (size_t i = 0; i < ids.size(); ++i) {
      bk.envs_host[i] = ids[i];
      bk.floats_fwd = std::max(bk.floats_fwd, fwd_of[ids[i]]);
      bk.floats_adj = std::max(bk.floats_adj, adj_of[ids[i]]);
      bk.ccap_max = std::max(bk.ccap_max, P.ccap_of[ids[i]]);
    }
    max_lds = std::max(max_lds, (int)std::max(adj_bytes(M, team, bk.floats_adj),
                                              fwd_bytes(M, team, bk.floats_fwd, bk.ccap_max)));
    h->buckets.push_back(bk);
  }
  // buckets run concurrently: one stream each (default priority), forked from
  // and joined back to the caller's stream with events
  if (h->buckets.size() > 1) {
    for (size_t i = 0; i < h->buckets.size(); ++i) {
      hipStream_t sx;
      hipEvent_t ex;
      if (hipStreamCreateWithFlags(&sx, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&ex, hipEventDisableTiming) != hipSuccess) {
        release(h);
        return fail(SIM_E_DEVICE, "cannot create bucket streams");
      }
      h->streams.push_back(sx);
      h->joins.push_back(ex);
    }
    if (hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess) {
      release(h);
      return fail(SIM_E_DEVICE, "cannot create fork event");
    }
  }
  sim_status st = SIM_OK;
  {
    // the camera's scene
    const int S = d->env_sphere_off[E];
    std::vector<int> env_sph(d->env_sphere_off, d->env_sphere_off + E + 1);
    std::vector<int> env_body(d->env_body_off, d->env_body_off + E + 1);
    std::vector<int> sph_body(d->sphere_body, d->sphere_body + S);
    std::vector<float4> sph(S);
    for (int k = 0; k < S; ++k)
      sph[k] = make_float4(d->sphere_offset[3 * k], d->sphere_offset[3 * k + 1], d->sphere_offset[3 * k + 2],
                           d->sphere_radius[k]);
    for (int e = 0; e < E; ++e) h->max_env_spheres = std::max(h->max_env_spheres, env_sph[e + 1] - env_sph[e]);
    if ((st = upload(&h->d_env_sph, env_sph)) != SIM_OK || (st = upload(&h->d_env_body, env_body)) != SIM_OK ||
        (st = upload(&h->d_sph_body, sph_body)) != SIM_OK || (st = upload(&h->d_sph, sph)) != SIM_OK) {
      release(h);
      return st;
    }
  }
  if ((st = upload(&h->d_hdr, P.hdr)) != SIM_OK || (st = upload(&h->d_topo, P.topo)) != SIM_OK ||
      (st = upload(&h->d_cst, P.cst)) != SIM_OK || (st = upload(&h->d_target, P.target)) != SIM_OK) {
    release(h);
    return st;
  }
  for (auto& b : h->buckets)
    if ((st = upload(&b.envs_dev, b.envs_host)) != SIM_OK) { release(h); return st; }
  if ((st = upload(&h->d_queue, std::vector<int>(std::max<size_t>(1, h->buckets.size()), 0))) != SIM_OK) {
    release(h);
    return st;
  }
  // controller: clock table, weight-gradient tiles and parameter map
  if (d->ctrl_kind == 1) {
    const int in = d->mlp_sizes[0], n1 = d->mlp_sizes[1], n2 = d->mlp_sizes[2], no = d->mlp_sizes[3];
    M.ctrl = 1; M.mlp_in = in; M.mlp_h1 = n1; M.mlp_h2 = n2; M.mlp_out = no; M.mlp_rec = d->mlp_rec;
    M.tape_stride = tape_len(in, n1, n2, no);
    std::vector<float> clock(2 * (size_t)std::max(d->T_max, 1));
    for (int t = 0; t < d->T_max; ++t) {
      const double ph = 2.0 * M_PI * (double)d->clock_hz * (double)t * (double)d->dt;
      clock[2 * t] = (float)std::sin(ph);
      clock[2 * t + 1] = (float)std::cos(ph);
    }
    if ((st = upload(&h->d_clock, clock)) != SIM_OK) { release(h); return st; }
    M.clock = h->d_clock;
    // layers: (delta offset, rows, activation offset, columns, weight offset, bias offset)
    const int lay[3][6] = {{tape_d1(M), n1, tape_s(M), in, 0, n1 * in},
                           {tape_d2(M), n2, tape_h1(M), n1, n1 * in + n1, n1 * in + n1 + n2 * n1},
                           {tape_du(M), no, tape_h2(M), n2, n1 * in + n1 + n2 * n1 + n2,
                            n1 * in + n1 + n2 * n1 + n2 + no * n2}};
    h->n_params = n1 * in + n1 + n2 * n1 + n2 + no * n2 + no;
    if (hipMalloc((void**)&h->d_wt, sizeof(float) * (size_t)(n1 * in + n2 * n1 + no * n2)) != hipSuccess) {
      release(h);
      return fail(SIM_E_NOMEM, "hipMalloc failed");
    }
    std::vector<WgradTile> tiles;
    std::vector<int> map(h->n_params, 0);
    for (int l = 0; l < 3; ++l) {
      const int Mr = lay[l][1], Kc = lay[l][3];
      for (int i0 = 0; i0 < Mr; i0 += 32)
        for (int k0 = 0; k0 <= Kc; k0 += 32) {
          const int tid = (int)tiles.size();
          tiles.push_back({lay[l][0], lay[l][2], Mr, Kc, i0, k0});
          for (int i = i0; i < std::min(Mr, i0 + 32); ++i)
            for (int k = k0; k <= std::min(Kc, k0 + 31); ++k) {
              const int p = k < Kc ? lay[l][4] + i * Kc + k : lay[l][5] + i;
              map[p] = tid * 1024 + (i - i0) * 32 + (k - k0);
            }
        }
    }
    h->n_wtiles = (int)tiles.size();
    if ((st = upload(&h->d_tiles, tiles)) != SIM_OK || (st = upload(&h->d_map, map)) != SIM_OK) {
      release(h);
      return st;
    }
  }
  if (d->ws_kind == SIM_WS_LEARNED) {
    std::vector<uint16_t> wb(SIM_WSN_PARAMS);
    for (int p = 0; p < SIM_WSN_PARAMS; ++p) {
      // bfloat16, nearest with ties to even
      uint32_t u;
      std::memcpy(&u, &d->ws_net[p], 4);
      u += 0x7FFFu + ((u >> 16) & 1u);
      wb[p] = (uint16_t)(u >> 16);
    }
    if ((st = upload(&h->d_wsn, wb)) != SIM_OK) { release(h); return st; }
    M.wsn = h->d_wsn;
  }
  M.dump = P.dump;
  h->tape_rows = P.tape_rows;
  h->seg_floats = (P.seg_total + 63) & ~63LL;
  h->tape_floats = M.ctrl ? ((P.tape_rows * M.tape_stride + 63) & ~63LL) : 0;
  if (max_lds > 65536 && allow_large_lds(std::min(max_lds, h->max_lds)) != hipSuccess) {
    release(h);
    return fail(SIM_E_DEVICE, "cannot raise the dynamic LDS limit");
  }
  h->lds_allowed = std::max(65536, max_lds);
  M.hdr = h->d_hdr; M.topo = h->d_topo; M.cst = h->d_cst; M.target = h->d_target;
  sim_info& I = h->info;
  I.n_envs = E; I.n_bodies = B; I.n_joints = J; I.lam_size = M.lam_tot;
  I.n_ckpt = d->T_max > 0 ? (d->T_max - 1) / d->ckpt_every + 1 : 1;
  I.ckpt_floats = (int64_t)I.n_ckpt * (18LL * B + M.lam_tot);
  {
    const long long n_chunks = M.ctrl ? (h->tape_rows + h->chunk - 1) / h->chunk : 0;
    I.workspace_bytes = 4LL * (std::max<long long>(h->seg_floats, 1) + h->tape_floats +
                               n_chunks * h->n_wtiles * 1024LL);
  }
  I.n_params = h->n_params;
  I.grad_store = M.dump == DUMP_TRAJECTORY ? SIM_GRAD_TRAJECTORY
                 : M.dump == DUMP_SEGMENT  ? SIM_GRAD_SEGMENT
                                           : SIM_GRAD_REPLAY;
  I.max_lds_bytes = max_lds;
  I.n_tiles = 0;
  for (auto& b : h->buckets) I.n_tiles += b.n_tiles;
  *out = h;
  return SIM_OK;
}

int32_t sim_describe_order(const sim_model_desc* d, int32_t env, int32_t* codes, int32_t* colours, int32_t cap) {
  if (!d || env < 0 || env >= d->n_envs) return fail(SIM_E_ARG, "sim_describe_order: bad arguments");
  PackedModel P;
  std::string perr;
  const sim_status st = pack_model(d, P, perr);
  if (st != SIM_OK) return fail(st, perr);
  const int* hd = &P.hdr[(size_t)env * H_COUNT];
  const int nj = hd[H_NJ], G = hd[H_G], Pn = hd[H_P], ncol = hd[H_NCOL], ncand = hd[H_NCAND];
  const int* tp = P.topo.data() + hd[H_TOPO];
  const int* gbody = tp + 2 * nj;
  const int* pcode = gbody + G;
  const int* colstart = pcode + Pn;
  const int* cand = colstart + ncol + 1;
  // ground index -> global sphere index
  std::vector<int> gsph;
  for (int s = d->env_sphere_off[env]; s < d->env_sphere_off[env + 1]; ++s)
    if ((d->sphere_flags[s] & 1) && d->ground) gsph.push_back(s);
  for (int c = 0; c < ncol; ++c)
    for (int i = colstart[c]; i < colstart[c + 1]; ++i) {
      if (i >= cap) continue;
      const int k = cand_kind(cand[i]), x = cand_idx(cand[i]);
      int v = x;
      if (k == K_JOINT) v = hd[H_J0] + x;
      else if (k == K_GROUND) v = gsph[x];
      else v = (pcode[x] & 0xFFFF) | ((pcode[x] >> 16) << 12);
      if (codes) codes[i] = (k << 24) | v;
      if (colours) colours[i] = c;
    }
  return ncand;
}

sim_status sim_destroy(sim_handle h) {
  if (!h) return fail(SIM_E_ARG, "sim_destroy: null handle");
  if (h->n_graphs > 0) return fail(SIM_E_STATE, "sim_destroy: step graphs of this handle are still alive");
  release(h);
  return SIM_OK;
}

sim_status sim_get_info(sim_handle h, sim_info* info) {
  if (!h || !info) return fail(SIM_E_ARG, "sim_get_info: null argument");
  *info = h->info;
  return SIM_OK;
}

sim_status sim_lambda_offsets(sim_handle h, int32_t* lam_off) {
  if (!h || !lam_off) return fail(SIM_E_ARG, "sim_lambda_offsets: null argument");
  std::copy(h->lam_off.begin(), h->lam_off.end(), lam_off);
  return SIM_OK;
}

sim_status sim_step(sim_handle h, const float* x_in, float* x_out, const float* u, const float* lam_in,
                    float* lam_out, int32_t t, uint32_t* env_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "sim_step: null handle");
  if (h->M.n_envs == 0) return SIM_OK;
  if (!x_in || !x_out || (h->M.lam_tot > 0 && (!lam_in || !lam_out)) || (h->M.J > 0 && !u))
    return fail(SIM_E_ARG, "sim_step: null array");
  if (x_in == x_out) return fail(SIM_E_ARG, "sim_step: x_in must not alias x_out");
  sim_status s = check_device("sim_step (earlier fault)");
  if (s != SIM_OK) return s;
  if (t < 0 || (h->M.ctrl && t >= std::max(h->M.T_max, 1))) return fail(SIM_E_ARG, "sim_step: step index out of range");
  return launch_steps(h, x_in, x_out, u, lam_in, lam_out, t, env_flags, (hipStream_t)stream);
}

sim_status rollout(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                   float* lam_final, float* ckpt, uint32_t* env_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout: null handle");
  if (h->M.n_envs == 0) return SIM_OK;
  if (!x0 || !loss_env) return fail(SIM_E_ARG, "rollout: null x0 or loss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, "rollout: null control tape");
  sim_status s = check_device("rollout (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  RolloutArgs a{x0, u, loss_env, x_final, lam_final, ckpt, env_flags, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0}};
  DevModel M = h->M;
  if (!prep_controls(h, M, u, st)) return check_device("rollout controls");
  return run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_rollout(h, i, M, a, sx); },
                     "rollout launch");
}

sim_status rollout_solve(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                         float* lam_final, uint32_t* env_flags, int32_t* iters_env, int32_t* fallbacks_env,
                         float* records, int64_t rec_cap, uint64_t* rec_count, int32_t rec_every, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_solve: null handle");
  if (h->M.solve_mode != SIM_SOLVE_TOL) return fail(SIM_E_STATE, "rollout_solve: the model is not in tolerance mode");
  if (h->M.n_envs == 0) return SIM_OK;
  if (!x0 || !loss_env) return fail(SIM_E_ARG, "rollout_solve: null x0 or loss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, "rollout_solve: null control tape");
  if (records && (rec_cap < 0 || !rec_count || rec_every < 1))
    return fail(SIM_E_ARG, "rollout_solve: records need rec_cap >= 0, rec_count and rec_every >= 1");
  sim_status s = check_device("rollout_solve (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  RolloutArgs a{x0, u, loss_env, x_final, lam_final, nullptr, env_flags, iters_env, fallbacks_env,
                RecArgs{records, (long long)rec_cap, (unsigned long long*)rec_count, records ? rec_every : 0}};
  DevModel M = h->M;
  if (!prep_controls(h, M, u, st)) return check_device("rollout_solve controls");
  return run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_rollout(h, i, M, a, sx); },
                     "rollout_solve launch");
}

}  // extern "C"

namespace {
// The reverse sweep with its workspace given (caller memory or the
// allocation-free scratch).  Nothing in the workspace needs to start at zero:
// the recompute writes every saved working set before the reverse reads it,
// the reverse writes every controller tape row it later contracts, and the
// contraction writes every partial tile before the reduction reads it.
// kept: the workspace holds the working sets rollout_keep wrote (no recompute).
sim_status rollout_grad_ws(sim_handle h, const float* x0, const float* u, const float* ckpt,
                           const float* dloss_env, float* g_x0, float* g_u, float* g_inv_mass, float* g_inv_inertia,
                           float* g_mu, float* g_damping, float* g_anchor_p, float* g_anchor_c, void* workspace,
                           uint32_t* env_flags, void* stream, bool kept = false) {
  sim_status s = check_device("rollout_grad (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)workspace;
  GradArgs a{x0,   u,         ckpt, dloss_env, g_x0,       g_u,        g_inv_mass, g_inv_inertia,
             g_mu, g_damping, g_anchor_p, g_anchor_c, ws, env_flags};
  DevModel M = h->M;
  if (!prep_controls(h, M, u, st)) return check_device("rollout_grad controls");
  M.tape = ws + h->seg_floats;
  auto mark = [&](int k) { return !h->tev[k] || hipEventRecord(h->tev[k], st) == hipSuccess; };
  if (!mark(0)) return check_device("rollout_grad timing event");
  if (M.dump == DUMP_TRAJECTORY && !kept)
    s = run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_recompute(h, i, M, a, sx); },
                    "rollout_grad recompute launch");
  if (s != SIM_OK) return s;
  if (!mark(1) || !mark(2)) return check_device("rollout_grad timing event");
  s = run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_reverse(h, i, M, a, sx); },
                  "rollout_grad launch");
  if (s != SIM_OK) return s;
  if (!mark(3)) return check_device("rollout_grad timing event");
  if (!M.ctrl || !g_u) return s;
  // dL/dW: contraction of the per env-step deltas and activations
  if (launch_wgrad(M.tape, M.tape_stride, (int)h->tape_rows, h->chunk, h->d_tiles, h->n_wtiles,
                   M.tape + h->tape_floats, h->d_map, h->n_params, g_u, st) != hipSuccess)
    return check_device("rollout_grad weight gradient");
  return SIM_OK;
}

// Argument checks shared by both entry points.
sim_status rollout_grad_args(sim_handle h, const char* who, const float* x0, const float* u, const float* ckpt,
                             const float* dloss_env) {
  if (h->M.solve_mode != SIM_SOLVE_FIXED)
    return fail(SIM_E_UNSUPPORTED, std::string(who) + ": the gradient is of the fixed-sweep step (solve_mode 0)");
  if (!x0 || !ckpt || !dloss_env) return fail(SIM_E_ARG, std::string(who) + ": null x0, ckpt or dloss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, std::string(who) + ": null control tape");
  return SIM_OK;
}
}  // namespace

extern "C" {

sim_status rollout_grad(sim_handle h, const float* x0, const float* u, const float* ckpt, const float* dloss_env,
                        float* g_x0, float* g_u, float* g_inv_mass, float* g_inv_inertia, float* g_mu,
                        float* g_damping, float* g_anchor_p, float* g_anchor_c, void* workspace,
                        size_t workspace_bytes, uint32_t* env_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_grad: null handle");
  if (h->M.n_envs == 0) return SIM_OK;
  sim_status s = rollout_grad_args(h, "rollout_grad", x0, u, ckpt, dloss_env);
  if (s != SIM_OK) return s;
  if (!workspace || (int64_t)workspace_bytes < h->info.workspace_bytes)
    return fail(SIM_E_NOMEM, "rollout_grad: workspace smaller than sim_info.workspace_bytes (" +
                                 std::to_string(h->info.workspace_bytes) + ")");
  return rollout_grad_ws(h, x0, u, ckpt, dloss_env, g_x0, g_u, g_inv_mass, g_inv_inertia, g_mu, g_damping,
                         g_anchor_p, g_anchor_c, workspace, env_flags, stream);
}

sim_status rollout_grad_noalloc(sim_handle h, const float* x0, const float* u, const float* ckpt,
                                const float* dloss_env, float* g_x0, float* g_u, float* g_inv_mass,
                                float* g_inv_inertia, float* g_mu, float* g_damping, float* g_anchor_p,
                                float* g_anchor_c, uint32_t* env_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_grad_noalloc: null handle");
  if (h->M.n_envs == 0) return SIM_OK;
  sim_status s = rollout_grad_args(h, "rollout_grad_noalloc", x0, u, ckpt, dloss_env);
  if (s != SIM_OK) return s;
  if (h->info.workspace_bytes > (int64_t)SIM_NOALLOC_SCRATCH_BYTES)
    return fail(SIM_E_NOMEM, "rollout_grad_noalloc: the model's workspace (" +
                                 std::to_string(h->info.workspace_bytes) + " bytes) exceeds the allocation-free "
                                 "scratch (" + std::to_string((long long)SIM_NOALLOC_SCRATCH_BYTES) +
                                 " bytes); set grad_store or grad_mem_limit so that sim_info.workspace_bytes fits");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return check_device("rollout_grad_noalloc");
  if (dev != h->device) return fail(SIM_E_STATE, "rollout_grad_noalloc: the handle's device is not current");
  void* ws = scratch_of(h->device);
  if (!ws) return fail(SIM_E_STATE, "rollout_grad_noalloc: no scratch address for this device");
  return rollout_grad_ws(h, x0, u, ckpt, dloss_env, g_x0, g_u, g_inv_mass, g_inv_inertia, g_mu, g_damping,
                         g_anchor_p, g_anchor_c, ws, env_flags, stream);
}

sim_status rollout_keep(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                        float* lam_final, float* ckpt, uint32_t* env_flags, void* workspace, size_t workspace_bytes,
                        void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_keep: null handle");
  if (h->M.solve_mode != SIM_SOLVE_FIXED)
    return fail(SIM_E_UNSUPPORTED, "rollout_keep: the working sets are of the fixed-sweep step (solve_mode 0)");
  if (h->M.dump != DUMP_TRAJECTORY)
    return fail(SIM_E_UNSUPPORTED, "rollout_keep: the model's reverse sweep is not in trajectory mode "
                                   "(sim_info.grad_store; raise grad_mem_limit or set SIM_GRAD_TRAJECTORY)");
  if (h->M.n_envs == 0) return SIM_OK;
  if (!x0 || !loss_env) return fail(SIM_E_ARG, "rollout_keep: null x0 or loss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, "rollout_keep: null control tape");
  if (!workspace || (int64_t)workspace_bytes < h->info.workspace_bytes)
    return fail(SIM_E_NOMEM, "rollout_keep: workspace smaller than sim_info.workspace_bytes (" +
                                 std::to_string(h->info.workspace_bytes) + ")");
  sim_status s = check_device("rollout_keep (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  RolloutArgs a{x0, u, loss_env, x_final, lam_final, ckpt, env_flags, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0},
                (float*)workspace};
  DevModel M = h->M;
  if (!prep_controls(h, M, u, st)) return check_device("rollout_keep controls");
  return run_buckets(h, st, [&](size_t i, hipStream_t sx) { return bucket_rollout(h, i, M, a, sx); },
                     "rollout_keep launch");
}

sim_status rollout_grad_kept(sim_handle h, const float* x0, const float* u, const float* dloss_env, float* g_x0,
                             float* g_u, float* g_inv_mass, float* g_inv_inertia, float* g_mu, float* g_damping,
                             float* g_anchor_p, float* g_anchor_c, void* workspace, size_t workspace_bytes,
                             uint32_t* env_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_grad_kept: null handle");
  if (h->M.dump != DUMP_TRAJECTORY)
    return fail(SIM_E_UNSUPPORTED, "rollout_grad_kept: the model's reverse sweep is not in trajectory mode");
  if (h->M.n_envs == 0) return SIM_OK;
  if (h->M.solve_mode != SIM_SOLVE_FIXED)
    return fail(SIM_E_UNSUPPORTED, "rollout_grad_kept: the gradient is of the fixed-sweep step (solve_mode 0)");
  if (!x0 || !dloss_env) return fail(SIM_E_ARG, "rollout_grad_kept: null x0 or dloss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, "rollout_grad_kept: null control tape");
  if (!workspace || (int64_t)workspace_bytes < h->info.workspace_bytes)
    return fail(SIM_E_NOMEM, "rollout_grad_kept: workspace smaller than sim_info.workspace_bytes (" +
                                 std::to_string(h->info.workspace_bytes) + ")");
  return rollout_grad_ws(h, x0, u, nullptr, dloss_env, g_x0, g_u, g_inv_mass, g_inv_inertia, g_mu, g_damping,
                         g_anchor_p, g_anchor_c, workspace, env_flags, stream, true);
}

sim_status rollout_and_grad(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                            float* lam_final, float* ckpt, uint32_t* env_flags, const float* dloss_env, float* g_x0,
                            float* g_u, float* g_inv_mass, float* g_inv_inertia, float* g_mu, float* g_damping,
                            float* g_anchor_p, float* g_anchor_c, void* workspace, size_t workspace_bytes,
                            uint32_t* grad_flags, void* stream) {
  if (!h) return fail(SIM_E_ARG, "rollout_and_grad: null handle");
  if (h->M.solve_mode != SIM_SOLVE_FIXED)
    return fail(SIM_E_UNSUPPORTED, "rollout_and_grad: the gradient is of the fixed-sweep step (solve_mode 0)");
  if (h->M.dump != DUMP_TRAJECTORY)
    return fail(SIM_E_UNSUPPORTED, "rollout_and_grad: the model's reverse sweep is not in trajectory mode "
                                   "(sim_info.grad_store; raise grad_mem_limit or set SIM_GRAD_TRAJECTORY)");
  if (h->M.n_envs == 0) return SIM_OK;
  if (!x0 || !loss_env || !dloss_env) return fail(SIM_E_ARG, "rollout_and_grad: null x0, loss_env or dloss_env");
  if (h->M.J > 0 && h->M.T_max > 0 && !u) return fail(SIM_E_ARG, "rollout_and_grad: null control tape");
  if (!workspace || (int64_t)workspace_bytes < h->info.workspace_bytes)
    return fail(SIM_E_NOMEM, "rollout_and_grad: workspace smaller than sim_info.workspace_bytes (" +
                                 std::to_string(h->info.workspace_bytes) + ")");
  sim_status s = check_device("rollout_and_grad (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)workspace;
  RolloutArgs ra{x0, u, loss_env, x_final, lam_final, ckpt, env_flags, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0},
                 ws};
  GradArgs ga{x0,   u,         nullptr,    dloss_env,  g_x0, g_u, g_inv_mass, g_inv_inertia,
              g_mu, g_damping, g_anchor_p, g_anchor_c, ws,   grad_flags};
  DevModel Mf = h->M;
  if (!prep_controls(h, Mf, u, st)) return check_device("rollout_and_grad controls");
  DevModel Mg = Mf;
  Mg.tape = ws + h->seg_floats;
  auto mark = [&](int k) { return !h->tev[k] || hipEventRecord(h->tev[k], st) == hipSuccess; };
  if (!mark(0) || !mark(1) || !mark(2)) return check_device("rollout_and_grad timing event");
  // a bucket's reverse follows its own forward on its stream; the buckets
  // join once, after both
  s = run_buckets(h, st, [&](size_t i, hipStream_t sx) {
        return bucket_rollout(h, i, Mf, ra, sx) && bucket_reverse(h, i, Mg, ga, sx);
      }, "rollout_and_grad launch");
  if (s != SIM_OK) return s;
  if (!mark(3)) return check_device("rollout_and_grad timing event");
  if (!Mg.ctrl || !g_u) return s;
  if (launch_wgrad(Mg.tape, Mg.tape_stride, (int)h->tape_rows, h->chunk, h->d_tiles, h->n_wtiles,
                   Mg.tape + h->tape_floats, h->d_map, h->n_params, g_u, st) != hipSuccess)
    return check_device("rollout_and_grad weight gradient");
  return SIM_OK;
}

sim_status sim_time_grad(sim_handle h, void* const* ev) {
  if (!h) return fail(SIM_E_ARG, "sim_time_grad: null handle");
  for (int k = 0; k < 4; ++k) {
    if (ev && !ev[k]) return fail(SIM_E_ARG, "sim_time_grad: null event");
    h->tev[k] = ev ? (hipEvent_t)ev[k] : nullptr;
  }
  return SIM_OK;
}

sim_status sim_time_buckets(sim_handle h, void* const* ev, int32_t n) {
  if (!h) return fail(SIM_E_ARG, "sim_time_buckets: null handle");
  if (!ev) {
    h->bev.clear();
    return SIM_OK;
  }
  if (n != (int32_t)h->buckets.size())
    return fail(SIM_E_SHAPE, "sim_time_buckets: expected " + std::to_string(h->buckets.size()) + " buckets");
  std::vector<hipEvent_t> v(2 * (size_t)n);
  for (size_t k = 0; k < v.size(); ++k) {
    if (!ev[k]) return fail(SIM_E_ARG, "sim_time_buckets: null event");
    v[k] = (hipEvent_t)ev[k];
  }
  h->bev.swap(v);
  return SIM_OK;
}

sim_status sim_env_buckets(sim_handle h, int32_t* bucket_of_env) {
  if (!h || !bucket_of_env) return fail(SIM_E_ARG, "sim_env_buckets: null argument");
  for (size_t i = 0; i < h->buckets.size(); ++i)
    for (int e : h->buckets[i].envs_host)
      if (e >= 0) bucket_of_env[e] = (int32_t)i;
  return SIM_OK;
}

// ------------------------------------------------------------- the camera
namespace {
sim_status render_args(sim_handle h, const float* x, const sim_camera* cam, const sim_textures* tex, const char* what,
                       RenderScene& sc, RenderCam& rc, RenderTex& rt) {
  if (!h || !x || !cam || !tex || !tex->sphere || !tex->ground)
    return fail(SIM_E_ARG, std::string(what) + ": null argument");
  if (cam->width < 1 || cam->height < 1 || !(cam->focal > 0.f) || !(cam->pitch > 0.f))
    return fail(SIM_E_ARG, std::string(what) + ": image size, focal length and pixel pitch must be positive");
  if ((long long)cam->width * cam->height > (1LL << 28))
    return fail(SIM_E_ARG, std::string(what) + ": image larger than 2^28 pixels");
  if (tex->sphere_nx < 2 || tex->sphere_ny < 2 || tex->ground_nx < 2 || tex->ground_ny < 2 ||
      !(tex->ground_cell > 0.f))
    return fail(SIM_E_ARG, std::string(what) + ": textures need at least 2 x 2 texels and a positive cell");
  sc = RenderScene{h->M.n_envs, h->M.B, h->M.ground, h->d_env_sph, h->d_env_body, h->d_sph_body, h->d_sph};
  for (int k = 0; k < 3; ++k) rc.pos[k] = cam->pos[k];
  for (int k = 0; k < 9; ++k) rc.axes[k] = cam->axes[k];
  rc.focal = cam->focal;
  rc.pitch = cam->pitch;
  rc.width = cam->width;
  rc.height = cam->height;
  rt = RenderTex{tex->sphere, tex->sphere_nx, tex->sphere_ny, tex->ground, tex->ground_nx, tex->ground_ny,
                 tex->ground_cell};
  return SIM_OK;
}
}  // namespace

sim_status sim_render(sim_handle h, const float* x, const sim_camera* cam, const sim_textures* tex, float* image,
                      void* stream) {
  RenderScene sc;
  RenderCam rc;
  RenderTex rt;
  sim_status st = render_args(h, x, cam, tex, "sim_render", sc, rc, rt);
  if (st != SIM_OK) return st;
  if (!image) return fail(SIM_E_ARG, "sim_render: null image");
  if (launch_render(sc, x, rc, rt, image, (hipStream_t)stream) != hipSuccess) return check_device("sim_render");
  return SIM_OK;
}

sim_status sim_render_grad(sim_handle h, const float* x, const sim_camera* cam, const sim_textures* tex,
                           const float* w, float* g_x, void* stream) {
  RenderScene sc;
  RenderCam rc;
  RenderTex rt;
  sim_status st = render_args(h, x, cam, tex, "sim_render_grad", sc, rc, rt);
  if (st != SIM_OK) return st;
  if (!w || !g_x) return fail(SIM_E_ARG, "sim_render_grad: null weights or gradient");
  static_assert(kRenderMaxSpheres == SIM_RENDER_MAX_SPHERES, "render sphere limit");
  if (h->max_env_spheres > kRenderMaxSpheres)
    return fail(SIM_E_UNSUPPORTED, "sim_render_grad: an env has " + std::to_string(h->max_env_spheres) +
                                       " spheres, more than " + std::to_string(kRenderMaxSpheres));
  if (launch_render_grad(sc, x, rc, rt, w, g_x, (hipStream_t)stream) != hipSuccess)
    return check_device("sim_render_grad");
  return SIM_OK;
}

// ------------------------------------------------------------- graphs, tuning
sim_status sim_step_graph(sim_handle h, int32_t n_steps, float* x, const float* u, float* lam, int32_t t0,
                          uint32_t* env_flags, sim_graph* out) {
  if (!h || !out) return fail(SIM_E_ARG, "sim_step_graph: null argument");
  *out = nullptr;
  if (n_steps < 1) return fail(SIM_E_ARG, "sim_step_graph: n_steps < 1");
  const DevModel& M = h->M;
  if (M.n_envs > 0 && (!x || (M.lam_tot > 0 && !lam) || (M.J > 0 && !u)))
    return fail(SIM_E_ARG, "sim_step_graph: null array");
  if (t0 < 0 || (M.ctrl && (long long)t0 + n_steps > std::max(M.T_max, 1)))
    return fail(SIM_E_ARG, "sim_step_graph: step indices outside [0, T_max)");
  sim_status s = check_device("sim_step_graph (earlier fault)");
  if (s != SIM_OK) return s;
  sim_graph_s* g = new sim_graph_s();
  g->h = h;
  ++h->n_graphs;
  if (M.n_envs == 0) {
    if (hipGraphCreate(&g->graph, 0) != hipSuccess ||
        hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
      sim_graph_destroy(g);
      return check_device("sim_step_graph instantiate");
    }
    *out = g;
    return SIM_OK;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    sim_graph_destroy(g);
    return fail(SIM_E_DEVICE, "sim_step_graph: cannot create the capture stream");
  }
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    sim_graph_destroy(g);
    return check_device("sim_step_graph begin capture");
  }
  const size_t xs = (size_t)18 * M.B;
  for (int k = 0; k < n_steps && s == SIM_OK; ++k) {
    const float* uk = M.ctrl ? u : (u ? u + (size_t)k * M.J : nullptr);
    s = launch_steps(h, x + (k & 1) * xs, x + ((k + 1) & 1) * xs, uk, lam, lam, t0 + k, env_flags, cs);
  }
  const hipError_t ec = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (s != SIM_OK || ec != hipSuccess || hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    sim_graph_destroy(g);
    return s != SIM_OK ? s : check_device("sim_step_graph capture");
  }
  *out = g;
  return SIM_OK;
}

sim_status sim_graph_launch(sim_graph g, void* stream) {
  if (!g || !g->exec) return fail(SIM_E_ARG, "sim_graph_launch: null graph");
  if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return check_device("sim_graph_launch");
  return SIM_OK;
}

sim_status sim_graph_destroy(sim_graph g) {
  if (!g) return fail(SIM_E_ARG, "sim_graph_destroy: null graph");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->h) --g->h->n_graphs;
  delete g;
  return SIM_OK;
}

int32_t sim_get_teams(sim_handle h, int32_t* teams, int32_t cap) {
  if (!h) return fail(SIM_E_ARG, "sim_get_teams: null handle");
  const int n = (int)h->buckets.size();
  for (int i = 0; i < n && teams && i < cap; ++i) teams[i] = h->buckets[i].team;
  return n;
}

sim_status sim_set_teams(sim_handle h, const int32_t* teams, int32_t n) {
  if (!h || (n > 0 && !teams)) return fail(SIM_E_ARG, "sim_set_teams: null argument");
  if (h->n_graphs > 0) return fail(SIM_E_STATE, "sim_set_teams: destroy the step graphs of this handle first");
  if (n != (int)h->buckets.size())
    return fail(SIM_E_SHAPE, "sim_set_teams: expected " + std::to_string(h->buckets.size()) + " team widths");
  for (int i = 0; i < n; ++i) {
    const auto ok = admissible_teams(h, h->buckets[i]);
    if (std::find(ok.begin(), ok.end(), teams[i]) == ok.end())
      return fail(SIM_E_ARG, "sim_set_teams: team " + std::to_string(teams[i]) + " not admissible for bucket " +
                                 std::to_string(i));
  }
  if (hipDeviceSynchronize() != hipSuccess) return check_device("sim_set_teams");
  for (int i = 0; i < n; ++i) {
    const sim_status s = retile(h, h->buckets[i], teams[i]);
    if (s != SIM_OK) return s;
  }
  return SIM_OK;
}

int32_t sim_tune(sim_handle h, const float* x0, const float* u, int32_t with_grad, int32_t max_candidates,
                 int32_t* teams, int32_t cap, void* stream) {
  if (!h) return fail(SIM_E_ARG, "sim_tune: null handle");
  const DevModel& M0 = h->M;
  const int n = (int)h->buckets.size();
  if (M0.n_envs == 0) return n;
  if (!x0 || (M0.J > 0 && M0.T_max > 0 && !u)) return fail(SIM_E_ARG, "sim_tune: null x0 or controls");
  if (max_candidates < 1) return fail(SIM_E_ARG, "sim_tune: max_candidates < 1");
  if (with_grad && M0.solve_mode != SIM_SOLVE_FIXED)
    return fail(SIM_E_UNSUPPORTED, "sim_tune: no gradient in tolerance mode (use with_grad = 0)");
  if (h->n_graphs > 0) return fail(SIM_E_STATE, "sim_tune: destroy the step graphs of this handle first");
  sim_status s = check_device("sim_tune (earlier fault)");
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  float *loss = nullptr, *dl = nullptr, *ck = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (float* p : {loss, dl, ck, ws})
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const int E = M0.n_envs;
  if (upload(&loss, std::vector<float>(E, 0.f)) != SIM_OK || upload(&dl, std::vector<float>(E, 1.f)) != SIM_OK ||
      hipMalloc((void**)&ck, (size_t)std::max<int64_t>(h->info.ckpt_floats, 1) * 4) != hipSuccess ||
      (with_grad && hipMalloc((void**)&ws, (size_t)h->info.workspace_bytes) != hipSuccess) ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(SIM_E_NOMEM, "sim_tune: cannot allocate temporaries");
  }
  DevModel M = M0;
  if (!prep_controls(h, M, u, st)) { cleanup(); return check_device("sim_tune controls"); }
  M.tape = ws ? ws + h->seg_floats : nullptr;
  const RolloutArgs ra{x0, u, loss, nullptr, nullptr, ck, nullptr, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0}};
  const GradArgs ga{x0, u, ck, dl, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, ws, nullptr};
  // every bucket once at its current width: warms the code and writes the checkpoints
  for (int i = 0; i < n; ++i)
    if (!bucket_rollout(h, i, M, ra, st)) { cleanup(); return check_device("sim_tune rollout"); }
  if (hipStreamSynchronize(st) != hipSuccess) { cleanup(); return check_device("sim_tune rollout"); }
  for (int i = 0; i < n; ++i) {
    const std::vector<int> cand = admissible_teams(h, h->buckets[i]);
    int best = h->buckets[i].team;
    float best_ms = -1.f;
    for (int c = 0; c < (int)cand.size() && c < max_candidates; ++c) {
      if ((s = retile(h, h->buckets[i], cand[c])) != SIM_OK) { cleanup(); return s; }
      if (hipEventRecord(e0, st) != hipSuccess || !bucket_rollout(h, i, M, ra, st) ||
          (with_grad && !bucket_grad(h, i, M, ga, st)) || hipEventRecord(e1, st) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess) {
        cleanup();
        return check_device("sim_tune timing");
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best_ms < 0.f || ms < best_ms) { best_ms = ms; best = cand[c]; }
    }
    if ((s = retile(h, h->buckets[i], best)) != SIM_OK) { cleanup(); return s; }
  }
  cleanup();
  for (int i = 0; i < n && teams && i < cap; ++i) teams[i] = h->buckets[i].team;
  return n;
}

// ------------------------------------------------------------- warm-start network
namespace {
int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    int n = 0;
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    cus[dev] = n > 0 ? n : 256;
  }
  return cus[dev];
}
}  // namespace

int64_t wsn_workspace_bytes(int64_t n) {
  if (n < 0) return fail(SIM_E_ARG, "wsn_workspace_bytes: n < 0");
  return (int64_t)wsn_parts(n, device_cus()) * (SIM_WSN_PARAMS + 1) * (int64_t)sizeof(float);
}

sim_status wsn_to_bf16(const float* w, uint16_t* w_bf16, void* stream) {
  if (!w || !w_bf16) return fail(SIM_E_ARG, "wsn_to_bf16: null argument");
  if (launch_wsn_to_bf16(w, w_bf16, (hipStream_t)stream) != hipSuccess) return check_device("wsn_to_bf16");
  return SIM_OK;
}

sim_status wsn_forward(const uint16_t* w_bf16, const float* x, int64_t stride, int64_t n, float* y, void* stream) {
  if (n < 0 || stride < SIM_WSN_IN) return fail(SIM_E_ARG, "wsn_forward: n < 0 or stride < 7");
  if (n == 0) return SIM_OK;
  if (!w_bf16 || !x || !y) return fail(SIM_E_ARG, "wsn_forward: null argument");
  if (launch_wsn_forward(w_bf16, x, stride, n, y, device_cus(), (hipStream_t)stream) != hipSuccess)
    return check_device("wsn_forward");
  return SIM_OK;
}

sim_status wsn_loss_grad(const uint16_t* w_bf16, const float* rec, int64_t stride, int64_t n, float huber,
                         int32_t relative, float* loss, float* grad, void* workspace, size_t workspace_bytes,
                         void* stream) {
  if (n < 0 || stride < SIM_WSN_IN + SIM_WSN_OUT) return fail(SIM_E_ARG, "wsn_loss_grad: n < 0 or stride < 10");
  if (!(huber >= 0.f)) return fail(SIM_E_ARG, "wsn_loss_grad: huber < 0");
  if (!w_bf16 || (n > 0 && !rec) || !workspace) return fail(SIM_E_ARG, "wsn_loss_grad: null argument");
  const int parts = wsn_parts(n, device_cus());
  if (workspace_bytes < (size_t)parts * (SIM_WSN_PARAMS + 1) * sizeof(float))
    return fail(SIM_E_NOMEM, "wsn_loss_grad: workspace smaller than wsn_workspace_bytes(n)");
  if (launch_wsn_loss_grad(w_bf16, rec, stride, n, huber, relative ? 1 : 0, (float*)workspace, parts, grad, loss,
                           (hipStream_t)stream) != hipSuccess)
    return check_device("wsn_loss_grad");
  return SIM_OK;
}

sim_status wsn_adam(float* w, uint16_t* w_bf16, const float* grad, float* m, float* v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* stream) {
  if (!w || !w_bf16 || !grad || !m || !v) return fail(SIM_E_ARG, "wsn_adam: null argument");
  if (step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return fail(SIM_E_ARG, "wsn_adam: step < 1 or beta outside [0, 1)");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  if (launch_wsn_adam(w, w_bf16, grad, m, v, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream) != hipSuccess)
    return check_device("wsn_adam");
  return SIM_OK;
}

sim_status sim_adam(float* w, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                    float beta1, float beta2, float eps, float max_norm, float* scratch, float* grad_norm,
                    void* stream) {
  if (n < 0) return fail(SIM_E_ARG, "sim_adam: n < 0");
  if (n == 0) return SIM_OK;
  if (!w || !grad || !m || !v || !scratch) return fail(SIM_E_ARG, "sim_adam: null argument");
  if (step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(max_norm >= 0.f))
    return fail(SIM_E_ARG, "sim_adam: step < 1, beta outside [0, 1) or max_norm < 0");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  hipStream_t st = (hipStream_t)stream;
  if (launch_adam(w, grad, m, v, n, lr, beta1, beta2, eps, c1, c2, max_norm, scratch, grad_norm, st) != hipSuccess)
    return check_device("sim_adam");
  return SIM_OK;
}

}  // extern "C"
