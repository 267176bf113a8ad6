// TEST INFRASTRUCTURE ONLY: the library's kernel source (step_core.h,
// drivers.h) compiled for the host in double precision, one env at a time
// with one-lane teams.  It checks the algebra of the forward step and of the
// hand-written adjoint against the FP64 oracle to ~1e-9 (what remains on the
// GPU is FP32 rounding).  Nothing in the product loads this library.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#define float double
#define sqrtf sqrt
#define fabsf fabs
#define fmaxf fmax
#include "../../paper_1611_01652_amd/csrc/drivers.h"
#include "../../paper_1611_01652_amd/csrc/model_pack.h"
#include "../../paper_1611_01652_amd/csrc/model_pack.cpp"
using namespace sim;
namespace {
struct TeamHost {
  int tl = 0, ts = 1;
  void sync() const {}
  bool any(bool p) const { return p; }
  int prefix(bool p, int& total) const { total = p ? 1 : 0; return 0; }
  double team_sum(double v) const { return v; }
  bool team_any(bool p) const { return p; }
};
struct Host { PackedModel P; DevModel M; };
bool make(const sim_model_desc* d, Host& h) {
  std::string err;
  if (pack_model(d, h.P, err) != SIM_OK) { fprintf(stderr, "pack: %s\n", err.c_str()); return false; }
  DevModel& M = h.M;
  M.n_envs = d->n_envs; M.B = d->env_body_off[d->n_envs]; M.J = d->env_joint_off[d->n_envs];
  M.T_max = d->T_max; M.n_iters = d->n_iters; M.ground = d->ground; M.loss_kind = d->loss_kind;
  M.loss_mask = d->loss_mask; M.ckpt_every = d->ckpt_every; M.dt = d->dt; M.gx = d->gravity[0];
  M.gy = d->gravity[1]; M.gz = d->gravity[2]; M.beta = d->beta; M.gamma = d->gamma; M.spec = d->spec_margin;
  M.warm = d->warm; M.lam_tot = h.P.lam_off[d->n_envs];
  M.hdr = h.P.hdr.data(); M.topo = h.P.topo.data(); M.cst = h.P.cst.data(); M.target = h.P.target.data();
  return true;
}
}  // namespace
extern "C" {
int kh_sizes(const sim_model_desc* d, long long* out) {
  Host h;
  if (!make(d, h)) return -1;
  const int n_ckpt = d->T_max > 0 ? (d->T_max - 1) / d->ckpt_every + 1 : 1;
  out[0] = h.M.lam_tot; out[1] = h.P.seg_total; out[2] = (long long)n_ckpt * (18LL * h.M.B + h.M.lam_tot);
  return 0;
}
int kh_rollout_grad(const sim_model_desc* d, const double* x0, const double* u, const double* dloss, double* loss,
                    double* xf, double* gx0, double* gu, double* gm, double* gI, double* gmu, double* gd) {
  Host h;
  if (!make(d, h)) return -1;
  const int n_ckpt = d->T_max > 0 ? (d->T_max - 1) / d->ckpt_every + 1 : 1;
  std::vector<double> ckpt((size_t)n_ckpt * (18 * h.M.B + h.M.lam_tot) + 1), lf(h.M.lam_tot + 1), seg(h.P.seg_total + 1);
  TeamHost tm;
  RolloutArgs ra{x0, u, loss, xf, lf.data(), ckpt.data(), nullptr};
  GradArgs ga{x0, u, ckpt.data(), dloss, gx0, gu, gm, gI, gmu, gd, seg.data()};
  for (int ie = 0; ie < d->n_envs; ++ie) {
    std::vector<double> lds(h.P.adj_of[ie] + 16);
    Env E = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
    env_rollout(tm, h.M, E, true, ra);
    Env EA = make_env(h.M, ie, lds.data(), h.M.n_iters, true);
    env_rollout_grad(tm, h.M, EA, true, ga);
  }
  return 0;
}
}
