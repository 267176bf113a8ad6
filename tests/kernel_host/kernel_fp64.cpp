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
#define tanhf tanh
#define atan2f atan2
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
struct Host { PackedModel P; DevModel M; std::vector<double> clock; };
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
  M.ctrl = d->ctrl_kind;
  if (M.ctrl) {
    M.mlp_in = d->mlp_sizes[0]; M.mlp_h1 = d->mlp_sizes[1]; M.mlp_h2 = d->mlp_sizes[2]; M.mlp_out = d->mlp_sizes[3];
    M.tape_stride = tape_len(M.mlp_in, M.mlp_h1, M.mlp_h2, M.mlp_out);
    h.clock.assign(2 * (size_t)std::max(d->T_max, 1), 0.0);
    for (int t = 0; t < d->T_max; ++t) {
      const double ph = 2.0 * M_PI * d->clock_hz * (t * d->dt);
      h.clock[2 * t] = std::sin(ph);
      h.clock[2 * t + 1] = std::cos(ph);
    }
    M.clock = h.clock.data();
  }
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
  std::vector<double> tape;
  if (h.M.ctrl) {
    tape.assign((size_t)h.P.tape_rows * h.M.tape_stride + 1, 0.0);
    h.M.W = u;
    h.M.tape = tape.data();
  }
  RolloutArgs ra{x0, u, loss, xf, lf.data(), ckpt.data(), nullptr};
  GradArgs ga{x0, u, ckpt.data(), dloss, gx0, gu, gm, gI, gmu, gd, seg.data()};
  for (int ie = 0; ie < d->n_envs; ++ie) {
    std::vector<double> lds(h.P.adj_of[ie] + 16);
    Env E = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
    env_rollout(tm, h.M, E, true, ra);
    Env EA = make_env(h.M, ie, lds.data(), h.M.n_iters, true);
    env_rollout_grad(tm, h.M, EA, true, ga);
  }
  if (h.M.ctrl) {
    // dL/dW: the same contraction the GPU does with MFMA, in plain loops
    const DevModel& M = h.M;
    const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
    const int lay[3][6] = {{tape_d1(M), n1, tape_s(M), in, 0, n1 * in},
                           {tape_d2(M), n2, tape_h1(M), n1, n1 * in + n1, n1 * in + n1 + n2 * n1},
                           {tape_du(M), no, tape_h2(M), n2, n1 * in + n1 + n2 * n1 + n2,
                            n1 * in + n1 + n2 * n1 + n2 + no * n2}};
    const int np = n1 * in + n1 + n2 * n1 + n2 + no * n2 + no;
    for (int p = 0; p < np; ++p) gu[p] = 0.0;
    for (long long r = 0; r < h.P.tape_rows; ++r) {
      const double* row = tape.data() + r * M.tape_stride;
      for (int l = 0; l < 3; ++l)
        for (int i = 0; i < lay[l][1]; ++i) {
          const double dl = row[lay[l][0] + i];
          for (int k = 0; k < lay[l][3]; ++k) gu[lay[l][4] + i * lay[l][3] + k] += dl * row[lay[l][2] + k];
          gu[lay[l][5] + i] += dl;
        }
    }
  }
  return 0;
}
}
