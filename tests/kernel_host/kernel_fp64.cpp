// TEST INFRASTRUCTURE ONLY: the library's kernel source (step_core.h,
// drivers.h) compiled for the host in double precision, one env at a time
// with one-lane teams.  It checks the algebra of the forward step and of the
// hand-written adjoint against the FP64 oracle to ~1e-9 (what remains on the
// GPU is FP32 rounding).  Nothing in the product loads this library.
#include "host_common.h"
using namespace sim;
namespace {
struct TeamHost {
  int tl = 0, ts = 1, team = 0, n_teams = 1;
  double* lds0 = nullptr;
  int* cnt = nullptr;
  int* map = nullptr;
  const double* net = nullptr;   // warm-start network parameters (bfloat16 values)
  void sync() const {}
  bool any(bool p) const { return p; }
  int prefix(bool p, int& total) const { total = p ? 1 : 0; return 0; }
  double team_sum(double v) const { return v; }
  double team_max(double v) const { return v; }
  bool team_any(bool p) const { return p; }
  double pair_swap(double v) const { return v; }   // one-lane teams never pair
  // the controller's layers in plain loops (the GPU does them as matrix-core
  // products over the envs of a wave)
  void ctrl_forward(const DevModel& M, const Env& E) const { host_ctrl_forward(M, E); }
  void ctrl_backward(const DevModel& M, const Env& E) const { host_ctrl_backward(M, E); }
  int* shared_cnt() const { return cnt; }
  int* shared_map() const { return map; }
  void wsn_rows(int total, const int* mp) const { host_wsn_rows(lds0, net, total, mp); }
  unsigned long long reserve(unsigned long long* ctr, int n) const {
    const unsigned long long v = *ctr;
    *ctr += (unsigned long long)n;
    return v;
  }
};
}  // namespace
extern "C" {
void kh_set_ring(int on) { g_force_ring = on; }
// 1: in trajectory mode the rollout keeps the working sets (rollout_keep) and
// the reverse reads them without a recompute (rollout_grad_kept)
static int g_keep = 0;
void kh_set_keep(int on) { g_keep = on; }
int kh_sizes(const sim_model_desc* d, long long* out) {
  Host h;
  if (!make(d, h)) return -1;
  const int n_ckpt = d->T_max > 0 ? (d->T_max - 1) / d->ckpt_every + 1 : 1;
  out[0] = h.M.lam_tot; out[1] = h.P.seg_total; out[2] = (long long)n_ckpt * (18LL * h.M.B + h.M.lam_tot);
  out[3] = h.P.dump;
  out[4] = *std::max_element(h.P.fwd_of.begin(), h.P.fwd_of.end());
  out[5] = *std::max_element(h.P.adj_of.begin(), h.P.adj_of.end());
  return 0;
}
int kh_rollout_grad(const sim_model_desc* d, const double* x0, const double* u, const double* dloss, double* loss,
                    double* xf, double* gx0, double* gu, double* gm, double* gI, double* gmu, double* gd,
                    double* gap, double* gac) {
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
  const bool keep = g_keep && h.M.dump == DUMP_TRAJECTORY;
  RolloutArgs ra{x0, u, loss, xf, lf.data(), ckpt.data(), nullptr, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0},
                 keep ? seg.data() : nullptr};
  GradArgs ga{x0, u, ckpt.data(), dloss, gx0, gu, gm, gI, gmu, gd, gap, gac, seg.data(), nullptr};
  for (int ie = 0; ie < d->n_envs; ++ie) {
    std::vector<double> lds(h.P.adj_of[ie] + 16);
    Env E = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
    if (keep) env_rollout_keep(tm, h.M, E, true, ra);
    else env_rollout(tm, h.M, E, true, ra);
    if (h.M.dump == DUMP_TRAJECTORY && !keep) {
      // every segment recomputed on its own from its checkpoint (last first:
      // the order must not matter)
      const int K = h.M.ckpt_every, nseg = (d->T_env[ie] + K - 1) / K;
      for (int sg = nseg - 1; sg >= 0; --sg) {
        std::fill(lds.begin(), lds.end(), std::nan(""));
        Env ER = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
        env_recompute(tm, h.M, ER, true, ga, sg);
      }
      std::fill(lds.begin(), lds.end(), std::nan(""));
    }
    Env EA = make_env(h.M, ie, lds.data(), h.M.n_iters, true);
    if (h.M.dump != DUMP_REPLAY) env_rollout_grad<true>(tm, h.M, EA, true, ga);
    else env_rollout_grad<false>(tm, h.M, EA, true, ga);
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

// Tolerance-mode forward rollout (plain or learned warm start) with sweep and
// fallback counts and training records; returns the number of records.
long long kh_rollout_solve(const sim_model_desc* d, const double* x0, const double* u, double* loss, double* xf,
                           int* iters, int* fbs, double* rec, long long rec_cap, int rec_every) {
  Host h;
  if (!make(d, h)) return -1;
  std::vector<double> lf(h.M.lam_tot + 1), net(4867, 0.0);
  if (d->ws_kind)
    for (int p = 0; p < 4867; ++p) net[p] = bf16r(d->ws_net[p]);
  unsigned long long count = 0;
  RolloutArgs ra{x0, u, loss, xf, lf.data(), nullptr, nullptr, iters, fbs,
                 RecArgs{rec, rec_cap, &count, rec ? rec_every : 0}};
  for (int ie = 0; ie < d->n_envs; ++ie) {
    std::vector<double> lds(h.P.fwd_of[ie] + 16);
    std::vector<int> cnt(64), map(h.P.ccap_of[ie] + 1);
    TeamHost tm;
    tm.lds0 = lds.data();
    tm.cnt = cnt.data();
    tm.map = map.data();
    tm.net = net.data();
    Env E = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
    env_rollout<TeamHost, true>(tm, h.M, E, true, ra);
  }
  return (long long)count;
}
}
