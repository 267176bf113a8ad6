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
// bfloat16 rounding of a double: 8 significant bits, nearest, ties to even
double bf16r(double x) {
  if (!std::isfinite(x) || x == 0.0) return x;
  int e;
  (void)std::frexp(x, &e);
  const double q = std::ldexp(1.0, e - 8);
  return std::nearbyint(x / q) * q;
}
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
  void ctrl_forward(const DevModel& M, const Env& E) const {
    const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
    const double *W1 = M.W, *b1 = W1 + n1 * in, *W2 = b1 + n1, *b2 = W2 + n2 * n1, *W3 = b2 + n2, *b3 = W3 + no * n2;
    double* s = E.mlp();
    double *h1 = s + mo_h1(M), *h2 = s + mo_h2(M), *u = s + mo_u(M);
    for (int i = 0; i < n1; ++i) {
      double a = b1[i];
      for (int k = 0; k < in; ++k) a += W1[i * in + k] * s[k];
      h1[i] = std::tanh(a);
    }
    for (int i = 0; i < n2; ++i) {
      double a = b2[i];
      for (int k = 0; k < n1; ++k) a += W2[i * n1 + k] * h1[k];
      h2[i] = std::tanh(a);
    }
    for (int i = 0; i < no; ++i) {
      double a = b3[i];
      for (int k = 0; k < n2; ++k) a += W3[i * n2 + k] * h2[k];
      u[i] = a;
    }
  }
  void ctrl_backward(const DevModel& M, const Env& E) const {
    const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
    const double *W1 = M.W, *W2 = W1 + n1 * in + n1, *W3 = W2 + n2 * n1 + n2;
    const double* s = E.mlp();
    const double *h1 = s + mo_h1(M), *h2 = s + mo_h2(M);
    double* du = E.mlpA();
    double *d2 = du + mo_d2(M), *d1 = du + mo_d1(M), *sb = du + mo_sb(M);
    for (int k = 0; k < n2; ++k) {
      double g = 0.0;
      for (int i = 0; i < no; ++i) g += W3[i * n2 + k] * du[i];
      d2[k] = g * (1.0 - h2[k] * h2[k]);
    }
    for (int k = 0; k < n1; ++k) {
      double g = 0.0;
      for (int i = 0; i < n2; ++i) g += W2[i * n1 + k] * d2[i];
      d1[k] = g * (1.0 - h1[k] * h1[k]);
    }
    for (int k = 0; k < in; ++k) {
      double g = 0.0;
      for (int i = 0; i < n1; ++i) g += W1[i * in + k] * d1[i];
      sb[k] = g;
    }
  }
  int* shared_cnt() const { return cnt; }
  int* shared_map() const { return map; }
  // the network in plain loops, with the rounding of the matrix-core kernel
  // (bfloat16 inputs and hidden activations); accumulation in double
  void wsn_rows(int total, const int* mp) const {
    for (int i = 0; i < total; ++i) {
      const double* x = lds0 + mp[i] + XF;
      double* y = lds0 + mp[i] + XY;
      const double *W1 = net, *b1 = W1 + 448, *W2 = b1 + 64, *b2 = W2 + 4096, *W3 = b2 + 64, *b3 = W3 + 192;
      double xi[7], h1[64], h2[64];
      for (int k = 0; k < 7; ++k) xi[k] = bf16r(x[k]);
      for (int h = 0; h < 64; ++h) {
        double s = b1[h];
        for (int k = 0; k < 7; ++k) s += W1[h * 7 + k] * xi[k];
        h1[h] = bf16r(std::max(s, 0.0));
      }
      for (int h = 0; h < 64; ++h) {
        double s = b2[h];
        for (int k = 0; k < 64; ++k) s += W2[h * 64 + k] * h1[k];
        h2[h] = bf16r(std::max(s, 0.0));
      }
      for (int o = 0; o < 3; ++o) {
        double s = b3[o];
        for (int k = 0; k < 64; ++k) s += W3[o * 64 + k] * h2[k];
        y[o] = s;
      }
    }
  }
  unsigned long long reserve(unsigned long long* ctr, int n) const {
    const unsigned long long v = *ctr;
    *ctr += (unsigned long long)n;
    return v;
  }
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
  M.dump = h.P.dump;
  M.decay = d->use_grad_decay ? d->grad_decay : 1.0;
  M.has_rest = desc_has_rest(d) ? 1 : 0;
  M.servo = d->servo;
  M.rest_th = d->rest_threshold;
  M.solve_mode = d->solve_mode; M.tol = d->tol; M.max_iters = d->max_iters;
  M.ws_kind = d->ws_kind; M.fb_iters = d->fb_iters; M.fb_tol = d->fb_tol;
  if (M.ctrl) {
    M.mlp_in = d->mlp_sizes[0]; M.mlp_h1 = d->mlp_sizes[1]; M.mlp_h2 = d->mlp_sizes[2]; M.mlp_out = d->mlp_sizes[3];
    M.mlp_rec = d->mlp_rec;
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
  RolloutArgs ra{x0, u, loss, xf, lf.data(), ckpt.data(), nullptr, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0}};
  GradArgs ga{x0, u, ckpt.data(), dloss, gx0, gu, gm, gI, gmu, gd, gap, gac, seg.data(), nullptr};
  for (int ie = 0; ie < d->n_envs; ++ie) {
    std::vector<double> lds(h.P.adj_of[ie] + 16);
    Env E = make_env(h.M, ie, lds.data(), h.M.n_iters, false);
    env_rollout(tm, h.M, E, true, ra);
    if (h.M.dump == DUMP_TRAJECTORY) {
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
