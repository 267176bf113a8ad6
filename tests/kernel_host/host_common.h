// TEST INFRASTRUCTURE ONLY: host-side pieces shared by the builds of the
// library's kernel source for the host (one-lane teams in kernel_fp64.cpp,
// multi-lane waves in kernel_lanes.cpp): the kernel source in double
// precision, the controller's layers and the warm-start network as plain
// loops, and the device model made from a description.
#pragma once
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
inline void host_ctrl_forward(const DevModel& M, const Env& E) {
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
inline void host_ctrl_backward(const DevModel& M, const Env& E) {
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
// the network in plain loops, with the rounding of the matrix-core kernel
// (bfloat16 inputs and hidden activations); accumulation in double
inline void host_wsn_rows(double* lds0, const double* net, int total, const int* mp) {
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
struct Host { PackedModel P; DevModel M; std::vector<double> clock; };
// 1: every env of a model whose reverse reads saved working sets keeps a ring
// of the impulse history (the library takes it where it lets a CU hold more
// envs); 0: none does
int g_force_ring = 0;
bool make(const sim_model_desc* d, Host& h) {
  std::string err;
  if (pack_model(d, h.P, err) != SIM_OK) { fprintf(stderr, "pack: %s\n", err.c_str()); return false; }
  if (g_force_ring && h.P.dump != DUMP_REPLAY) {
    for (int e = 0; e < d->n_envs; ++e) h.P.hdr[(size_t)e * H_COUNT + H_RING] = 1;
    h.P.adj_of = h.P.adj_ring_of;
  }
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
