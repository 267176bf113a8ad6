// Host-side packing of a model description into the per-env topology and
// constants the kernels read (no device calls: also used by host-only tools).
#include "model_pack.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace sim {
namespace {

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct HostEnv {
  int nb = 0, nj = 0, G = 0, P = 0, ncol = 0, ncand = 0, ccap = 0, nslot = 0, lam = 0;
  std::vector<int> topo;   // jpar, jchi, gbody, pcode, colstart, cand
  std::vector<float> cst;
  int team = 1;
  int fwd_floats = 0, adj_floats = 0, adj_floats_ring = 0;
  int dump_floats = 0;     // one step's saved working set (see drivers.h)
};

std::string* g_msg = nullptr;
sim_status fail(sim_status s, const std::string& m) {
  if (g_msg) *g_msg = m;
  return s;
}

// Canonical colour-major order of one env (the same definition as the
// oracle's, implemented independently here):
//  joints: greedy colour in joint order, smallest colour not used by an
//          earlier joint sharing a non-world body;
//  ground: colour = rank of the sphere among its body's ground spheres;
//  pairs:  round-robin edge colouring of the env's bodies (padded to even);
// empty colours are dropped (they do not change the order).
sim_status build_env(const sim_model_desc& d, int e, bool keep_v, HostEnv& H) {
  const int b0 = d.env_body_off[e], b1 = d.env_body_off[e + 1];
  const int j0 = d.env_joint_off[e], j1 = d.env_joint_off[e + 1];
  const int s0 = d.env_sphere_off[e], s1 = d.env_sphere_off[e + 1];
  H.nb = b1 - b0;
  H.nj = j1 - j0;
  if (H.nb > 65535) return fail(SIM_E_UNSUPPORTED, "env " + std::to_string(e) + ": more than 65535 bodies");
  std::vector<int> jpar(H.nj), jchi(H.nj);
  for (int j = 0; j < H.nj; ++j) {
    const int p = d.joint_parent[j0 + j], c = d.joint_child[j0 + j];
    if (c < b0 || c >= b1) return fail(SIM_E_SHAPE, "joint " + std::to_string(j0 + j) + ": child outside its env");
    if (p != -1 && (p < b0 || p >= b1))
      return fail(SIM_E_SHAPE, "joint " + std::to_string(j0 + j) + ": parent outside its env");
    if (p == c) return fail(SIM_E_SHAPE, "joint " + std::to_string(j0 + j) + ": parent == child");
    jpar[j] = p < 0 ? -1 : p - b0;
    jchi[j] = c - b0;
  }
  // joint colours
  std::vector<int> jcol(H.nj, 0);
  int njc = 0;
  for (int j = 0; j < H.nj; ++j) {
    std::vector<char> used(H.nj + 1, 0);
    for (int k = 0; k < j; ++k) {
      const bool share = (jpar[j] >= 0 && (jpar[j] == jpar[k] || jpar[j] == jchi[k])) ||
                         (jchi[j] == jpar[k] || jchi[j] == jchi[k]);
      if (share) used[jcol[k]] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    jcol[j] = c;
    njc = std::max(njc, c + 1);
  }
  // spheres
  std::vector<int> gsph, gsub, psph(H.nb, -1);
  int nsub = 0;
  for (int s = s0; s < s1; ++s) {
    const int b = d.sphere_body[s];
    if (b < b0 || b >= b1) return fail(SIM_E_SHAPE, "sphere " + std::to_string(s) + ": body outside its env");
    if (!(d.sphere_radius[s] >= 0.f) || !std::isfinite(d.sphere_radius[s]))
      return fail(SIM_E_ARG, "sphere " + std::to_string(s) + ": invalid radius");
    if ((d.sphere_flags[s] & 1) && d.ground) {
      int rank = 0;
      for (int q = s0; q < s; ++q)
        if ((d.sphere_flags[q] & 1) && d.sphere_body[q] == b) ++rank;
      gsph.push_back(s);
      gsub.push_back(rank);
      nsub = std::max(nsub, rank + 1);
    }
    if (d.sphere_flags[s] & 2) {
      if (psph[b - b0] >= 0)
        return fail(SIM_E_SHAPE, "body " + std::to_string(b) + ": more than one sphere-sphere contact sphere");
      psph[b - b0] = s;
    }
  }
  H.G = (int)gsph.size();
  // pair candidates, (a, b) lexicographic
  std::vector<int> pcode;
  std::vector<std::vector<int>> pidx(H.nb);
  auto joined = [&](int a, int b) {
    for (int j = 0; j < H.nj; ++j)
      if ((jpar[j] == a && jchi[j] == b) || (jpar[j] == b && jchi[j] == a)) return true;
    return false;
  };
  for (int a = 0; a < H.nb; ++a) {
    pidx[a].assign(H.nb, -1);
    for (int b = a + 1; b < H.nb; ++b) {
      if (psph[a] < 0 || psph[b] < 0 || joined(a, b)) continue;
      pidx[a][b] = (int)pcode.size();
      pcode.push_back(a | (b << 16));
    }
  }
  H.P = (int)pcode.size();
  // colour-major candidate list
  std::vector<int> colstart, cand;
  int max_col = 1;
  for (int c = 0; c < njc; ++c) {
    colstart.push_back((int)cand.size());
    for (int j = 0; j < H.nj; ++j)
      if (jcol[j] == c) cand.push_back((K_JOINT << 24) | j);
    max_col = std::max(max_col, (int)cand.size() - colstart.back());
  }
  for (int k = 0; k < nsub; ++k) {
    colstart.push_back((int)cand.size());
    for (int g = 0; g < H.G; ++g)
      if (gsub[g] == k) cand.push_back((K_GROUND << 24) | g);
  }
  if (H.P > 0) {
    const int Bp = H.nb + (H.nb & 1);
    for (int k = 0; k <= Bp - 2; ++k) {
      const int start = (int)cand.size();
      auto emit = [&](int x, int y) {
        if (x > y) std::swap(x, y);
        if (y >= H.nb) return;
        if (pidx[x][y] >= 0) cand.push_back((K_PAIR << 24) | pidx[x][y]);
      };
      emit(k, Bp - 1);
      for (int i = 1; i <= Bp / 2 - 1; ++i) emit((k + i) % (Bp - 1), ((k - i) % (Bp - 1) + (Bp - 1)) % (Bp - 1));
      if ((int)cand.size() > start) colstart.push_back(start);
    }
  }
  H.ncol = (int)colstart.size();
  colstart.push_back((int)cand.size());
  H.ncand = (int)cand.size();
  const int jr = d.servo ? 6 : 5;   // rows per joint (a servo adds its motor row)
  H.lam = jr * H.nj + 4 * H.G + 4 * H.P;
  // contact capacity per env: every candidate when few, else 2 per body + 4
  H.ccap = std::min(H.G + H.P, 2 * H.nb + 4);
  H.nslot = jr * H.nj + 4 * H.ccap;
  H.topo.clear();
  H.topo.insert(H.topo.end(), jpar.begin(), jpar.end());
  H.topo.insert(H.topo.end(), jchi.begin(), jchi.end());
  for (int g = 0; g < H.G; ++g) H.topo.push_back(d.sphere_body[gsph[g]] - b0);
  H.topo.insert(H.topo.end(), pcode.begin(), pcode.end());
  H.topo.insert(H.topo.end(), colstart.begin(), colstart.end());
  H.topo.insert(H.topo.end(), cand.begin(), cand.end());
  // constants
  H.cst.assign(cst_size(H.nb, H.nj, H.G), 0.f);
  for (int b = 0; b < H.nb; ++b) {
    const float im = d.inv_mass[b0 + b];
    if (!(im > 0.f) || !std::isfinite(im)) return fail(SIM_E_ARG, "body " + std::to_string(b0 + b) + ": inv_mass must be > 0");
    H.cst[b] = im;
    for (int k = 0; k < 3; ++k) {
      const float ii = d.inv_inertia[3 * (b0 + b) + k];
      if (!(ii >= 0.f) || !std::isfinite(ii)) return fail(SIM_E_ARG, "body " + std::to_string(b0 + b) + ": invalid inv_inertia");
      H.cst[H.nb + 3 * b + k] = ii;
    }
    if (psph[b] >= 0) {
      for (int k = 0; k < 3; ++k) H.cst[4 * H.nb + 3 * b + k] = d.sphere_offset[3 * psph[b] + k];
      H.cst[7 * H.nb + b] = d.sphere_radius[psph[b]];
    }
  }
  for (int j = 0; j < H.nj; ++j) {
    float* c = H.cst.data() + 8 * H.nb + JS * j;
    const int gj = j0 + j;
    for (int k = 0; k < 3; ++k) {
      c[JAP + k] = d.anchor_p[3 * gj + k];
      c[JAC + k] = d.anchor_c[3 * gj + k];
      c[JXP + k] = d.axis_p[3 * gj + k];
      c[JXC + k] = d.axis_c[3 * gj + k];
      c[JUP + k] = d.perp_p[3 * gj + k];
      c[JUC + k] = d.perp_c[3 * gj + k];
    }
    c[JD] = d.damping[gj];
    if (d.servo) {
      const float g = d.servo_gain[gj], tq = d.servo_torque[gj], vm = d.servo_vmax[gj];
      if (!(g >= 0.f && tq >= 0.f && vm >= 0.f) || !std::isfinite(g) || !std::isfinite(tq) || !std::isfinite(vm))
        return fail(SIM_E_ARG, "joint " + std::to_string(gj) + ": servo gain, torque and vmax must be finite and >= 0");
      c[JG] = g; c[JT] = tq; c[JV] = vm;
    }
  }
  for (int g = 0; g < H.G; ++g) {
    float* c = H.cst.data() + 8 * H.nb + JS * H.nj + 4 * g;
    for (int k = 0; k < 3; ++k) c[k] = d.sphere_offset[3 * gsph[g] + k];
    c[3] = d.sphere_radius[gsph[g]];
  }
  H.cst[8 * H.nb + JS * H.nj + 4 * H.G] = d.mu[e];
  H.cst[8 * H.nb + JS * H.nj + 4 * H.G + 1] = d.restitution ? d.restitution[e] : 0.f;
  // team size: enough lanes for the widest joint colour and half the bodies
  H.team = std::min(64, next_pow2(std::max({1, max_col, (H.nb + 1) / 2})));
  int mf = 0, ma = 0;
  if (d.ctrl_kind == 1) {
    const int rec = d.mlp_rec;
    if (d.mlp_sizes[3] != H.nj + rec || d.mlp_sizes[0] != 2 * H.nj + 2 + rec)
      return fail(SIM_E_SHAPE, "env " + std::to_string(e) +
                                   ": controller needs out = joints + rec and in = 2 joints + 2 + rec");
    H.lam += rec;   // the recurrent state rides after the impulses
    mf = mlp_fwd_floats(d.mlp_sizes[0], d.mlp_sizes[1], d.mlp_sizes[2], d.mlp_sizes[3]);
    ma = mlp_adj_floats(d.mlp_sizes[0], d.mlp_sizes[1], d.mlp_sizes[2], d.mlp_sizes[3]);
  }
  const int vs = vsave_floats(keep_v, H.nb);
  H.fwd_floats = make_lay(H.nb, H.nj, H.G, H.P, H.ncol, H.ncand, H.nj + H.ccap, H.nslot, H.lam, d.n_iters, false, mf, ma, vs).total;
  H.adj_floats = make_lay(H.nb, H.nj, H.G, H.P, H.ncol, H.ncand, H.nj + H.ccap, H.nslot, H.lam, d.n_iters, true, mf, ma, vs).total;
  H.adj_floats_ring =
      make_lay(H.nb, H.nj, H.G, H.P, H.ncol, H.ncand, H.nj + H.ccap, H.nslot, H.lam, d.n_iters, true, mf, ma, vs, true).total;
  H.dump_floats = dump_stride_of(H.fwd_floats, d.n_iters, H.nslot, H.nb);
  return SIM_OK;
}

}  // namespace

sim_status pack_model(const sim_model_desc* d, PackedModel& P, std::string& err) {
  g_msg = &err;
  const int E = d->n_envs;
  P.hdr.assign((size_t)E * H_COUNT, 0);
  P.topo.clear();
  P.cst.clear();
  P.target.assign(3 * (size_t)E, 0.f);
  P.lam_off.assign(E + 1, 0);
  P.team_of.assign(E, 1);
  P.fwd_of.assign(E, 0);
  P.adj_of.assign(E, 0);
  P.adj_ring_of.assign(E, 0);
  P.ccap_of.assign(E, 0);
  P.seg_total = 0;
  P.tape_rows = 0;
  if (d->ctrl_kind != 0 && d->ctrl_kind != 1) { g_msg = nullptr; err = "unknown ctrl_kind"; return SIM_E_ARG; }
  if (d->ctrl_kind == 1) {
    for (int k = 0; k < 4; ++k)
      if (d->mlp_sizes[k] <= 0) { g_msg = nullptr; err = "controller sizes must be > 0"; return SIM_E_ARG; }
    if (d->mlp_sizes[1] > 256 || d->mlp_sizes[2] > 256) { g_msg = nullptr; err = "controller hidden width > 256"; return SIM_E_UNSUPPORTED; }
    if (d->mlp_rec < 0) { g_msg = nullptr; err = "mlp_rec < 0"; return SIM_E_ARG; }
  }
  // per-env buffer sizes of the three reverse sweep modes
  std::vector<long long> sz_replay(E), sz_segment(E), sz_traj(E);
  const bool keep_v = d->ws_kind || desc_has_rest(d);   // as make_env sizes the LDS layout
  for (int e = 0; e < E; ++e) {
    HostEnv H;
    const sim_status st = build_env(*d, e, keep_v, H);
    if (st != SIM_OK) { g_msg = nullptr; return st; }
    int* hd = &P.hdr[(size_t)e * H_COUNT];
    hd[H_B0] = d->env_body_off[e]; hd[H_NB] = H.nb; hd[H_J0] = d->env_joint_off[e]; hd[H_NJ] = H.nj;
    hd[H_LAMOFF] = P.lam_off[e]; hd[H_LAMSZ] = H.lam; hd[H_G] = H.G; hd[H_P] = H.P; hd[H_NCOL] = H.ncol;
    hd[H_TOPO] = (int)P.topo.size(); hd[H_CST] = (int)P.cst.size(); hd[H_T] = d->T_env[e];
    hd[H_LB] = d->loss_body[e] - d->env_body_off[e]; hd[H_CCAP] = H.ccap; hd[H_NCAND] = H.ncand;
    hd[H_ENV] = e; hd[H_NSLOT] = H.nslot;
    sz_replay[e] = (long long)d->ckpt_every * (18 * H.nb + H.lam);
    sz_segment[e] = (long long)d->ckpt_every * H.dump_floats;
    sz_traj[e] = (long long)d->T_env[e] * H.dump_floats + SEG_TAIL;
    hd[H_TAPE] = (int)P.tape_rows;
    if (d->ctrl_kind == 1) P.tape_rows += d->T_env[e];
    P.topo.insert(P.topo.end(), H.topo.begin(), H.topo.end());
    P.cst.insert(P.cst.end(), H.cst.begin(), H.cst.end());
    for (int k = 0; k < 3; ++k) P.target[3 * e + k] = d->target[3 * e + k];
    P.lam_off[e + 1] = P.lam_off[e] + H.lam;
    P.team_of[e] = H.team;
    P.fwd_of[e] = H.fwd_floats;
    P.adj_of[e] = H.adj_floats;
    P.adj_ring_of[e] = H.adj_floats_ring;
    P.ccap_of[e] = H.ccap;
  }
  // Each env's block starts on a SEG_UNIT boundary; the header holds its
  // offset in those units.
  auto total_of = [&](const std::vector<long long>& sz) {
    long long t = 0;
    for (int e = 0; e < E; ++e) t += (sz[e] + SEG_UNIT - 1) / SEG_UNIT * SEG_UNIT;
    return t;
  };
  const long long tot[3] = {total_of(sz_replay), total_of(sz_segment), total_of(sz_traj)};
  const long long limit = (d->grad_mem_limit > 0 ? d->grad_mem_limit : kGradMemDefault) / 4;
  if (d->grad_store == SIM_GRAD_AUTO) {
    // the fastest mode that fits: no replay, and recomputes in parallel
    P.dump = tot[2] <= limit ? DUMP_TRAJECTORY : (tot[1] <= limit ? DUMP_SEGMENT : DUMP_REPLAY);
  } else {
    P.dump = d->grad_store == SIM_GRAD_TRAJECTORY ? DUMP_TRAJECTORY
             : d->grad_store == SIM_GRAD_SEGMENT  ? DUMP_SEGMENT
                                                  : DUMP_REPLAY;
  }
  const std::vector<long long>& sz = P.dump == DUMP_TRAJECTORY ? sz_traj
                                     : P.dump == DUMP_SEGMENT  ? sz_segment
                                                               : sz_replay;
  long long off = 0;
  for (int e = 0; e < E; ++e) {
    if (off / SEG_UNIT > 0x7fffffffLL) { g_msg = nullptr; err = "reverse sweep buffer exceeds 2^31 x 64 floats"; return SIM_E_UNSUPPORTED; }
    P.hdr[(size_t)e * H_COUNT + H_SEG] = (int)(off / SEG_UNIT);
    off += (sz[e] + SEG_UNIT - 1) / SEG_UNIT * SEG_UNIT;
  }
  P.seg_total = off;
  g_msg = nullptr;
  return SIM_OK;
}

}  // namespace sim
