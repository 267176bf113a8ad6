// FP64 CPU oracle of the differentiable rigid-body time step.
//
// TEST INFRASTRUCTURE ONLY. Tests, the smoke check and the benchmark's CPU
// baseline leg call this; the product library never includes, links or runs
// it, and it shares no code with the GPU path.  Only the seeded input
// generators serve both sides.
//
// What it computes (paper section 2.1 and eq. (L)/(g) of section 2.2):
//   x^{t+1} = f_ph(x^t, u^t): bodies with 6 DOF (position, rotation matrix,
//   linear and angular velocity) exchange impulses under hinge and sphere
//   contact constraints; the impulses solve the LCP approximately by a fixed
//   number of projected Gauss-Seidel sweeps with softened (Baumgarte)
//   constraints; the new velocities are integrated by semi-implicit Euler and
//   the rotation matrix is renormalised (eq. (1), read as
//   N(A) = (3A - A A^T A)/2).  L = sum_t l(x^t, p); the gradient is the exact
//   reverse-mode derivative of the unrolled discrete map (BPTT, section 2.1.1),
//   derived mechanically by the operator-overloading tape in scalar.hpp from
//   this same code, one step at a time from stored step-start states.
//
// Every choice the paper leaves open (softening constants, sweep order, warm
// start, friction model, tie-breaks at kinks) is fixed in the design notes
// and implemented here in the most direct form.
//
// Parity pins live in tests/test_oracle_*.py: free fall and ballistic closed
// forms, a ball at rest, sliding-to-rolling at 5/7 of the initial speed,
// momentum conservation, pendulum period, spin angle n*atan(dt*w), LCP brute
// force, central finite differences of the gradient; the controller's
// sensor and clock inputs read back through routing weights, the loss kinds
// on straight-line flight (values and gradients), motor torque, damping decay
// and the world inertia about a hinge, the angular-momentum balance of a
// free chain, and pair friction (momentum, the Coulomb disk, independence of
// the tangent basis).
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "oracle.h"
#include "scalar.hpp"

namespace orc {

// ------------------------------------------------------------------ vectors
template <class S> struct V3 {
  S x, y, z;
  V3() : x(0.0), y(0.0), z(0.0) {}
  V3(S a, S b, S c) : x(a), y(b), z(c) {}
};
template <class S> V3<S> operator+(const V3<S>& a, const V3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> V3<S> operator-(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> V3<S> operator-(const V3<S>& a) { return {-a.x, -a.y, -a.z}; }
template <class S> V3<S> operator*(const S& s, const V3<S>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class S> V3<S> cvt(const double* p) { return {S(p[0]), S(p[1]), S(p[2])}; }

template <class S> struct M3 {
  S m[3][3];
  M3() { for (auto& r : m) for (auto& e : r) e = S(0.0); }
};
template <class S> V3<S> operator*(const M3<S>& A, const V3<S>& v) {
  return {A.m[0][0] * v.x + A.m[0][1] * v.y + A.m[0][2] * v.z,
          A.m[1][0] * v.x + A.m[1][1] * v.y + A.m[1][2] * v.z,
          A.m[2][0] * v.x + A.m[2][1] * v.y + A.m[2][2] * v.z};
}
template <class S> M3<S> matmul(const M3<S>& A, const M3<S>& B) {
  M3<S> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
  return C;
}
template <class S> M3<S> transpose(const M3<S>& A) {
  M3<S> T;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T.m[i][j] = A.m[j][i];
  return T;
}
template <class S> M3<S> skew(const V3<S>& w) {
  M3<S> K;
  K.m[0][1] = -w.z; K.m[0][2] = w.y;
  K.m[1][0] = w.z;  K.m[1][2] = -w.x;
  K.m[2][0] = -w.y; K.m[2][1] = w.x;
  return K;
}

// ------------------------------------------------------------------ model
struct Model {
  oracle_model c;
  int n_bodies = 0, n_joints = 0, n_spheres = 0;
};

// Per-env static topology: contact candidates and the canonical sweep order.
struct PairCand { int sa, sb, ba, bb; };  // spheres (global), bodies (global), ba < bb
struct Con { int kind, idx; };            // kind 0 joint (global idx), 1 ground (sphere), 2 pair (cand idx)
struct EnvTopo {
  int b0, nb, j0, nj, s0, ns;
  std::vector<int> ground;      // global sphere ids with the ground flag, sphere order
  std::vector<PairCand> pairs;  // candidate pairs, (local a, local b) lexicographic
  std::vector<Con> order;       // canonical colour-major order of all candidate constraints
  int lam_off, lam_size;        // carried-state block: warm-start impulses, then the controller's h
  int lam_imp;                  // impulses in it (the rest is h)
  int jr;                       // rows (and carried impulses) per joint: 5, 6 with servos
};

static bool joined(const Model& M, const EnvTopo& E, int ga, int gb) {
  for (int j = E.j0; j < E.j0 + E.nj; ++j) {
    const int p = M.c.joint_parent[j], c = M.c.joint_child[j];
    if ((p == ga && c == gb) || (p == gb && c == ga)) return true;
  }
  return false;
}

// Canonical order (the paper fixes none; sweep order is part of the result
// after a fixed number of Gauss-Seidel sweeps):
//  1. joints, greedy colours in joint order (smallest colour not used by an
//     earlier joint sharing a non-world body);
//  2. ground contacts, colour = rank of the sphere among its body's ground spheres;
//  3. sphere pairs, round-robin edge colouring of the env's bodies.
// Inside one colour constraints touch disjoint bodies, so their order is
// immaterial; here they are listed by index.
static EnvTopo build_topo(const Model& M, int e, int lam_off) {
  const oracle_model& c = M.c;
  EnvTopo E;
  E.b0 = c.env_body_off[e]; E.nb = c.env_body_off[e + 1] - E.b0;
  E.j0 = c.env_joint_off[e]; E.nj = c.env_joint_off[e + 1] - E.j0;
  E.s0 = c.env_sphere_off[e]; E.ns = c.env_sphere_off[e + 1] - E.s0;
  // joint colours
  std::vector<int> jcol(E.nj, 0);
  int njc = 0;
  for (int j = 0; j < E.nj; ++j) {
    std::vector<char> used(E.nj + 1, 0);
    const int pj = c.joint_parent[E.j0 + j], cj = c.joint_child[E.j0 + j];
    for (int k = 0; k < j; ++k) {
      const int pk = c.joint_parent[E.j0 + k], ck = c.joint_child[E.j0 + k];
      bool share = false;
      for (int x : {pj, cj})
        for (int y : {pk, ck})
          if (x >= 0 && x == y) share = true;
      if (share) used[jcol[k]] = 1;
    }
    int col = 0;
    while (used[col]) ++col;
    jcol[j] = col;
    njc = std::max(njc, col + 1);
  }
  for (int col = 0; col < njc; ++col)
    for (int j = 0; j < E.nj; ++j)
      if (jcol[j] == col) E.order.push_back({0, E.j0 + j});
  // ground contacts
  if (c.ground) {
    std::vector<int> sub;
    int nsub = 0;
    for (int s = E.s0; s < E.s0 + E.ns; ++s) {
      if (!(c.sphere_flags[s] & 1)) continue;
      int rank = 0;
      for (int q = E.s0; q < s; ++q)
        if ((c.sphere_flags[q] & 1) && c.sphere_body[q] == c.sphere_body[s]) ++rank;
      E.ground.push_back(s);
      sub.push_back(rank);
      nsub = std::max(nsub, rank + 1);
    }
    for (int k = 0; k < nsub; ++k)
      for (size_t g = 0; g < E.ground.size(); ++g)
        if (sub[g] == k) E.order.push_back({1, (int)g});
  }
  // sphere pairs: one pair sphere per body at most
  std::vector<int> psph(E.nb, -1);
  for (int s = E.s0; s < E.s0 + E.ns; ++s)
    if (c.sphere_flags[s] & 2) psph[c.sphere_body[s] - E.b0] = s;
  std::vector<std::vector<int>> cand_of(E.nb, std::vector<int>(E.nb, -1));
  for (int a = 0; a < E.nb; ++a)
    for (int b = a + 1; b < E.nb; ++b) {
      if (psph[a] < 0 || psph[b] < 0) continue;
      if (joined(M, E, E.b0 + a, E.b0 + b)) continue;
      cand_of[a][b] = (int)E.pairs.size();
      E.pairs.push_back({psph[a], psph[b], E.b0 + a, E.b0 + b});
    }
  if (!E.pairs.empty()) {
    const int Bp = E.nb + (E.nb & 1);
    for (int k = 0; k <= Bp - 2; ++k) {
      auto emit = [&](int x, int y) {
        if (x > y) std::swap(x, y);
        if (y >= E.nb) return;  // padded body
        if (cand_of[x][y] >= 0) E.order.push_back({2, cand_of[x][y]});
      };
      emit(k, Bp - 1);
      for (int i = 1; i <= Bp / 2 - 1; ++i) emit((k + i) % (Bp - 1), ((k - i) % (Bp - 1) + (Bp - 1)) % (Bp - 1));
    }
  }
  E.lam_off = lam_off;
  E.jr = c.servo ? 6 : 5;
  E.lam_imp = E.jr * E.nj + 4 * (int)E.ground.size() + 4 * (int)E.pairs.size();
  E.lam_size = E.lam_imp + (c.ctrl_kind == 1 ? c.mlp_rec : 0);
  return E;
}

// ------------------------------------------------------------------ rows
template <class S> struct Row {
  int a = -1, b = -1;           // local bodies, -1 = world
  V3<S> la, aa, lb, ab;         // Jacobian: linear/angular for a and b
  V3<S> Wla, Waa, Wlb, Wab;     // W = M^-1 J^T
  S m = S(0.0), bias = S(0.0), lam = S(0.0);
  double lo = -INFINITY, hi = INFINITY;
};
template <class S> struct ConRows {
  int kind;       // 0 joint (5 scalar rows, 6 with a servo), 1 contact (normal + friction block)
  int store;      // offset into the warm-start block
  int nrows;
  Row<S> r[6];
  V3<S> t1, t2;   // contact tangents (for the tangent impulse carry)
  S mt = S(0.0);  // friction block effective mass
  S gap = S(0.0); // contact gap
  int code = 0;   // candidate code: kind << 24 | id (ground: the env's ground-sphere index, pair: local a | local b << 12)
};

// Solver statistics and training records of one step (tolerance mode).
struct StepStats {
  int env = 0;
  int sweeps = 0;                      // Gauss-Seidel sweeps, discarded ones included
  int fallbacks = 0;                   // learned warm starts rejected
  int rec_every = 0;                   // records at steps t with t % rec_every == 0 (0: none)
  std::vector<double>* recs = nullptr;
};

// bfloat16: 8 significant bits, nearest with ties to even (the default
// floating-point rounding mode of nearbyint).  Values below the bfloat16
// normal range are not expected here and are rounded as if normal.
static double bf16(double x) {
  if (!std::isfinite(x) || x == 0.0) return x;
  int e;
  (void)std::frexp(x, &e);
  const double q = std::ldexp(1.0, e - 8);
  return std::nearbyint(x / q) * q;
}

// Warm-start network: y = W3 h2 + b3, h2 = relu(W2 h1 + b2), h1 = relu(W1 x + b1)
// with weights, input and hidden activations rounded to bfloat16.
static void wsn_eval(const double* w, const double* f, double* y) {
  const int I = ORACLE_WSN_IN, H = ORACLE_WSN_HID, O = ORACLE_WSN_OUT;
  const double *W1 = w, *b1 = W1 + H * I, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + O * H;
  double x[ORACLE_WSN_IN], h1[ORACLE_WSN_HID], h2[ORACLE_WSN_HID];
  for (int k = 0; k < I; ++k) x[k] = bf16(f[k]);
  for (int i = 0; i < H; ++i) {
    double s = bf16(b1[i]);
    for (int k = 0; k < I; ++k) s += bf16(W1[i * I + k]) * x[k];
    h1[i] = bf16(std::max(s, 0.0));
  }
  for (int i = 0; i < H; ++i) {
    double s = bf16(b2[i]);
    for (int k = 0; k < H; ++k) s += bf16(W2[i * H + k]) * h1[k];
    h2[i] = bf16(std::max(s, 0.0));
  }
  for (int o = 0; o < O; ++o) {
    double s = bf16(b3[o]);
    for (int k = 0; k < H; ++k) s += bf16(W3[o * H + k]) * h2[k];
    y[o] = s;
  }
}

template <class S> struct Bodies {
  std::vector<V3<S>> p, v, w;
  std::vector<M3<S>> R, Iw;
  std::vector<S> invm;
};

template <class S> S jdotv(const Row<S>& r, const Bodies<S>& B) {
  S s = S(0.0);
  if (r.a >= 0) s = s + dot(r.la, B.v[r.a]) + dot(r.aa, B.w[r.a]);
  s = s + dot(r.lb, B.v[r.b]) + dot(r.ab, B.w[r.b]);
  return s;
}
template <class S> void apply(const Row<S>& r, Bodies<S>& B, const S& d) {
  if (r.a >= 0) { B.v[r.a] = B.v[r.a] + d * r.Wla; B.w[r.a] = B.w[r.a] + d * r.Waa; }
  B.v[r.b] = B.v[r.b] + d * r.Wlb; B.w[r.b] = B.w[r.b] + d * r.Wab;
}
// W = M^-1 J^T and J W (the constraint-space inverse mass of the row)
template <class S> S finish_row(Row<S>& r, const Bodies<S>& B) {
  S k = S(0.0);
  if (r.a >= 0) {
    r.Wla = B.invm[r.a] * r.la; r.Waa = B.Iw[r.a] * r.aa;
    k = k + dot(r.la, r.Wla) + dot(r.aa, r.Waa);
  }
  r.Wlb = B.invm[r.b] * r.lb; r.Wab = B.Iw[r.b] * r.ab;
  k = k + dot(r.lb, r.Wlb) + dot(r.ab, r.Wab);
  return k;
}

// ------------------------------------------------------------------ controller
// eq. (g): u^t = g_deep(s(x^t), h^t) with s = joint angles, joint rates and a
// sine/cosine clock; tanh hidden layers; the output's first J entries are the
// torques (linear), the rest give the next recurrent state h^{t+1} = tanh(.)
// (h and hn: the controller's recurrent state before and after the step).
template <class S>
void mlp_controls(const Model& M, const EnvTopo& E, int t, const Bodies<S>& B, const S* W, S* u, const S* h = nullptr,
                  S* hn = nullptr) {
  const oracle_model& c = M.c;
  const int nin = c.mlp_in, h1 = c.mlp_h1, h2 = c.mlp_h2, nout = c.mlp_out;
  std::vector<S> s(nin, S(0.0));
  for (int j = 0; j < E.nj; ++j) {
    const int gj = E.j0 + j;
    const int pa = c.joint_parent[gj], ch = c.joint_child[gj] - E.b0;
    const int a = pa >= 0 ? pa - E.b0 : -1;
    V3<S> na = cvt<S>(c.axis_p + 3 * gj), ua = cvt<S>(c.perp_p + 3 * gj), wa;
    if (a >= 0) { na = B.R[a] * na; ua = B.R[a] * ua; wa = B.w[a]; }
    const V3<S> ub = B.R[ch] * cvt<S>(c.perp_c + 3 * gj);
    s[j] = atan2(dot(cross(ua, ub), na), dot(ua, ub));
    s[E.nj + j] = dot(B.w[ch] - wa, na);
  }
  const double ph = 2.0 * M_PI * c.clock_hz * (t * c.dt);
  s[2 * E.nj] = S(std::sin(ph));
  s[2 * E.nj + 1] = S(std::cos(ph));
  for (int i = 0; i < c.mlp_rec; ++i) s[2 * E.nj + 2 + i] = h[i];
  const S* W1 = W;
  const S* b1 = W1 + h1 * nin;
  const S* W2 = b1 + h1;
  const S* b2 = W2 + h2 * h1;
  const S* W3 = b2 + h2;
  const S* b3 = W3 + nout * h2;
  std::vector<S> z1(h1), z2(h2);
  for (int i = 0; i < h1; ++i) {
    S a = b1[i];
    for (int k = 0; k < nin; ++k) a = a + W1[i * nin + k] * s[k];
    z1[i] = tanh(a);
  }
  for (int i = 0; i < h2; ++i) {
    S a = b2[i];
    for (int k = 0; k < h1; ++k) a = a + W2[i * h1 + k] * z1[k];
    z2[i] = tanh(a);
  }
  for (int i = 0; i < nout; ++i) {
    S a = b3[i];
    for (int k = 0; k < h2; ++k) a = a + W3[i * h2 + k] * z2[k];
    if (i < E.nj) u[i] = a;
    else hn[i - E.nj] = tanh(a);
  }
}

// ------------------------------------------------------------------ one step
// Differentiable inputs of one env step: state, warm-start block, controls and
// the per-body / per-joint / per-env model parameters (the hinge anchors are
// the model's link lengths, section 4).
template <class S> struct StepIn {
  const S* x;      // [nb][18]
  const S* lam;    // [lam_size]
  const S* u;      // [nj]
  const S* invm;   // [nb]
  const S* invI;   // [nb][3]
  const S* damp;   // [nj]
  S mu;
  const S* anc_p;  // [nj][3] hinge point in the parent (or world) frame
  const S* anc_c;  // [nj][3] hinge point in the child frame
  double rest = 0.0;  // restitution coefficient of the env's contacts
};

template <class S>
void step_env(const Model& M, const EnvTopo& E, const StepIn<S>& in, S* xn, S* lamn,
              const S* W = nullptr, int t = 0, StepStats* stats = nullptr) {
  const oracle_model& c = M.c;
  const int nb = E.nb;
  const S dt = S(c.dt);
  Bodies<S> B;
  B.p.resize(nb); B.v.resize(nb); B.w.resize(nb); B.R.resize(nb); B.Iw.resize(nb); B.invm.resize(nb);
  for (int b = 0; b < nb; ++b) {
    const S* xb = in.x + 18 * b;
    B.p[b] = {xb[0], xb[1], xb[2]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B.R[b].m[i][j] = xb[3 + 3 * i + j];
    B.v[b] = {xb[12], xb[13], xb[14]};
    B.w[b] = {xb[15], xb[16], xb[17]};
    B.invm[b] = in.invm[b];
  }
  // S0 controls: tape, or the controller evaluated on x^t
  std::vector<S> u(E.nj), hn(c.ctrl_kind == 1 ? c.mlp_rec : 0);
  if (c.ctrl_kind == 1) mlp_controls(M, E, t, B, W, u.data(), in.lam + E.lam_imp, hn.data());
  else for (int j = 0; j < E.nj; ++j) u[j] = in.u[j];
  // S1 world inverse inertia R diag(1/I) R^T and sphere centres
  for (int b = 0; b < nb; ++b) {
    M3<S> D;
    for (int k = 0; k < 3; ++k) D.m[k][k] = in.invI[3 * b + k];
    B.Iw[b] = matmul(matmul(B.R[b], D), transpose(B.R[b]));
  }
  std::vector<V3<S>> cen(E.ns);
  for (int s = 0; s < E.ns; ++s) {
    const int gs = E.s0 + s, b = c.sphere_body[gs] - E.b0;
    cen[s] = B.p[b] + B.R[b] * cvt<S>(c.sphere_offset + 3 * gs);
  }
  // S2 joint torques (motor input minus viscous damping about the hinge axis),
  // equal and opposite on child and parent
  std::vector<V3<S>> tq(nb);
  for (int j = 0; j < E.nj; ++j) {
    const int gj = E.j0 + j;
    const int pa = c.joint_parent[gj], b = c.joint_child[gj] - E.b0;
    const int a = pa >= 0 ? pa - E.b0 : -1;
    V3<S> n = cvt<S>(c.axis_p + 3 * gj), wa;
    if (a >= 0) { n = B.R[a] * n; wa = B.w[a]; }
    // (a servo's target angle is not a torque: its joint takes the damping alone)
    const S tau = (c.servo ? S(0.0) : u[j]) - in.damp[j] * dot(B.w[b] - wa, n);
    tq[b] = tq[b] + tau * n;
    if (a >= 0) tq[a] = tq[a] - tau * n;
  }
  // S3 velocity prediction with gravity and torques (no gyroscopic term)
  const V3<S> g = {S(c.gravity[0]), S(c.gravity[1]), S(c.gravity[2])};
  for (int b = 0; b < nb; ++b) {
    B.v[b] = B.v[b] + dt * g;
    B.w[b] = B.w[b] + dt * (B.Iw[b] * tq[b]);
  }
  // S4/S5 constraint rows at x^t in canonical order
  const S beta = S(c.beta), gam = S(c.gamma);
  std::vector<ConRows<S>> cons;
  std::vector<char> active_ground(E.ground.size(), 0), active_pair(E.pairs.size(), 0);
  const V3<S> ex(S(1.0), S(0.0), S(0.0)), ey(S(0.0), S(1.0), S(0.0)), ez(S(0.0), S(0.0), S(1.0));
  for (const Con& k : E.order) {
    ConRows<S> C;
    if (k.kind == 0) {
      const int gj = k.idx, jl = gj - E.j0;
      const int pa = c.joint_parent[gj], b = c.joint_child[gj] - E.b0;
      const int a = pa >= 0 ? pa - E.b0 : -1;
      C.kind = 0; C.nrows = E.jr; C.store = E.jr * jl;
      const V3<S> rb = B.R[b] * V3<S>(in.anc_c[3 * jl], in.anc_c[3 * jl + 1], in.anc_c[3 * jl + 2]);
      V3<S> ra, Pa = V3<S>(in.anc_p[3 * jl], in.anc_p[3 * jl + 1], in.anc_p[3 * jl + 2]);
      if (a >= 0) { ra = B.R[a] * Pa; Pa = B.p[a] + ra; }
      const V3<S> err = (B.p[b] + rb) - Pa;
      const V3<S> e3[3] = {ex, ey, ez};
      const S ev[3] = {err.x, err.y, err.z};
      for (int q = 0; q < 3; ++q) {
        Row<S>& r = C.r[q];
        r.a = a; r.b = b;
        r.la = -e3[q]; r.aa = -cross(ra, e3[q]); r.lb = e3[q]; r.ab = cross(rb, e3[q]);
        r.bias = beta * ev[q] / dt;
      }
      V3<S> na = cvt<S>(c.axis_p + 3 * gj), ua = cvt<S>(c.perp_p + 3 * gj);
      V3<S> t2 = cross(na, ua);
      if (a >= 0) { na = B.R[a] * na; ua = B.R[a] * ua; t2 = B.R[a] * t2; }
      const V3<S> nb_w = B.R[b] * cvt<S>(c.axis_c + 3 * gj);
      const V3<S> ax = cross(na, nb_w);
      const V3<S> tk[2] = {ua, t2};
      for (int q = 0; q < 2; ++q) {
        Row<S>& r = C.r[3 + q];
        r.a = a; r.b = b;
        r.aa = -tk[q]; r.ab = tk[q];
        r.bias = beta * dot(tk[q], ax) / dt;
      }
      if (c.servo) {
        // velocity motor: target rate from the hinge angle, clipped; impulse
        // within the torque limit over the step
        const V3<S> ub = B.R[b] * cvt<S>(c.perp_c + 3 * gj);
        const S theta = atan2(dot(cross(ua, ub), na), dot(ua, ub));
        S rate = S(c.servo_gain[gj]) * (u[jl] - theta);
        const double vmax = c.servo_vmax[gj];
        if (val(rate) > vmax) rate = S(vmax);
        else if (val(rate) < -vmax) rate = S(-vmax);
        Row<S>& r = C.r[5];
        r.a = a; r.b = b;
        r.aa = -na; r.ab = na;
        r.bias = -rate;
        r.hi = c.servo_torque[gj] * c.dt;
        r.lo = -r.hi;
      }
      for (int q = 0; q < C.nrows; ++q) {
        Row<S>& r = C.r[q];
        r.m = S(1.0) / (finish_row(r, B) + gam);
        r.lam = S(c.warm) * in.lam[C.store + q];  // joints are always active: plain warm start
      }
    } else {
      int a = -1, b;
      V3<S> n, ra_, rb_;
      S gap;
      int store;
      if (k.kind == 1) {
        const int gs = E.ground[k.idx], s = gs - E.s0;
        b = c.sphere_body[gs] - E.b0;
        const S rad = S(c.sphere_radius[gs]);
        gap = cen[s].z - rad;
        if (!(val(gap) < c.spec_margin)) continue;  // inactive candidate
        active_ground[k.idx] = 1;
        n = ez;
        rb_ = (cen[s] - rad * n) - B.p[b];
        store = E.jr * E.nj + 4 * k.idx;
        C.code = (1 << 24) | k.idx;
      } else {
        const PairCand& pc = E.pairs[k.idx];
        a = pc.ba - E.b0; b = pc.bb - E.b0;
        const V3<S> ca = cen[pc.sa - E.s0], cb = cen[pc.sb - E.s0];
        const S raa = S(c.sphere_radius[pc.sa]), rbb = S(c.sphere_radius[pc.sb]);
        const V3<S> d = cb - ca;
        const S L = sqrt(dot(d, d));
        gap = L - raa - rbb;
        if (!(val(gap) < c.spec_margin)) continue;
        active_pair[k.idx] = 1;
        C.code = (2 << 24) | (pc.ba - E.b0) | ((pc.bb - E.b0) << 12);
        n = val(L) < 1e-9 ? ez : (S(1.0) / L) * d;
        ra_ = (ca + raa * n) - B.p[a];
        rb_ = (cb - rbb * n) - B.p[b];
        store = E.jr * E.nj + 4 * (int)E.ground.size() + 4 * k.idx;
      }
      C.kind = 1; C.nrows = 3; C.store = store; C.gap = gap;
      // tangent basis
      V3<S> t1, t2;
      if (k.kind == 1) { t1 = ex; t2 = ey; }
      else {
        const V3<S> w = std::fabs(val(n.z)) < 0.9 ? cross(n, ez) : cross(n, ex);
        t1 = (S(1.0) / sqrt(dot(w, w))) * w;
        t2 = cross(n, t1);
      }
      C.t1 = t1; C.t2 = t2;
      const V3<S> dirs[3] = {n, t1, t2};
      S K[3];
      for (int q = 0; q < 3; ++q) {
        Row<S>& r = C.r[q];
        r.a = a; r.b = b;
        if (a >= 0) { r.la = -dirs[q]; r.aa = -cross(ra_, dirs[q]); }
        r.lb = dirs[q]; r.ab = cross(rb_, dirs[q]);
        K[q] = finish_row(r, B);
      }
      // normal row: speculative when separated, Baumgarte when penetrating
      // (C = 0 takes the penetrating branch).  Restitution: a contact that
      // the predicted velocities would close within this step (touching ones
      // included) and that approaches faster than the threshold aims at e
      // times its approach speed, unless the Baumgarte push-out is faster.
      Row<S>& rn = C.r[0];
      rn.m = S(1.0) / (K[0] + gam);
      rn.bias = (val(gap) > 0.0 ? gap : beta * gap) / dt;
      if (in.rest > 0.0) {
        const S vn = jdotv(rn, B);   // at the predicted velocities (before the warm start)
        if (val(vn) < -c.rest_threshold && val(vn) * c.dt + val(gap) < 0.0) {
          const S rb = S(in.rest) * vn;
          if (val(rb) < val(rn.bias)) rn.bias = rb;
        }
      }
      rn.lo = 0.0; rn.hi = INFINITY;
      C.mt = S(2.0) / (K[1] + K[2]);
      // warm start: previous normal impulse and the tangent impulse carried as
      // a world vector, re-projected on the new tangents
      const V3<S> Lt = {in.lam[store + 1], in.lam[store + 2], in.lam[store + 3]};
      rn.lam = S(c.warm) * in.lam[store];
      C.r[1].lam = S(c.warm) * dot(t1, Lt);
      C.r[2].lam = S(c.warm) * dot(t2, Lt);
    }
    cons.push_back(C);
  }
  // S6 warm start.  Plain: the carried impulses.  Learned (tolerance mode):
  // contact impulses from the warm-start network on per-contact features,
  // projected onto lambda_n >= 0, |lambda_t| <= mu lambda_n.
  const S mu = in.mu;
  const bool tolmode = c.solve_mode == 1;
  const size_t nc = cons.size();
  std::vector<std::array<S, 6>> plain(nc);
  for (size_t i = 0; i < nc; ++i)
    for (int q = 0; q < cons[i].nrows; ++q) plain[i][q] = cons[i].r[q].lam;
  std::vector<V3<S>> v_pred, w_pred;
  std::vector<std::array<double, ORACLE_WSN_IN>> feat(nc);
  if (tolmode) {
    v_pred = B.v;
    w_pred = B.w;
    for (size_t i = 0; i < nc; ++i) {
      const ConRows<S>& C = cons[i];
      if (C.kind != 1) continue;
      const double mn = val(C.r[0].m), mt = val(C.mt);
      feat[i] = {val(C.gap) / c.dt, val(jdotv(C.r[0], B)), val(jdotv(C.r[1], B)), val(jdotv(C.r[2], B)),
                 val(plain[i][0]) / mn, val(plain[i][1]) / mt, val(plain[i][2]) / mt};
    }
  }
  if (tolmode && c.ws_kind == 1) {
    for (size_t i = 0; i < nc; ++i) {
      ConRows<S>& C = cons[i];
      if (C.kind != 1) continue;
      // the network predicts the correction to the carried impulses, in
      // velocity units (impulse over effective mass)
      double y[ORACLE_WSN_OUT];
      wsn_eval(c.ws_w, feat[i].data(), y);
      const double ln = std::max(val(C.r[0].m) * (feat[i][4] + y[0]), 0.0);
      double l1 = val(C.mt) * (feat[i][5] + y[1]), l2 = val(C.mt) * (feat[i][6] + y[2]);
      const double rho = val(mu) * ln, nrm = std::sqrt(l1 * l1 + l2 * l2);
      if (!(nrm <= rho)) { l1 *= rho / nrm; l2 *= rho / nrm; }
      C.r[0].lam = S(ln);
      C.r[1].lam = S(l1);
      C.r[2].lam = S(l2);
    }
  }
  for (auto& C : cons)
    for (int q = 0; q < C.nrows; ++q) apply(C.r[q], B, C.r[q].lam);
  // S7 projected Gauss-Seidel.  One sweep visits every constraint in the
  // canonical order and returns the residual: the largest |delta lambda| / m
  // over the scalar rows and |delta lambda_t| / m_t over the friction blocks.
  double res_c = 0.0;   // residual of the contact rows in the last sweep
  auto sweep = [&]() -> double {
    double res = 0.0;
    res_c = 0.0;
    for (auto& C : cons) {
      const int nscalar = C.kind == 0 ? C.nrows : 1;
      for (int q = 0; q < nscalar; ++q) {
        Row<S>& r = C.r[q];
        const S s = jdotv(r, B) + r.bias + gam * r.lam;
        const S lt = r.lam - r.m * s;
        S ln;
        if (val(lt) <= r.lo) ln = S(r.lo);
        else if (val(lt) >= r.hi) ln = S(r.hi);
        else ln = lt;
        apply(r, B, ln - r.lam);
        const double rr = std::fabs(val(ln) - val(r.lam)) / val(r.m);
        res = std::max(res, rr);
        if (C.kind == 1) res_c = std::max(res_c, rr);
        r.lam = ln;
      }
      if (C.kind == 1) {
        // friction block: isotropic Coulomb disk |lambda_t| <= mu lambda_n
        Row<S>& r1 = C.r[1];
        Row<S>& r2 = C.r[2];
        const S l1 = r1.lam - C.mt * jdotv(r1, B);
        const S l2 = r2.lam - C.mt * jdotv(r2, B);
        const S rho = mu * C.r[0].lam;
        const S nrm = sqrt(l1 * l1 + l2 * l2);
        S n1 = l1, n2 = l2;
        if (!(val(nrm) <= val(rho))) {
          const S sc = rho / nrm;
          n1 = sc * l1;
          n2 = sc * l2;
        }
        apply(r1, B, n1 - r1.lam);
        apply(r2, B, n2 - r2.lam);
        const double d1 = val(n1) - val(r1.lam), d2 = val(n2) - val(r2.lam);
        const double rt = std::sqrt(d1 * d1 + d2 * d2) / val(C.mt);
        res = std::max(res, rt);
        res_c = std::max(res_c, rt);
        r1.lam = n1;
        r2.lam = n2;
      }
    }
    return res;
  };
  if (!tolmode) {
    for (int it = 0; it < c.n_iters; ++it) (void)sweep();
  } else if (nc > 0) {
    int it = 0;
    double res = INFINITY;
    if (c.ws_kind == 1) {
      // the test looks at the rows the network started: the contacts
      while (it < c.fb_iters && res > c.tol) { res = sweep(); ++it; }
      const double test = it > 0 ? res_c : INFINITY;
      if (res > c.tol && test > c.fb_tol) {
        // rejected: restart this env's solve from the plain warm start
        if (stats) { stats->sweeps += it; stats->fallbacks += 1; }
        B.v = v_pred;
        B.w = w_pred;
        for (size_t i = 0; i < nc; ++i)
          for (int q = 0; q < cons[i].nrows; ++q) cons[i].r[q].lam = plain[i][q];
        for (auto& C : cons)
          for (int q = 0; q < C.nrows; ++q) apply(C.r[q], B, C.r[q].lam);
        it = 0;
        res = INFINITY;
      }
    }
    while (res > c.tol && it < c.max_iters) { res = sweep(); ++it; }
    if (stats) stats->sweeps += it;
    if (stats && stats->recs && stats->rec_every > 0 && t % stats->rec_every == 0 && res <= c.tol) {
      for (size_t i = 0; i < nc; ++i) {
        const ConRows<S>& C = cons[i];
        if (C.kind != 1) continue;
        const double mn = val(C.r[0].m), mt = val(C.mt);
        std::vector<double>& R = *stats->recs;
        for (int k = 0; k < ORACLE_WSN_IN; ++k) R.push_back(feat[i][k]);
        R.push_back(val(C.r[0].lam) / mn);
        R.push_back(val(C.r[1].lam) / mt);
        R.push_back(val(C.r[2].lam) / mt);
        R.push_back(mn);
        R.push_back(mt);
        R.push_back(stats->env);
        R.push_back(t);
        R.push_back(C.code);
        R.push_back(0.0);
      }
    }
  }
  // S8 semi-implicit Euler and rotation renormalisation
  for (int b = 0; b < nb; ++b) {
    B.p[b] = B.p[b] + dt * B.v[b];
    M3<S> A = B.R[b];
    const M3<S> WR = matmul(skew(B.w[b]), B.R[b]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A.m[i][j] = A.m[i][j] + dt * WR.m[i][j];
    const M3<S> AAtA = matmul(matmul(A, transpose(A)), A);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B.R[b].m[i][j] = (S(3.0) * A.m[i][j] - AAtA.m[i][j]) * S(0.5);
  }
  for (int b = 0; b < nb; ++b) {
    S* xb = xn + 18 * b;
    xb[0] = B.p[b].x; xb[1] = B.p[b].y; xb[2] = B.p[b].z;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) xb[3 + 3 * i + j] = B.R[b].m[i][j];
    xb[12] = B.v[b].x; xb[13] = B.v[b].y; xb[14] = B.v[b].z;
    xb[15] = B.w[b].x; xb[16] = B.w[b].y; xb[17] = B.w[b].z;
  }
  // S9 store impulses for the next step's warm start (zero when inactive),
  // and the controller's next recurrent state
  for (int i = 0; i < E.lam_imp; ++i) lamn[i] = S(0.0);
  for (size_t i = 0; i < hn.size(); ++i) lamn[E.lam_imp + i] = hn[i];
  for (auto& C : cons) {
    if (C.kind == 0) {
      for (int q = 0; q < C.nrows; ++q) lamn[C.store + q] = C.r[q].lam;
    } else {
      const V3<S> Lt = C.r[1].lam * C.t1 + C.r[2].lam * C.t2;
      lamn[C.store] = C.r[0].lam;
      lamn[C.store + 1] = Lt.x; lamn[C.store + 2] = Lt.y; lamn[C.store + 3] = Lt.z;
    }
  }
}

// ------------------------------------------------------------------ loss
// Loss contribution l(x^{t}, p) of the state reached after step t (1-based),
// eq. (L); `x0` only enters the mean-velocity kind.
template <class S>
S loss_term(const Model& M, const EnvTopo& E, int e, int t, int T, const S* xt, const S* x0) {
  const oracle_model& c = M.c;
  const int lb = c.loss_body[e] - E.b0;
  const S* p = xt + 18 * lb;
  const double* tg = c.target + 3 * e;
  if (c.loss_kind == 0) {
    if (t != T) return S(0.0);
    S L = S(0.0);
    for (int k = 0; k < 3; ++k)
      if (c.loss_mask & (1 << k)) { const S d = p[k] - S(tg[k]); L = L + d * d; }
    return L;
  }
  if (c.loss_kind == 1) {
    S q = S(0.0);
    for (int k = 0; k < 3; ++k)
      if (c.loss_mask & (1 << k)) { const S d = p[k] - S(tg[k]); q = q + d * d; }
    if (val(q) <= 0.0) return S(0.0);
    return sqrt(q) / S(double(T));
  }
  if (t != T) return S(0.0);
  if (c.loss_kind == 3) {
    S L = S(0.0);
    for (int k = 0; k < 3; ++k)
      if (c.loss_mask & (1 << k)) { const S d = p[k] - S(tg[k]); L = L + d * d; }
    for (int k = 12; k < 18; ++k) L = L + p[k] * p[k];   // |v|^2 + |omega|^2 (p = the body's record)
    return L;
  }
  const S* p0 = x0 + 18 * lb;
  return -(p[0] - p0[0]) / S(T * c.dt);
}

// ------------------------------------------------------------------ drivers
struct Ctx {
  Model M;
  std::vector<EnvTopo> topo;
  int lam_total = 0;
};

static void build_ctx(const oracle_model* m, Ctx& C) {
  C.M.c = *m;
  C.M.n_bodies = m->env_body_off[m->n_envs];
  C.M.n_joints = m->env_joint_off[m->n_envs];
  C.M.n_spheres = m->env_sphere_off[m->n_envs];
  int off = 0;
  C.topo.clear();
  for (int e = 0; e < m->n_envs; ++e) {
    C.topo.push_back(build_topo(C.M, e, off));
    off += C.topo.back().lam_size;
  }
  C.lam_total = off;
}

template <class F> static void parallel_envs(int n_envs, int n_threads, F f) {
  if (n_threads <= 1 || n_envs <= 1) {
    for (int e = 0; e < n_envs; ++e) f(e);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int i = 0; i < n_threads; ++i)
    th.emplace_back([&]() {
      for (int e; (e = next.fetch_add(1)) < n_envs;) f(e);
    });
  for (auto& t : th) t.join();
}

template <class S> static std::vector<S> to_s(const double* p, int n) {
  std::vector<S> v(n);
  for (int i = 0; i < n; ++i) v[i] = S(p[i]);
  return v;
}

// Test aid for judging conditioning (never part of the method): multiply each
// state component after a step by (1 + noise * r), r in [-1, 1) from a
// counter-based hash of (env, step, component) (splitmix64), which mimics
// the rounding of a single-precision run.
static double noise_r(uint64_t seed, uint64_t e, uint64_t t, uint64_t i) {
  uint64_t z = (e * 0x9E3779B97F4A7C15ULL) ^ (t * 0xBF58476D1CE4E5B9ULL) ^ (i * 0x94D049BB133111EBULL) ^
               (seed * 0xD6E8FEB86659FD93ULL);
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Forward rollout of one env in type S; optionally records step-start states.
template <class S>
static S rollout_env(const Ctx& C, int e, std::vector<S>& x, std::vector<S>& lam,
                     std::vector<double>* xs, std::vector<double>* ls, double* traj,
                     StepStats* stats = nullptr) {
  const oracle_model& c = C.M.c;
  const EnvTopo& E = C.topo[e];
  const int T = c.T_env[e];
  const int n = 18 * E.nb;
  std::vector<S> x0 = x, xn(n), ln(E.lam_size);
  const std::vector<S> invm = to_s<S>(c.inv_mass + E.b0, E.nb);
  const std::vector<S> invI = to_s<S>(c.inv_inertia + 3 * E.b0, 3 * E.nb);
  const std::vector<S> damp = to_s<S>(c.damping + E.j0, E.nj);
  const std::vector<S> ap = to_s<S>(c.anchor_p + 3 * E.j0, 3 * E.nj);
  const std::vector<S> ac = to_s<S>(c.anchor_c + 3 * E.j0, 3 * E.nj);
  std::vector<S> W;
  if (c.ctrl_kind == 1) W = to_s<S>(c.mlp_w, c.mlp_n_params);
  S L = S(0.0);
  for (int t = 0; t < T; ++t) {
    if (xs) for (int i = 0; i < n; ++i) xs->push_back(val(x[i]));
    if (ls) for (int i = 0; i < E.lam_size; ++i) ls->push_back(val(lam[i]));
    std::vector<S> u(E.nj);
    if (c.ctrl_kind == 0)
      for (int j = 0; j < E.nj; ++j) u[j] = S(c.u[(size_t)t * c.u_stride + E.j0 + j]);
    StepIn<S> in{x.data(), lam.data(), u.data(), invm.data(), invI.data(), damp.data(), S(c.mu[e]),
                 ap.data(), ac.data()};
    in.rest = c.restitution ? c.restitution[e] : 0.0;
    step_env(C.M, E, in, xn.data(), ln.data(), W.data(), t, stats);
    if (c.noise > 0.0)
      for (int i = 0; i < n; ++i) xn[i] = xn[i] * S(1.0 + c.noise * noise_r(c.noise_seed, e, t, i));
    x.swap(xn);
    lam.swap(ln);
    L = L + loss_term(C.M, E, e, t + 1, T, x.data(), x0.data());
    if (traj)
      for (int i = 0; i < n; ++i) traj[((size_t)(t + 1) * C.M.n_bodies + E.b0) * 18 + i] = val(x[i]);
  }
  return L;
}

// Warm-start impulses of an env at the start of a rollout: given, or zeros.
static std::vector<double> start_impulses(const oracle_model& m, const EnvTopo& E) {
  if (!m.lam0) return std::vector<double>(E.lam_size, 0.0);
  return std::vector<double>(m.lam0 + E.lam_off, m.lam0 + E.lam_off + E.lam_size);
}

}  // namespace orc

using namespace orc;

extern "C" {

int oracle_lambda_size(const oracle_model* m, int* out_offsets) {
  Ctx C;
  build_ctx(m, C);
  if (out_offsets)
    for (int e = 0; e <= m->n_envs; ++e) out_offsets[e] = e < m->n_envs ? C.topo[e].lam_off : C.lam_total;
  return C.lam_total;
}

int oracle_order(const oracle_model* m, int env, int* kinds, int* idx, int cap) {
  Ctx C;
  build_ctx(m, C);
  const EnvTopo& E = C.topo[env];
  const int n = (int)E.order.size();
  for (int i = 0; i < n && i < cap; ++i) {
    kinds[i] = E.order[i].kind;
    int v = E.order[i].idx;
    if (E.order[i].kind == 1) v = E.ground[v];
    if (E.order[i].kind == 2) v = E.pairs[v].ba * 65536 + E.pairs[v].bb;
    idx[i] = v;
  }
  return n;
}

int oracle_step(const oracle_model* m, const double* x, const double* lam, const double* u, double* xn,
                double* lamn, int t) {
  Ctx C;
  build_ctx(m, C);
  for (int e = 0; e < m->n_envs; ++e) {
    const EnvTopo& E = C.topo[e];
    StepIn<double> in{x + 18 * E.b0, lam + E.lam_off, u + E.j0, m->inv_mass + E.b0, m->inv_inertia + 3 * E.b0,
                      m->damping + E.j0, m->mu[e], m->anchor_p + 3 * E.j0, m->anchor_c + 3 * E.j0};
    in.rest = m->restitution ? m->restitution[e] : 0.0;
    step_env<double>(C.M, E, in, xn + 18 * E.b0, lamn + E.lam_off, m->mlp_w, t);
  }
  return 0;
}

int oracle_rollout(const oracle_model* m, const double* x0, double* loss_env, double* x_final,
                   double* lam_final, double* traj, int n_threads) {
  Ctx C;
  build_ctx(m, C);
  if (traj)
    for (int b = 0; b < 18 * C.M.n_bodies; ++b) traj[b] = x0[b];
  parallel_envs(m->n_envs, n_threads, [&](int e) {
    const EnvTopo& E = C.topo[e];
    std::vector<double> x(x0 + 18 * E.b0, x0 + 18 * (E.b0 + E.nb));
    std::vector<double> lam = start_impulses(*m, E);
    const double L = rollout_env<double>(C, e, x, lam, nullptr, nullptr, traj);
    if (loss_env) loss_env[e] = L;
    if (x_final) std::copy(x.begin(), x.end(), x_final + 18 * E.b0);
    if (lam_final) std::copy(lam.begin(), lam.end(), lam_final + E.lam_off);
  });
  return 0;
}

long long oracle_rollout_ex(const oracle_model* m, const double* x0, double* loss_env, double* x_final,
                            double* lam_final, int* iters_env, int* fallbacks_env, int rec_every, double* recs,
                            long long rec_cap, int n_threads) {
  Ctx C;
  build_ctx(m, C);
  std::vector<std::vector<double>> rec_env(m->n_envs);
  parallel_envs(m->n_envs, n_threads, [&](int e) {
    const EnvTopo& E = C.topo[e];
    std::vector<double> x(x0 + 18 * E.b0, x0 + 18 * (E.b0 + E.nb));
    std::vector<double> lam = start_impulses(*m, E);
    StepStats st;
    st.env = e;
    st.rec_every = recs ? rec_every : 0;
    st.recs = &rec_env[e];
    const double L = rollout_env<double>(C, e, x, lam, nullptr, nullptr, nullptr, &st);
    if (loss_env) loss_env[e] = L;
    if (x_final) std::copy(x.begin(), x.end(), x_final + 18 * E.b0);
    if (lam_final) std::copy(lam.begin(), lam.end(), lam_final + E.lam_off);
    if (iters_env) iters_env[e] = st.sweeps;
    if (fallbacks_env) fallbacks_env[e] = st.fallbacks;
  });
  long long n = 0;
  for (const auto& r : rec_env)
    for (size_t k = 0; k < r.size(); k += ORACLE_REC, ++n)
      if (recs && n < rec_cap) std::copy(r.begin() + k, r.begin() + k + ORACLE_REC, recs + n * ORACLE_REC);
  return n;
}

// The controller's outputs u^t for env `env` at state x (global [B][18]) and
// step t, with the recurrent state h^t from lam0 (zeros without): eq. (g)
// evaluated on the joint sensors, the clock and h^t.  A test hook for pinning
// the controller's inputs.
int oracle_controls(const oracle_model* m, int env, const double* x, int t, double* u_out) {
  if (m->ctrl_kind != 1 || env < 0 || env >= m->n_envs) return -1;
  Ctx C;
  build_ctx(m, C);
  const EnvTopo& E = C.topo[env];
  Bodies<double> B;
  B.p.resize(E.nb); B.v.resize(E.nb); B.w.resize(E.nb); B.R.resize(E.nb); B.Iw.resize(E.nb); B.invm.resize(E.nb);
  for (int b = 0; b < E.nb; ++b) {
    const double* xb = x + 18 * (E.b0 + b);
    B.p[b] = {xb[0], xb[1], xb[2]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B.R[b].m[i][j] = xb[3 + 3 * i + j];
    B.v[b] = {xb[12], xb[13], xb[14]};
    B.w[b] = {xb[15], xb[16], xb[17]};
  }
  std::vector<double> h(m->mlp_rec, 0.0), hn(m->mlp_rec, 0.0);
  if (m->lam0)
    for (int i = 0; i < m->mlp_rec; ++i) h[i] = m->lam0[E.lam_off + E.lam_imp + i];
  mlp_controls<double>(C.M, E, t, B, m->mlp_w, u_out, h.data(), hn.data());
  return E.nj;
}

double oracle_bf16(double x) { return bf16(x); }

void oracle_wsn_forward(const double* w, const double* x, int stride, int n, double* y) {
  for (int i = 0; i < n; ++i) wsn_eval(w, x + (size_t)i * stride, y + 3 * (size_t)i);
}

// Reverse mode over the unrolled trajectory: forward once storing step-start
// states, then one tape per step, last step first, carrying the adjoints of
// the state and of the warm-start impulses.
int oracle_rollout_grad(const oracle_model* m, const double* x0, const double* dloss, double* loss_env,
                        double* g_x0, double* g_u, double* g_inv_mass, double* g_inv_inertia, double* g_mu,
                        double* g_damping, double* g_w, double* g_anchor_p, double* g_anchor_c, int n_threads) {
  if (m->solve_mode != 0) return -1;  // the gradient is of the fixed-sweep map
  Ctx C;
  build_ctx(m, C);
  const oracle_model& c = C.M.c;
  if (g_u) std::fill(g_u, g_u + (size_t)c.T_max * c.u_stride, 0.0);
  std::vector<std::vector<double>> gw_env;
  if (c.ctrl_kind == 1) gw_env.assign(m->n_envs, {});
  parallel_envs(m->n_envs, n_threads, [&](int e) {
    const EnvTopo& E = C.topo[e];
    const int n = 18 * E.nb, T = c.T_env[e];
    std::vector<double> xs, ls;
    std::vector<double> x(x0 + 18 * E.b0, x0 + 18 * (E.b0 + E.nb)), lam = start_impulses(*m, E);
    xs.reserve((size_t)T * n);
    ls.reserve((size_t)T * E.lam_size);
    const double L = rollout_env<double>(C, e, x, lam, &xs, &ls, nullptr);
    if (loss_env) loss_env[e] = L;
    const double dl = dloss ? dloss[e] : 1.0;
    std::vector<double> xbar(n, 0.0), lbar(E.lam_size, 0.0);
    std::vector<double> gm(E.nb, 0.0), gI(3 * E.nb, 0.0), gd(E.nj, 0.0), gap(3 * E.nj, 0.0), gac(3 * E.nj, 0.0), gW;
    double gmu = 0.0;
    if (c.ctrl_kind == 1) gW.assign(c.mlp_n_params, 0.0);
    Tape tp;
    tape() = &tp;
    for (int t = T - 1; t >= 0; --t) {
      // gradient decay: the carry from the later steps shrinks by alpha per
      // step (section 3.2); at t = T - 1 there is no carry yet
      if (t < T - 1 && c.grad_decay != 1.0) {
        for (double& v : xbar) v *= c.grad_decay;
        for (double& v : lbar) v *= c.grad_decay;
      }
      tp.clear();
      std::vector<Var> xv(n), lv(E.lam_size), uv(E.nj), mv(E.nb), Iv(3 * E.nb), dv(E.nj), apv(3 * E.nj),
          acv(3 * E.nj), Wv;
      for (int i = 0; i < n; ++i) xv[i] = Var::input(xs[(size_t)t * n + i]);
      for (int i = 0; i < E.lam_size; ++i) lv[i] = Var::input(ls[(size_t)t * E.lam_size + i]);
      for (int j = 0; j < E.nj; ++j)
        uv[j] = Var::input(c.ctrl_kind == 0 ? c.u[(size_t)t * c.u_stride + E.j0 + j] : 0.0);
      for (int b = 0; b < E.nb; ++b) mv[b] = Var::input(c.inv_mass[E.b0 + b]);
      for (int i = 0; i < 3 * E.nb; ++i) Iv[i] = Var::input(c.inv_inertia[3 * E.b0 + i]);
      for (int j = 0; j < E.nj; ++j) dv[j] = Var::input(c.damping[E.j0 + j]);
      for (int i = 0; i < 3 * E.nj; ++i) apv[i] = Var::input(c.anchor_p[3 * E.j0 + i]);
      for (int i = 0; i < 3 * E.nj; ++i) acv[i] = Var::input(c.anchor_c[3 * E.j0 + i]);
      const Var muv = Var::input(c.mu[e]);
      if (c.ctrl_kind == 1) {
        Wv.resize(c.mlp_n_params);
        for (int i = 0; i < c.mlp_n_params; ++i) Wv[i] = Var::input(c.mlp_w[i]);
      }
      // the state x^0 enters the mean-velocity loss directly
      std::vector<Var> x0v(n);
      for (int i = 0; i < n; ++i) x0v[i] = Var(x0[18 * E.b0 + i]);
      std::vector<Var> xn(n), ln(E.lam_size);
      StepIn<Var> in{xv.data(), lv.data(), uv.data(), mv.data(), Iv.data(), dv.data(), muv, apv.data(), acv.data()};
      in.rest = c.restitution ? c.restitution[e] : 0.0;
      step_env<Var>(C.M, E, in, xn.data(), ln.data(), Wv.data(), t);
      const Var lt = loss_term<Var>(C.M, E, e, t + 1, T, xn.data(), x0v.data());
      tp.adj.assign(tp.nodes.size(), 0.0);
      for (int i = 0; i < n; ++i) if (xn[i].id >= 0) tp.adj[xn[i].id] += xbar[i];
      for (int i = 0; i < E.lam_size; ++i) if (ln[i].id >= 0) tp.adj[ln[i].id] += lbar[i];
      if (lt.id >= 0) tp.adj[lt.id] += dl;
      tp.sweep();
      for (int i = 0; i < n; ++i) xbar[i] = tp.adj[xv[i].id];
      for (int i = 0; i < E.lam_size; ++i) lbar[i] = tp.adj[lv[i].id];
      if (g_u && c.ctrl_kind == 0)
        for (int j = 0; j < E.nj; ++j) g_u[(size_t)t * c.u_stride + E.j0 + j] = tp.adj[uv[j].id];
      for (int b = 0; b < E.nb; ++b) gm[b] += tp.adj[mv[b].id];
      for (int i = 0; i < 3 * E.nb; ++i) gI[i] += tp.adj[Iv[i].id];
      for (int j = 0; j < E.nj; ++j) gd[j] += tp.adj[dv[j].id];
      for (int i = 0; i < 3 * E.nj; ++i) gap[i] += tp.adj[apv[i].id];
      for (int i = 0; i < 3 * E.nj; ++i) gac[i] += tp.adj[acv[i].id];
      gmu += tp.adj[muv.id];
      if (c.ctrl_kind == 1)
        for (int i = 0; i < c.mlp_n_params; ++i) gW[i] += tp.adj[Wv[i].id];
    }
    tape() = nullptr;
    // direct dependence of the mean-velocity loss on x^0
    if (c.loss_kind == 2 && T > 0) {
      const int lb = c.loss_body[e] - E.b0;
      xbar[18 * lb + 0] += dl / (T * c.dt);
    }
    if (g_x0) std::copy(xbar.begin(), xbar.end(), g_x0 + 18 * E.b0);
    if (g_inv_mass) std::copy(gm.begin(), gm.end(), g_inv_mass + E.b0);
    if (g_inv_inertia) std::copy(gI.begin(), gI.end(), g_inv_inertia + 3 * E.b0);
    if (g_damping) std::copy(gd.begin(), gd.end(), g_damping + E.j0);
    if (g_anchor_p) std::copy(gap.begin(), gap.end(), g_anchor_p + 3 * E.j0);
    if (g_anchor_c) std::copy(gac.begin(), gac.end(), g_anchor_c + 3 * E.j0);
    if (g_mu) g_mu[e] = gmu;
    if (c.ctrl_kind == 1) gw_env[e] = std::move(gW);
  });
  if (g_w && c.ctrl_kind == 1) {
    std::fill(g_w, g_w + c.mlp_n_params, 0.0);
    for (int e = 0; e < m->n_envs; ++e)
      for (int i = 0; i < c.mlp_n_params; ++i) g_w[i] += gw_env[e][i];
  }
  return 0;
}

// Arithmetic operations of one step of env `env` from state x / warm start lam.
long long oracle_count_flops(const oracle_model* m, int env, const double* x, const double* lam,
                             const double* u, int t) {
  Ctx C;
  build_ctx(m, C);
  const EnvTopo& E = C.topo[env];
  std::vector<Cnt> xv(x + 18 * E.b0, x + 18 * (E.b0 + E.nb)), lv(lam + E.lam_off, lam + E.lam_off + E.lam_size);
  std::vector<Cnt> uv(E.nj), mv(E.nb), Iv(3 * E.nb), dv(E.nj), Wv;
  for (int j = 0; j < E.nj; ++j) uv[j] = u ? u[E.j0 + j] : 0.0;
  for (int b = 0; b < E.nb; ++b) mv[b] = m->inv_mass[E.b0 + b];
  for (int i = 0; i < 3 * E.nb; ++i) Iv[i] = m->inv_inertia[3 * E.b0 + i];
  for (int j = 0; j < E.nj; ++j) dv[j] = m->damping[E.j0 + j];
  if (m->ctrl_kind == 1) Wv.assign(m->mlp_w, m->mlp_w + m->mlp_n_params);
  std::vector<Cnt> xn(18 * E.nb), ln(E.lam_size);
  std::vector<Cnt> apv(m->anchor_p + 3 * E.j0, m->anchor_p + 3 * (E.j0 + E.nj));
  std::vector<Cnt> acv(m->anchor_c + 3 * E.j0, m->anchor_c + 3 * (E.j0 + E.nj));
  StepIn<Cnt> in{xv.data(), lv.data(), uv.data(), mv.data(), Iv.data(), dv.data(), Cnt(m->mu[env]), apv.data(),
                 acv.data()};
  in.rest = m->restitution ? m->restitution[env] : 0.0;
  flop_counter() = 0;
  step_env<Cnt>(C.M, E, in, xn.data(), ln.data(), Wv.data(), t);
  return (long long)flop_counter();
}

// Reverse-mode cost of one step: edges of its tape (one multiply-add each in
// the reverse sweep); also returns the forward operation count.
long long oracle_count_tape_edges(const oracle_model* m, int env, const double* x, const double* lam,
                                  const double* u, int t) {
  Ctx C;
  build_ctx(m, C);
  const EnvTopo& E = C.topo[env];
  Tape tp;
  tape() = &tp;
  std::vector<Var> xv(18 * E.nb), lv(E.lam_size), uv(E.nj), mv(E.nb), Iv(3 * E.nb), dv(E.nj), Wv;
  for (int i = 0; i < 18 * E.nb; ++i) xv[i] = Var::input(x[18 * E.b0 + i]);
  for (int i = 0; i < E.lam_size; ++i) lv[i] = Var::input(lam[E.lam_off + i]);
  for (int j = 0; j < E.nj; ++j) uv[j] = Var::input(u ? u[E.j0 + j] : 0.0);
  for (int b = 0; b < E.nb; ++b) mv[b] = Var::input(m->inv_mass[E.b0 + b]);
  for (int i = 0; i < 3 * E.nb; ++i) Iv[i] = Var::input(m->inv_inertia[3 * E.b0 + i]);
  for (int j = 0; j < E.nj; ++j) dv[j] = Var::input(m->damping[E.j0 + j]);
  if (m->ctrl_kind == 1) {
    Wv.resize(m->mlp_n_params);
    for (int i = 0; i < m->mlp_n_params; ++i) Wv[i] = Var::input(m->mlp_w[i]);
  }
  std::vector<Var> xn(18 * E.nb), ln(E.lam_size), apv(3 * E.nj), acv(3 * E.nj);
  for (int i = 0; i < 3 * E.nj; ++i) apv[i] = Var::input(m->anchor_p[3 * E.j0 + i]);
  for (int i = 0; i < 3 * E.nj; ++i) acv[i] = Var::input(m->anchor_c[3 * E.j0 + i]);
  StepIn<Var> in{xv.data(), lv.data(), uv.data(), mv.data(), Iv.data(), dv.data(), Var::input(m->mu[env]),
                 apv.data(), acv.data()};
  in.rest = m->restitution ? m->restitution[env] : 0.0;
  step_env<Var>(C.M, E, in, xn.data(), ln.data(), Wv.data(), t);
  long long edges = 0;
  for (const auto& n : tp.nodes) edges += (n.a >= 0) + (n.b >= 0);
  tape() = nullptr;
  return edges;
}

}  // extern "C"
