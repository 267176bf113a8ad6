// Per-environment time step and its hand-written adjoint, for one "team" of
// lanes that owns one env.  All of the env's working set lives in LDS.
//
// The step (paper section 2.1): joint torques -> velocity prediction ->
// contact candidates / gap test -> constraint rows -> warm start -> fixed
// projected Gauss-Seidel sweeps in colour-major order -> semi-implicit Euler
// + rotation renormalisation N(A) = (3A - A A^T A)/2 (eq. (1)).
//
// Parallelism inside a team: bodies, joints and candidates are strided over
// the team's lanes; the Gauss-Seidel sweep runs colour by colour, and the
// constraints of one colour (which touch disjoint bodies, so the result does
// not depend on their order) run on different lanes at once.  The rows of one
// constraint are updated in sequence by the lane that owns it.
//
// The adjoint reverses one step given dL/dx^{t+1} and dL/dlambda^t: the
// forward step is first replayed on chip from the stored step-start state
// while the pre-projection impulse of every row update is recorded; then the
// integration, the sweeps (iterations, colours and rows exactly reversed,
// velocities reconstructed by undoing each update, clamp / disk branches
// taken from the recorded values), the warm start, the row set-up, the
// velocity prediction and the torques are differentiated in turn.
//
// This header compiles both as HIP device code and as plain host C++ (a team
// of one lane), so the arithmetic can be checked on a CPU during development.
#pragma once
#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define SHD __host__ __device__ inline
#define SHD_NOINLINE __host__ __device__ __attribute__((noinline))
// The per-env drivers are inlined into their kernels: as real calls they keep
// the caller's live state in a stack frame (hundreds of bytes of scratch per
// lane).
#define SHD_FLAT __host__ __device__ inline __attribute__((always_inline))
#else
#define SHD inline
#define SHD_NOINLINE inline
#define SHD_FLAT inline
#endif

namespace sim {

// Product of two non-negative ints below 2^24 (LDS indices).  The masks
// tell the compiler the operands' range, so the GPU code uses a full-rate
// 24-bit multiply instead of a quarter-rate 32-bit one.
SHD int mul24(int a, int b) { return (int)(((unsigned)a & 0xFFFFFFu) * ((unsigned)b & 0xFFFFFFu)); }

// ------------------------------------------------------------------ small vectors
struct f3 { float x, y, z; };
SHD f3 mk3(float x, float y, float z) { f3 r; r.x = x; r.y = y; r.z = z; return r; }
SHD f3 operator+(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
SHD f3 operator-(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
SHD f3 operator-(f3 a) { return mk3(-a.x, -a.y, -a.z); }
SHD f3 operator*(float s, f3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
SHD float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
SHD f3 cross(f3 a, f3 b) { return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
SHD f3 ld3(const float* p) { return mk3(p[0], p[1], p[2]); }
SHD void st3(float* p, f3 v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }
// 16-byte vector for batched LDS access (ds_read_b128 / ds_write_b128)
struct alignas(16) f4 { float x, y, z, w; };
SHD f4 ld4(const float* p) { return *reinterpret_cast<const f4*>(p); }
SHD void st4(float* p, f4 v) { *reinterpret_cast<f4*>(p) = v; }
struct alignas(8) f2 { float x, y; };
SHD void st2(float* p, f2 v) { *reinterpret_cast<f2*>(p) = v; }
SHD void add3(float* p, f3 v) { p[0] += v.x; p[1] += v.y; p[2] += v.z; }
// R (row-major 9) times v, and R^T times v
SHD f3 mv(const float* R, f3 v) {
  return mk3(R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
             R[6] * v.x + R[7] * v.y + R[8] * v.z);
}
SHD f3 mtv(const float* R, f3 v) {
  return mk3(R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
             R[2] * v.x + R[5] * v.y + R[8] * v.z);
}
// symmetric 3x3 stored as xx yy zz xy xz yz
SHD f3 sv(const float* S, f3 v) {
  return mk3(S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
             S[4] * v.x + S[5] * v.y + S[2] * v.z);
}
// M += a b^T  (full 3x3 row-major)
SHD void add_outer(float* M, f3 a, f3 b) {
  M[0] += a.x * b.x; M[1] += a.x * b.y; M[2] += a.x * b.z;
  M[3] += a.y * b.x; M[4] += a.y * b.y; M[5] += a.y * b.z;
  M[6] += a.z * b.x; M[7] += a.z * b.y; M[8] += a.z * b.z;
}

// compensated accumulation: *sum += x, with the rounding error kept in *c
SHD void kahan_add(float* sum, float* c, float x) {
  const float y = x - *c;
  const float t = *sum + y;
  *c = (t - *sum) - y;
  *sum = t;
}

// ------------------------------------------------------------------ model in global memory
enum { H_B0, H_NB, H_J0, H_NJ, H_LAMOFF, H_LAMSZ, H_G, H_P, H_NCOL, H_TOPO, H_CST, H_T, H_LB, H_CCAP,
       H_NCAND, H_ENV, H_SEG, H_NSLOT, H_TAPE, H_RING, H_COUNT };
// candidate code: kind in the top byte
enum { K_JOINT = 0, K_GROUND = 1, K_PAIR = 2 };
SHD int cand_kind(int c) { return c >> 24; }
SHD int cand_idx(int c) { return c & 0xFFFFFF; }

struct DevModel {
  int n_envs, B, J, lam_tot, T_max, n_iters, ground, loss_kind, loss_mask, ckpt_every;
  float dt, gx, gy, gz, beta, gamma, spec, warm;
  const int* hdr;     // [E][H_COUNT]
  const int* topo;    // per-env topology ints
  const float* cst;   // per-env constants
  const float* target;// [E][3]
  // controller (ctrl == 1): [u, a] = MLP(s(x), h), weights W shared by all
  // envs; mlp_rec recurrent units h^{t+1} = tanh(a), carried after the
  // impulses in the env's carried-state block
  int ctrl, mlp_in, mlp_h1, mlp_h2, mlp_out, tape_stride, mlp_rec;
  const float* clock; // [T_max][2] sin, cos of 2 pi f t dt
  const float* W;     // weights (set per call)
  const float* Wt;    // their transposes W1^T, W2^T, W3^T (made per call, device)
  float* tape;        // per env-step activations and deltas (reverse only)
  // solve to a residual tolerance (forward only) and learned warm start
  int solve_mode, max_iters, ws_kind, fb_iters;
  float tol, fb_tol;
  const uint16_t* wsn; // warm-start network, bfloat16 [4867]
  int dump;           // reverse sweep buffer: DUMP_REPLAY, DUMP_SEGMENT or DUMP_TRAJECTORY
  float decay;        // gradient decay per reversed step (1: the exact derivative)
  int has_rest;       // some env has restitution > 0 (the predicted velocities are kept)
  int servo;          // every hinge is a servo motor: u holds target angles, 6 rows per joint
  float rest_th;      // approach speed below which contacts do not bounce
};
// Reverse sweep buffer modes: step-start states of one segment (each step is
// replayed), saved working sets of one segment, or of the whole trajectory
// (all segments recomputed in a separate launch).  An env's block starts on a
// SEG_UNIT-float boundary; in trajectory mode its last SEG_TAIL floats hold
// the loss body's final state record.
enum { DUMP_REPLAY = 0, DUMP_SEGMENT = 1, DUMP_TRAJECTORY = 2 };
enum { SEG_UNIT = 64, SEG_TAIL = 20 };
// tape row: s, h1, h2, du, d2, d1 (pre-activation adjoints)
SHD int tape_s(const DevModel&) { return 0; }
SHD int tape_h1(const DevModel& M) { return M.mlp_in; }
SHD int tape_h2(const DevModel& M) { return M.mlp_in + M.mlp_h1; }
SHD int tape_du(const DevModel& M) { return M.mlp_in + M.mlp_h1 + M.mlp_h2; }
SHD int tape_d2(const DevModel& M) { return tape_du(M) + M.mlp_out; }
SHD int tape_d1(const DevModel& M) { return tape_d2(M) + M.mlp_h2; }
SHD int tape_len(int in, int h1, int h2, int out) { return (in + 2 * h1 + 2 * h2 + out + 3) & ~3; }

// ------------------------------------------------------------------ LDS layout
// body record (forward)
enum { BP = 0, BR = 3, BV = 12, BW = 15, BI = 18, BIM = 24, BII = 25, BTQ = 28, BPR = 31, BPO = 32, BS = 36 };
// body record (adjoint)
// AIM/AII collect the current step's parameter adjoints; ATM/ATI hold the
// running totals over the trajectory and ACM/ACI their compensation terms
// (Kahan summation: a trajectory's parameter gradient is a long sum of terms
// that largely cancel).
enum { AP = 0, AR = 3, AV = 12, AW = 15, AIW = 18, AIM = 27, AII = 28, ATQ = 31, AW0 = 34,
       ATM = 37, ATI = 38, ACM = 41, ACI = 42, BSA = 48 };
// joint constants: anchors, axes and perpendiculars (parent, child frames),
// damping, the step's control, and the servo's gain, torque and rate limits
enum { JAP = 0, JAC = 3, JXP = 6, JXC = 9, JUP = 12, JUC = 15, JD = 18, JU = 19, JG = 20, JT = 21, JV = 22, JS = 24 };
// row slot; a contact uses 4 slots: normal, tangent 1, tangent 2, extras.
// Each body's part of the row is two aligned float4: (Ja, m) (Wa, bias) for
// body a and (Jb, m) (Wb, bias) for body b, so a lane that handles one body
// reads its part with two 16-byte loads; m and bias are kept in both
// (RMA, RBA: the copies of body a's part).  Then (Jl, lambda), lambda0.
enum { RJA = 0, RMA = 3, RWA = 4, RBA = 7, RJB = 8, RM = 11, RWB = 12, RBI = 15, RJL = 16, RL = 19, RL0 = 20, RS = 24 };
// a servo's motor row (a hinge's sixth) also holds its impulse bound
// torque * dt and 1 where the target rate was clipped to the rate limit
enum { RHI = 21, RCLIP = 22 };
// contact extras slot: tangents, friction mass, gap, store offset, code,
// (tolerance mode) the warm-start features XF[7] and network outputs XY[3],
// and 1 where restitution set the normal bias
enum { XT1 = 0, XT2 = 3, XMT = 6, XGAP = 7, XSTORE = 8, XCODE = 9, XF = 10, XY = 17, XREST = 20 };
// row adjoint slot, in the same shape: (Ja-bar, -) (Wa-bar, -) (Jb-bar, m-bar)
// (Wb-bar, bias-bar) (Jl-bar, lambda-bar)
enum { QJA = 0, QWA = 4, QJB = 8, QM = 11, QWB = 12, QB = 15, QJL = 16, QL = 19, RSA = 20 };

// Sweep plan entries (16 bytes, one LDS load): per live colour (start in the
// active list, count, 1 for a colour of hinges, -); per active constraint
// (slot, body a, body b, code), body a being the world slot nb where the
// constraint has no body a.
struct alignas(16) i4 { int x, y, z, w; };

struct Lay {
  int body, jc, gs, topo, ws, rows, act_cnt, act_slot, act_code, live, plan, vis, misc, grp, mlp, vsave;  // forward
  int bodyA, rowsA, hist, wsA, jA, mlpA;                                     // adjoint
  int hring;   // 0: the sweep history of the step in LDS; HRING: a ring of sweeps (the rest in global memory)
  int total_fwd, total;
};
// Sweeps of the impulse history held in LDS when the reverse reads the saved
// working sets: the current sweep's, the previous one's and the one loaded next.
constexpr int HRING = 3;
enum { MISC_LOSS = 0, MISC_FLAGS = 1, MISC_NCON = 2, MISC_MU = 3, MISC_GMU = 4, MISC_GMUC = 5, MISC_ITERS = 6,
       MISC_FB = 7, MISC_REST = 8, MISC_N = 12 };

SHD int align4(int x) { return (x + 3) & ~3; }
// Per-joint parameter adjoints of the reverse sweep, running totals over the
// trajectory with their compensation terms (Kahan), in units of nj floats:
// damping total [0, 1), damping compensation [1, 2), anchor in the parent
// frame (3 per joint) [2, 5), anchor in the child frame [5, 8), and the
// compensations of the anchors [8, 11) and [11, 14).
enum { JA_DAMP = 0, JA_DAMPC = 1, JA_ANCP = 2, JA_ANCC = 5, JA_ANC_COMP = 6, JA_FLOATS = 14 };
// mlp_f / mlp_a: controller floats per env (s, h1, h2 / du, d2, d1, sbar), 0 without one
// vs_f: floats of saved predicted velocities (learned warm start, restitution), 0 without
// ring: the adjoint layout holds HRING sweeps of the impulse history instead
// of all of them and the start impulses
SHD Lay make_lay(int nb, int nj, int G, int P, int ncol, int ncand, int nvis, int nslot, int lam, int n_iters,
                 bool adj,
                 int mlp_f = 0, int mlp_a = 0, int vs_f = 0, bool ring = false) {
  Lay L;
  L.hring = adj && ring ? HRING : 0;
  int o = 0;
  L.body = o; o += align4((nb + 1) * BS);   // bodies and the world slot (index nb)
  L.jc = o; o += align4(nj * JS);
  L.gs = o; o += align4(G * 4);
  L.topo = o; o += align4(2 * nj + G + P + ncol + 1 + ncand);
  L.ws = o; o += align4(lam);
  L.rows = o; o += align4(nslot * RS);
  L.act_cnt = o; o += align4(ncol);
  L.act_slot = o; o += align4(ncand);
  L.act_code = o; o += align4(ncand);
  L.live = o; o += align4(ncol + 3);
  L.plan = o; o += 4 * ncol;
  L.vis = o; o += 4 * nvis;   // the constraints a step places: every joint and up to ccap contacts
  L.misc = o; o += MISC_N;
  L.grp = o; o += align4(nb + 1);
  L.mlp = o; o += align4(mlp_f);
  L.vsave = o; o += align4(vs_f);
  L.total_fwd = o;
  if (adj) {
    L.bodyA = o; o += align4((nb + 1) * BSA);
    L.rowsA = o; o += align4(nslot * RSA);
    if (L.hring) {
      L.hist = o; o += align4(HRING * nslot);
    } else {
      o += align4(nslot);   // hist(-1): the sweeps' start impulses (reverse only)
      L.hist = o; o += align4(n_iters * nslot);
    }
    L.wsA = o; o += align4(lam);
    L.jA = o; o += align4(JA_FLOATS * nj);   // per-joint parameter adjoint totals and compensations
    L.mlpA = o; o += align4(mlp_a);
  } else {
    L.bodyA = L.rowsA = L.hist = L.wsA = L.jA = L.mlpA = o;
  }
  L.total = o;
  return L;
}

// ------------------------------------------------------------------ env view
struct Env {
  int b0, nb, j0, nj, lam_off, lam_size, G, P, ncol, T, lb, ccap, ncand, e, nslot, seg_off, tape_off;
  int lam_imp;        // impulses in the carried-state block (the rest: the controller's h)
  int jr;             // rows (and carried impulses) per joint: 5, 6 with servo motors
  const int* gtopo;   // global topology of the env
  const float* gcst;  // global constants of the env
  float* L;           // LDS base of the env
  Lay lay;
  // LDS accessors
  SHD float* body(int b) const { return L + lay.body + mul24(b, BS); }
  SHD float* bodyA(int b) const { return L + lay.bodyA + mul24(b, BSA); }
  SHD float* jc(int j) const { return L + lay.jc + mul24(j, JS); }
  SHD float* gsph(int g) const { return L + lay.gs + 4 * g; }
  SHD int* topo() const { return (int*)(L + lay.topo); }
  SHD int jpar(int j) const { return topo()[j]; }
  SHD int jchi(int j) const { return topo()[nj + j]; }
  SHD int gbody(int g) const { return topo()[2 * nj + g]; }
  SHD int pcode(int p) const { return topo()[2 * nj + G + p]; }
  SHD int colstart(int c) const { return topo()[2 * nj + G + P + c]; }
  SHD int cand(int i) const { return topo()[2 * nj + G + P + ncol + 1 + i]; }
  SHD float* ws() const { return L + lay.ws; }
  SHD float* wsA() const { return L + lay.wsA; }
  SHD float* row(int s) const { return L + lay.rows + mul24(s, RS); }
  SHD float* rowA(int s) const { return L + lay.rowsA + mul24(s, RSA); }
  // (it >= -1: the row before the first sweep's holds the start impulses; in
  // a ring, sweep it sits in slot it mod HRING)
  SHD float* hist(int it) const {
    if (lay.hring) {
      int k = it % HRING;
      if (k < 0) k += HRING;
      return L + lay.hist + k * nslot;
    }
    return L + lay.hist + it * nslot;
  }
  SHD int* act_cnt() const { return (int*)(L + lay.act_cnt); }
  SHD int* act_slot() const { return (int*)(L + lay.act_slot); }
  SHD int* act_code() const { return (int*)(L + lay.act_code); }
  // [0] colours with an active constraint this step, [1] joint colours (the
  // first colours of the canonical order), [2..2+ncol) the active colours in
  // order, [2+ncol] the entries of the sweep plan
  SHD int* live() const { return (int*)(L + lay.live); }
  // sweep plan of the step (built with the live list): plan()[g] = (start in
  // vis, count, 1 for hinges, -) for its g-th visit; vis() the step's active
  // constraints, visit by visit
  SHD i4* plan() const { return (i4*)(L + lay.plan); }
  SHD i4* vis() const { return (i4*)(L + lay.vis); }
  // (row set-up) the plan entry that last took each body, the world slot's
  // included
  SHD int* grp() const { return (int*)(L + lay.grp); }
  SHD float* misc() const { return L + lay.misc; }
  SHD float* jA() const { return L + lay.jA; }
  SHD float* mlp() const { return L + lay.mlp; }
  SHD float* mlpA() const { return L + lay.mlpA; }
  SHD float* vsave(int b) const { return L + lay.vsave + 6 * b; }
  // first float of the env's block of the reverse sweep buffer
  SHD size_t seg_base() const { return (size_t)seg_off * SEG_UNIT; }
  // warm-start store offset of a candidate
  SHD int store_of(int code) const {
    const int k = cand_kind(code), i = cand_idx(code);
    if (k == K_JOINT) return jr * i;
    if (k == K_GROUND) return jr * nj + 4 * i;
    return jr * nj + 4 * G + 4 * i;
  }
};

// Controller LDS regions of an env, each array starting on a float4:
//   forward  s[in], h1[h1], h2[h2], u[out]
//   adjoint  du[out], d2[h2], d1[h1], sbar[in]
SHD int mlp_fwd_floats(int in, int h1, int h2, int out) { return align4(in) + align4(h1) + align4(h2) + align4(out); }
SHD int mlp_adj_floats(int in, int h1, int h2, int out) { return align4(out) + align4(h2) + align4(h1) + align4(in); }
SHD int mlp_floats_fwd(const DevModel& M) {
  return M.ctrl ? mlp_fwd_floats(M.mlp_in, M.mlp_h1, M.mlp_h2, M.mlp_out) : 0;
}
SHD int mlp_floats_adj(const DevModel& M) {
  return M.ctrl ? mlp_adj_floats(M.mlp_in, M.mlp_h1, M.mlp_h2, M.mlp_out) : 0;
}
SHD int mo_h1(const DevModel& M) { return align4(M.mlp_in); }
SHD int mo_h2(const DevModel& M) { return align4(M.mlp_in) + align4(M.mlp_h1); }
SHD int mo_u(const DevModel& M) { return mo_h2(M) + align4(M.mlp_h2); }
SHD int mo_d2(const DevModel& M) { return align4(M.mlp_out); }
SHD int mo_d1(const DevModel& M) { return align4(M.mlp_out) + align4(M.mlp_h2); }
SHD int mo_sb(const DevModel& M) { return mo_d1(M) + align4(M.mlp_h1); }
SHD int vsave_floats(bool keep, int nb) { return keep ? 6 * nb : 0; }
// Floats of one step's saved working set: the forward LDS region, the sweep
// history and the step-start angular velocities.
SHD int dump_stride_of(int total_fwd, int n_iters, int nslot, int nb) {
  return total_fwd + align4(n_iters * nslot) + align4(3 * nb);
}

SHD Env make_env(const DevModel& M, int ie, float* lds, int n_iters, bool adj) {
  const int* h = M.hdr + (size_t)ie * H_COUNT;
  Env E;
  E.b0 = h[H_B0]; E.nb = h[H_NB]; E.j0 = h[H_J0]; E.nj = h[H_NJ];
  E.lam_off = h[H_LAMOFF]; E.lam_size = h[H_LAMSZ]; E.G = h[H_G]; E.P = h[H_P]; E.ncol = h[H_NCOL];
  E.lam_imp = E.lam_size - (M.ctrl ? M.mlp_rec : 0);
  E.jr = M.servo ? 6 : 5;
  E.T = h[H_T]; E.lb = h[H_LB]; E.ccap = h[H_CCAP]; E.ncand = h[H_NCAND]; E.e = h[H_ENV];
  E.nslot = h[H_NSLOT]; E.seg_off = h[H_SEG]; E.tape_off = h[H_TAPE];
  E.gtopo = M.topo + h[H_TOPO];
  E.gcst = M.cst + h[H_CST];
  E.L = lds;
  // (the reverse of saved working sets may keep a ring of the impulse
  // history: an env flagged for it in its header)
  E.lay = make_lay(E.nb, E.nj, E.G, E.P, E.ncol, E.ncand, E.nj + E.ccap, E.nslot, E.lam_size, n_iters, adj,
                   mlp_floats_fwd(M),
                   mlp_floats_adj(M), vsave_floats(M.ws_kind || M.has_rest, E.nb),
                   M.dump != DUMP_REPLAY && h[H_RING] != 0);
  return E;
}

// Colours with at least one active constraint this step (built by f_rows):
// the sweeps visit only these, in canonical order, which changes nothing but
// the number of (empty) colour passes.
SHD int n_live(const Env& E, bool act) { return act ? E.live()[0] : 0; }
SHD int n_plan(const Env& E, bool act) { return act ? E.live()[2 + E.ncol] : 0; }
SHD int live_col(const Env& E, int i) { return E.live()[2 + i]; }
SHD int n_joint_cols(const Env& E, bool act) { return act ? E.live()[1] : 0; }

// per-env constants in global memory:
//   bodies  invm[nb], invI[3][nb], pair-sphere offset[3][nb], pair-sphere radius[nb]
//   joints  20 floats each (JAP..JD layout, JU unused)
//   ground  offset(3), radius  per ground sphere
//   env     mu, restitution
SHD int cst_joint(const Env& E) { return 8 * E.nb; }
SHD int cst_ground(const Env& E) { return 8 * E.nb + JS * E.nj; }
SHD int cst_env(const Env& E) { return 8 * E.nb + JS * E.nj + 4 * E.G; }
SHD int cst_size(int nb, int nj, int G) { return 8 * nb + JS * nj + 4 * G + 4; }
SHD int topo_size(int nj, int G, int P, int ncol, int ncand) { return 2 * nj + G + P + ncol + 1 + ncand; }

// Load topology and constants of the env into LDS (team-parallel).
template <class Team>
SHD void load_env_static(const Team& tm, const DevModel& M, const Env& E) {
  const int ntopo = topo_size(E.nj, E.G, E.P, E.ncol, E.ncand);
  int* tp = E.topo();
  for (int i = tm.tl; i < ntopo; i += tm.ts) tp[i] = E.gtopo[i];
  for (int b = tm.tl; b < E.nb; b += tm.ts) {
    float* B = E.body(b);
    B[BIM] = E.gcst[b];
    for (int k = 0; k < 3; ++k) B[BII + k] = E.gcst[E.nb + 3 * b + k];
    for (int k = 0; k < 3; ++k) B[BPO + k] = E.gcst[4 * E.nb + 3 * b + k];
    B[BPR] = E.gcst[7 * E.nb + b];
  }
  // the world slot: a body at rest with zero inverse mass and inertia, the
  // second body of world-attached joints and ground contacts in the sweeps
  for (int i = tm.tl; i < BS; i += tm.ts) E.body(E.nb)[i] = 0.f;
  for (int i = tm.tl; i < JS * E.nj; i += tm.ts) E.L[E.lay.jc + i] = E.gcst[cst_joint(E) + i];
  for (int i = tm.tl; i < 4 * E.G; i += tm.ts) E.L[E.lay.gs + i] = E.gcst[cst_ground(E) + i];
  if (tm.tl == 0) {
    int m = 0;
    while (m < E.ncol && E.gtopo[2 * E.nj + E.G + E.P + m] < E.gtopo[2 * E.nj + E.G + E.P + m + 1] &&
           cand_kind(E.gtopo[2 * E.nj + E.G + E.P + E.ncol + 1 + E.gtopo[2 * E.nj + E.G + E.P + m]]) == K_JOINT)
      ++m;
    E.live()[0] = 0;
    E.live()[1] = m;
    E.live()[2 + E.ncol] = 0;
    E.misc()[MISC_MU] = E.gcst[cst_env(E)];
    E.misc()[MISC_REST] = E.gcst[cst_env(E) + 1];
    E.misc()[MISC_LOSS] = 0.f;
    (*reinterpret_cast<int*>(E.misc() + MISC_FLAGS)) = 0;
    (*reinterpret_cast<int*>(E.misc() + MISC_ITERS)) = 0;
    (*reinterpret_cast<int*>(E.misc() + MISC_FB)) = 0;
  }
}

// state x[18][B] (SoA, global) <-> LDS body records
template <class Team>
SHD void load_state(const Team& tm, const Env& E, const float* x, int B) {
  for (int b = tm.tl; b < E.nb; b += tm.ts) {
    float* R = E.body(b);
    for (int k = 0; k < 18; ++k) R[k] = x[(size_t)k * B + E.b0 + b];
  }
}
template <class Team>
SHD void store_state(const Team& tm, const Env& E, float* x, int B) {
  for (int b = tm.tl; b < E.nb; b += tm.ts) {
    const float* R = E.body(b);
    for (int k = 0; k < 18; ++k) x[(size_t)k * B + E.b0 + b] = R[k];
  }
}
template <class Team>
SHD void load_ws(const Team& tm, const Env& E, const float* lam) {
  for (int i = tm.tl; i < E.lam_size; i += tm.ts) E.ws()[i] = lam[E.lam_off + i];
}
template <class Team>
SHD void store_ws(const Team& tm, const Env& E, float* lam) {
  for (int i = tm.tl; i < E.lam_size; i += tm.ts) lam[E.lam_off + i] = E.ws()[i];
}

// ------------------------------------------------------------------ row helpers
// two-body row: a may be -1 (world)
struct RowB { int a, b; };

SHD float row_jv(const float* r, const float* va, const float* wa, const float* vb, const float* wb, bool has_a) {
  // J v = Jl.(vb - va) + Jaa.wa + Jab.wb
  float s = r[RJL] * vb[0] + r[RJL + 1] * vb[1] + r[RJL + 2] * vb[2];
  s += r[RJB] * wb[0] + r[RJB + 1] * wb[1] + r[RJB + 2] * wb[2];
  if (has_a) {
    s -= r[RJL] * va[0] + r[RJL + 1] * va[1] + r[RJL + 2] * va[2];
    s += r[RJA] * wa[0] + r[RJA + 1] * wa[1] + r[RJA + 2] * wa[2];
  }
  return s;
}
SHD void row_apply(const float* r, float* va, float* wa, float* vb, float* wb, bool has_a, float ima, float imb,
                   float d) {
  // (row slots are 16-byte aligned: Jl, W_b and W_a are read as float4)
  const f4 jl = ld4(r + RJL), wr = ld4(r + RWB);
  const float cb = imb * d;
  vb[0] += cb * jl.x; vb[1] += cb * jl.y; vb[2] += cb * jl.z;
  wb[0] += d * wr.x; wb[1] += d * wr.y; wb[2] += d * wr.z;
  if (has_a) {
    const f4 wl = ld4(r + RWA);
    const float ca = ima * d;
    va[0] -= ca * jl.x; va[1] -= ca * jl.y; va[2] -= ca * jl.z;
    wa[0] += d * wl.x; wa[1] += d * wl.y; wa[2] += d * wl.z;
  }
}
// W = M^-1 J^T (angular parts stored), returns K = J W
SHD float row_finish(float* r, const float* Ba, const float* Bb, bool has_a) {
  const f3 jl = ld3(r + RJL);
  const f3 jb = ld3(r + RJB);
  const f3 wb = sv(Bb + BI, jb);
  st3(r + RWB, wb);
  float im = Bb[BIM];
  float k = dot(jb, wb);
  if (has_a) {
    const f3 ja = ld3(r + RJA);
    const f3 wa = sv(Ba + BI, ja);
    st3(r + RWA, wa);
    k += dot(ja, wa);
    im += Ba[BIM];
  } else {
    // no body a: both of its parts are zero (the world slot's velocity is
    // zero, so these rows act on body b alone)
    st3(r + RJA, mk3(0.f, 0.f, 0.f));
    st3(r + RWA, mk3(0.f, 0.f, 0.f));
  }
  return k + im * dot(jl, jl);
}

// The lane-local copy of the two bodies' velocities used while one lane
// updates the rows of one constraint.
struct Vel {
  float va[3], wa[3], vb[3], wb[3];
};
SHD void vel_load(Vel& V, const Env& E, int a, int b) {
  const float* Bb = E.body(b);
  for (int k = 0; k < 3; ++k) { V.vb[k] = Bb[BV + k]; V.wb[k] = Bb[BW + k]; }
  if (a >= 0) {
    const float* Ba = E.body(a);
    for (int k = 0; k < 3; ++k) { V.va[k] = Ba[BV + k]; V.wa[k] = Ba[BW + k]; }
  } else {
    for (int k = 0; k < 3; ++k) { V.va[k] = 0.f; V.wa[k] = 0.f; }
  }
}
SHD void vel_store(const Vel& V, const Env& E, int a, int b) {
  float* Bb = E.body(b);
  for (int k = 0; k < 3; ++k) { Bb[BV + k] = V.vb[k]; Bb[BW + k] = V.wb[k]; }
  if (a >= 0) {
    float* Ba = E.body(a);
    for (int k = 0; k < 3; ++k) { Ba[BV + k] = V.va[k]; Ba[BW + k] = V.wa[k]; }
  }
}

// bodies of a candidate constraint
SHD RowB cand_bodies(const Env& E, int code) {
  const int k = cand_kind(code), i = cand_idx(code);
  RowB r;
  if (k == K_JOINT) { r.a = E.jpar(i); r.b = E.jchi(i); }
  else if (k == K_GROUND) { r.a = -1; r.b = E.gbody(i); }
  else { const int pc = E.pcode(i); r.a = pc & 0xFFFF; r.b = pc >> 16; }
  return r;
}

// disk projection of the tangent impulse: inside iff |l| <= rho
SHD void disk(float l1, float l2, float rho, float& o1, float& o2) {
  const float n = sqrtf(l1 * l1 + l2 * l2);
  if (n <= rho) { o1 = l1; o2 = l2; }
  else { const float s = rho / n; o1 = s * l1; o2 = s * l2; }
}

// ------------------------------------------------------------------ forward phases
// F1: world inverse inertia R diag(1/I) R^T; torque accumulators cleared.
template <class Team>
SHD void f_body_setup(const Team& tm, const Env& E, bool act, bool rec) {
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    float* B = E.body(b);
    const float* R = B + BR;
    const float d0 = B[BII], d1 = B[BII + 1], d2 = B[BII + 2];
    // S = R D R^T
    float S[6];
    S[0] = R[0] * R[0] * d0 + R[1] * R[1] * d1 + R[2] * R[2] * d2;
    S[1] = R[3] * R[3] * d0 + R[4] * R[4] * d1 + R[5] * R[5] * d2;
    S[2] = R[6] * R[6] * d0 + R[7] * R[7] * d1 + R[8] * R[8] * d2;
    S[3] = R[0] * R[3] * d0 + R[1] * R[4] * d1 + R[2] * R[5] * d2;
    S[4] = R[0] * R[6] * d0 + R[1] * R[7] * d1 + R[2] * R[8] * d2;
    S[5] = R[3] * R[6] * d0 + R[4] * R[7] * d1 + R[5] * R[8] * d2;
    for (int k = 0; k < 6; ++k) B[BI + k] = S[k];
    B[BTQ] = B[BTQ + 1] = B[BTQ + 2] = 0.f;
    if (rec) {
      float* A = E.bodyA(b);
      A[AW0] = B[BW]; A[AW0 + 1] = B[BW + 1]; A[AW0 + 2] = B[BW + 2];
    }
  }
}

// hinge axis in world coordinates (parent frame rotated, or the world axis)
SHD f3 joint_axis_w(const Env& E, int j) {
  const float* C = E.jc(j);
  const int a = E.jpar(j);
  const f3 n = ld3(C + JXP);
  return a >= 0 ? mv(E.body(a) + BR, n) : n;
}

// F2: motor torque minus viscous damping, equal and opposite on child and
// parent.  Joints run colour by colour so no two lanes touch one body.
template <class Team>
SHD void f_torques(const Team& tm, const Env& E, bool act) {
  // joints occupy the first colours of the canonical order; a joint colour
  // holds only joints
  const int njc = n_joint_cols(E, act);
  for (int c = 0; tm.any(c < njc); ++c) {
    int lo = 0, hi = 0;
    if (c < njc) { lo = E.colstart(c); hi = E.colstart(c + 1); }
    for (int i = lo + tm.tl; i < hi; i += tm.ts) {
      const int j = cand_idx(E.cand(i));
      const float* C = E.jc(j);
      const int a = E.jpar(j), b = E.jchi(j);
      const f3 n = joint_axis_w(E, j);
      float* Bb = E.body(b);
      f3 wrel = ld3(Bb + BW);
      if (a >= 0) wrel = wrel - ld3(E.body(a) + BW);
      // (a servo's control is its target angle, not a torque)
      const float tau = (E.jr == 6 ? 0.f : C[JU]) - C[JD] * dot(wrel, n);
      add3(Bb + BTQ, tau * n);
      if (a >= 0) add3(E.body(a) + BTQ, -(tau * n));
    }
    tm.sync();
  }
}

// F3: v* = v + dt g ; w* = w + dt Iw tq
template <class Team>
SHD void f_predict(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    float* B = E.body(b);
    B[BV] += M.dt * M.gx; B[BV + 1] += M.dt * M.gy; B[BV + 2] += M.dt * M.gz;
    const f3 dw = sv(B + BI, ld3(B + BTQ));
    B[BW] += M.dt * dw.x; B[BW + 1] += M.dt * dw.y; B[BW + 2] += M.dt * dw.z;
  }
}

// Build the rows of one joint into slots s..s+4 (s+5: a servo's motor row).  Each row is formed in
// registers (W = M^-1 J^T, K = J W, m = 1 / (K + gamma), as row_finish forms
// them, in the same order) and written with 16-byte stores.
static_assert(RMA == RJA + 3 && RBA == RWA + 3 && RM == RJB + 3 && RBI == RWB + 3 && RL == RJL + 3 &&
                  RJA % 4 == 0 && RWA % 4 == 0 && RJB % 4 == 0 && RWB % 4 == 0 && RJL % 4 == 0,
              "row slot layout");
SHD void build_joint(const DevModel& M, const Env& E, int j, int s) {
  const float* C = E.jc(j);
  const int a = E.jpar(j), b = E.jchi(j);
  const bool ha = a >= 0;
  const float* Bb = E.body(b);
  const float* Ba = ha ? E.body(a) : nullptr;
  float Ib[6], Ia[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < 6; ++k) Ib[k] = Bb[BI + k];
  if (ha)
    for (int k = 0; k < 6; ++k) Ia[k] = Ba[BI + k];
  const float imb = Bb[BIM], ima = ha ? Ba[BIM] : 0.f;
  const f3 rb = mv(Bb + BR, ld3(C + JAC));
  f3 ra = mk3(0.f, 0.f, 0.f), Pa = ld3(C + JAP);
  if (ha) { ra = mv(Ba + BR, Pa); Pa = ld3(Ba + BP) + ra; }
  const f3 err = (ld3(Bb + BP) + rb) - Pa;
  const float kb = M.beta / M.dt;
  f3 na = ld3(C + JXP), ua = ld3(C + JUP);
  f3 t2 = cross(na, ua);
  if (ha) { na = mv(Ba + BR, na); ua = mv(Ba + BR, ua); t2 = mv(Ba + BR, t2); }
  const f3 nbw = mv(Bb + BR, ld3(C + JXC));
  const f3 ax = cross(na, nbw);
  const float* w0 = E.ws() + E.jr * j;
  // (unrolled: the row index is a constant in each copy, so nothing indexed
  // by it leaves the registers; the sixth row only with a servo)
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q == 5 && E.jr != 6) break;
    f3 jl, ja, jb;
    float bias;
    float clip = 0.f;
    if (q == 5) {
      // servo: relative rate about the parent's axis driven toward
      // gain (theta* - theta), clipped to the rate limit
      const f3 ub = mv(Bb + BR, ld3(C + JUC));
      const float th = atan2f(dot(cross(ua, ub), na), dot(ua, ub));
      float rate = C[JG] * (C[JU] - th);
      if (rate > C[JV]) { rate = C[JV]; clip = 1.f; }
      else if (rate < -C[JV]) { rate = -C[JV]; clip = 1.f; }
      jl = mk3(0.f, 0.f, 0.f);
      ja = -na;
      jb = na;
      bias = -rate;
    } else if (q < 3) {
      const f3 e = mk3(q == 0 ? 1.f : 0.f, q == 1 ? 1.f : 0.f, q == 2 ? 1.f : 0.f);
      jl = e;
      ja = cross(e, ra);
      jb = cross(rb, e);
      bias = kb * (q == 0 ? err.x : (q == 1 ? err.y : err.z));
    } else {
      const f3 tk = q == 3 ? ua : t2;
      jl = mk3(0.f, 0.f, 0.f);
      ja = -tk;
      jb = tk;
      bias = kb * dot(tk, ax);
    }
    const f3 wb = sv(Ib, jb);
    float im = imb;
    float K = dot(jb, wb);
    f3 wa = mk3(0.f, 0.f, 0.f);
    if (ha) {
      wa = sv(Ia, ja);
      K += dot(ja, wa);
      im += ima;
    } else {
      // no body a: both of its parts are zero (the world slot's velocity is
      // zero, so these rows act on body b alone)
      ja = mk3(0.f, 0.f, 0.f);
    }
    K = K + im * dot(jl, jl);
    const float m = 1.f / (K + M.gamma);
    const float l0 = M.warm * w0[q];
    float* r = E.row(s + q);
    st4(r + RJA, f4{ja.x, ja.y, ja.z, m});
    st4(r + RWA, f4{wa.x, wa.y, wa.z, bias});
    st4(r + RJB, f4{jb.x, jb.y, jb.z, m});
    st4(r + RWB, f4{wb.x, wb.y, wb.z, bias});
    st4(r + RJL, f4{jl.x, jl.y, jl.z, l0});
    r[RL0] = l0;
    if (q == 5) {
      r[RHI] = C[JT] * M.dt;
      r[RCLIP] = clip;
    }
  }
}

// Gap and geometry of a contact candidate; returns the gap.
struct CGeo {
  f3 n, ra, rb;   // normal, lever arms (contact point minus body centre)
  f3 ca, cb;      // sphere centres (pair), or cb for ground
  float L, gap;
};
SHD CGeo contact_geo(const Env& E, int code) {
  CGeo g;
  const int k = cand_kind(code), i = cand_idx(code);
  if (k == K_GROUND) {
    const int b = E.gbody(i);
    const float* Bb = E.body(b);
    const float* S = E.gsph(i);
    g.cb = ld3(Bb + BP) + mv(Bb + BR, ld3(S));
    g.gap = g.cb.z - S[3];
    g.n = mk3(0.f, 0.f, 1.f);
    g.rb = (g.cb - S[3] * g.n) - ld3(Bb + BP);
    g.ra = mk3(0.f, 0.f, 0.f);
    g.ca = g.ra;
    g.L = 0.f;
  } else {
    const int pc = E.pcode(i), a = pc & 0xFFFF, b = pc >> 16;
    const float* Ba = E.body(a);
    const float* Bb = E.body(b);
    g.ca = ld3(Ba + BP) + mv(Ba + BR, ld3(Ba + BPO));
    g.cb = ld3(Bb + BP) + mv(Bb + BR, ld3(Bb + BPO));
    const f3 d = g.cb - g.ca;
    g.L = sqrtf(dot(d, d));
    g.gap = g.L - Ba[BPR] - Bb[BPR];
    g.n = g.L < 1e-9f ? mk3(0.f, 0.f, 1.f) : (1.f / g.L) * d;
    g.ra = (g.ca + Ba[BPR] * g.n) - ld3(Ba + BP);
    g.rb = (g.cb - Bb[BPR] * g.n) - ld3(Bb + BP);
  }
  return g;
}
SHD void tangents(f3 n, bool ground, f3& t1, f3& t2) {
  if (ground) { t1 = mk3(1.f, 0.f, 0.f); t2 = mk3(0.f, 1.f, 0.f); return; }
  const f3 w = fabsf(n.z) < 0.9f ? cross(n, mk3(0.f, 0.f, 1.f)) : cross(n, mk3(1.f, 0.f, 0.f));
  t1 = (1.f / sqrtf(dot(w, w))) * w;
  t2 = cross(n, t1);
}

// Build an active contact into slots s..s+3.
SHD void build_contact(const DevModel& M, const Env& E, int code, int s, const CGeo& g) {
  const RowB rb = cand_bodies(E, code);
  const bool ground = cand_kind(code) == K_GROUND;
  const float* Bb = E.body(rb.b);
  const float* Ba = rb.a >= 0 ? E.body(rb.a) : nullptr;
  f3 t1, t2;
  tangents(g.n, ground, t1, t2);
  const f3 dirs[3] = {g.n, t1, t2};
  float K[3];
  for (int q = 0; q < 3; ++q) {
    float* r = E.row(s + q);
    st3(r + RJL, dirs[q]);
    st3(r + RJA, ground ? mk3(0.f, 0.f, 0.f) : cross(dirs[q], g.ra));
    st3(r + RJB, cross(g.rb, dirs[q]));
    K[q] = row_finish(r, Ba, Bb, !ground);
  }
  float* x = E.row(s + 3);
  st3(x + XT1, t1);
  st3(x + XT2, t2);
  x[XMT] = 2.f / (K[1] + K[2]);
  x[XGAP] = g.gap;
  const int st = E.store_of(code);
  *reinterpret_cast<int*>(x + XSTORE) = st;
  *reinterpret_cast<int*>(x + XCODE) = code;
  float* rn = E.row(s);
  rn[RM] = rn[RMA] = 1.f / (K[0] + M.gamma);
  float bias = (g.gap > 0.f ? g.gap : M.beta * g.gap) / M.dt;
  // restitution: a contact that the predicted velocities (the body records
  // now) would close within the step, approaching faster than the threshold,
  // leaves at e times its approach speed unless the push-out is faster
  float rest = 0.f;
  const float e = E.misc()[MISC_REST];
  if (e > 0.f) {
    const float vn = row_jv(rn, Ba ? Ba + BV : nullptr, Ba ? Ba + BW : nullptr, Bb + BV, Bb + BW, !ground);
    if (vn < -M.rest_th && vn * M.dt + g.gap < 0.f && e * vn < bias) {
      bias = e * vn;
      rest = 1.f;
    }
  }
  x[XREST] = rest;
  rn[RBI] = rn[RBA] = bias;
  const float* w = E.ws() + st;
  const f3 Lt = mk3(w[1], w[2], w[3]);
  rn[RL] = rn[RL0] = M.warm * w[0];
  E.row(s + 1)[RL] = E.row(s + 1)[RL0] = M.warm * dot(t1, Lt);
  E.row(s + 2)[RL] = E.row(s + 2)[RL0] = M.warm * dot(t2, Lt);
  E.row(s + 1)[RM] = E.row(s + 1)[RMA] = x[XMT];
  E.row(s + 2)[RM] = E.row(s + 2)[RMA] = x[XMT];
  E.row(s + 1)[RBI] = E.row(s + 1)[RBA] = 0.f;
  E.row(s + 2)[RBI] = E.row(s + 2)[RBA] = 0.f;
}

// F4: per colour, test candidates, compact the active ones, build rows.
// Inactive contact candidates have their stored impulses cleared.  A colour
// holds only joints or only contacts.
//
// The sweep plan lists the step's visits: each joint colour with an active
// constraint, and runs of consecutive live contact colours merged into one
// visit where no constraint of a later colour touches a body that an earlier
// colour of the run touches (the world slot aside).  Such constraints commute
// with everything before them in the run (each update reads and writes only
// its own row and its two bodies), so a merged visit gives the same bits as
// the colours one after another, with fewer visits per sweep: a long chain's
// pair contacts fall into many colours with one or two active pairs each.
// vis() holds the placed constraints contiguously, visit by visit: every
// active joint and the active contacts that found a row slot (a contact
// beyond the env's capacity is dropped and the env flagged, and gets no
// entry), so it needs nj + ccap entries; the colour's active lists
// (act_code, act_slot, act_cnt) keep every active constraint.
template <class Team>
SHD void f_rows(const Team& tm, const DevModel& M, const Env& E, bool act) {
  // Joint rows depend only on the step's body state, so all joints are built
  // at once, lanes over joints; the colour loop below lists them.
  const int nj = act ? E.nj : 0;
  for (int j = tm.tl; j < nj; j += tm.ts) build_joint(M, E, j, E.jr * j);
  for (int b = tm.tl; b <= (act ? E.nb : -1); b += tm.ts) E.grp()[b] = -2;
  tm.sync();
  int ncon = 0;                    // active contacts so far, placed while below ccap (team-uniform)
  int voff = 0;                    // entries of vis() so far
  int np = 0;                      // plan entries opened so far
  int gstart = 0, gcnt = 0, gkind = -1;   // the open plan entry
  for (int c = 0; tm.any(c < E.ncol && act); ++c) {
    int lo = 0, hi = 0;
    if (act && c < E.ncol) { lo = E.colstart(c); hi = E.colstart(c + 1); }
    const bool jcol = hi > lo && cand_kind(E.cand(lo)) == K_JOINT;
    int cnt = 0;          // active constraints of this colour
    int vcnt = 0;         // of them placed (vis entries)
    bool clash = false;   // this lane's constraints touch a body of the open entry
    for (int base = lo; tm.any(base < hi); base += tm.ts) {
      const int i = base + tm.tl;
      const bool live = i < hi;
      const int code = live ? E.cand(i) : 0;
      bool on = false;
      CGeo g;
      if (live) {
        if (jcol) on = true;
        else {
          g = contact_geo(E, code);
          on = g.gap < M.spec;
          if (!on) {
            float* w = E.ws() + E.store_of(code);
            w[0] = w[1] = w[2] = w[3] = 0.f;
          }
        }
      }
      int total = 0;
      const int pos = tm.prefix(on, total);
      // placed: every joint; the contacts while the capacity lasts, i.e. the
      // first `room` active ones of this pass (team-uniform)
      const int room = jcol ? total : (E.ccap - ncon <= 0 ? 0 : (E.ccap - ncon < total ? E.ccap - ncon : total));
      if (on) {
        const int li = lo + cnt + pos;   // position in the colour's active list
        E.act_code()[li] = code;
        int s = -1;
        if (jcol) {
          s = E.jr * cand_idx(code);
        } else if (pos < room) {
          s = E.jr * E.nj + 4 * (ncon + pos);
          build_contact(M, E, code, s, g);
        } else {
          // beyond the env's contact capacity: dropped, env flagged
          float* w = E.ws() + E.store_of(code);
          w[0] = w[1] = w[2] = w[3] = 0.f;
          (*reinterpret_cast<int*>(E.misc() + MISC_FLAGS)) |= 2;
        }
        E.act_slot()[li] = s;
        if (pos < room) {
          const RowB rb = cand_bodies(E, code);
          E.vis()[voff + vcnt + pos] = i4{s, rb.a >= 0 ? rb.a : E.nb, rb.b, code};
          if (!jcol) clash = clash || (rb.a >= 0 && E.grp()[rb.a] == np - 1) || E.grp()[rb.b] == np - 1;
        }
      }
      cnt += total;
      vcnt += room;
      if (!jcol) ncon += total;
    }
    if (act && c < E.ncol) E.act_cnt()[c] = cnt;
    const bool merge = !tm.team_any(clash) && !jcol && gkind == 0;
    if (vcnt > 0) {
      if (!merge) {
        if (gcnt > 0 && tm.tl == 0) E.plan()[np - 1] = i4{gstart, gcnt, gkind, 0};
        ++np;
        gstart = voff;
        gcnt = 0;
        gkind = jcol ? 1 : 0;
      }
      gcnt += vcnt;
      // the open entry's bodies: this colour's constraints touch distinct
      // bodies (the world slot aside, which is not marked)
      if (!jcol)
        for (int k = tm.tl; k < vcnt; k += tm.ts) {
          const i4 v = E.vis()[voff + k];
          E.grp()[v.z] = np - 1;
          if (v.y < E.nb) E.grp()[v.y] = np - 1;
        }
      voff += vcnt;
    }
    tm.sync();
  }
  if (act && tm.tl == 0) {
    if (gcnt > 0) E.plan()[np - 1] = i4{gstart, gcnt, gkind, 0};
    E.live()[2 + E.ncol] = np;
    int m = 0;
    for (int c = 0; c < E.ncol; ++c)
      if (E.act_cnt()[c] > 0) E.live()[2 + m++] = c;
    E.live()[0] = m;
  }
  tm.sync();
}

// The colour visits of n_iters sweeps over the live colours, first to last
// (DIR = 1) or last to first (DIR = -1).  The plan does not change during the
// sweeps, so the loads of the next visit's entries (this lane's first
// constraint of the next colour, the plan of the colour after it) are issued
// before the current visit runs and are not waited for at its start.
template <int DIR>
struct SweepCursor {
  int nl, left;   // live colours; visits left, the current one included
  int it, ci;     // iteration and live colour of the current visit
  int cn, c2;     // live colours of the next two visits
  i4 pc, vc, pn;  // plan and this lane's first entry of the current colour, plan of the next
  SHD int step(int c) const { return DIR > 0 ? (c + 1 == nl ? 0 : c + 1) : (c == 0 ? nl - 1 : c - 1); }
  // Hinges are visited by lane pairs (one body each) when the team has two
  // lanes or more: lane tl takes constraints l0(tl) + k * step(tl).
  template <class Team>
  SHD static bool paired(const Team& tm, const i4& p) { return p.z != 0 && tm.ts >= 2; }
  template <class Team>
  SHD static int l0(const Team& tm, const i4& p) { return paired(tm, p) ? tm.tl >> 1 : tm.tl; }
  template <class Team>
  SHD static int stride(const Team& tm, const i4& p) { return paired(tm, p) ? tm.ts >> 1 : tm.ts; }
  // (written with plain branches: a conditional expression over two 16-byte
  // lvalues makes the compiler keep the cursor in scratch memory)
  template <class Team>
  SHD i4 first(const Team& tm, const Env& E, const i4& p, bool ok) const {
    const int i = l0(tm, p);
    i4 r{-1, 0, 0, 0};
    if (ok && i < p.y) r = E.vis()[p.x + i];
    return r;
  }
  template <class Team>
  SHD void start(const Team& tm, const Env& E, int n_iters, int n_live_cols) {
    nl = n_live_cols;
    left = nl * n_iters;
    it = DIR > 0 ? 0 : n_iters - 1;
    ci = DIR > 0 ? 0 : nl - 1;
    cn = step(ci);
    c2 = step(cn);
    pc = i4{0, 0, 0, 0};
    if (left > 0) pc = E.plan()[ci];
    vc = first(tm, E, pc, left > 0);
    pn = i4{0, 0, 0, 0};
    if (left > 1) pn = E.plan()[cn];
  }
  // loads for the next visit (call before the current one runs)
  template <class Team>
  SHD void prefetch(const Team& tm, const Env& E, i4& vn, i4& p2) const {
    vn = first(tm, E, pn, left > 1);
    p2 = i4{0, 0, 0, 0};
    if (left > 2) p2 = E.plan()[c2];
  }
  // this lane's k-th constraint of the current colour (k >= 1: not prefetched)
  template <class Team>
  SHD i4 entry(const Team& tm, const Env& E, int k) const {
    if (k == 0) return vc;
    return E.vis()[pc.x + l0(tm, pc) + k * stride(tm, pc)];
  }
  // constraints of the current colour this lane takes part in (the stride
  // is a power of two, as team widths are, so the quotient is a shift)
  template <class Team>
  SHD int count(const Team& tm) const {
    const int n = left > 0 ? pc.y : 0, i = l0(tm, pc), sh = __builtin_ctz(stride(tm, pc));
    return i < n ? (n - i + (1 << sh) - 1) >> sh : 0;
  }
  SHD void advance(const i4& vn, const i4& p2) {
    if (cn == (DIR > 0 ? 0 : nl - 1)) it += DIR;
    --left;
    ci = cn;
    cn = c2;
    c2 = step(c2);
    pc = pn;
    vc = vn;
    pn = p2;
  }
};

// Velocities of a constraint's two bodies in registers.
struct VR { float va[3], wa[3], vb[3], wb[3]; };
SHD void vr_load(VR& V, const Env& E, int a, int b) {
  const float* Bb = E.body(b) + BV;   // v(3), w(3) contiguous, 16-byte aligned
  const f4 q0 = ld4(Bb);
  V.vb[0] = q0.x; V.vb[1] = q0.y; V.vb[2] = q0.z; V.wb[0] = q0.w; V.wb[1] = Bb[4]; V.wb[2] = Bb[5];
  if (a >= 0) {
    const float* Ba = E.body(a) + BV;
    const f4 p0 = ld4(Ba);
    V.va[0] = p0.x; V.va[1] = p0.y; V.va[2] = p0.z; V.wa[0] = p0.w; V.wa[1] = Ba[4]; V.wa[2] = Ba[5];
  } else {
    for (int k = 0; k < 3; ++k) { V.va[k] = 0.f; V.wa[k] = 0.f; }
  }
}
SHD void vr_store(const VR& V, const Env& E, int a, int b) {
  float* Bb = E.body(b) + BV;
  f4 q0; q0.x = V.vb[0]; q0.y = V.vb[1]; q0.z = V.vb[2]; q0.w = V.wb[0];
  st4(Bb, q0); Bb[4] = V.wb[1]; Bb[5] = V.wb[2];
  if (a >= 0) {
    float* Ba = E.body(a) + BV;
    f4 p0; p0.x = V.va[0]; p0.y = V.va[1]; p0.z = V.va[2]; p0.w = V.wa[0];
    st4(Ba, p0); Ba[4] = V.wa[1]; Ba[5] = V.wa[2];
  }
}
// Both bodies of a sweep visit (body a may be the world slot).
SHD void vr_load_ab(VR& V, const Env& E, int a, int b) {
  const float* Bb = E.body(b) + BV;
  const float* Ba = E.body(a) + BV;
  const f4 q0 = ld4(Bb), p0 = ld4(Ba);
  V.vb[0] = q0.x; V.vb[1] = q0.y; V.vb[2] = q0.z; V.wb[0] = q0.w; V.wb[1] = Bb[4]; V.wb[2] = Bb[5];
  V.va[0] = p0.x; V.va[1] = p0.y; V.va[2] = p0.z; V.wa[0] = p0.w; V.wa[1] = Ba[4]; V.wa[2] = Ba[5];
}
// Body b alone (a ground contact: body a is the world slot, whose velocity
// is zero and stays zero).
SHD void vr_load_b(VR& V, const Env& E, int b) {
  const float* Bb = E.body(b) + BV;
  const f4 q0 = ld4(Bb);
  V.vb[0] = q0.x; V.vb[1] = q0.y; V.vb[2] = q0.z; V.wb[0] = q0.w; V.wb[1] = Bb[4]; V.wb[2] = Bb[5];
  for (int k = 0; k < 3; ++k) { V.va[k] = 0.f; V.wa[k] = 0.f; }
}
SHD void vr_store_b(const VR& V, const Env& E, int b) {
  float* Bb = E.body(b) + BV;
  f4 q0; q0.x = V.vb[0]; q0.y = V.vb[1]; q0.z = V.vb[2]; q0.w = V.wb[0];
  st4(Bb, q0); Bb[4] = V.wb[1]; Bb[5] = V.wb[2];
}
SHD void vr_store_ab(const VR& V, const Env& E, int a, int b) {
  float* Bb = E.body(b) + BV;
  float* Ba = E.body(a) + BV;
  f4 q0; q0.x = V.vb[0]; q0.y = V.vb[1]; q0.z = V.vb[2]; q0.w = V.wb[0];
  f4 p0; p0.x = V.va[0]; p0.y = V.va[1]; p0.z = V.va[2]; p0.w = V.wa[0];
  st4(Bb, q0); Bb[4] = V.wb[1]; Bb[5] = V.wb[2];
  st4(Ba, p0); Ba[4] = V.wa[1]; Ba[5] = V.wa[2];
}
// One row slot in registers: Jl, Ja, Jb, Wa, Wb, m, bias, lam (lam0 not needed).
struct RR { float jl[3], ja[3], jb[3], wa[3], wb[3], m, bias, lam; };
SHD void rr_load(RR& R, const float* p) {
  const f4 a = ld4(p + RJA), b = ld4(p + RWA), c = ld4(p + RJB), d = ld4(p + RWB), e = ld4(p + RJL);
  R.ja[0] = a.x; R.ja[1] = a.y; R.ja[2] = a.z;
  R.wa[0] = b.x; R.wa[1] = b.y; R.wa[2] = b.z;
  R.jb[0] = c.x; R.jb[1] = c.y; R.jb[2] = c.z; R.m = c.w;
  R.wb[0] = d.x; R.wb[1] = d.y; R.wb[2] = d.z; R.bias = d.w;
  R.jl[0] = e.x; R.jl[1] = e.y; R.jl[2] = e.z; R.lam = e.w;
}
SHD float rr_jv(const RR& R, const VR& V, bool ha) {
  float s = R.jl[0] * V.vb[0] + R.jl[1] * V.vb[1] + R.jl[2] * V.vb[2];
  s += R.jb[0] * V.wb[0] + R.jb[1] * V.wb[1] + R.jb[2] * V.wb[2];
  if (ha) {
    s -= R.jl[0] * V.va[0] + R.jl[1] * V.va[1] + R.jl[2] * V.va[2];
    s += R.ja[0] * V.wa[0] + R.ja[1] * V.wa[1] + R.ja[2] * V.wa[2];
  }
  return s;
}
SHD void rr_apply(const RR& R, VR& V, bool ha, float ima, float imb, float d) {
  const float cb = imb * d;
  for (int k = 0; k < 3; ++k) { V.vb[k] += cb * R.jl[k]; V.wb[k] += d * R.wb[k]; }
  if (ha) {
    const float ca = ima * d;
    for (int k = 0; k < 3; ++k) { V.va[k] -= ca * R.jl[k]; V.wa[k] += d * R.wa[k]; }
  }
}

// ------------------------------------------------------------------ hinge visits
// A hinge row's arithmetic split by body.  Its point rows have Jl = e_S (axis
// S = 0, 1, 2) and its angular rows Jl = 0 (S = 3), so the row's J v is the
// sum of side b's part v_b,S + Jb . w_b and side a's part -v_a,S + Ja . w_a
// (side a is the world slot when there is no body a), always added as
// (part b) + (part a); W . vbar in the reverse likewise.  A visit runs with
// both sides in one lane (NS = 2) or with one side on each lane of a pair
// (2m: a, 2m+1: b; NS = 1) whose lanes swap their parts.  IEEE addition is
// commutative and each side's arithmetic applies its sign to one exact
// leaf (sg = +-1 times a value), so both forms give the same bits: results do
// not depend on the team width.  The adjoint of Jl, a constant, is skipped.
struct HS { float v[3], w[3]; };  // a side's body velocity (or its adjoint)
struct HR { float j[3], W[3], m, bias; };  // a side's angular Jacobian part, W = I^-1 j, and the row's m and bias
struct HQ { float j[3], W[3], m, b; };     // a side's adjoint accumulators of j and W (and, side b, of m and bias)

SHD void hs_load(HS& x, const float* p) {   // p: v(3), w(3), 16-byte aligned
  const f4 q = ld4(p);
  x.v[0] = q.x; x.v[1] = q.y; x.v[2] = q.z; x.w[0] = q.w; x.w[1] = p[4]; x.w[2] = p[5];
}
SHD void hs_store(const HS& x, float* p) {
  f4 q; q.x = x.v[0]; q.y = x.v[1]; q.z = x.v[2]; q.w = x.w[0];
  st4(p, q); p[4] = x.w[1]; p[5] = x.w[2];
}
// Side b's part of a row or row adjoint sits HSIDE floats after side a's, so
// a lane addresses its side as (row + HSIDE * side) + the side-a offset.
constexpr int HSIDE = RJB - RJA;
static_assert(RWB - RWA == HSIDE && QJB - QJA == HSIDE && QWB - QWA == HSIDE, "side layout");
// p: a row + HSIDE * side (side 1: body b, side 0: body a); two 16-byte loads or stores each
SHD void hr_load(HR& r, const float* p) {
  const f4 a = ld4(p + RJA), b = ld4(p + RWA);
  r.j[0] = a.x; r.j[1] = a.y; r.j[2] = a.z; r.m = a.w;
  r.W[0] = b.x; r.W[1] = b.y; r.W[2] = b.z; r.bias = b.w;
}
SHD void hq_load(HQ& q, const float* p) {
  const f4 a = ld4(p + QJA), b = ld4(p + QWA);
  q.j[0] = a.x; q.j[1] = a.y; q.j[2] = a.z; q.m = a.w;
  q.W[0] = b.x; q.W[1] = b.y; q.W[2] = b.z; q.b = b.w;
}
// (side a's slots for m-bar and bias-bar are padding: what is written there is unused)
SHD void hq_store(const HQ& q, float* p) {
  f4 a, b;
  a.x = q.j[0]; a.y = q.j[1]; a.z = q.j[2]; a.w = q.m;
  b.x = q.W[0]; b.y = q.W[1]; b.z = q.W[2]; b.w = q.b;
  st4(p + QJA, a);
  st4(p + QWA, b);
}
// The sides of a visit held by this lane: index i has side sd[i] (1 = b),
// body bd[i], sign sg[i], inverse mass im[i] and signed inverse mass sim[i].
template <int NS>
struct HSides {
  int sd[NS], bd[NS], so[NS];   // so: HSIDE * sd
  float sg[NS], im[NS], sim[NS];
  template <class Team>
  SHD void init(const Team& tm, const Env& E, int a, int b) {
    for (int i = 0; i < NS; ++i) {
      sd[i] = NS == 2 ? 1 - i : (tm.tl & 1);
      bd[i] = sd[i] ? b : a;
      so[i] = HSIDE * sd[i];
      sg[i] = sd[i] ? 1.f : -1.f;
      im[i] = E.body(bd[i])[BIM];
      sim[i] = sg[i] * im[i];
    }
  }
};
// part b + part a: both in this lane, or this lane's part and its partner's
template <int NS, class Team>
SHD float h_sum(const Team& tm, const float* p) {
  if (NS == 2) return p[0] + p[1];
  return p[0] + tm.pair_swap(p[0]);
}
template <int S>
SHD float h_jpart(const HR& r, const HS& x, float sg) {
  float p = S < 3 ? sg * x.v[S] : 0.f;
  p += r.j[0] * x.w[0];
  p += r.j[1] * x.w[1];
  p += r.j[2] * x.w[2];
  return p;
}
template <int S>
SHD void h_apply(const HR& r, HS& x, float sim, float d) {
  if (S < 3) x.v[S] += sim * d;
  for (int k = 0; k < 3; ++k) x.w[k] += d * r.W[k];
}
template <int S, int NS, class Team>
SHD void h_row_fwd(const Team& tm, const DevModel& M, const HR* r, HS* x, const HSides<NS>& sd, float m, float bias,
                   float& lam, float* h, float* rmax) {
  float p[NS];
  for (int i = 0; i < NS; ++i) p[i] = h_jpart<S>(r[i], x[i], sd.sg[i]);
  const float sv_ = h_sum<NS>(tm, p) + bias + M.gamma * lam;
  const float lt = lam - m * sv_;
  if (h) *h = lt;
  if (rmax) *rmax = fmaxf(*rmax, fabsf(lt - lam) / m);
  const float d = lt - lam;
  for (int i = 0; i < NS; ++i) h_apply<S>(r[i], x[i], sd.sim[i], d);
  lam = lt;
}

// A servo's motor row: as h_row_fwd, the impulse clamped to [-hi, hi]
// (the recorded value is the impulse before the clamp).
template <int NS, class Team>
SHD void h_row_box(const Team& tm, const DevModel& M, const HR* r, HS* x, const HSides<NS>& sd, float m, float bias,
                   float hi, float& lam, float* h, float* rmax) {
  float p[NS];
  for (int i = 0; i < NS; ++i) p[i] = h_jpart<3>(r[i], x[i], sd.sg[i]);
  const float sv_ = h_sum<NS>(tm, p) + bias + M.gamma * lam;
  const float lt = lam - m * sv_;
  const float ln = lt <= -hi ? -hi : (lt >= hi ? hi : lt);
  if (h) *h = lt;
  if (rmax) *rmax = fmaxf(*rmax, fabsf(ln - lam) / m);
  const float d = ln - lam;
  for (int i = 0; i < NS; ++i) h_apply<3>(r[i], x[i], sd.sim[i], d);
  lam = ln;
}

// One forward visit of a hinge (5 unbounded rows, then a servo's clamped
// motor row) with all data in
// registers; a: body index or the world slot.  rmax (tolerance mode, NS = 2):
// running maximum of |delta lambda| / m over the rows.
template <int NS, class Team>
SHD void hinge_fwd(const Team& tm, const DevModel& M, const Env& E, int s, int a, int b, float* H,
                   float* rmax = nullptr) {
  HSides<NS> sd;
  sd.init(tm, E, a, b);
  HS x[NS];
  for (int i = 0; i < NS; ++i) hs_load(x[i], E.body(sd.bd[i]) + BV);
  HR r[5][NS];
  float m[5], bias[5], lam[5];
  float* R0 = E.row(s);
  for (int q = 0; q < 5; ++q) {
    for (int i = 0; i < NS; ++i) hr_load(r[q][i], R0 + sd.so[i] + q * RS);
    m[q] = r[q][0].m; bias[q] = r[q][0].bias; lam[q] = R0[q * RS + RL];
  }
  // The rows' impulses are the same in both lanes of a pair (they are formed
  // from the same sums in the same order), so both lanes store them.
  float* Hw = H ? H + s : nullptr;
  h_row_fwd<0, NS>(tm, M, r[0], x, sd, m[0], bias[0], lam[0], Hw ? Hw : nullptr, rmax);
  h_row_fwd<1, NS>(tm, M, r[1], x, sd, m[1], bias[1], lam[1], Hw ? Hw + 1 : nullptr, rmax);
  h_row_fwd<2, NS>(tm, M, r[2], x, sd, m[2], bias[2], lam[2], Hw ? Hw + 2 : nullptr, rmax);
  h_row_fwd<3, NS>(tm, M, r[3], x, sd, m[3], bias[3], lam[3], Hw ? Hw + 3 : nullptr, rmax);
  h_row_fwd<3, NS>(tm, M, r[4], x, sd, m[4], bias[4], lam[4], Hw ? Hw + 4 : nullptr, rmax);
  for (int q = 0; q < 5; ++q) R0[q * RS + RL] = lam[q];
  if (E.jr == 6) {
    const float* R5 = R0 + 5 * RS;
    HR r5[NS];
    for (int i = 0; i < NS; ++i) hr_load(r5[i], R5 + sd.so[i]);
    float l5 = R5[RL];
    h_row_box<NS>(tm, M, r5, x, sd, r5[0].m, r5[0].bias, R5[RHI], l5, Hw ? Hw + 5 : nullptr, rmax);
    R0[5 * RS + RL] = l5;
  }
  for (int i = 0; i < NS; ++i) hs_store(x[i], E.body(sd.bd[i]) + BV);
}

// A hinge's warm start v += W lambda0 over its five rows, by side (see
// hinge_fwd): a lane of a pair updates its own body, one lane alone both, with
// the same arithmetic.  a: body index or the world slot.
template <int NS, class Team>
SHD void hinge_warm(const Team& tm, const Env& E, int s, int a, int b) {
  HSides<NS> sd;
  sd.init(tm, E, a, b);
  const float* R0 = E.row(s);
  for (int i = 0; i < NS; ++i) {
    HS x;
    hs_load(x, E.body(sd.bd[i]) + BV);
    HR r[5];
    for (int q = 0; q < 5; ++q) hr_load(r[q], R0 + sd.so[i] + q * RS);
    h_apply<0>(r[0], x, sd.sim[i], R0[RL0]);
    h_apply<1>(r[1], x, sd.sim[i], R0[RS + RL0]);
    h_apply<2>(r[2], x, sd.sim[i], R0[2 * RS + RL0]);
    h_apply<3>(r[3], x, sd.sim[i], R0[3 * RS + RL0]);
    h_apply<3>(r[4], x, sd.sim[i], R0[4 * RS + RL0]);
    if (E.jr == 6) {
      HR r5;
      hr_load(r5, R0 + 5 * RS + sd.so[i]);
      h_apply<3>(r5, x, sd.sim[i], R0[5 * RS + RL0]);
    }
    hs_store(x, E.body(sd.bd[i]) + BV);
  }
}

// F5: warm start, v += W lambda0 for every row, colour by colour; a hinge
// colour is taken by lane pairs when the team has two lanes, as in the sweeps.
template <class Team>
SHD void f_warm(const Team& tm, const Env& E, bool act) {
  const int nl = n_plan(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    i4 pl{0, 0, 0, 0};
    if (ci < nl) pl = E.plan()[ci];
    const int n = pl.y, lo = pl.x;
    const bool pr = pl.z != 0 && tm.ts >= 2;
    const int k0 = pr ? tm.tl >> 1 : tm.tl, kst = pr ? tm.ts >> 1 : tm.ts;
    for (int k = k0; k < n; k += kst) {
      const i4 v = E.vis()[lo + k];
      const int s = v.x;
      if (s < 0) continue;
      const int code = v.w;
      if (cand_kind(code) == K_JOINT) {
        if (pr) hinge_warm<1>(tm, E, s, v.y, v.z);
        else hinge_warm<2>(tm, E, s, v.y, v.z);
        continue;
      }
      const RowB rb{v.y == E.nb ? -1 : v.y, v.z};
      Vel V;
      vel_load(V, E, rb.a, rb.b);
      const float ima = rb.a >= 0 ? E.body(rb.a)[BIM] : 0.f, imb = E.body(rb.b)[BIM];
      for (int q = 0; q < 3; ++q) {
        const float* r = E.row(s + q);
        row_apply(r, V.va, V.wa, V.vb, V.wb, rb.a >= 0, ima, imb, r[RL0]);
      }
      vel_store(V, E, rb.a, rb.b);
    }
    tm.sync();
  }
}

// One visit of a contact: normal row clamped at 0, then the friction disk.
// HA = false: a ground contact (body a is the world slot), whose body-a terms
// are zeros and are skipped (the same bits: x - 0 + 0 is x).
template <bool HA = true>
SHD void pgs_contact(const DevModel& M, const Env& E, int s, int a, int b, float mu, float* H,
                     float* rmax = nullptr) {
  constexpr bool ha = HA;
  VR V;
  if constexpr (HA) vr_load_ab(V, E, a, b);
  else vr_load_b(V, E, b);
  RR R[3];
  for (int q = 0; q < 3; ++q) rr_load(R[q], E.row(s + q));
  const float mt = E.row(s + 3)[XMT];
  const float ima = HA ? E.body(a)[BIM] : 0.f, imb = E.body(b)[BIM];
  {
    const float sv_ = rr_jv(R[0], V, ha) + R[0].bias + M.gamma * R[0].lam;
    const float lt = R[0].lam - R[0].m * sv_;
    const float ln = lt <= 0.f ? 0.f : lt;
    if (H) H[s] = lt;
    if (rmax) *rmax = fmaxf(*rmax, fabsf(ln - R[0].lam) / R[0].m);
    rr_apply(R[0], V, ha, ima, imb, ln - R[0].lam);
    R[0].lam = ln;
  }
  const float l1 = R[1].lam - mt * rr_jv(R[1], V, ha);
  const float l2 = R[2].lam - mt * rr_jv(R[2], V, ha);
  float n1, n2;
  disk(l1, l2, mu * R[0].lam, n1, n2);
  if (H) { H[s + 1] = l1; H[s + 2] = l2; }
  if (rmax) {
    const float d1 = n1 - R[1].lam, d2 = n2 - R[2].lam;
    *rmax = fmaxf(*rmax, sqrtf(d1 * d1 + d2 * d2) / mt);
  }
  rr_apply(R[1], V, ha, ima, imb, n1 - R[1].lam);
  rr_apply(R[2], V, ha, ima, imb, n2 - R[2].lam);
  E.row(s)[RL] = R[0].lam;
  E.row(s + 1)[RL] = n1;
  E.row(s + 2)[RL] = n2;
  if constexpr (HA) vr_store_ab(V, E, a, b);
  else vr_store_b(V, E, b);
}

// F6: projected Gauss-Seidel sweeps.  With hist, the pre-projection impulse of
// every row update is recorded there, n_iters rows of nslot floats (in LDS or
// global memory).
template <class Team>
SHD void f_pgs(const Team& tm, const DevModel& M, const Env& E, bool act, float* hist) {
  const float mu = E.misc()[MISC_MU];
  SweepCursor<1> sw;
  sw.start(tm, E, M.n_iters, n_plan(E, act));
  while (tm.any(sw.left > 0)) {
    i4 vn, p2;
    sw.prefetch(tm, E, vn, p2);
    float* H = hist ? hist + (size_t)sw.it * E.nslot : nullptr;
    const int nk = sw.count(tm);
    for (int k = 0; k < nk; ++k) {
      const i4 v = sw.entry(tm, E, k);
      if (v.x < 0) continue;
      // a hinge colour is visited by lane pairs whenever the team has two lanes
      if (cand_kind(v.w) != K_JOINT) {
        if (v.y == E.nb) pgs_contact<false>(M, E, v.x, v.y, v.z, mu, H);
        else pgs_contact<true>(M, E, v.x, v.y, v.z, mu, H);
      }
      else if (tm.ts >= 2) hinge_fwd<1>(tm, M, E, v.x, v.y, v.z, H);
      else hinge_fwd<2>(tm, M, E, v.x, v.y, v.z, H);
    }
    tm.sync();
    sw.advance(vn, p2);
  }
}

// F7: semi-implicit Euler and renormalisation of R.
template <class Team>
SHD void f_integrate(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    float* B = E.body(b);
    for (int k = 0; k < 3; ++k) B[BP + k] += M.dt * B[BV + k];
    const float* R = B + BR;
    const float h = M.dt, w0 = B[BW], w1 = B[BW + 1], w2 = B[BW + 2];
    // A = R + dt [w]x R
    float A[9];
    for (int j = 0; j < 3; ++j) {
      const float r0 = R[j], r1 = R[3 + j], r2 = R[6 + j];
      A[j] = r0 + h * (-w2 * r1 + w1 * r2);
      A[3 + j] = r1 + h * (w2 * r0 - w0 * r2);
      A[6 + j] = r2 + h * (-w1 * r0 + w0 * r1);
    }
    // G = A^T A ; N = (3A - A G)/2
    float G[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) G[3 * i + j] = A[i] * A[j] + A[3 + i] * A[3 + j] + A[6 + i] * A[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const float ag = A[3 * i] * G[j] + A[3 * i + 1] * G[3 + j] + A[3 * i + 2] * G[6 + j];
        B[BR + 3 * i + j] = 0.5f * (3.f * A[3 * i + j] - ag);
      }
  }
}

// F8: store impulses for the next warm start.
template <class Team>
SHD void f_store(const Team& tm, const Env& E, bool act) {
  const int nl = n_plan(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    i4 pl{0, 0, 0, 0};
    if (ci < nl) pl = E.plan()[ci];
    const int n = pl.y, lo = pl.x;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const i4 v = E.vis()[lo + k];
      const int s = v.x;
      if (s < 0) continue;
      const int code = v.w;
      float* w = E.ws() + E.store_of(code);
      if (cand_kind(code) == K_JOINT) {
        for (int q = 0; q < E.jr; ++q) w[q] = E.row(s + q)[RL];
      } else {
        const float* x = E.row(s + 3);
        const float l1 = E.row(s + 1)[RL], l2 = E.row(s + 2)[RL];
        w[0] = E.row(s)[RL];
        const f3 Lt = l1 * ld3(x + XT1) + l2 * ld3(x + XT2);
        w[1] = Lt.x; w[2] = Lt.y; w[3] = Lt.z;
      }
    }
  }
  tm.sync();
}

// Joint sensor of the controller: hinge angle (from the perpendicular unit
// vectors of the two frames, about the parent's axis) and hinge rate.
struct Sensor { f3 na, ua, ub, wrel; float y, x; };
SHD Sensor joint_sensor(const Env& E, int j, const float* wa_src, const float* wb_src) {
  const float* C = E.jc(j);
  const int a = E.jpar(j), b = E.jchi(j);
  Sensor S;
  S.na = ld3(C + JXP);
  S.ua = ld3(C + JUP);
  f3 wa = mk3(0.f, 0.f, 0.f);
  if (a >= 0) {
    S.na = mv(E.body(a) + BR, S.na);
    S.ua = mv(E.body(a) + BR, S.ua);
    wa = ld3(wa_src == nullptr ? E.body(a) + BW : wa_src);
  }
  S.ub = mv(E.body(b) + BR, ld3(C + JUC));
  S.wrel = ld3(wb_src == nullptr ? E.body(b) + BW : wb_src) - wa;
  S.y = dot(cross(S.ua, S.ub), S.na);
  S.x = dot(S.ua, S.ub);
  return S;
}

// Controls of step t into the joint records: the tape row, or the
// controller evaluated on x^t (eq. (g) without the recurrent state).
template <class Team>
SHD void f_controls(const Team& tm, const DevModel& M, const Env& E, const float* u_row, bool act, int t = 0) {
  const int nj = act ? E.nj : 0;
  if (!M.ctrl) {
    for (int j = tm.tl; j < nj; j += tm.ts) E.jc(j)[JU] = u_row ? u_row[E.j0 + j] : 0.f;
    return;
  }
  float* sv_ = E.mlp();
  for (int j = tm.tl; j < nj; j += tm.ts) {
    const Sensor S = joint_sensor(E, j, nullptr, nullptr);
    sv_[j] = atan2f(S.y, S.x);
    sv_[E.nj + j] = dot(S.wrel, S.na);
  }
  if (act && tm.tl == 0) {
    sv_[2 * E.nj] = M.clock[2 * t];
    sv_[2 * E.nj + 1] = M.clock[2 * t + 1];
  }
  // the recurrent state h^t
  const int rec = act ? M.mlp_rec : 0;
  for (int i = tm.tl; i < rec; i += tm.ts) sv_[2 * E.nj + 2 + i] = E.ws()[E.lam_imp + i];
  for (int k = M.mlp_in + tm.tl; k < align4(M.mlp_in); k += tm.ts) sv_[k] = 0.f;
  tm.sync();
  // h1 = tanh(W1 s + b1), h2 = tanh(W2 h1 + b2), [u, a] = W3 h2 + b3 for
  // every env of the wave at once (a team whose env is idle gets values it
  // ignores)
  tm.ctrl_forward(M, E);
  const float* u = sv_ + mo_u(M);
  for (int i = tm.tl; i < nj; i += tm.ts) E.jc(i)[JU] = u[i];
  // h^{t+1} = tanh(a) replaces h^t in the carried state (nothing later in the
  // step reads h)
  for (int i = tm.tl; i < rec; i += tm.ts) E.ws()[E.lam_imp + i] = tanhf(u[E.nj + i]);
}

// Loss term of the state after step t (1-based) for the loss body; p is its
// record (position, rotation, velocity, angular velocity).
SHD float loss_term(const DevModel& M, const Env& E, int t1, const float* p, const float* p0) {
  const float* tg = M.target + 3 * E.e;
  if (M.loss_kind == 0) {
    if (t1 != E.T) return 0.f;
    float L = 0.f;
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) { const float d = p[k] - tg[k]; L += d * d; }
    return L;
  }
  if (M.loss_kind == 1) {
    float q = 0.f;
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) { const float d = p[k] - tg[k]; q += d * d; }
    return q > 0.f ? sqrtf(q) / (float)E.T : 0.f;
  }
  if (t1 != E.T) return 0.f;
  if (M.loss_kind == 3) {
    float L = 0.f;
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) { const float d = p[k] - tg[k]; L += d * d; }
    for (int k = BV; k < BW + 3; ++k) L += p[k] * p[k];
    return L;
  }
  return -(p[0] - p0[0]) / ((float)E.T * M.dt);
}

// One full forward step (no recording): x^t (LDS) -> x^{t+1} (LDS).
template <class Team>
SHD void env_step(const Team& tm, const DevModel& M, const Env& E, const float* u_row, bool act, int t = 0) {
  f_controls(tm, M, E, u_row, act, t);
  f_body_setup(tm, E, act, false);
  tm.sync();
  f_torques(tm, E, act);
  f_predict(tm, M, E, act);
  tm.sync();
  if (M.has_rest) f_save_vel(tm, E, act);
  f_rows(tm, M, E, act);
  f_warm(tm, E, act);
  f_pgs(tm, M, E, act, nullptr);
  f_integrate(tm, M, E, act);
  f_store(tm, E, act);
}

// ------------------------------------------------------------------ solve to a tolerance
// Training records of converged contacts (tolerance mode).
struct RecArgs {
  float* rec;                    // [cap][16] or null
  long long cap;
  unsigned long long* count;     // device counter
  int every;                     // steps t with t % every == 0
};

SHD bool is_contact_colour(const Env& E, int c) {
  const int lo = E.colstart(c), hi = E.colstart(c + 1);
  return hi > lo && cand_kind(E.cand(lo)) != K_JOINT;
}

// Warm-start features of every active contact, at the predicted velocities
// and the plain warm-start impulses, into its extras slot: gap / dt, J v of the
// normal and both tangent rows, and the three plain impulses over their
// effective masses.
template <class Team>
SHD void f_features(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nl = n_live(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    const int c = ci < nl ? live_col(E, ci) : 0;
    const bool cc = ci < nl && is_contact_colour(E, c);
    const int n = cc ? E.act_cnt()[c] : 0;
    const int lo = cc ? E.colstart(c) : 0;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const int s = E.act_slot()[lo + k];
      if (s < 0) continue;
      const RowB rb = cand_bodies(E, E.act_code()[lo + k]);
      const bool ha = rb.a >= 0;
      VR V;
      vr_load(V, E, rb.a, rb.b);
      RR R0, R1, R2;
      rr_load(R0, E.row(s));
      rr_load(R1, E.row(s + 1));
      rr_load(R2, E.row(s + 2));
      float* x = E.row(s + 3);
      const float mt = x[XMT];
      x[XF + 0] = x[XGAP] / M.dt;
      x[XF + 1] = rr_jv(R0, V, ha);
      x[XF + 2] = rr_jv(R1, V, ha);
      x[XF + 3] = rr_jv(R2, V, ha);
      x[XF + 4] = E.row(s)[RL0] / R0.m;
      x[XF + 5] = E.row(s + 1)[RL0] / mt;
      x[XF + 6] = E.row(s + 2)[RL0] / mt;
    }
  }
  tm.sync();
}

// Predicted velocities, kept for a restart from the plain warm start and for
// the adjoint of restitution.
template <class Team>
SHD void f_save_vel(const Team& tm, const Env& E, bool act) {
  if (act)
    for (int b = tm.tl; b < E.nb; b += tm.ts)
      for (int k = 0; k < 6; ++k) E.vsave(b)[k] = E.body(b)[BV + k];
}

// Learned warm start: the network on the features of every contact of the
// wave (matrix cores, 16 contacts per tile); its outputs correct the carried
// impulses (in velocity units: impulse over effective mass), and the result,
// projected onto lambda_n >= 0, |lambda_t| <= mu lambda_n, replaces the
// contacts' warm-start impulses.
// Contacts placed in row slots (team-uniform): the first ccap active contacts
// in colour-major order; any beyond the capacity were dropped and flagged.
SHD int placed_contacts(const Env& E, bool act) {
  int n = 0;
  for (int c = 0; c < E.ncol && act; ++c)
    if (is_contact_colour(E, c)) n += E.act_cnt()[c];
  return n < E.ccap ? n : E.ccap;
}

template <class Team>
SHD void f_learned_ws(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int n_e = placed_contacts(E, act);
  int* cnt = tm.shared_cnt();
  int* map = tm.shared_map();
  if (tm.tl == 0) cnt[tm.team] = act ? n_e : 0;
  tm.sync();
  int base = 0, total = 0;
  for (int q = 0; q < tm.n_teams; ++q) {
    const int v = cnt[q];
    if (q < tm.team) base += v;
    total += v;
  }
  int idx = base;
  const int nl = n_live(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    const int c = ci < nl ? live_col(E, ci) : 0;
    const bool cc = ci < nl && is_contact_colour(E, c);
    const int n = cc ? E.act_cnt()[c] : 0;
    const int lo = cc ? E.colstart(c) : 0;
    for (int k = tm.tl; k < n; k += tm.ts)
      if (idx + k < base + n_e) map[idx + k] = (int)(E.row(E.act_slot()[lo + k] + 3) - tm.lds0);
    idx += n;
  }
  tm.sync();
  tm.wsn_rows(total, map);
  tm.sync();
  const float mu = E.misc()[MISC_MU];
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    const int c = ci < nl ? live_col(E, ci) : 0;
    const bool cc = ci < nl && is_contact_colour(E, c);
    const int n = cc ? E.act_cnt()[c] : 0;
    const int lo = cc ? E.colstart(c) : 0;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const int s = E.act_slot()[lo + k];
      if (s < 0) continue;
      // outputs: corrections to the carried impulses over their effective masses
      const float* x = E.row(s + 3);
      const float ln = fmaxf(E.row(s)[RM] * (x[XF + 4] + x[XY]), 0.f);
      float l1 = x[XMT] * (x[XF + 5] + x[XY + 1]), l2 = x[XMT] * (x[XF + 6] + x[XY + 2]);
      const float rho = mu * ln, nrm = sqrtf(l1 * l1 + l2 * l2);
      if (!(nrm <= rho)) { l1 *= rho / nrm; l2 *= rho / nrm; }
      E.row(s)[RL] = E.row(s)[RL0] = ln;
      E.row(s + 1)[RL] = E.row(s + 1)[RL0] = l1;
      E.row(s + 2)[RL] = E.row(s + 2)[RL0] = l2;
    }
  }
  tm.sync();
}

// Restart from the plain warm start: predicted velocities back, every row's
// impulse back to the carried one (joints never changed theirs).
template <class Team>
SHD void f_restart(const Team& tm, const DevModel& M, const Env& E, bool act) {
  if (act)
    for (int b = tm.tl; b < E.nb; b += tm.ts)
      for (int k = 0; k < 6; ++k) E.body(b)[BV + k] = E.vsave(b)[k];
  const int nl = n_live(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    const int c = ci < nl ? live_col(E, ci) : 0;
    const int n = ci < nl ? E.act_cnt()[c] : 0;
    const int lo = ci < nl ? E.colstart(c) : 0;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const int s = E.act_slot()[lo + k];
      if (s < 0) continue;
      if (cand_kind(E.act_code()[lo + k]) == K_JOINT) {
        for (int q = 0; q < E.jr; ++q) E.row(s + q)[RL] = E.row(s + q)[RL0];
      } else {
        const float* x = E.row(s + 3);
        const float* w = E.ws() + *reinterpret_cast<const int*>(x + XSTORE);
        const f3 Lt = mk3(w[1], w[2], w[3]);
        E.row(s)[RL] = E.row(s)[RL0] = M.warm * w[0];
        E.row(s + 1)[RL] = E.row(s + 1)[RL0] = M.warm * dot(ld3(x + XT1), Lt);
        E.row(s + 2)[RL] = E.row(s + 2)[RL0] = M.warm * dot(ld3(x + XT2), Lt);
      }
    }
  }
  tm.sync();
}

// Sweeps until the residual (largest |delta lambda| / m of a sweep) is at most
// tol or `limit` sweeps have run; it / res carry the count and the last
// residual, res_c (if given) the last residual of the contact rows alone
// (team-uniform).
template <class Team>
SHD void f_pgs_tol(const Team& tm, const DevModel& M, const Env& E, bool live, int& it, float& res, int limit,
                   float* res_c = nullptr) {
  const float mu = E.misc()[MISC_MU];
  for (;;) {
    const bool run = live && res > M.tol && it < limit;
    if (!tm.any(run)) break;
    float r = 0.f, rc = 0.f;
    const int nl = n_live(E, run);
    for (int ci = 0; tm.any(ci < nl); ++ci) {
      const int c = ci < nl ? live_col(E, ci) : 0;
      const int n = ci < nl ? E.act_cnt()[c] : 0;
      const int lo = ci < nl ? E.colstart(c) : 0;
      for (int k = tm.tl; k < n; k += tm.ts) {
        const int s = E.act_slot()[lo + k];
        if (s < 0) continue;
        const int code = E.act_code()[lo + k];
        const RowB rb = cand_bodies(E, code);
        const int a = rb.a >= 0 ? rb.a : E.nb;
        if (cand_kind(code) == K_JOINT) hinge_fwd<2>(tm, M, E, s, a, rb.b, nullptr, &r);
        else pgs_contact(M, E, s, a, rb.b, mu, nullptr, &rc);
      }
      tm.sync();
    }
    if (run) {
      res = tm.team_max(fmaxf(r, rc));
      if (res_c) *res_c = tm.team_max(rc);
      ++it;
    }
  }
}

// One record per active contact of a converged step: features, converged
// impulses over their effective masses, m_n, m_t, env, step, code (the last
// three as int32 bit patterns).
template <class Team>
SHD void f_records(const Team& tm, const DevModel& M, const Env& E, bool act, int t, const RecArgs& ra) {
  const int n_e = placed_contacts(E, act);
  const unsigned long long base = tm.reserve(ra.count, act ? n_e : 0);
  long long idx = (long long)base;
  const int nl = n_live(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    const int c = ci < nl ? live_col(E, ci) : 0;
    const bool cc = ci < nl && is_contact_colour(E, c);
    const int n = cc ? E.act_cnt()[c] : 0;
    const int lo = cc ? E.colstart(c) : 0;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const int s = E.act_slot()[lo + k];
      const long long i = idx + k;
      if (s < 0 || i >= ra.cap) continue;
      const float* x = E.row(s + 3);
      const float mn = E.row(s)[RM], mt = x[XMT];
      float* o = ra.rec + (size_t)i * 16;
      for (int q = 0; q < 7; ++q) o[q] = x[XF + q];
      o[7] = E.row(s)[RL] / mn;
      o[8] = E.row(s + 1)[RL] / mt;
      o[9] = E.row(s + 2)[RL] / mt;
      o[10] = mn;
      o[11] = mt;
      *reinterpret_cast<int*>(o + 12) = E.e;
      *reinterpret_cast<int*>(o + 13) = t;
      *reinterpret_cast<int*>(o + 14) = E.act_code()[lo + k];
      o[15] = 0.f;
    }
    idx += n;
  }
}

// One forward step solved to the residual tolerance, with the plain or the
// learned warm start (and its fallback); counts sweeps and fallbacks in the
// env's misc slots and writes training records when asked.
template <class Team>
SHD void env_step_solve(const Team& tm, const DevModel& M, const Env& E, const float* u_row, bool act, int t,
                        const RecArgs* ra) {
  f_controls(tm, M, E, u_row, act, t);
  f_body_setup(tm, E, act, false);
  tm.sync();
  f_torques(tm, E, act);
  f_predict(tm, M, E, act);
  tm.sync();
  if (M.ws_kind || M.has_rest) f_save_vel(tm, E, act);
  f_rows(tm, M, E, act);
  const bool rec = ra && ra->rec && ra->every > 0 && t % ra->every == 0;
  if (M.ws_kind || rec) f_features(tm, M, E, act);
  if (M.ws_kind) f_learned_ws(tm, M, E, act);
  f_warm(tm, E, act);
  int nrows = 0;
  for (int c = 0; c < E.ncol && act; ++c) nrows += E.act_cnt()[c];
  const bool live = act && nrows > 0;
  int it = 0, wasted = 0, fb = 0;
  float res = 3.0e38f;
  if (M.ws_kind) {
    // the test of the learned start looks at the rows it started: the contacts
    float res_c = 3.0e38f;
    f_pgs_tol(tm, M, E, live, it, res, M.fb_iters, &res_c);
    const bool rej = live && res > M.tol && (it > 0 ? res_c : 3.0e38f) > M.fb_tol;
    if (tm.any(rej)) {
      f_restart(tm, M, E, rej);
      f_warm(tm, E, rej);
      if (rej) {
        wasted = it;
        fb = 1;
        it = 0;
        res = 3.0e38f;
      }
    }
  }
  f_pgs_tol(tm, M, E, live, it, res, M.max_iters);
  if (act && tm.tl == 0) {
    *reinterpret_cast<int*>(E.misc() + MISC_ITERS) += it + wasted;
    *reinterpret_cast<int*>(E.misc() + MISC_FB) += fb;
  }
  if (tm.any(rec && live && res <= M.tol)) f_records(tm, M, E, rec && live && res <= M.tol, t, *ra);
  f_integrate(tm, M, E, act);
  f_store(tm, E, act);
}

// ------------------------------------------------------------------ adjoint
// Adjoint of the linear part of W = M^-1 J^T folded at accumulation time:
// W_lin_a = -invm_a Jl, W_lin_b = invm_b Jl.
struct VelA {
  float va[3], wa[3], vb[3], wb[3];
};
SHD void vela_load(VelA& V, const Env& E, int a, int b) {
  const float* Bb = E.bodyA(b);
  for (int k = 0; k < 3; ++k) { V.vb[k] = Bb[AV + k]; V.wb[k] = Bb[AW + k]; }
  if (a >= 0) {
    const float* Ba = E.bodyA(a);
    for (int k = 0; k < 3; ++k) { V.va[k] = Ba[AV + k]; V.wa[k] = Ba[AW + k]; }
  } else {
    for (int k = 0; k < 3; ++k) { V.va[k] = 0.f; V.wa[k] = 0.f; }
  }
}
SHD void vela_store(const VelA& V, const Env& E, int a, int b) {
  float* Bb = E.bodyA(b);
  for (int k = 0; k < 3; ++k) { Bb[AV + k] = V.vb[k]; Bb[AW + k] = V.wb[k]; }
  if (a >= 0) {
    float* Ba = E.bodyA(a);
    for (int k = 0; k < 3; ++k) { Ba[AV + k] = V.va[k]; Ba[AW + k] = V.wa[k]; }
  }
}
// W . vbar (the adjoint seen through v += W d)
SHD float row_wvbar(const float* r, const VelA& A, bool ha, float ima, float imb) {
  float s = imb * (r[RJL] * A.vb[0] + r[RJL + 1] * A.vb[1] + r[RJL + 2] * A.vb[2]);
  s += r[RWB] * A.wb[0] + r[RWB + 1] * A.wb[1] + r[RWB + 2] * A.wb[2];
  if (ha) {
    s -= ima * (r[RJL] * A.va[0] + r[RJL + 1] * A.va[1] + r[RJL + 2] * A.va[2]);
    s += r[RWA] * A.wa[0] + r[RWA + 1] * A.wa[1] + r[RWA + 2] * A.wa[2];
  }
  return s;
}
// accumulate the adjoint of W from v += W d (given vbar after the update)
SHD void row_wbar(float* q, const float* r, const VelA& A, bool ha, float ima, float imb, float d,
                  float* imbar_a, float* imbar_b) {
  // angular parts
  q[QWB] += A.wb[0] * d; q[QWB + 1] += A.wb[1] * d; q[QWB + 2] += A.wb[2] * d;
  // linear parts: W_lin_b = imb Jl
  q[QJL] += imb * A.vb[0] * d; q[QJL + 1] += imb * A.vb[1] * d; q[QJL + 2] += imb * A.vb[2] * d;
  *imbar_b += d * (r[RJL] * A.vb[0] + r[RJL + 1] * A.vb[1] + r[RJL + 2] * A.vb[2]);
  if (ha) {
    q[QWA] += A.wa[0] * d; q[QWA + 1] += A.wa[1] * d; q[QWA + 2] += A.wa[2] * d;
    q[QJL] -= ima * A.va[0] * d; q[QJL + 1] -= ima * A.va[1] * d; q[QJL + 2] -= ima * A.va[2] * d;
    *imbar_a -= d * (r[RJL] * A.va[0] + r[RJL + 1] * A.va[1] + r[RJL + 2] * A.va[2]);
  }
}
// vbar += J^T sb ; Jbar += sb v
SHD void row_jbar(float* q, const float* r, VelA& A, const Vel& V, bool ha, float sb) {
  for (int k = 0; k < 3; ++k) {
    A.vb[k] += r[RJL + k] * sb;
    A.wb[k] += r[RJB + k] * sb;
    q[QJL + k] += sb * V.vb[k];
    q[QJB + k] += sb * V.wb[k];
    if (ha) {
      A.va[k] -= r[RJL + k] * sb;
      A.wa[k] += r[RJA + k] * sb;
      q[QJL + k] -= sb * V.va[k];
      q[QJA + k] += sb * V.wa[k];
    }
  }
}
// undo v += W d
SHD void row_unapply(const float* r, Vel& V, bool ha, float ima, float imb, float d) {
  row_apply(r, V.va, V.wa, V.vb, V.wb, ha, ima, imb, -d);
}

// Clear the per-step adjoint accumulators (rows, body extras).
template <class Team>
SHD void a_clear_step(const Team& tm, const Env& E, bool act) {
  // row adjoints and the world slot's adjoint with 16-byte stores (both
  // regions start on a float4 boundary and span whole float4)
  static_assert(RSA % 4 == 0 && BSA % 4 == 0, "float4 spans");
  const f4 z{0.f, 0.f, 0.f, 0.f};
  const int ns4 = act ? E.nslot * (RSA / 4) : 0;
  for (int i = tm.tl; i < ns4; i += tm.ts) st4(E.rowA(0) + 4 * i, z);
  // hist(-1) = the start impulses, so that in the reversed sweeps a hinge
  // row's impulse before its update is the previous sweep's record in every
  // sweep, the first included
  // (a ring takes them when it is filled)
  const int nsl = act && !E.lay.hring ? E.nslot : 0;
  for (int s = tm.tl; s < nsl; s += tm.ts) E.hist(-1)[s] = E.row(s)[RL0];
  // the world slot's adjoint is a sink of the sweeps: cleared every step so
  // that it stays finite (it only ever meets zero inverse masses)
  const int nw4 = act ? BSA / 4 : 0;
  for (int i = tm.tl; i < nw4; i += tm.ts) st4(E.bodyA(E.nb) + 4 * i, z);
  // per body: the inverse-inertia, inverse-mass and torque adjoints, floats
  // AIW .. ATQ + 2, one 8-byte, three 16-byte and one 8-byte store
  static_assert(AIW % 4 == 2 && AIM == AIW + 9 && AII == AIM + 1 && ATQ == AII + 3, "body adjoint layout");
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    float* A = E.bodyA(b);
    st2(A + AIW, f2{0.f, 0.f});
    st4(A + AIW + 2, z);
    st4(A + AIW + 6, z);
    st4(A + AIW + 10, z);
    st2(A + AIW + 14, f2{0.f, 0.f});
  }
}

// Gradient decay (section 3.2): the adjoints carried back from the later
// steps, the state's and the carried impulses', shrink by M.decay.
template <class Team>
SHD void a_decay(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nb = act ? E.nb : 0;
  for (int i = tm.tl; i < 18 * nb; i += tm.ts) E.bodyA(i / 18)[AP + i % 18] *= M.decay;
  const int nl = act ? E.lam_size : 0;
  for (int i = tm.tl; i < nl; i += tm.ts) E.wsA()[i] *= M.decay;
}

// B8: adjoint of the impulse store; lambda bar of each active row starts from
// the stored output's adjoint.  Inactive candidates' stored outputs were
// constants (zeros): their adjoint is dropped here.
template <class Team>
SHD void a_store(const Team& tm, const Env& E, bool act) {
  const int nl = n_plan(E, act);
  for (int ci = 0; tm.any(ci < nl); ++ci) {
    i4 pl{0, 0, 0, 0};
    if (ci < nl) pl = E.plan()[ci];
    const int n = pl.y, lo = pl.x;
    for (int k = tm.tl; k < n; k += tm.ts) {
      const i4 v = E.vis()[lo + k];
      const int s = v.x;
      if (s < 0) continue;
      const int code = v.w;
      float* wA = E.wsA() + E.store_of(code);
      if (cand_kind(code) == K_JOINT) {
        for (int q = 0; q < E.jr; ++q) E.rowA(s + q)[QL] = wA[q];
      } else {
        const float* x = E.row(s + 3);
        float* xa = E.rowA(s + 3);
        const f3 Lb = mk3(wA[1], wA[2], wA[3]);
        const f3 t1 = ld3(x + XT1), t2 = ld3(x + XT2);
        const float l1 = E.row(s + 1)[RL], l2 = E.row(s + 2)[RL];
        E.rowA(s)[QL] = wA[0];
        E.rowA(s + 1)[QL] = dot(t1, Lb);
        E.rowA(s + 2)[QL] = dot(t2, Lb);
        add3(xa + XT1, l1 * Lb);
        add3(xa + XT2, l2 * Lb);
      }
    }
  }
  tm.sync();
  // the adjoint of the incoming store is rebuilt by the warm-start reverse
  // (the recurrent state's adjoint, after the impulses', stays: it is the
  // carry of the controller's reverse)
  const int nls = act ? E.lam_imp : 0;
  for (int i = tm.tl; i < nls; i += tm.ts) E.wsA()[i] = 0.f;
  tm.sync();
}

// B7: adjoint of integration and renormalisation (per body); leaves
// vbar, wbar of the post-sweep velocities and pbar, Rbar of x^t.
template <class Team>
SHD void a_integrate(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    float* B = E.body(b);
    float* A = E.bodyA(b);
    const float h = M.dt;
    for (int k = 0; k < 3; ++k) A[AV + k] += h * A[AP + k];   // p' = p + h v'
    const float* R = B + BR;
    const float w0 = B[BW], w1 = B[BW + 1], w2 = B[BW + 2];
    float Am[9];
    for (int j = 0; j < 3; ++j) {
      const float r0 = R[j], r1 = R[3 + j], r2 = R[6 + j];
      Am[j] = r0 + h * (-w2 * r1 + w1 * r2);
      Am[3 + j] = r1 + h * (w2 * r0 - w0 * r2);
      Am[6 + j] = r2 + h * (-w1 * r0 + w0 * r1);
    }
    float Nb[9];
    for (int k = 0; k < 9; ++k) Nb[k] = A[AR + k];
    // Abar = 1.5 Nb - 0.5 (Nb A^T A + A Nb^T A + A A^T Nb)
    float AtA[9], AAt[9], NtA[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        AtA[3 * i + j] = Am[i] * Am[j] + Am[3 + i] * Am[3 + j] + Am[6 + i] * Am[6 + j];
        AAt[3 * i + j] = Am[3 * i] * Am[3 * j] + Am[3 * i + 1] * Am[3 * j + 1] + Am[3 * i + 2] * Am[3 * j + 2];
        NtA[3 * i + j] = Nb[i] * Am[j] + Nb[3 + i] * Am[3 + j] + Nb[6 + i] * Am[6 + j];   // Nb^T A
      }
    float Ab[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float t1 = 0.f, t2 = 0.f, t3 = 0.f;
        for (int k = 0; k < 3; ++k) {
          t1 += Nb[3 * i + k] * AtA[3 * k + j];
          t2 += Am[3 * i + k] * NtA[3 * k + j];
          t3 += AAt[3 * i + k] * Nb[3 * k + j];
        }
        Ab[3 * i + j] = 1.5f * Nb[3 * i + j] - 0.5f * (t1 + t2 + t3);
      }
    // A = R + h S(w) R : Rbar = Abar - h S(w) Abar ; wbar += h * d<Abar, S R>/dw
    float Mx[9];   // Abar R^T
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Mx[3 * i + j] = Ab[3 * i] * R[3 * j] + Ab[3 * i + 1] * R[3 * j + 1] + Ab[3 * i + 2] * R[3 * j + 2];
    A[AW] += h * (Mx[7] - Mx[5]);
    A[AW + 1] += h * (Mx[2] - Mx[6]);
    A[AW + 2] += h * (Mx[3] - Mx[1]);
    for (int j = 0; j < 3; ++j) {
      const float a0 = Ab[j], a1 = Ab[3 + j], a2 = Ab[6 + j];
      A[AR + j] = a0 - h * (-w2 * a1 + w1 * a2);
      A[AR + 3 + j] = a1 - h * (w2 * a0 - w0 * a2);
      A[AR + 6 + j] = a2 - h * (-w1 * a0 + w0 * a1);
    }
  }
  tm.sync();
}

// Row adjoint accumulators in registers (layout of a row adjoint slot).
struct QR { float jl[3], ja[3], jb[3], wa[3], wb[3], m, b, l; };
SHD void qr_load(QR& Q, const float* p) {
  const f4 a = ld4(p + QJA), b = ld4(p + QWA), c = ld4(p + QJB), d = ld4(p + QWB), e = ld4(p + QJL);
  Q.ja[0] = a.x; Q.ja[1] = a.y; Q.ja[2] = a.z;
  Q.wa[0] = b.x; Q.wa[1] = b.y; Q.wa[2] = b.z;
  Q.jb[0] = c.x; Q.jb[1] = c.y; Q.jb[2] = c.z; Q.m = c.w;
  Q.wb[0] = d.x; Q.wb[1] = d.y; Q.wb[2] = d.z; Q.b = d.w;
  Q.jl[0] = e.x; Q.jl[1] = e.y; Q.jl[2] = e.z; Q.l = e.w;
}
SHD void qr_store(const QR& Q, float* p) {
  f4 a, b, c, d, e;
  a.x = Q.ja[0]; a.y = Q.ja[1]; a.z = Q.ja[2]; a.w = 0.f;
  b.x = Q.wa[0]; b.y = Q.wa[1]; b.z = Q.wa[2]; b.w = 0.f;
  c.x = Q.jb[0]; c.y = Q.jb[1]; c.z = Q.jb[2]; c.w = Q.m;
  d.x = Q.wb[0]; d.y = Q.wb[1]; d.z = Q.wb[2]; d.w = Q.b;
  e.x = Q.jl[0]; e.y = Q.jl[1]; e.z = Q.jl[2]; e.w = Q.l;
  st4(p + QJA, a); st4(p + QWA, b); st4(p + QJB, c); st4(p + QWB, d); st4(p + QJL, e);
}
SHD void vra_load(VR& A, const Env& E, int a, int b) {
  const float* Bb = E.bodyA(b) + AV;   // vbar(3), wbar(3) contiguous, 16-byte aligned
  const f4 q0 = ld4(Bb);
  A.vb[0] = q0.x; A.vb[1] = q0.y; A.vb[2] = q0.z; A.wb[0] = q0.w; A.wb[1] = Bb[4]; A.wb[2] = Bb[5];
  if (a >= 0) {
    const float* Ba = E.bodyA(a) + AV;
    const f4 p0 = ld4(Ba);
    A.va[0] = p0.x; A.va[1] = p0.y; A.va[2] = p0.z; A.wa[0] = p0.w; A.wa[1] = Ba[4]; A.wa[2] = Ba[5];
  } else {
    for (int k = 0; k < 3; ++k) { A.va[k] = 0.f; A.wa[k] = 0.f; }
  }
}
SHD void vra_load_ab(VR& A, const Env& E, int a, int b) {
  const float* Bb = E.bodyA(b) + AV;
  const float* Ba = E.bodyA(a) + AV;
  const f4 q0 = ld4(Bb), p0 = ld4(Ba);
  A.vb[0] = q0.x; A.vb[1] = q0.y; A.vb[2] = q0.z; A.wb[0] = q0.w; A.wb[1] = Bb[4]; A.wb[2] = Bb[5];
  A.va[0] = p0.x; A.va[1] = p0.y; A.va[2] = p0.z; A.wa[0] = p0.w; A.wa[1] = Ba[4]; A.wa[2] = Ba[5];
}
SHD void vra_load_b(VR& A, const Env& E, int b) {
  const float* Bb = E.bodyA(b) + AV;
  const f4 q0 = ld4(Bb);
  A.vb[0] = q0.x; A.vb[1] = q0.y; A.vb[2] = q0.z; A.wb[0] = q0.w; A.wb[1] = Bb[4]; A.wb[2] = Bb[5];
  for (int k = 0; k < 3; ++k) { A.va[k] = 0.f; A.wa[k] = 0.f; }
}
SHD void vra_store_b(const VR& A, const Env& E, int b) {
  float* Bb = E.bodyA(b) + AV;
  f4 q0; q0.x = A.vb[0]; q0.y = A.vb[1]; q0.z = A.vb[2]; q0.w = A.wb[0];
  st4(Bb, q0); Bb[4] = A.wb[1]; Bb[5] = A.wb[2];
}
SHD void vra_store_ab(const VR& A, const Env& E, int a, int b) {
  float* Bb = E.bodyA(b) + AV;
  float* Ba = E.bodyA(a) + AV;
  f4 q0; q0.x = A.vb[0]; q0.y = A.vb[1]; q0.z = A.vb[2]; q0.w = A.wb[0];
  f4 p0; p0.x = A.va[0]; p0.y = A.va[1]; p0.z = A.va[2]; p0.w = A.wa[0];
  st4(Bb, q0); Bb[4] = A.wb[1]; Bb[5] = A.wb[2];
  st4(Ba, p0); Ba[4] = A.wa[1]; Ba[5] = A.wa[2];
}
SHD void vra_store(const VR& A, const Env& E, int a, int b) {
  float* Bb = E.bodyA(b) + AV;
  f4 q0; q0.x = A.vb[0]; q0.y = A.vb[1]; q0.z = A.vb[2]; q0.w = A.wb[0];
  st4(Bb, q0); Bb[4] = A.wb[1]; Bb[5] = A.wb[2];
  if (a >= 0) {
    float* Ba = E.bodyA(a) + AV;
    f4 p0; p0.x = A.va[0]; p0.y = A.va[1]; p0.z = A.va[2]; p0.w = A.wa[0];
    st4(Ba, p0); Ba[4] = A.wa[1]; Ba[5] = A.wa[2];
  }
}
// W . vbar through v += W d
SHD float rr_wv(const RR& R, const VR& A, bool ha, float ima, float imb) {
  float s = imb * (R.jl[0] * A.vb[0] + R.jl[1] * A.vb[1] + R.jl[2] * A.vb[2]);
  s += R.wb[0] * A.wb[0] + R.wb[1] * A.wb[1] + R.wb[2] * A.wb[2];
  if (ha) {
    s -= ima * (R.jl[0] * A.va[0] + R.jl[1] * A.va[1] + R.jl[2] * A.va[2]);
    s += R.wa[0] * A.wa[0] + R.wa[1] * A.wa[1] + R.wa[2] * A.wa[2];
  }
  return s;
}
// adjoint of W from v += W d (linear parts folded into Jl and the inverse masses)
SHD void rr_wbar(QR& Q, const RR& R, const VR& A, bool ha, float ima, float imb, float d, float& imA, float& imB) {
  for (int k = 0; k < 3; ++k) { Q.wb[k] += A.wb[k] * d; Q.jl[k] += imb * A.vb[k] * d; }
  imB += d * (R.jl[0] * A.vb[0] + R.jl[1] * A.vb[1] + R.jl[2] * A.vb[2]);
  if (ha) {
    for (int k = 0; k < 3; ++k) { Q.wa[k] += A.wa[k] * d; Q.jl[k] -= ima * A.va[k] * d; }
    imA -= d * (R.jl[0] * A.va[0] + R.jl[1] * A.va[1] + R.jl[2] * A.va[2]);
  }
}
// vbar += J^T sb ; Jbar += sb v
SHD void rr_jbar(QR& Q, const RR& R, VR& A, const VR& V, bool ha, float sb) {
  for (int k = 0; k < 3; ++k) {
    A.vb[k] += R.jl[k] * sb;
    A.wb[k] += R.jb[k] * sb;
    Q.jl[k] += sb * V.vb[k];
    Q.jb[k] += sb * V.wb[k];
  }
  if (ha)
    for (int k = 0; k < 3; ++k) {
      A.va[k] -= R.jl[k] * sb;
      A.wa[k] += R.ja[k] * sb;
      Q.jl[k] -= sb * V.va[k];
      Q.ja[k] += sb * V.wa[k];
    }
}
// Reverse of one scalar row update; lt is the recorded pre-projection
// impulse, lp the impulse before the update, unbounded for hinge rows.
SHD void rev_scalar(const RR& R, QR& Q, VR& V, VR& A, bool ha, float ima, float imb, float lt, float lp,
                    bool unbounded, float gamma, float& imA, float& imB) {
  const float ln = unbounded ? lt : fmaxf(lt, 0.f);
  const float d = ln - lp;
  rr_apply(R, V, ha, ima, imb, -d);   // v before the update
  rr_wbar(Q, R, A, ha, ima, imb, d, imA, imB);
  const float wv = rr_wv(R, A, ha, ima, imb);
  const float g = Q.l + wv;
  const float ltb = (unbounded || lt > 0.f) ? g : 0.f;
  const float sb = -R.m * ltb;
  const float sval = rr_jv(R, V, ha) + R.bias + gamma * lp;
  Q.m += -sval * ltb;
  Q.b += sb;
  rr_jbar(Q, R, A, V, ha, sb);
  Q.l = -wv + ltb + gamma * sb;
}

// Reverse of one hinge row update, by side (see hinge_fwd).
template <int S>
SHD float h_wpart(const HR& r, const HS& A, float sim) {
  float p = S < 3 ? sim * A.v[S] : 0.f;
  p += r.W[0] * A.w[0];
  p += r.W[1] * A.w[1];
  p += r.W[2] * A.w[2];
  return p;
}
// Row-shared data of one hinge row in the reverse: mass, bias, recorded
// pre-projection impulse lt and the impulse before the update lp, and the
// adjoint accumulators of m, bias and lambda.
struct HRow { float m, bias, lt, lp, qm, qb, ql; };
template <int S, int NS, class Team>
SHD void h_row_rev(const Team& tm, const HR* r, HQ* q, HS* x, HS* A, const HSides<NS>& sd, float* imx, HRow& c,
                   float gamma) {
  const float d = c.lt - c.lp;
  for (int i = 0; i < NS; ++i) h_apply<S>(r[i], x[i], sd.sim[i], -d);   // v before the update
  // adjoint of W from v += W d (the linear part folded into the inverse masses)
  for (int i = 0; i < NS; ++i) {
    for (int k = 0; k < 3; ++k) q[i].W[k] += A[i].w[k] * d;
    if (S < 3) imx[i] += (sd.sg[i] * d) * A[i].v[S];
  }
  float p[NS];
  for (int i = 0; i < NS; ++i) p[i] = h_wpart<S>(r[i], A[i], sd.sim[i]);
  const float wv = h_sum<NS>(tm, p);
  const float ltb = c.ql + wv;
  const float sb = -c.m * ltb;
  for (int i = 0; i < NS; ++i) p[i] = h_jpart<S>(r[i], x[i], sd.sg[i]);
  const float sval = h_sum<NS>(tm, p) + c.bias + gamma * c.lp;
  c.qm += -sval * ltb;
  c.qb += sb;
  // vbar += J^T sb ; Jbar += sb v
  for (int i = 0; i < NS; ++i) {
    if (S < 3) A[i].v[S] += sd.sg[i] * sb;
    for (int k = 0; k < 3; ++k) {
      A[i].w[k] += r[i].j[k] * sb;
      q[i].j[k] += sb * x[i].w[k];
    }
  }
  c.ql = -wv + ltb + gamma * sb;
}
// Row q of a visit whose first row is at R0 / Q0 (row slots and adjoint
// slots) and whose records start at H and Hp.
template <int NS>
SHD void h_rev_load(const HSides<NS>& sd, const float* R0, const float* Q0, int q, const float* H, const float* Hp,
                    HR* r, HQ* qa, HRow& c) {
  const float* R = R0 + q * RS;
  const float* Q = Q0 + q * RSA;
  for (int i = 0; i < NS; ++i) {
    hr_load(r[i], R + sd.so[i]);
    hq_load(qa[i], Q + sd.so[i]);
  }
  // m and bias from this lane's part; the m and bias adjoints are side b's
  // (index 0 is side b in a one-lane visit; a lane of a pair that holds side a
  // computes nothing from them)
  c.m = r[0].m; c.bias = r[0].bias;
  c.qm = qa[0].m; c.qb = qa[0].b; c.ql = Q[QL];
  c.lt = H[q];
  c.lp = Hp[q];
}

// Reverse of a servo's motor row update (see h_row_box): c.lp is the impulse
// before the update, c.lt the recorded one before the clamp; the adjoint
// passes the clamp only strictly inside the bounds.
template <int NS, class Team>
SHD void h_row_rev_box(const Team& tm, const HR* r, HQ* q, HS* x, HS* A, const HSides<NS>& sd, HRow& c, float gamma,
                       float hi) {
  const float ln = c.lt <= -hi ? -hi : (c.lt >= hi ? hi : c.lt);
  const float d = ln - c.lp;
  for (int i = 0; i < NS; ++i) h_apply<3>(r[i], x[i], sd.sim[i], -d);   // v before the update
  for (int i = 0; i < NS; ++i)
    for (int k = 0; k < 3; ++k) q[i].W[k] += A[i].w[k] * d;
  float p[NS];
  for (int i = 0; i < NS; ++i) p[i] = h_wpart<3>(r[i], A[i], sd.sim[i]);
  const float wv = h_sum<NS>(tm, p);
  const float g = c.ql + wv;
  const float ltb = (c.lt > -hi && c.lt < hi) ? g : 0.f;
  const float sb = -c.m * ltb;
  for (int i = 0; i < NS; ++i) p[i] = h_jpart<3>(r[i], x[i], sd.sg[i]);
  const float sval = h_sum<NS>(tm, p) + c.bias + gamma * c.lp;
  c.qm += -sval * ltb;
  c.qb += sb;
  for (int i = 0; i < NS; ++i)
    for (int k = 0; k < 3; ++k) {
      A[i].w[k] += r[i].j[k] * sb;
      q[i].j[k] += sb * x[i].w[k];
    }
  c.ql = -wv + ltb + gamma * sb;
}

// Reverse of one hinge visit (rows 4..0).  Row data and row adjoint
// accumulators are streamed: row q-1 is loaded while row q is reversed.
// A servo's motor row (clamped to [-hi, hi]) is reversed first, on its own.
// a: body index or the world slot (whose adjoint slot is a sink).  H: this
// sweep's records, Hp: the previous sweep's (the start impulses before the
// first sweep).
template <int NS, class Team>
SHD void hinge_rev(const Team& tm, const DevModel& M, const Env& E, int s, int a, int b, const float* H,
                   const float* Hp, bool first) {
  HSides<NS> sd;
  sd.init(tm, E, a, b);
  HS x[NS], A[NS];
  float imx[NS];
  for (int i = 0; i < NS; ++i) {
    hs_load(x[i], E.body(sd.bd[i]) + BV);
    hs_load(A[i], E.bodyA(sd.bd[i]) + AV);
    imx[i] = 0.f;
  }
  const float* R0 = E.row(s);
  float* Q0 = E.rowA(s);
  const float* Hs = H + s;
  const float* Hps = Hp + s;
  if (E.jr == 6) {
    HR r5[NS];
    HQ q5[NS];
    HRow c5;
    h_rev_load<NS>(sd, R0, Q0, 5, Hs, Hps, r5, q5, c5);
    const float hi = R0[5 * RS + RHI];
    // the impulse before this sweep's update: the previous sweep's clamped
    // result, or the start impulse
    if (!first) c5.lp = c5.lp <= -hi ? -hi : (c5.lp >= hi ? hi : c5.lp);
    h_row_rev_box<NS>(tm, r5, q5, x, A, sd, c5, M.gamma, hi);
    float* Q = Q0 + 5 * RSA;
    for (int i = 0; i < NS; ++i) {
      q5[i].m = c5.qm;
      q5[i].b = c5.qb;
      hq_store(q5[i], Q + sd.so[i]);
    }
    Q[QL] = c5.ql;
  }
  // Rows are loaded AH rows ahead of their reversal: a lane of a pair holds
  // all five rows from the start of the visit (one LDS round trip), a
  // one-lane visit (two sides per lane) streams them one row ahead.
  constexpr int AH = NS == 1 ? 5 : 1;
  HR rr[5][NS];
  HQ qq[5][NS];
  HRow cr[5];
#pragma unroll
  for (int q = 4; q > 4 - AH; --q) h_rev_load<NS>(sd, R0, Q0, q, Hs, Hps, rr[q], qq[q], cr[q]);
#pragma unroll
  for (int q = 4; q >= 0; --q) {
    if (q - AH >= 0) h_rev_load<NS>(sd, R0, Q0, q - AH, Hs, Hps, rr[q - AH], qq[q - AH], cr[q - AH]);
    HRow& cc = cr[q];
    if (q >= 3) h_row_rev<3, NS>(tm, rr[q], qq[q], x, A, sd, imx, cc, M.gamma);
    else if (q == 2) h_row_rev<2, NS>(tm, rr[q], qq[q], x, A, sd, imx, cc, M.gamma);
    else if (q == 1) h_row_rev<1, NS>(tm, rr[q], qq[q], x, A, sd, imx, cc, M.gamma);
    else h_row_rev<0, NS>(tm, rr[q], qq[q], x, A, sd, imx, cc, M.gamma);
    // (the row-shared adjoints are the same in both lanes of a pair)
    float* Q = Q0 + q * RSA;
    for (int i = 0; i < NS; ++i) {
      qq[q][i].m = cc.qm;
      qq[q][i].b = cc.qb;
      hq_store(qq[q][i], Q + sd.so[i]);
    }
    Q[QL] = cc.ql;
  }
  for (int i = 0; i < NS; ++i) {
    hs_store(x[i], E.body(sd.bd[i]) + BV);
    hs_store(A[i], E.bodyA(sd.bd[i]) + AV);
    E.bodyA(sd.bd[i])[AIM] += imx[i];
  }
}

// Reverse of one contact visit: friction disk, then the normal row.  HA =
// false: a ground contact, body a's terms skipped (they go to the world
// slot's velocity, zero, and its adjoint, a sink, and to the row's body-a
// Jacobian adjoints, which a ground contact's set-up adjoint does not read).
template <bool HA = true>
SHD void rev_contact(const DevModel& M, const Env& E, int s, int a, int b, float mu, const float* H,
                     const float* Hp, float& gmu) {
  constexpr bool ha = HA;
  VR V, A;
  if constexpr (HA) {
    vr_load_ab(V, E, a, b);
    vra_load_ab(A, E, a, b);
  } else {
    vr_load_b(V, E, b);
    vra_load_b(A, E, b);
  }
  RR R1, R2;
  QR Q1, Q2;
  rr_load(R1, E.row(s + 1));
  rr_load(R2, E.row(s + 2));
  qr_load(Q1, E.rowA(s + 1));
  qr_load(Q2, E.rowA(s + 2));
  float* xa = E.rowA(s + 3);
  const float mt = E.row(s + 3)[XMT];
  const float ima = HA ? E.body(a)[BIM] : 0.f, imb = E.body(b)[BIM];
  float imA = 0.f, imB = 0.f;
  const float ltn = H[s], l1t = H[s + 1], l2t = H[s + 2];
  const float ln = fmaxf(ltn, 0.f);
  const float rho = mu * ln;
  float n1, n2, p1, p2, lpn;
  disk(l1t, l2t, rho, n1, n2);
  if (Hp) {
    lpn = fmaxf(Hp[s], 0.f);
    disk(Hp[s + 1], Hp[s + 2], mu * lpn, p1, p2);
  } else {
    lpn = E.row(s)[RL0];
    p1 = E.row(s + 1)[RL0];
    p2 = E.row(s + 2)[RL0];
  }
  const float d1 = n1 - p1, d2 = n2 - p2;
  rr_apply(R2, V, ha, ima, imb, -d2);
  rr_apply(R1, V, ha, ima, imb, -d1);
  rr_wbar(Q1, R1, A, ha, ima, imb, d1, imA, imB);
  rr_wbar(Q2, R2, A, ha, ima, imb, d2, imA, imB);
  const float wv1 = rr_wv(R1, A, ha, ima, imb);
  const float wv2 = rr_wv(R2, A, ha, ima, imb);
  const float g1 = Q1.l + wv1, g2 = Q2.l + wv2;
  const float nrm = sqrtf(l1t * l1t + l2t * l2t);
  float tb1 = g1, tb2 = g2, lnb = 0.f;
  if (!(nrm <= rho)) {
    const float u1 = l1t / nrm, u2 = l2t / nrm, sc = rho / nrm;
    const float ug = u1 * g1 + u2 * g2;
    tb1 = sc * (g1 - u1 * ug);
    tb2 = sc * (g2 - u2 * ug);
    gmu += ug * ln;
    lnb = ug * mu;   // adjoint of this iteration's normal impulse
  }
  const float jv1 = rr_jv(R1, V, ha), jv2 = rr_jv(R2, V, ha);
  xa[XMT] += -(tb1 * jv1 + tb2 * jv2);
  rr_jbar(Q1, R1, A, V, ha, -mt * tb1);
  rr_jbar(Q2, R2, A, V, ha, -mt * tb2);
  Q1.l = -wv1 + tb1;
  Q2.l = -wv2 + tb2;
  qr_store(Q1, E.rowA(s + 1));
  qr_store(Q2, E.rowA(s + 2));
  RR R0;
  QR Q0;
  rr_load(R0, E.row(s));
  qr_load(Q0, E.rowA(s));
  Q0.l += lnb;
  rev_scalar(R0, Q0, V, A, ha, ima, imb, ltn, lpn, false, M.gamma, imA, imB);
  qr_store(Q0, E.rowA(s));
  if constexpr (HA) {
    vr_store_ab(V, E, a, b);
    vra_store_ab(A, E, a, b);
    E.bodyA(a)[AIM] += imA;
  } else {
    vr_store_b(V, E, b);
    vra_store_b(A, E, b);
  }
  E.bodyA(b)[AIM] += imB;
}

// Sweep it of the impulse history into its ring slot: from the step's
// history in global memory, or (it = -1) the start impulses.
template <class Team>
SHD void hist_fill(const Team& tm, const Env& E, const float* gh, int it) {
  float* dst = E.hist(it);
  if (it >= 0) {
    const float* src = gh + (size_t)it * E.nslot;
    for (int s = tm.tl; s < E.nslot; s += tm.ts) dst[s] = src[s];
  } else {
    for (int s = tm.tl; s < E.nslot; s += tm.ts) dst[s] = E.row(s)[RL0];
  }
}

// B6: adjoint of the sweeps (iterations, colours and rows exactly reversed).
// gh: the step's impulse history in global memory, n_iters rows of nslot
// floats, when the env keeps only a ring of it in LDS: the last two sweeps
// are loaded first, and at the start of each reversed sweep it the sweep it-2
// (or the start impulses) takes the slot sweep it+1 no longer needs.
template <class Team>
SHD void a_pgs(const Team& tm, const DevModel& M, const Env& E, bool act, const float* gh = nullptr) {
  const float mu = E.misc()[MISC_MU];
  float gmu = 0.f;
  const bool ring = E.lay.hring != 0 && act && M.n_iters > 0;
  if (ring) {
    hist_fill(tm, E, gh, M.n_iters - 1);
    hist_fill(tm, E, gh, M.n_iters - 2);
  }
  tm.sync();
  SweepCursor<-1> sw;
  sw.start(tm, E, M.n_iters, n_plan(E, act));
  while (tm.any(sw.left > 0)) {
    i4 vn, p2;
    sw.prefetch(tm, E, vn, p2);
    // (the slot is read by no visit of this sweep; the barrier after the
    // visit orders the writes before the next sweep's reads)
    if (ring && sw.left > 0 && sw.ci == sw.nl - 1 && sw.it >= 1) hist_fill(tm, E, gh, sw.it - 2);
    const float* H = E.hist(sw.it);
    const float* Hp = E.hist(sw.it - 1);
    const int nk = sw.count(tm);
    for (int k = 0; k < nk; ++k) {
      const i4 v = sw.entry(tm, E, k);
      if (v.x < 0) continue;
      if (cand_kind(v.w) != K_JOINT) {
        if (v.y == E.nb) rev_contact<false>(M, E, v.x, v.y, v.z, mu, H, sw.it > 0 ? Hp : nullptr, gmu);
        else rev_contact<true>(M, E, v.x, v.y, v.z, mu, H, sw.it > 0 ? Hp : nullptr, gmu);
      }
      else if (tm.ts >= 2) hinge_rev<1>(tm, M, E, v.x, v.y, v.z, H, Hp, sw.it == 0);
      else hinge_rev<2>(tm, M, E, v.x, v.y, v.z, H, Hp, sw.it == 0);
    }
    tm.sync();
    sw.advance(vn, p2);
  }
  // friction coefficient adjoint (one lane per team holds it after a reduction)
  float tot = tm.team_sum(gmu);
  if (tm.tl == 0 && act) kahan_add(E.misc() + MISC_GMU, E.misc() + MISC_GMUC, tot);
  tm.sync();
}

// Adjoint of a hinge's warm start (see hinge_warm), by side: each side adds
// its part of W-bar and of its body's inverse-mass adjoint; a row's impulse
// adjoint takes (part b) + (part a) of W^T v-bar, exchanged within a pair, so
// both lanes hold the same value.
template <int S, int NS, class Team>
SHD float hinge_warm_row(const Team& tm, const HSides<NS>& sd, const float* R, float* Q, const HS* A, float* imx) {
  const float d = R[RL0];
  float p[NS];
  for (int i = 0; i < NS; ++i) {
    HR r;
    hr_load(r, R + sd.so[i]);
    float* qw = Q + QWA + sd.so[i];
    f4 w4 = ld4(qw);
    w4.x += A[i].w[0] * d; w4.y += A[i].w[1] * d; w4.z += A[i].w[2] * d;
    st4(qw, w4);
    if (S < 3) imx[i] += (sd.sg[i] * d) * A[i].v[S];
    p[i] = h_wpart<S>(r, A[i], sd.sim[i]);
  }
  return Q[QL] + h_sum<NS>(tm, p);
}
template <int NS, class Team>
SHD void hinge_warm_rev(const Team& tm, const DevModel& M, const Env& E, int s, int a, int b, int code) {
  HSides<NS> sd;
  sd.init(tm, E, a, b);
  const float* R0 = E.row(s);
  float* Q0 = E.rowA(s);
  HS A[NS];
  float imx[NS];
  for (int i = 0; i < NS; ++i) {
    hs_load(A[i], E.bodyA(sd.bd[i]) + AV);
    imx[i] = 0.f;
  }
  float l0b[6];
  l0b[0] = hinge_warm_row<0, NS>(tm, sd, R0, Q0, A, imx);
  l0b[1] = hinge_warm_row<1, NS>(tm, sd, R0 + RS, Q0 + RSA, A, imx);
  l0b[2] = hinge_warm_row<2, NS>(tm, sd, R0 + 2 * RS, Q0 + 2 * RSA, A, imx);
  l0b[3] = hinge_warm_row<3, NS>(tm, sd, R0 + 3 * RS, Q0 + 3 * RSA, A, imx);
  l0b[4] = hinge_warm_row<3, NS>(tm, sd, R0 + 4 * RS, Q0 + 4 * RSA, A, imx);
  if (E.jr == 6) l0b[5] = hinge_warm_row<3, NS>(tm, sd, R0 + 5 * RS, Q0 + 5 * RSA, A, imx);
  // Both lanes of a pair hold the same values; one of them (side b's) adds
  // them: a read-modify-write by both lanes would count them once only where
  // the two lanes' reads precede both writes, as in a wave's lockstep.
  if (NS == 2 || sd.sd[0] == 1) {
    float* wA = E.wsA() + E.store_of(code);
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (q < 5 || E.jr == 6) wA[q] += M.warm * l0b[q];
  }
  for (int i = 0; i < NS; ++i) E.bodyA(sd.bd[i])[AIM] += imx[i];
}

// B5: adjoint of the warm start v += W lambda0 and of lambda0 = warm * store.
template <class Team>
SHD void a_warm(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nl = n_plan(E, act);
  for (int ci = nl - 1; tm.any(ci >= 0); --ci) {
    i4 pl{0, 0, 0, 0};
    if (ci >= 0) pl = E.plan()[ci];
    const int n = pl.y, lo = pl.x;
    const bool pr = pl.z != 0 && tm.ts >= 2;
    const int k0 = pr ? tm.tl >> 1 : tm.tl, kst = pr ? tm.ts >> 1 : tm.ts;
    for (int k = k0; k < n; k += kst) {
      const i4 v = E.vis()[lo + k];
      const int s = v.x;
      if (s < 0) continue;
      const int code = v.w;
      if (cand_kind(code) == K_JOINT) {
        if (pr) hinge_warm_rev<1>(tm, M, E, s, v.y, v.z, code);
        else hinge_warm_rev<2>(tm, M, E, s, v.y, v.z, code);
        continue;
      }
      const RowB rb{v.y == E.nb ? -1 : v.y, v.z};
      const bool ha = rb.a >= 0;
      const int nr = 3;
      VelA A;
      vela_load(A, E, rb.a, rb.b);
      float imA = 0.f, imB = 0.f;
      const float ima = ha ? E.body(rb.a)[BIM] : 0.f, imb = E.body(rb.b)[BIM];
      float l0b[5];
      for (int q = 0; q < nr; ++q) {
        const float* r = E.row(s + q);
        float* qa = E.rowA(s + q);
        row_wbar(qa, r, A, ha, ima, imb, r[RL0], &imA, &imB);
        l0b[q] = qa[QL] + row_wvbar(r, A, ha, ima, imb);
      }
      float* wA = E.wsA() + E.store_of(code);
      {
        const float* x = E.row(s + 3);
        float* xa = E.rowA(s + 3);
        const float* w = E.ws() + E.store_of(code);
        const f3 Lt = mk3(w[1], w[2], w[3]);
        const f3 t1 = ld3(x + XT1), t2 = ld3(x + XT2);
        wA[0] += M.warm * l0b[0];
        const f3 Lb = (M.warm * l0b[1]) * t1 + (M.warm * l0b[2]) * t2;
        wA[1] += Lb.x; wA[2] += Lb.y; wA[3] += Lb.z;
        add3(xa + XT1, (M.warm * l0b[1]) * Lt);
        add3(xa + XT2, (M.warm * l0b[2]) * Lt);
      }
      if (ha) E.bodyA(rb.a)[AIM] += imA;
      E.bodyA(rb.b)[AIM] += imB;
    }
    tm.sync();
  }
}

// Adjoint of row_finish: K = im |Jl|^2 + Ja^T Iw_a Ja + Jb^T Iw_b Jb, W = Iw J.
// Kb is the adjoint of K; adds into Jbar and body Iw-bar / invm-bar.
SHD void a_row_finish(const Env& E, const float* r, float* q, int a, int b, float Kb) {
  const bool ha = a >= 0;
  float* Ab = E.bodyA(b);
  const float* Bb = E.body(b);
  const f3 jl = ld3(r + RJL), jb = ld3(r + RJB);
  float im = Bb[BIM];
  const float jl2 = dot(jl, jl);
  Ab[AIM] += Kb * jl2;
  // Jb: W = Iw Jb, K += Jb.W  ->  Jbbar += Iw (Wbar + 2 Kb Jb); Iwbar += (Wbar + Kb Jb) Jb^T
  {
    const f3 wbb = ld3(q + QWB);
    const f3 tmp = wbb + (2.f * Kb) * jb;
    add3(q + QJB, sv(Bb + BI, tmp));
    add_outer(Ab + AIW, wbb + Kb * jb, jb);
  }
  if (ha) {
    float* Aa = E.bodyA(a);
    const float* Ba = E.body(a);
    const f3 ja = ld3(r + RJA);
    im += Ba[BIM];
    Aa[AIM] += Kb * jl2;
    const f3 wab = ld3(q + QWA);
    const f3 tmp = wab + (2.f * Kb) * ja;
    add3(q + QJA, sv(Ba + BI, tmp));
    add_outer(Aa + AIW, wab + Kb * ja, ja);
  }
  add3(q + QJL, (2.f * Kb * im) * jl);
}

// The body adjoint's position, rotation, inverse-inertia and inverse-mass
// parts (floats AP .. AR + 8 and AIW .. AIM), read and written as two
// aligned runs: three float4, then a float2 and two float4.
static_assert(AP == 0 && AR == 3 && AIW == 18 && AIM == 27 && BSA % 4 == 0, "body adjoint layout");
struct BodyAdjHead { float ap[3], ar[9], aiw[9], aim; };
SHD float f3_at(f3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
SHD void bah_load(BodyAdjHead& h, const float* A) {
  const f4 a0 = ld4(A), a1 = ld4(A + 4), a2 = ld4(A + 8);
  const f2 b0 = *reinterpret_cast<const f2*>(A + 18);
  const f4 b1 = ld4(A + 20), b2 = ld4(A + 24);
  h.ap[0] = a0.x; h.ap[1] = a0.y; h.ap[2] = a0.z; h.ar[0] = a0.w;
  h.ar[1] = a1.x; h.ar[2] = a1.y; h.ar[3] = a1.z; h.ar[4] = a1.w;
  h.ar[5] = a2.x; h.ar[6] = a2.y; h.ar[7] = a2.z; h.ar[8] = a2.w;
  h.aiw[0] = b0.x; h.aiw[1] = b0.y;
  h.aiw[2] = b1.x; h.aiw[3] = b1.y; h.aiw[4] = b1.z; h.aiw[5] = b1.w;
  h.aiw[6] = b2.x; h.aiw[7] = b2.y; h.aiw[8] = b2.z; h.aim = b2.w;
}
SHD void bah_store(const BodyAdjHead& h, float* A) {
  st4(A, f4{h.ap[0], h.ap[1], h.ap[2], h.ar[0]});
  st4(A + 4, f4{h.ar[1], h.ar[2], h.ar[3], h.ar[4]});
  st4(A + 8, f4{h.ar[5], h.ar[6], h.ar[7], h.ar[8]});
  st2(A + 18, f2{h.aiw[0], h.aiw[1]});
  st4(A + 20, f4{h.aiw[2], h.aiw[3], h.aiw[4], h.aiw[5]});
  st4(A + 24, f4{h.aiw[6], h.aiw[7], h.aiw[8], h.aim});
}
SHD void outer_acc(float* O, f3 a, f3 b) {
  O[0] += a.x * b.x; O[1] += a.x * b.y; O[2] += a.x * b.z;
  O[3] += a.y * b.x; O[4] += a.y * b.y; O[5] += a.y * b.z;
  O[6] += a.z * b.x; O[7] += a.z * b.y; O[8] += a.z * b.z;
}
// Adjoint of build_joint.  The five rows' row_finish adjoints (see
// a_row_finish) are accumulated in registers and added to the bodies once;
// the rows' Jacobian adjoints stay in registers for the geometry below (the
// adjoint of Jl, a constant for a hinge, is not formed).  Like the sweeps, a
// hinge colour can be taken by lane pairs: each lane of a pair forms its own
// body's terms (NS = 1), and one lane alone forms both (NS = 2, index 0 =
// body b), with the same expressions in the same order, so the results do
// not depend on the form.  Side a needs side b's Jacobian adjoints of the
// two angular rows, which a pair exchanges with the DPP swap.
template <int NS, class Team>
SHD void a_joint(const Team& tm, const DevModel& M, const Env& E, int j, int s) {
  const float* C = E.jc(j);
  const int a = E.jpar(j), b = E.jchi(j);
  const bool ha = a >= 0;
  const float* Bb = E.body(b);
  const float* Ba = ha ? E.body(a) : nullptr;
  static_assert(QM == QJB + 3 && QB == QWB + 3 && QJA % 4 == 0 && QWA % 4 == 0, "row adjoint layout");
  int sd[NS];        // 1: body b's side
  bool on[NS];       // the side has a body (side a of a world-attached joint has none)
  float I[NS][6];    // the side's body inverse inertia (world frame)
  for (int i = 0; i < NS; ++i) {
    sd[i] = NS == 2 ? 1 - i : (tm.tl & 1);
    on[i] = sd[i] || ha;
    // (side a of a world-attached joint reads the world slot: zero inertia)
    const float* B = sd[i] ? Bb : (ha ? Ba : E.body(E.nb));
    for (int k = 0; k < 6; ++k) I[i][k] = B[BI + k];
  }
  f3 qj[NS][6];
  float qbias[6];
  float O[NS][9];
  float imx[NS];
  for (int i = 0; i < NS; ++i) {
    imx[i] = 0.f;
    for (int k = 0; k < 9; ++k) O[i][k] = 0.f;
  }
  // (unrolled: qj and qbias stay in registers; the sixth row only with a servo)
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q == 5 && E.jr != 6) break;
    const float* r = E.row(s + q);
    const float* qa = E.rowA(s + q);
    const float qm = qa[QM];
    qbias[q] = qa[QB];
    // Jl is a unit axis for the point rows and zero for the angular rows
    const float jl2 = q < 3 ? 1.f : 0.f;
    for (int i = 0; i < NS; ++i) {
      const int so = HSIDE * sd[i];
      const f4 rj = ld4(r + RJA + so), qj4 = ld4(qa + QJA + so), qw4 = ld4(qa + QWA + so);
      const float m = rj.w;   // (RMA / RM: the same value)
      const float Kb = -m * m * qm;
      qj[i][q] = mk3(qj4.x, qj4.y, qj4.z);
      if (on[i]) {
        // J: W = Iw J, K += J.W  ->  Jbar += Iw (Wbar + 2 Kb J); Iwbar += (Wbar + Kb J) J^T
        const f3 jx = mk3(rj.x, rj.y, rj.z), wx = mk3(qw4.x, qw4.y, qw4.z);
        imx[i] += Kb * jl2;
        qj[i][q] = qj[i][q] + sv(I[i], wx + (2.f * Kb) * jx);
        outer_acc(O[i], wx + Kb * jx, jx);
      }
    }
  }
  const float kb = M.beta / M.dt;
  const f3 rbl = ld3(C + JAC), ral = ld3(C + JAP);
  f3 rx[NS], errb = mk3(0.f, 0.f, 0.f);
  for (int i = 0; i < NS; ++i) rx[i] = mk3(0.f, 0.f, 0.f);
  for (int q = 0; q < 3; ++q) {
    const f3 e = mk3(q == 0 ? 1.f : 0.f, q == 1 ? 1.f : 0.f, q == 2 ? 1.f : 0.f);
    // Ja = e x ra ; Jb = rb x e
    for (int i = 0; i < NS; ++i) rx[i] = rx[i] + (sd[i] ? cross(e, qj[i][q]) : cross(qj[i][q], e));
    errb = errb + (kb * qbias[q]) * e;
  }
  for (int i = 0; i < NS; ++i) rx[i] = sd[i] ? rx[i] + errb : rx[i] - errb;
  // angular rows
  f3 na = ld3(C + JXP), ua = ld3(C + JUP);
  const f3 t2l = cross(na, ua);
  f3 t2 = t2l;
  const f3 nal = na, ual = ua;
  if (ha) { na = mv(Ba + BR, na); ua = mv(Ba + BR, ua); t2 = mv(Ba + BR, t2); }
  const f3 nbl = ld3(C + JXC);
  const f3 nbw = mv(Bb + BR, nbl);
  const f3 ax = cross(na, nbw);
  // side b's and side a's Jacobian adjoints of the angular rows
  // (index 2: a servo's motor row, J = (-na, na))
  f3 qjb[3], qja[3];
  const int nq = E.jr == 6 ? 3 : 2;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q == 2 && nq != 3) break;
    if (NS == 2) {
      qjb[q] = qj[0][3 + q];
      qja[q] = qj[NS - 1][3 + q];
    } else {
      const f3 own = qj[0][3 + q];
      const f3 other = mk3(tm.pair_swap(own.x), tm.pair_swap(own.y), tm.pair_swap(own.z));
      qjb[q] = sd[0] ? own : other;
      qja[q] = sd[0] ? other : own;
    }
  }
  f3 axb = mk3(0.f, 0.f, 0.f), tb[2];
  for (int q = 0; q < 2; ++q) {
    const float cb = kb * qbias[3 + q];
    const f3 tk = q == 0 ? ua : t2;
    tb[q] = qjb[q] - qja[q] + cb * ax;
    axb = axb + cb * tk;
  }
  // ax = na x nbw ; a motor row's Jacobian is na itself
  f3 nab = cross(nbw, axb);
  if (nq == 3) nab = nab + (qjb[2] - qja[2]);
  const f3 nbb = cross(axb, na);
  // The anchors (the link lengths): r_b = R_b a_c and r_a = R_a a_p give
  // a_c-bar = R_b^T r_b-bar and a_p-bar = R_a^T r_a-bar; a world-attached
  // joint's point a_p enters the error alone, -errbar.  Each side adds its
  // own anchor's totals (a lane of a pair: its side only).
  for (int i = 0; i < NS; ++i) {
    const f3 g = sd[i] ? mtv(Bb + BR, rx[i]) : (ha ? mtv(Ba + BR, rx[i]) : -errb);
    float* tot = E.jA() + (sd[i] ? JA_ANCC : JA_ANCP) * E.nj + 3 * j;
    float* cmp = tot + JA_ANC_COMP * E.nj;
    kahan_add(tot, cmp, g.x);
    kahan_add(tot + 1, cmp + 1, g.y);
    kahan_add(tot + 2, cmp + 2, g.z);
  }
  // The bodies' adjoints, each read and written once with 16-byte accesses;
  // every element takes its additions in the order of the adjoint's terms.
  for (int i = 0; i < NS; ++i) {
    if (!on[i]) continue;
    float* A = E.bodyA(sd[i] ? b : a);
    BodyAdjHead h;
    bah_load(h, A);
    h.aim += imx[i];
    for (int k = 0; k < 9; ++k) h.aiw[k] += O[i][k];
    if (sd[i]) {
      for (int k = 0; k < 3; ++k) h.ap[k] += f3_at(errb, k);
      outer_acc(h.ar, rx[i], rbl);
      outer_acc(h.ar, nbb, nbl);
    } else {
      for (int k = 0; k < 3; ++k) h.ap[k] += -f3_at(errb, k);
      outer_acc(h.ar, rx[i], ral);
      outer_acc(h.ar, nab, nal);
      outer_acc(h.ar, tb[0], ual);
      outer_acc(h.ar, tb[1], t2l);
    }
    bah_store(h, A);
  }
}

// Adjoint of build_contact (+ the tangent adjoints collected from the store
// and warm-start reverses).
SHD void a_contact(const DevModel& M, const Env& E, int code, int s) {
  const RowB rb = cand_bodies(E, code);
  const bool ground = cand_kind(code) == K_GROUND;
  const CGeo g = contact_geo(E, code);
  const float* x = E.row(s + 3);
  const float* xa = E.rowA(s + 3);
  const bool rest = x[XREST] != 0.f;
  if (rest) {
    // bias = e v_n, v_n = Jl.(vb - va) + Ja.wa + Jb.wb at the predicted
    // velocities: adjoints of the normal row's Jacobian and of v*, w*
    float* q = E.rowA(s);
    const float* r = E.row(s);
    const float vnb = E.misc()[MISC_REST] * q[QB];
    const float* sb = E.vsave(rb.b);
    float* Ab = E.bodyA(rb.b);
    for (int k = 0; k < 3; ++k) {
      q[QJL + k] += vnb * sb[k];
      q[QJB + k] += vnb * sb[3 + k];
      Ab[AV + k] += vnb * r[RJL + k];
      Ab[AW + k] += vnb * r[RJB + k];
    }
    if (!ground) {
      const float* sa = E.vsave(rb.a);
      float* Aa = E.bodyA(rb.a);
      for (int k = 0; k < 3; ++k) {
        q[QJL + k] -= vnb * sa[k];
        q[QJA + k] += vnb * sa[3 + k];
        Aa[AV + k] -= vnb * r[RJL + k];
        Aa[AW + k] += vnb * r[RJA + k];
      }
    }
  }
  // row_finish adjoints: normal via m, tangents via mt = 2/(K1+K2)
  {
    const float m = E.row(s)[RM];
    a_row_finish(E, E.row(s), E.rowA(s), rb.a, rb.b, -m * m * E.rowA(s)[QM]);
    const float mt = x[XMT];
    const float Kt = -0.5f * mt * mt * xa[XMT];
    a_row_finish(E, E.row(s + 1), E.rowA(s + 1), rb.a, rb.b, Kt);
    a_row_finish(E, E.row(s + 2), E.rowA(s + 2), rb.a, rb.b, Kt);
  }
  const f3 t1 = ld3(x + XT1), t2 = ld3(x + XT2);
  const f3 dirs[3] = {g.n, t1, t2};
  f3 dirb[3], rab = mk3(0.f, 0.f, 0.f), rbb = mk3(0.f, 0.f, 0.f);
  for (int q = 0; q < 3; ++q) {
    const float* qa = E.rowA(s + q);
    const f3 jab = ld3(qa + QJA), jbb = ld3(qa + QJB);
    dirb[q] = ld3(qa + QJL);
    // Jb = rb x dir
    rbb = rbb + cross(dirs[q], jbb);
    dirb[q] = dirb[q] + cross(jbb, g.rb);
    if (!ground) {
      // Ja = dir x ra
      dirb[q] = dirb[q] + cross(g.ra, jab);
      rab = rab + cross(jab, dirs[q]);
    }
  }
  const float gapb = rest ? 0.f : E.rowA(s)[QB] * (g.gap > 0.f ? 1.f : M.beta) / M.dt;
  float* Ab = E.bodyA(rb.b);
  const float* Bb = E.body(rb.b);
  if (ground) {
    const int i = cand_idx(code);
    const f3 off = ld3(E.gsph(i));
    // rb = R o - r n (n constant) ; gap = p_z + (R o)_z - r
    add_outer(Ab + AR, rbb, off);
    Ab[AP + 2] += gapb;
    add_outer(Ab + AR, mk3(0.f, 0.f, gapb), off);
    return;
  }
  float* Aa = E.bodyA(rb.a);
  const float* Ba = E.body(rb.a);
  f3 nb_ = dirb[0];
  f3 t1b = dirb[1] + ld3(xa + XT1);
  const f3 t2b = dirb[2] + ld3(xa + XT2);
  // t2 = n x t1
  nb_ = nb_ + cross(t1, t2b);
  t1b = t1b + cross(t2b, g.n);
  // t1 = w / |w|, w = n x e
  {
    const bool zsel = fabsf(g.n.z) < 0.9f;
    const f3 e = zsel ? mk3(0.f, 0.f, 1.f) : mk3(1.f, 0.f, 0.f);
    const f3 w = cross(g.n, e);
    const float wl = sqrtf(dot(w, w));
    const f3 wb = (1.f / wl) * (t1b - dot(t1, t1b) * t1);
    nb_ = nb_ + cross(e, wb);
  }
  // ra = R_a o_a + r_a n ; rb = R_b o_b - r_b n
  const f3 oa = ld3(Ba + BPO), ob = ld3(Bb + BPO);
  add_outer(Aa + AR, rab, oa);
  add_outer(Ab + AR, rbb, ob);
  nb_ = nb_ + Ba[BPR] * rab - Bb[BPR] * rbb;
  // n = d / L, gap = L - r_a - r_b
  f3 db = gapb * g.n;
  if (g.L >= 1e-9f) db = db + (1.f / g.L) * (nb_ - dot(g.n, nb_) * g.n);
  // d = c_b - c_a, c = p + R o
  add3(Ab + AP, db);
  add_outer(Ab + AR, db, ob);
  add3(Aa + AP, -db);
  add_outer(Aa + AR, -db, oa);
}

// B4: adjoint of the row set-up, colour by colour (disjoint bodies).
template <class Team>
SHD void a_rows(const Team& tm, const DevModel& M, const Env& E, bool act) {
  const int nl = n_plan(E, act);
  for (int ci = nl - 1; tm.any(ci >= 0); --ci) {
    i4 pl{0, 0, 0, 0};
    if (ci >= 0) pl = E.plan()[ci];
    const int n = pl.y, lo = pl.x;
    // a hinge colour is taken by lane pairs (one body each) when the team has
    // a pair of lanes for each of its joints; otherwise one lane per joint
    const bool pr = pl.z != 0 && tm.ts >= 2 && 2 * n <= tm.ts;
    const int k0 = pr ? tm.tl >> 1 : tm.tl, kst = pr ? tm.ts >> 1 : tm.ts;
    for (int k = k0; k < n; k += kst) {
      const i4 v = E.vis()[lo + k];
      const int s = v.x;
      if (s < 0) continue;
      const int code = v.w;
      if (cand_kind(code) != K_JOINT) a_contact(M, E, code, s);
      else if (pr) a_joint<1>(tm, M, E, cand_idx(code), s);
      else a_joint<2>(tm, M, E, cand_idx(code), s);
    }
    tm.sync();
  }
}

// B3: adjoint of the prediction; B2: torques (per joint colour); B1: Iw.
// Largest adjoint magnitude a gradient keeps.  Beyond it an env's gradient is
// treated as overflowed: its products with the controller's activations (|s|
// up to ~1e2), summed over ~1e6 env-steps, would no longer be representable.
#define ADJ_LIMIT 1.0e30f

// bad (per lane): set when a control adjoint this lane writes exceeds ADJ_LIMIT
SHD void a_predict_torques_flag(bool* bad, float v) {
  if (bad && !(fabsf(v) <= ADJ_LIMIT)) *bad = true;
}
template <class Team>
SHD void a_predict_torques(const Team& tm, const DevModel& M, const Env& E, bool act, float* g_u_row,
                           float* g_damp, bool* bad = nullptr) {
  const int nb = act ? E.nb : 0;
  for (int b = tm.tl; b < nb; b += tm.ts) {
    const float* B = E.body(b);
    float* A = E.bodyA(b);
    const f3 wb = ld3(A + AW);
    // w* = w + dt Iw tq
    const f3 tqb = M.dt * sv(B + BI, wb);
    st3(A + ATQ, tqb);
    BodyAdjHead h;
    bah_load(h, A);
    outer_acc(h.aiw, M.dt * wb, ld3(B + BTQ));
    bah_store(h, A);
  }
  tm.sync();
  const int njc = n_joint_cols(E, act);
  for (int c = 0; tm.any(c < njc); ++c) {
    int lo = 0, hi = 0;
    if (c < njc) { lo = E.colstart(c); hi = E.colstart(c + 1); }
    for (int i = lo + tm.tl; i < hi; i += tm.ts) {
      const int j = cand_idx(E.cand(i));
      const float* C = E.jc(j);
      const int a = E.jpar(j), b = E.jchi(j);
      const f3 n = joint_axis_w(E, j);
      float* Ab = E.bodyA(b);
      f3 wrel = ld3(Ab + AW0);
      f3 tqd = ld3(Ab + ATQ);
      if (a >= 0) { wrel = wrel - ld3(E.bodyA(a) + AW0); tqd = tqd - ld3(E.bodyA(a) + ATQ); }
      const float dmp = C[JD];
      const bool servo = E.jr == 6;
      const float tau = (servo ? 0.f : C[JU]) - dmp * dot(wrel, n);
      const float taub = dot(n, tqd);
      f3 nb_ = tau * tqd - (taub * dmp) * wrel;
      // the control's adjoint: the torque's, or a servo's through the target
      // rate of its motor row, bias = -gain (u - theta) where not clipped
      float cb = taub;
      if (servo) {
        const int s5 = E.jr * j + 5;
        const float bb = E.row(s5)[RCLIP] != 0.f ? 0.f : E.rowA(s5)[QB];
        cb = -C[JG] * bb;
        // theta = atan2(y, x), y = (ua x ub).na, x = ua.ub, at x^t
        const float thb = C[JG] * bb;
        const Sensor S = joint_sensor(E, j, nullptr, nullptr);
        const float r2 = S.x * S.x + S.y * S.y;
        const float yb = r2 > 0.f ? thb * S.x / r2 : 0.f;
        const float xb = r2 > 0.f ? -thb * S.y / r2 : 0.f;
        add_outer(Ab + AR, yb * cross(S.na, S.ua) + xb * S.ua, ld3(C + JUC));
        if (a >= 0) {
          float* Aa = E.bodyA(a);
          add_outer(Aa + AR, yb * cross(S.ub, S.na) + xb * S.ub, ld3(C + JUP));
          add_outer(Aa + AR, yb * cross(S.ua, S.ub), ld3(C + JXP));
        }
      }
      if (M.ctrl) E.mlpA()[j] = cb;
      else if (g_u_row) {
        g_u_row[E.j0 + j] = cb;
        a_predict_torques_flag(bad, cb);
      }
      kahan_add(E.jA() + JA_DAMP * E.nj + j, E.jA() + JA_DAMPC * E.nj + j, -taub * dot(wrel, n));
      add3(Ab + AW, -(taub * dmp) * n);
      if (a >= 0) {
        float* Aa = E.bodyA(a);
        add3(Aa + AW, (taub * dmp) * n);
        add_outer(Aa + AR, nb_, ld3(C + JXP));
      }
    }
    tm.sync();
  }
  (void)g_damp;
  // B1: Iw = R D R^T -> Rbar += (Iwbar + Iwbar^T) R D ; invIbar_k += (R^T Iwbar R)_kk
  for (int b = tm.tl; b < nb; b += tm.ts) {
    const float* B = E.body(b);
    float* A = E.bodyA(b);
    // (the body's position and rotation are floats 0..11 of its record, the
    // adjoint's likewise: read and written as float4)
    static_assert(BP == 0 && BR == 3 && BS % 4 == 0 && AII % 4 == 0, "body record layout");
    BodyAdjHead h;
    bah_load(h, A);
    const f4 r0 = ld4(B), r1 = ld4(B + 4), r2 = ld4(B + 8);
    const float R[9] = {r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
    const float* G = h.aiw;
    float Sy[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Sy[3 * i + j] = G[3 * i + j] + G[3 * j + i];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        const float srk = Sy[3 * i] * R[k] + Sy[3 * i + 1] * R[3 + k] + Sy[3 * i + 2] * R[6 + k];
        h.ar[3 * i + k] += srk * B[BII + k];
      }
    bah_store(h, A);
    f4 ii = ld4(A + AII);   // the inverse-inertia adjoint (and, untouched, the torque adjoint's x)
    float acc3[3];
    for (int k = 0; k < 3; ++k) {
      // (R^T G R)_kk = sum_ij R_ik G_ij R_jk
      float acc = 0.f;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc += R[3 * i + k] * G[3 * i + j] * R[3 * j + k];
      acc3[k] = acc;
    }
    ii.x += acc3[0]; ii.y += acc3[1]; ii.z += acc3[2];
    st4(A + AII, ii);
    kahan_add(A + ATM, A + ACM, A[AIM]);
    for (int k = 0; k < 3; ++k) kahan_add(A + ATI + k, A + ACI + k, A[AII + k]);
  }
  tm.sync();
}

// Adjoint of the controller of step t: layer deltas (written with the
// activations to the env-step tape for the weight-gradient contraction) and
// the adjoint of the sensors into the state adjoint of x^t.
template <class Team>
SHD void a_controller(const Team& tm, const DevModel& M, const Env& E, bool act, int t, bool* bad = nullptr) {
  if (!M.ctrl) return;
  const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
  const float* sv_ = E.mlp();
  float* du = E.mlpA();
  const float* sb = du + mo_sb(M);
  // the recurrent head: a-bar = h-bar^{t+1} (1 - (h^{t+1})^2); the carried
  // state holds h^{t+1} after the step's controls
  const int rec = act ? M.mlp_rec : 0;
  for (int i = tm.tl; i < rec; i += tm.ts) {
    const float hn = E.ws()[E.lam_imp + i];
    du[E.nj + i] = E.wsA()[E.lam_imp + i] * (1.f - hn * hn);
  }
  for (int k = no + tm.tl; k < align4(no); k += tm.ts) du[k] = 0.f;
  tm.sync();
  // d2 = (W3^T du) (1 - h2^2), d1 = (W2^T d2) (1 - h1^2), sbar = W1^T d1 for
  // every env of the wave at once
  tm.ctrl_backward(M, E);
  if (act) {
    // tape row: s, h1, h2, du, d2, d1 (unpadded)
    float* row = M.tape + (size_t)(E.tape_off + t) * M.tape_stride;
    const int len = tape_d1(M) + n1;
    for (int k = tm.tl; k < len; k += tm.ts) {
      float v;
      if (k < tape_h1(M)) v = sv_[k];
      else if (k < tape_h2(M)) v = sv_[mo_h1(M) + k - tape_h1(M)];
      else if (k < tape_du(M)) v = sv_[mo_h2(M) + k - tape_h2(M)];
      else {
        if (k < tape_d2(M)) v = du[k - tape_du(M)];
        else if (k < tape_d1(M)) v = du[mo_d2(M) + k - tape_d2(M)];
        else v = du[mo_d1(M) + k - tape_d1(M)];
        a_predict_torques_flag(bad, v);
      }
      row[k] = v;
    }
  }
  // h-bar^t, carried to the reverse of step t - 1
  for (int i = tm.tl; i < rec; i += tm.ts) E.wsA()[E.lam_imp + i] = sb[2 * E.nj + 2 + i];
  tm.sync();
  // sensors: theta = atan2(y, x), y = (ua x ub).na, x = ua.ub ; rate = wrel.na
  const int njc = n_joint_cols(E, act);
  for (int c = 0; tm.any(c < njc); ++c) {
    int lo = 0, hi = 0;
    if (c < njc) { lo = E.colstart(c); hi = E.colstart(c + 1); }
    for (int i = lo + tm.tl; i < hi; i += tm.ts) {
      const int j = cand_idx(E.cand(i));
      const int a = E.jpar(j), b = E.jchi(j);
      const Sensor S = joint_sensor(E, j, a >= 0 ? E.bodyA(a) + AW0 : nullptr, E.bodyA(b) + AW0);
      const float thb = sb[j], rb = sb[E.nj + j];
      const float r2 = S.x * S.x + S.y * S.y;
      const float yb = r2 > 0.f ? thb * S.x / r2 : 0.f;
      const float xb = r2 > 0.f ? -thb * S.y / r2 : 0.f;
      const f3 uab = yb * cross(S.ub, S.na) + xb * S.ub;
      const f3 ubb = yb * cross(S.na, S.ua) + xb * S.ua;
      const f3 nab = yb * cross(S.ua, S.ub) + rb * S.wrel;
      const float* C = E.jc(j);
      float* Ab = E.bodyA(b);
      add3(Ab + AW, rb * S.na);
      add_outer(Ab + AR, ubb, ld3(C + JUC));
      if (a >= 0) {
        float* Aa = E.bodyA(a);
        add3(Aa + AW, -(rb * S.na));
        add_outer(Aa + AR, uab, ld3(C + JUP));
        add_outer(Aa + AR, nab, ld3(C + JXP));
      }
    }
    tm.sync();
  }
}

}  // namespace sim
