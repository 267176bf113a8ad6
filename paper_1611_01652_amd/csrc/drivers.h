// Env-level drivers built from the step phases: a forward rollout with
// checkpoints, a single step, and the reverse sweep over checkpointed
// segments (back-propagation through time, paper section 2.1.1).  The reverse
// recovers each step's working set from the checkpoints in one of three ways
// (DUMP_*): a segment at a time, replaying every step; a segment at a time,
// saving every step's working set during the recompute; or all segments
// recomputed at once by env_recompute in an earlier launch.
#pragma once
#include "step_core.h"

namespace sim {

struct RolloutArgs {
  const float* x0;     // [18][B]
  const float* u;      // [T_max][J] or null
  float* loss;         // [E]
  float* x_final;      // [18][B] or null
  float* lam_final;    // [lam_tot] or null
  float* ckpt;         // [n_ckpt][18 B + lam_tot] or null
  uint32_t* flags;     // [E] or null
  // tolerance mode: sweeps and fallbacks per env, training records
  int* iters;          // [E] or null
  int* fallbacks;      // [E] or null
  RecArgs rec;
  // the reverse sweep's buffer in trajectory mode: the rollout writes every
  // step's saved working set there as it goes (null: it does not)
  float* seg;
};

struct GradArgs {
  const float* x0;
  const float* u;
  const float* ckpt;
  const float* dloss;  // [E]
  float* g_x0;         // [18][B]
  float* g_u;          // [T_max][J]
  float* g_invm;       // [B]
  float* g_invI;       // [B][3]
  float* g_mu;         // [E]
  float* g_damp;       // [J]
  float* g_anc_p;      // [J][3] hinge anchors in the parent (world) frame
  float* g_anc_c;      // [J][3] hinge anchors in the child frame
  float* seg;          // per-env segment buffers
  uint32_t* flags;     // [E] or null: SIM_FLAG_GRAD_NONFINITE for envs whose adjoint overflowed
};

struct StepArgs {
  const float* x_in;
  float* x_out;
  const float* u;      // [J] (null with a controller)
  const float* lam_in;
  float* lam_out;
  uint32_t* flags;
  int t;               // step index (clock input of a controller)
};

SHD size_t ckpt_stride(const DevModel& M) { return (size_t)18 * M.B + M.lam_tot; }

template <class Team>
SHD void write_ckpt(const Team& tm, const DevModel& M, const Env& E, float* dst) {
  store_state(tm, E, dst, M.B);
  store_ws(tm, E, dst + (size_t)18 * M.B);
}
template <class Team>
SHD void read_ckpt(const Team& tm, const DevModel& M, const Env& E, const float* src) {
  load_state(tm, E, src, M.B);
  load_ws(tm, E, src + (size_t)18 * M.B);
}

template <class Team>
SHD uint32_t nonfinite_flag(const Team& tm, const Env& E) {
  bool bad = false;
  for (int b = tm.tl; b < E.nb; b += tm.ts) {
    const float* B = E.body(b);
    for (int k = 0; k < 18; ++k) bad = bad || !(fabsf(B[k]) <= 3.0e38f);
  }
  return tm.team_any(bad) ? 1u : 0u;
}

// SOLVE: the model solves to a residual tolerance (a separate instantiation,
// so the fixed-sweep kernels carry none of its state).
template <class Team, bool SOLVE = false>
SHD_FLAT void env_rollout(const Team& tm, const DevModel& M, const Env& E, bool valid, const RolloutArgs& a) {
  if (valid) {
    load_env_static(tm, M, E);
    load_state(tm, E, a.x0, M.B);
    for (int i = tm.tl; i < E.lam_size; i += tm.ts) E.ws()[i] = 0.f;
  }
  tm.sync();
  float p0x = valid ? E.body(E.lb)[BP] : 0.f;
  float loss = 0.f;
  const int K = M.ckpt_every;
  const int T = valid ? E.T : 0;
  for (int t = 0; tm.any(t < T); ++t) {
    const bool act = t < T;
    if (act && a.ckpt && t % K == 0) write_ckpt(tm, M, E, a.ckpt + (size_t)(t / K) * ckpt_stride(M));
    tm.sync();
    const float* u_row = (a.u && !M.ctrl) ? a.u + (size_t)t * M.J : nullptr;
    if (SOLVE) env_step_solve(tm, M, E, u_row, act, t, &a.rec);
    else env_step(tm, M, E, u_row, act, t);
    if (act && tm.tl == 0) {
      const float* p = E.body(E.lb) + BP;
      const float p0[3] = {p0x, 0.f, 0.f};
      loss += loss_term(M, E, t + 1, p, p0);
    }
  }
  tm.sync();
  uint32_t fl = valid ? nonfinite_flag(tm, E) : 0u;
  if (valid) {
    if (a.x_final) store_state(tm, E, a.x_final, M.B);
    if (a.lam_final) store_ws(tm, E, a.lam_final);
    if (tm.tl == 0) {
      a.loss[E.e] = loss;
      fl |= (uint32_t)(*reinterpret_cast<int*>(E.misc() + MISC_FLAGS));
      if (a.flags) a.flags[E.e] = fl;
      if (a.iters) a.iters[E.e] = *reinterpret_cast<int*>(E.misc() + MISC_ITERS);
      if (a.fallbacks) a.fallbacks[E.e] = *reinterpret_cast<int*>(E.misc() + MISC_FB);
    }
  }
}

template <class Team, bool SOLVE = false>
SHD_FLAT void env_single_step(const Team& tm, const DevModel& M, const Env& E, bool valid, const StepArgs& a) {
  if (valid) {
    load_env_static(tm, M, E);
    load_state(tm, E, a.x_in, M.B);
    load_ws(tm, E, a.lam_in);
  }
  tm.sync();
  if (SOLVE) env_step_solve(tm, M, E, a.u, valid, a.t, nullptr);
  else env_step(tm, M, E, a.u, valid, a.t);
  tm.sync();
  uint32_t fl = valid ? nonfinite_flag(tm, E) : 0u;
  if (valid) {
    store_state(tm, E, a.x_out, M.B);
    store_ws(tm, E, a.lam_out);
    if (tm.tl == 0 && a.flags) a.flags[E.e] = fl | (uint32_t)(*reinterpret_cast<int*>(E.misc() + MISC_FLAGS));
  }
}

// loss adjoint into the adjoint record pbar of the loss body for the state
// after step t1 (1-based), p its record (the final-state kind reads the
// velocities; the others the position only); tg: the env's target (held in registers by the caller: a global
// load inside the step loop would wait for the reverse sweep's in-flight
// fetches)
SHD void loss_adj(const DevModel& M, const Env& E, int t1, const float* p, const float* tg, float dl, float* pbar) {
  if (M.loss_kind == 0) {
    if (t1 != E.T) return;
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) pbar[k] += dl * 2.f * (p[k] - tg[k]);
    return;
  }
  if (M.loss_kind == 1) {
    float d[3] = {0.f, 0.f, 0.f}, q = 0.f;
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) { d[k] = p[k] - tg[k]; q += d[k] * d[k]; }
    if (q <= 0.f) return;
    const float s = dl / (sqrtf(q) * (float)E.T);
    for (int k = 0; k < 3; ++k) pbar[k] += s * d[k];
    return;
  }
  if (t1 != E.T) return;
  if (M.loss_kind == 3) {
    for (int k = 0; k < 3; ++k)
      if (M.loss_mask & (1 << k)) pbar[k] += dl * 2.f * (p[k] - tg[k]);
    for (int k = BV; k < BW + 3; ++k) pbar[k] += dl * 2.f * p[k];
    return;
  }
  pbar[0] += -dl / ((float)E.T * M.dt);
}

// Saved working set of one step (reverse sweep without replays): the forward
// LDS region, the sweep history and the step-start angular velocities, as
// they stand after the sweeps (before integration and the impulse store).
template <class Team>
SHD void save_step(const Team& tm, const DevModel& M, const Env& E, float* dst) {
  const int nf = E.lay.total_fwd, nh = align4(M.n_iters * E.nslot);
  for (int i = tm.tl; i < nf / 4; i += tm.ts) st4(dst + 4 * i, ld4(E.L + 4 * i));
  // (with a history ring the sweeps wrote the history to dst themselves)
  const float* hs = E.L + E.lay.hist;
  const int nh4 = E.lay.hring ? 0 : nh / 4;
  for (int i = tm.tl; i < nh4; i += tm.ts) st4(dst + nf + 4 * i, ld4(hs + 4 * i));
  for (int b = tm.tl; b < E.nb; b += tm.ts)
    for (int k = 0; k < 3; ++k) dst[nf + nh + 3 * b + k] = E.bodyA(b)[AW0 + k];
}
// Copy n4 float4 from global memory to LDS, skipping float4 [s0, s1): each
// lane issues LOAD_BATCH loads before it waits for the first, so a copy costs
// a few memory round trips instead of one per float4.
constexpr int LOAD_BATCH = 20;
template <class Team>
SHD void copy_to_lds(const Team& tm, float* dst, const float* src, int n4, int s0 = 0, int s1 = 0) {
  for (int i0 = tm.tl; i0 < n4; i0 += LOAD_BATCH * tm.ts) {
    f4 v[LOAD_BATCH];
#pragma unroll
    for (int u = 0; u < LOAD_BATCH; ++u) {
      const int i = i0 + u * tm.ts;
      if (i < n4) v[u] = ld4(src + 4 * i);
    }
#pragma unroll
    for (int u = 0; u < LOAD_BATCH; ++u) {
      const int i = i0 + u * tm.ts;
      if (i < n4 && (i < s0 || i >= s1)) st4(dst + 4 * i, v[u]);
    }
  }
}
// The misc slots are not restored: the reverse keeps running totals there
// (the friction coefficient's adjoint).
template <class Team>
SHD void load_step(const Team& tm, const DevModel& M, const Env& E, const float* src) {
  const int nf = E.lay.total_fwd, nh = align4(M.n_iters * E.nslot);
  // the first body's step-start angular velocity is loaded before the copies
  const bool b0 = tm.tl < E.nb;
  float w[3] = {0.f, 0.f, 0.f};
  if (b0)
    for (int k = 0; k < 3; ++k) w[k] = src[nf + nh + 3 * tm.tl + k];
  copy_to_lds(tm, E.L, src, nf / 4, E.lay.misc / 4, (E.lay.misc + MISC_N) / 4);
  // (a history ring is filled sweep by sweep by the sweeps' reverse)
  if (!E.lay.hring) copy_to_lds(tm, E.L + E.lay.hist, src + nf, nh / 4);
  if (b0)
    for (int k = 0; k < 3; ++k) E.bodyA(tm.tl)[AW0 + k] = w[k];
  for (int b = tm.tl + tm.ts; b < E.nb; b += tm.ts) {
    const float w0 = src[nf + nh + 3 * b], w1 = src[nf + nh + 3 * b + 1], w2 = src[nf + nh + 3 * b + 2];
    float* A = E.bodyA(b);
    A[AW0] = w0; A[AW0 + 1] = w1; A[AW0 + 2] = w2;
  }
}

// Step t up to the end of its sweeps, recording what the reverse needs: the
// sweep history at hist and, with rec_w0, the step-start angular velocities
// in the adjoint body slots.  u: the control tape (null with a controller).
template <class Team>
SHD void replay_to_sweeps(const Team& tm, const DevModel& M, const Env& E, const float* u, bool act, int t,
                          float* hist, bool rec_w0) {
  f_controls(tm, M, E, (u && !M.ctrl) ? u + (size_t)t * M.J : nullptr, act, t);
  f_body_setup(tm, E, act, rec_w0);
  tm.sync();
  f_torques(tm, E, act);
  f_predict(tm, M, E, act);
  tm.sync();
  if (M.has_rest) f_save_vel(tm, E, act);
  f_rows(tm, M, E, act);
  f_warm(tm, E, act);
  f_pgs(tm, M, E, act, hist);
}

// One step of the env with its working set saved at dst (trajectory layout:
// the forward LDS region after the sweeps, the sweep history, written by the
// sweeps themselves, and the step-start angular velocities); dst is null for
// a lane whose env takes no step.
template <class Team>
SHD void recorded_step(const Team& tm, const DevModel& M, const Env& E, const float* u, bool act, int t, float* dst) {
  const int nf = E.lay.total_fwd, nh = align4(M.n_iters * E.nslot);
  if (act)
    for (int b = tm.tl; b < E.nb; b += tm.ts)
      for (int k = 0; k < 3; ++k) dst[nf + nh + 3 * b + k] = E.body(b)[BW + k];
  replay_to_sweeps(tm, M, E, u, act, t, dst ? dst + nf : nullptr, false);
  tm.sync();
  if (act)
    for (int i = tm.tl; i < nf / 4; i += tm.ts) st4(dst + 4 * i, ld4(E.L + 4 * i));
  tm.sync();   // the copy reads bodies and rows that integration rewrites
  f_integrate(tm, M, E, act);
  f_store(tm, E, act);
  tm.sync();
}

// Trajectory mode: recompute segment sg of the env from its checkpoint with
// the forward LDS layout, writing each step's working set straight into the
// env's block (the sweep history and step-start angular velocities go to
// global memory as they are produced), and, for the last segment, the loss
// body's final record after it.
template <class Team>
SHD_FLAT void env_recompute(const Team& tm, const DevModel& M, const Env& E, bool valid, const GradArgs& a, int sg) {
  const int K = M.ckpt_every;
  const int T = valid ? E.T : 0;
  const int t0 = sg * K;
  const bool live = t0 < T;
  if (live) {
    load_env_static(tm, M, E);
    read_ckpt(tm, M, E, a.ckpt + (size_t)sg * ckpt_stride(M));
  }
  tm.sync();
  const int t1 = live ? (t0 + K < T ? t0 + K : T) : 0;
  const int sstride = live ? dump_stride_of(E.lay.total_fwd, M.n_iters, E.nslot, E.nb) : 0;
  float* seg = live ? a.seg + E.seg_base() : nullptr;
  for (int t = t0; tm.any(t < t1); ++t) {
    const bool act = t < t1;
    recorded_step(tm, M, E, a.u, act, t, act ? seg + (size_t)t * sstride : nullptr);
  }
  if (live && t1 == T && tm.tl == 0)
    for (int k = 0; k < 18; ++k) seg[(size_t)T * sstride + k] = E.body(E.lb)[k];
}

// The fixed-sweep rollout of env_rollout that also writes, in trajectory
// mode, every step's saved working set to the reverse sweep's buffer a.seg as
// the recompute would (the same arithmetic: the recompute starts from the
// checkpoints this rollout writes), so that the reverse needs no recompute.
template <class Team>
SHD_FLAT void env_rollout_keep(const Team& tm, const DevModel& M, const Env& E, bool valid, const RolloutArgs& a) {
  if (valid) {
    load_env_static(tm, M, E);
    load_state(tm, E, a.x0, M.B);
    for (int i = tm.tl; i < E.lam_size; i += tm.ts) E.ws()[i] = 0.f;
  }
  tm.sync();
  float p0x = valid ? E.body(E.lb)[BP] : 0.f;
  float loss = 0.f;
  const int K = M.ckpt_every;
  const int T = valid ? E.T : 0;
  const int sstride = valid ? dump_stride_of(E.lay.total_fwd, M.n_iters, E.nslot, E.nb) : 0;
  float* seg = valid ? a.seg + E.seg_base() : nullptr;
  for (int t = 0; tm.any(t < T); ++t) {
    const bool act = t < T;
    if (act && a.ckpt && t % K == 0) write_ckpt(tm, M, E, a.ckpt + (size_t)(t / K) * ckpt_stride(M));
    tm.sync();
    recorded_step(tm, M, E, a.u, act, t, act ? seg + (size_t)t * sstride : nullptr);
    if (act && tm.tl == 0) {
      const float* p = E.body(E.lb) + BP;
      const float p0[3] = {p0x, 0.f, 0.f};
      loss += loss_term(M, E, t + 1, p, p0);
    }
  }
  if (valid && T > 0 && tm.tl == 0)
    for (int k = 0; k < 18; ++k) seg[(size_t)T * sstride + k] = E.body(E.lb)[k];
  tm.sync();
  uint32_t fl = valid ? nonfinite_flag(tm, E) : 0u;
  if (valid) {
    if (a.x_final) store_state(tm, E, a.x_final, M.B);
    if (a.lam_final) store_ws(tm, E, a.lam_final);
    if (tm.tl == 0) {
      a.loss[E.e] = loss;
      fl |= (uint32_t)(*reinterpret_cast<int*>(E.misc() + MISC_FLAGS));
      if (a.flags) a.flags[E.e] = fl;
    }
  }
}

// SAVED: the working sets are saved (segment or trajectory mode, M.dump !=
// DUMP_REPLAY), else replayed; a separate instantiation each, so neither
// carries the other's code.
template <bool SAVED, class Team>
SHD_FLAT void env_rollout_grad(const Team& tm, const DevModel& M, const Env& E, bool valid, const GradArgs& a) {
  if (valid) {
    load_env_static(tm, M, E);
    for (int i = tm.tl; i < (E.nb + 1) * BSA; i += tm.ts) E.L[E.lay.bodyA + i] = 0.f;
    for (int i = tm.tl; i < E.lam_size; i += tm.ts) E.wsA()[i] = 0.f;
    for (int i = tm.tl; i < JA_FLOATS * E.nj; i += tm.ts) E.jA()[i] = 0.f;
    if (tm.tl == 0) E.misc()[MISC_GMU] = E.misc()[MISC_GMUC] = 0.f;
  }
  tm.sync();
  const int K = M.ckpt_every;
  const int T = valid ? E.T : 0;
  const float dl = valid ? a.dloss[E.e] : 0.f;
  float tg[3] = {0.f, 0.f, 0.f};
  if (valid)
    for (int k = 0; k < 3; ++k) tg[k] = M.target[3 * E.e + k];
  const int nseg = (T + K - 1) / K;
  const bool traj = SAVED && M.dump == DUMP_TRAJECTORY;
  const int sstride = !valid ? 0 : (SAVED ? dump_stride_of(E.lay.total_fwd, M.n_iters, E.nslot, E.nb)
                                          : 18 * E.nb + E.lam_size);
  float* seg = valid ? a.seg + E.seg_base() : nullptr;
  // zero the control gradient rows beyond T (and all rows of idle envs)
  if (valid && a.g_u && !M.ctrl)
    for (int t = T; t < M.T_max; ++t)
      for (int j = tm.tl; j < E.nj; j += tm.ts) a.g_u[(size_t)t * M.J + E.j0 + j] = 0.f;
  bool bad = false;   // this lane saw a non-finite adjoint (checked after every reversed step)
  for (int sg = nseg - 1; tm.any(sg >= 0); --sg) {
    const bool sact = sg >= 0;
    const int t0 = sact ? sg * K : 0;
    const int t1 = sact ? (t0 + K < T ? t0 + K : T) : 0;
    if (sact && !traj) read_ckpt(tm, M, E, a.ckpt + (size_t)sg * ckpt_stride(M));
    tm.sync();
    // recompute the segment, keeping each step-start state, or (segment mode)
    // each step's working set after its sweeps; in trajectory mode it is done
    for (int t = t0; !traj && tm.any(t < t1); ++t) {
      const bool act = t < t1;
      if (SAVED) {
        // (with a history ring the sweeps write the history to the step's
        // saved working set directly)
        float* dst = act ? seg + (size_t)(t - t0) * sstride : nullptr;
        replay_to_sweeps(tm, M, E, a.u, act, t, E.lay.hring ? (dst ? dst + E.lay.total_fwd : nullptr) : E.hist(0),
                         true);
        if (act) save_step(tm, M, E, dst);
        tm.sync();   // the copy reads bodies and rows that integration rewrites
        f_integrate(tm, M, E, act);
        f_store(tm, E, act);
        tm.sync();
        continue;
      }
      if (act) {
        float* dst = seg + (size_t)(t - t0) * sstride;
        for (int i = tm.tl; i < 18 * E.nb; i += tm.ts) dst[i] = E.body(i / 18)[i % 18];
        for (int i = tm.tl; i < E.lam_size; i += tm.ts) dst[18 * E.nb + i] = E.ws()[i];
      }
      tm.sync();
      env_step(tm, M, E, (a.u && !M.ctrl) ? a.u + (size_t)t * M.J : nullptr, act, t);
    }
    tm.sync();
    if (sact && sg == nseg - 1 && tm.tl == 0 && M.loss_kind != 1)
      loss_adj(M, E, T, traj ? seg + (size_t)T * sstride : E.body(E.lb) + BP, tg, dl, E.bodyA(E.lb) + AP);
    tm.sync();
    // reverse the segment's steps
    for (int t = t1 - 1; tm.any(t >= t0 && sact); --t) {
      const bool act = sact && t >= t0;
      if (SAVED) {
        // the saved working set of step t replaces its replay
        if (act) load_step(tm, M, E, seg + (size_t)(traj ? t : t - t0) * sstride);
        tm.sync();
      } else {
        if (act) {
          const float* src = seg + (size_t)(t - t0) * sstride;
          for (int i = tm.tl; i < 18 * E.nb; i += tm.ts) E.body(i / 18)[i % 18] = src[i];
          for (int i = tm.tl; i < E.lam_size; i += tm.ts) E.ws()[i] = src[18 * E.nb + i];
        }
        tm.sync();
        // replay step t with recording (no integration, no store)
        replay_to_sweeps(tm, M, E, a.u, act, t, E.hist(0), true);
      }
      // gradient decay of the carry from the later steps (none before the last step)
      if (M.decay != 1.f) {
        a_decay(tm, M, E, act && t < T - 1);
        tm.sync();
      }
      // loss on x^{t+1}: p(t+1) = p(t) + dt v'
      if (act && tm.tl == 0 && M.loss_kind == 1) {
        const float* B = E.body(E.lb);
        const float p1[3] = {B[BP] + M.dt * B[BV], B[BP + 1] + M.dt * B[BV + 1], B[BP + 2] + M.dt * B[BV + 2]};
        loss_adj(M, E, t + 1, p1, tg, dl, E.bodyA(E.lb) + AP);
      }
      a_clear_step(tm, E, act);
      tm.sync();
      a_store(tm, E, act);
      a_integrate(tm, M, E, act);
      a_pgs(tm, M, E, act,
            (SAVED && act) ? seg + (size_t)(traj ? t : t - t0) * sstride + E.lay.total_fwd : nullptr);
      a_warm(tm, M, E, act);
      a_rows(tm, M, E, act);
      // an overflow can later be dropped by a clamp's or a contact's select,
      // so it is caught where it leaves the env: in the control adjoints and
      // the controller's deltas, as each lane writes them
      a_predict_torques(tm, M, E, act, (act && a.g_u && !M.ctrl) ? a.g_u + (size_t)t * M.J : nullptr, nullptr,
                        &bad);
      a_controller(tm, M, E, act, t, &bad);
    }
    tm.sync();
  }
  if (valid && M.loss_kind == 2 && T > 0 && tm.tl == 0) E.bodyA(E.lb)[AP] += dl / ((float)T * M.dt);
  tm.sync();
  // An adjoint that overflowed (the gradient of a chaotic trajectory grows
  // exponentially with the horizon) carries inf / NaN, or values beyond
  // ADJ_LIMIT, back to x0 and into the parameter totals: such an env's
  // gradient is zeroed and flagged, so that it cannot poison sums over envs.
  if (valid) {
    for (int b = tm.tl; b < E.nb; b += tm.ts) {
      const float* A = E.bodyA(b);
      for (int k = 0; k < 18; ++k) bad = bad || !(fabsf(A[k]) <= ADJ_LIMIT);
      for (int k = 0; k < 4; ++k) bad = bad || !(fabsf(A[ATM + k]) <= ADJ_LIMIT);
    }
    for (int j = tm.tl; j < E.nj; j += tm.ts) {
      bad = bad || !(fabsf(E.jA()[JA_DAMP * E.nj + j]) <= ADJ_LIMIT);
      for (int k = 0; k < 3; ++k)
        bad = bad || !(fabsf(E.jA()[JA_ANCP * E.nj + 3 * j + k]) <= ADJ_LIMIT) ||
              !(fabsf(E.jA()[JA_ANCC * E.nj + 3 * j + k]) <= ADJ_LIMIT);
    }
    if (tm.tl == 0) bad = bad || !(fabsf(E.misc()[MISC_GMU]) <= ADJ_LIMIT);
  }
  bad = tm.team_any(bad);
  if (valid) {
    for (int b = tm.tl; b < E.nb; b += tm.ts) {
      const float* A = E.bodyA(b);
      if (a.g_x0)
        for (int k = 0; k < 18; ++k) a.g_x0[(size_t)k * M.B + E.b0 + b] = bad ? 0.f : A[k];
      if (a.g_invm) a.g_invm[E.b0 + b] = bad ? 0.f : A[ATM];
      if (a.g_invI)
        for (int k = 0; k < 3; ++k) a.g_invI[3 * (E.b0 + b) + k] = bad ? 0.f : A[ATI + k];
    }
    if (a.g_damp)
      for (int j = tm.tl; j < E.nj; j += tm.ts) a.g_damp[E.j0 + j] = bad ? 0.f : E.jA()[JA_DAMP * E.nj + j];
    if (a.g_anc_p)
      for (int i = tm.tl; i < 3 * E.nj; i += tm.ts) a.g_anc_p[3 * E.j0 + i] = bad ? 0.f : E.jA()[JA_ANCP * E.nj + i];
    if (a.g_anc_c)
      for (int i = tm.tl; i < 3 * E.nj; i += tm.ts) a.g_anc_c[3 * E.j0 + i] = bad ? 0.f : E.jA()[JA_ANCC * E.nj + i];
    if (tm.tl == 0 && a.g_mu) a.g_mu[E.e] = bad ? 0.f : E.misc()[MISC_GMU];
    if (tm.tl == 0 && a.flags) a.flags[E.e] = bad ? 4u : 0u;
    if (bad && a.g_u && !M.ctrl)
      for (int t = 0; t < T; ++t)
        for (int j = tm.tl; j < E.nj; j += tm.ts) a.g_u[(size_t)t * M.J + E.j0 + j] = 0.f;
    if (bad && M.ctrl) {
      // the env's deltas leave the weight-gradient contraction
      const int c0 = tape_du(M), c1 = tape_d1(M) + M.mlp_h1;
      for (int t = 0; t < T; ++t) {
        float* row = M.tape + (size_t)(E.tape_off + t) * M.tape_stride;
        for (int c = c0 + tm.tl; c < c1; c += tm.ts) row[c] = 0.f;
      }
    }
  }
}

}  // namespace sim
