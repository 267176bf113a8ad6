// TEST INFRASTRUCTURE ONLY: the library's kernel source (step_core.h,
// drivers.h) run on the host in double precision with whole teams of lanes,
// several teams per wave, each lane a fiber (ucontext) with a stack of its
// own, all on one thread.  The lanes of a wave run one at a time: a lane runs
// until it reaches a collective (a barrier, a vote, a prefix count, a team
// reduction, the pair exchange, the wave's controller or warm-start network,
// a record reservation), and a collective is resolved once every lane of its
// scope has reached it.  Which of the lanes that may run runs next (the
// schedule) is the lowest, the highest or a seeded-random one: a lane that
// reads what another lane writes between two collectives (a missing barrier)
// gives results that depend on it.  Lanes that reach different collectives (a
// barrier under divergent control flow) are reported.  Each team's LDS region is followed by a guard region; built with
// AddressSanitizer the guards are poisoned, so an access past a region, and
// any out-of-bounds access to the global buffers (exact-size allocations),
// stops the run.  Nothing in the product loads this library.
#include <setjmp.h>
#include <ucontext.h>

#include <functional>
#include <stdexcept>

#include "host_common.h"
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/asan_interface.h>
#define KL_POISON(p, n) __asan_poison_memory_region((p), (n))
#define KL_UNPOISON(p, n) __asan_unpoison_memory_region((p), (n))
#else
#define KL_POISON(p, n) ((void)0)
#define KL_UNPOISON(p, n) ((void)0)
#endif
#include <random>

using namespace sim;
namespace {
enum Op { OP_SYNC = 1, OP_ANY, OP_PREFIX, OP_TSUM, OP_TMAX, OP_TANY, OP_SWAP, OP_CTRL_F, OP_CTRL_B, OP_WSN,
          OP_RESERVE };
struct WaveFail {};

#if defined(__SANITIZE_ADDRESS__)
#define KL_FIBER_START(save, bottom, size) __sanitizer_start_switch_fiber((save), (bottom), (size))
#define KL_FIBER_FINISH(save, bottom, size) __sanitizer_finish_switch_fiber((save), (bottom), (size))
#else
#define KL_FIBER_START(save, bottom, size) ((void)0)
#define KL_FIBER_FINISH(save, bottom, size) ((void)0)
#endif

// The lanes of one wave as fibers run one at a time by a scheduler on the
// calling thread.  A lane runs until it reaches a collective; the
// collective's scope is the wave (barrier, vote, the controller's and the
// warm-start network's wave-wide products), the lane's team (prefix count,
// team reductions, record reservation) or the lane's pair (the DPP exchange);
// the lanes of that scope wait until all of them have reached it, then it is
// resolved and they may run again.  The next lane to run is the lowest, the
// highest or a random one of those that may (the schedule).  A scope whose
// lanes reach different collectives, or lanes that can no longer all
// proceed, stop the run.
struct Wave {
  enum { READY, BLOCK, DONE };
  int n, ts, n_teams, sched;
  std::mt19937 rng;
  std::vector<int> st, op, scope;
  std::vector<double> val, res;
  std::vector<long long> ires, ires2;
  std::vector<unsigned long long> ures;
  std::vector<const DevModel*> pm;
  std::vector<const Env*> pe;
  std::vector<int> rn, wtot;
  std::vector<const int*> wmap;
  bool failed = false;
  std::string why;
  double* lds0 = nullptr;
  const double* net = nullptr;
  unsigned long long* ctr = nullptr;
  long long resolved = 0;
  // fibers: started once with swapcontext, then switched with _setjmp /
  // _longjmp (no signal-mask system call per switch)
  ucontext_t main_ctx;
  std::vector<ucontext_t> ctx;
  jmp_buf main_jb;
  std::vector<jmp_buf> lane_jb;
  std::vector<char> started;
  std::vector<std::vector<char>> stacks;
  std::vector<void*> fake;
  const void* main_bottom = nullptr;
  size_t main_size = 0;

  Wave(int n_, int ts_, int sched_, unsigned seed)
      : n(n_), ts(ts_), n_teams(n_ / ts_), sched(sched_), rng(seed), st(n_, READY), op(n_), scope(n_), val(n_),
        res(n_), ires(n_), ires2(n_), ures(n_), pm(n_), pe(n_), rn(n_), wtot(n_), wmap(n_), ctx(n_), lane_jb(n_),
        started(n_, 0), stacks(n_), fake(n_, nullptr) {}
  // scope ids: 0 the wave, 1 + t team t, 1 + n_teams + q pair q
  bool in_scope(int lane, int sc) const {
    if (sc == 0) return true;
    if (sc <= n_teams) return lane / ts == sc - 1;
    return lane / 2 == sc - 1 - n_teams;
  }
  void fail(const std::string& w) {
    if (!failed) { failed = true; why = w; }
  }
  // back to the scheduler (from a lane)
  void yield(int lane) {
    KL_FIBER_START(&fake[lane], main_bottom, main_size);
    if (!_setjmp(lane_jb[lane])) _longjmp(main_jb, 1);
    KL_FIBER_FINISH(fake[lane], &main_bottom, &main_size);
  }
  // a lane's fiber ends: back to the scheduler for good
  [[noreturn]] void finish(int lane) {
    KL_FIBER_START(nullptr, main_bottom, main_size);
    _longjmp(main_jb, 1);
  }
  // the scheduler: run lanes until all are done or none may run
  void run() {
    for (;;) {
      std::vector<int> ready;
      for (int i = 0; i < n; ++i)
        if (st[i] == READY) ready.push_back(i);
      if (failed) return;
      if (ready.empty()) {
        std::string who;
        for (int i = 0; i < n; ++i)
          if (st[i] != DONE)
            who += " lane " + std::to_string(i) + ":op " + std::to_string(op[i]) + "/scope " + std::to_string(scope[i]);
        if (!who.empty()) fail("lanes can no longer proceed (a collective reached by part of its scope):" + who);
        return;
      }
      int pick = ready.front();
      if (sched == 1) pick = ready.back();
      else if (sched == 2) pick = ready[std::uniform_int_distribution<int>(0, (int)ready.size() - 1)(rng)];
      void* save = nullptr;
      KL_FIBER_START(&save, stacks[pick].data(), stacks[pick].size());
      if (!_setjmp(main_jb)) {
        if (!started[pick]) {
          started[pick] = 1;
          swapcontext(&main_ctx, &ctx[pick]);
        } else {
          _longjmp(lane_jb[pick], 1);
        }
      }
      KL_FIBER_FINISH(save, nullptr, nullptr);
    }
  }
  double arrive(int lane, int o, int sc, double v) {
    if (failed) throw WaveFail{};
    op[lane] = o;
    scope[lane] = sc;
    val[lane] = v;
    st[lane] = BLOCK;
    bool complete = true;
    for (int i = 0; i < n && complete; ++i)
      if (in_scope(i, sc)) complete = st[i] == BLOCK && scope[i] == sc;
    if (complete) {
      for (int i = 0; i < n; ++i)
        if (in_scope(i, sc) && op[i] != o) {
          fail("lanes of a scope reached different collectives: lane " + std::to_string(lane) + " op " +
               std::to_string(o) + ", lane " + std::to_string(i) + " op " + std::to_string(op[i]));
          break;
        }
      if (!failed) {
        resolve(o, sc);
        ++resolved;
        for (int i = 0; i < n; ++i)
          if (in_scope(i, sc)) st[i] = READY;
      }
    }
    yield(lane);
    if (failed) throw WaveFail{};
    return res[lane];
  }
  void resolve(int o, int sc) {
    std::vector<int> L;
    for (int i = 0; i < n; ++i)
      if (in_scope(i, sc)) L.push_back(i);
    if (o == OP_ANY) {
      bool a = false;
      for (int i : L) a = a || val[i] != 0.0;
      for (int i : L) res[i] = a ? 1.0 : 0.0;
    } else if (o == OP_PREFIX) {
      long long c = 0;
      for (int i : L) {
        ires[i] = c;
        if (val[i] != 0.0) ++c;
      }
      for (int i : L) ires2[i] = c;
    } else if (o == OP_TSUM || o == OP_TMAX || o == OP_TANY) {
      double r = val[L[0]];
      for (size_t k = 1; k < L.size(); ++k) {
        const double x = val[L[k]];
        if (o == OP_TSUM) r += x;
        else if (o == OP_TMAX) r = std::fmax(r, x);
        else r = (r != 0.0 || x != 0.0) ? 1.0 : 0.0;
      }
      if (o == OP_TANY) r = r != 0.0 ? 1.0 : 0.0;
      for (int i : L) res[i] = r;
    } else if (o == OP_SWAP) {
      res[L[0]] = val[L[1]];
      res[L[1]] = val[L[0]];
    } else if (o == OP_CTRL_F || o == OP_CTRL_B) {
      for (int t = 0; t < n_teams; ++t) {
        const int l0 = t * ts;
        for (int l = 1; l < ts; ++l)
          if (pe[l0 + l]->L != pe[l0]->L || pe[l0 + l]->e != pe[l0]->e) {
            failed = true;
            why = "team lanes passed different envs";
            return;
          }
        if (o == OP_CTRL_F) host_ctrl_forward(*pm[l0], *pe[l0]);
        else host_ctrl_backward(*pm[l0], *pe[l0]);
      }
    } else if (o == OP_WSN) {
      for (int i = 1; i < n; ++i)
        if (wtot[i] != wtot[0] || wmap[i] != wmap[0]) { failed = true; why = "lanes passed different contact lists"; return; }
      host_wsn_rows(lds0, net, wtot[0], wmap[0]);
    } else if (o == OP_RESERVE) {
      const unsigned long long base = *ctr;
      *ctr += (unsigned long long)rn[L[0]];
      for (int i : L) ures[i] = base;
    }
  }
};

struct TeamLanes {
  int tl, ts, lane, team, n_teams;
  Wave* w;
  double* lds0 = nullptr;
  int* cnt = nullptr;
  int* map = nullptr;
  const double* net = nullptr;
  int tsc() const { return 1 + team; }                      // this lane's team scope
  int psc() const { return 1 + n_teams + lane / 2; }       // this lane's pair scope
  void sync() const { w->arrive(lane, OP_SYNC, 0, 0.0); }
  bool any(bool p) const { return w->arrive(lane, OP_ANY, 0, p ? 1.0 : 0.0) != 0.0; }
  int prefix(bool p, int& total) const {
    w->arrive(lane, OP_PREFIX, tsc(), p ? 1.0 : 0.0);
    total = (int)w->ires2[lane];
    return (int)w->ires[lane];
  }
  double team_sum(double v) const { return w->arrive(lane, OP_TSUM, tsc(), v); }
  double team_max(double v) const { return w->arrive(lane, OP_TMAX, tsc(), v); }
  bool team_any(bool p) const { return w->arrive(lane, OP_TANY, tsc(), p ? 1.0 : 0.0) != 0.0; }
  double pair_swap(double v) const {
    if (ts < 2) throw std::logic_error("pair exchange in a one-lane team");
    return w->arrive(lane, OP_SWAP, psc(), v);
  }
  void ctrl_forward(const DevModel& M, const Env& E) const {
    w->pm[lane] = &M;
    w->pe[lane] = &E;
    w->arrive(lane, OP_CTRL_F, 0, 0.0);
  }
  void ctrl_backward(const DevModel& M, const Env& E) const {
    w->pm[lane] = &M;
    w->pe[lane] = &E;
    w->arrive(lane, OP_CTRL_B, 0, 0.0);
  }
  int* shared_cnt() const { return cnt; }
  int* shared_map() const { return map; }
  void wsn_rows(int total, const int* mp) const {
    w->wtot[lane] = total;
    w->wmap[lane] = mp;
    w->arrive(lane, OP_WSN, 0, 0.0);
  }
  unsigned long long reserve(unsigned long long* ctr, int n) const {
    w->ctr = ctr;
    w->rn[lane] = tl == 0 ? n : 0;
    w->arrive(lane, OP_RESERVE, tsc(), 0.0);
    return w->ures[lane];
  }
};

constexpr int GUARD = 64;   // floats of poisoned guard after each team's LDS region

struct Launch {
  const Host* h;
  int sched = 0;
  unsigned seed = 1;
  int teams_per_wave = 2;
  long long phases = 0;
  std::string err;
};

// One lane's fiber: its arguments, and the trampoline that runs the body.
struct LaneStart {
  std::function<void(int)> fn;
  int lane;
};
void lane_entry(unsigned lo, unsigned hi) {
  LaneStart* ls = reinterpret_cast<LaneStart*>(((uintptr_t)hi << 32) | (uintptr_t)lo);
  ls->fn(ls->lane);
}

// One wave: `tile` holds the env of each team (-1: none); body(t, E, valid)
// runs every lane.  Returns false (err set) if the lanes diverged.
template <class Body>
bool run_wave(Launch& L, int team, const std::vector<int>& tile, bool adj, bool ws, const double* net, Body body) {
  const Host& h = *L.h;
  const int nt = (int)tile.size(), n = nt * team;
  int stride = 0, ccap = 1;
  for (int ie : tile)
    if (ie >= 0) {
      stride = std::max(stride, adj ? h.P.adj_of[ie] : h.P.fwd_of[ie]);
      ccap = std::max(ccap, h.P.ccap_of[ie]);
    }
  stride = (stride + 3) & ~3;
  const size_t region = (size_t)stride + GUARD;
  std::vector<double> lds((size_t)nt * region, std::nan(""));
  for (int t = 0; t < nt; ++t) KL_POISON(lds.data() + t * region + stride, GUARD * sizeof(double));
  std::vector<int> cnt(64), map((size_t)nt * ccap + 1);
  Wave w(n, team, L.sched, L.seed++);
  w.lds0 = lds.data();
  w.net = net;
  std::vector<LaneStart> starts(n);
  for (int lane = 0; lane < n; ++lane) {
    starts[lane].lane = lane;
    starts[lane].fn = [&](int ln) {
      KL_FIBER_FINISH(nullptr, &w.main_bottom, &w.main_size);
      try {
        TeamLanes t{ln % team, team, ln, ln / team, nt, &w};
        if (ws) {
          t.lds0 = lds.data();
          t.cnt = cnt.data();
          t.map = map.data();
          t.net = net;
        }
        const int ie = tile[ln / team];
        const bool valid = ie >= 0;
        // (a team without an env takes the tile's first env's layout, as on the GPU)
        Env E = make_env(h.M, valid ? ie : tile[0], lds.data() + (size_t)(ln / team) * region, h.M.n_iters, adj);
        body(t, E, valid);
      } catch (const WaveFail&) {
      } catch (const std::exception& ex) {
        w.fail(ex.what());
      }
      w.st[ln] = Wave::DONE;
      w.finish(ln);
    };
    w.stacks[lane].resize(1 << 20);
    getcontext(&w.ctx[lane]);
    w.ctx[lane].uc_stack.ss_sp = w.stacks[lane].data();
    w.ctx[lane].uc_stack.ss_size = w.stacks[lane].size();
    w.ctx[lane].uc_link = &w.main_ctx;
    const uintptr_t a = (uintptr_t)&starts[lane];
    makecontext(&w.ctx[lane], (void (*)())lane_entry, 2, (unsigned)(a & 0xffffffffu), (unsigned)(a >> 32));
  }
  w.run();
  for (int t = 0; t < nt; ++t) KL_UNPOISON(lds.data() + t * region + stride, GUARD * sizeof(double));
  L.phases += w.resolved;
  if (w.failed) {
    L.err = w.why;
    return false;
  }
  return true;
}

// Envs grouped by team width (at least `min_team`; -n: exactly n lanes) into
// tiles of teams_per_wave envs, in env order.
std::vector<std::pair<int, std::vector<int>>> make_tiles(const Launch& L, int n_envs, int min_team) {
  std::vector<std::pair<int, std::vector<int>>> tiles;
  for (int team = 1; team <= 64; team *= 2) {
    std::vector<int> ids;
    for (int e = 0; e < n_envs; ++e)
      if ((min_team < 0 ? -min_team : std::max(L.h->P.team_of[e], min_team)) == team) ids.push_back(e);
    const int per = std::max(1, std::min(L.teams_per_wave, 64 / team));
    for (size_t i = 0; i < ids.size(); i += per) {
      std::vector<int> t(per, -1);
      for (int k = 0; k < per && i + k < ids.size(); ++k) t[k] = ids[i + k];
      tiles.push_back({team, t});
    }
  }
  return tiles;
}
}  // namespace

extern "C" {
void kl_set_ring(int on) { g_force_ring = on; }
// Forward rollout, trajectory recompute (every segment) and reverse sweep of
// every env, with the given schedule (0 ascending, 1 descending, 2 random
// with `seed`), teams of at least `min_team` lanes and `teams_per_wave` envs
// per wave.  Outputs as kh_rollout_grad.  Returns the number of phases run,
// or -1 with the reason in `err` (size `err_cap`).
long long kl_rollout_grad(const sim_model_desc* d, const double* x0, const double* u, const double* dloss, double* loss,
                          double* xf, double* gx0, double* gu, double* gm, double* gI, double* gmu, double* gd,
                          double* gap, double* gac, int sched, unsigned seed, int min_team, int teams_per_wave,
                          char* err, int err_cap) {
  Host h;
  if (!make(d, h)) return -1;
  Launch L;
  L.h = &h;
  L.sched = sched;
  L.seed = seed;
  L.teams_per_wave = teams_per_wave;
  const int n_ckpt = d->T_max > 0 ? (d->T_max - 1) / d->ckpt_every + 1 : 1;
  std::vector<double> ckpt((size_t)n_ckpt * (18 * h.M.B + h.M.lam_tot)), lf(h.M.lam_tot), seg(h.P.seg_total);
  std::vector<double> tape;
  if (h.M.ctrl) {
    tape.assign((size_t)h.P.tape_rows * h.M.tape_stride, 0.0);
    h.M.W = u;
    h.M.tape = tape.data();
  }
  RolloutArgs ra{x0, u, loss, xf, lf.data(), ckpt.data(), nullptr, nullptr, nullptr, RecArgs{nullptr, 0, nullptr, 0}};
  GradArgs ga{x0, u, ckpt.data(), dloss, gx0, gu, gm, gI, gmu, gd, gap, gac, seg.data(), nullptr};
  const auto tiles = make_tiles(L, d->n_envs, min_team);
  bool ok = true;
  for (const auto& tl : tiles)
    ok = ok && run_wave(L, tl.first, tl.second, false, false, nullptr,
                        [&](TeamLanes& t, Env& E, bool valid) { env_rollout(t, h.M, E, valid, ra); });
  if (ok && h.M.dump == DUMP_TRAJECTORY) {
    int nseg = 0;
    for (int e = 0; e < d->n_envs; ++e) nseg = std::max(nseg, (d->T_env[e] + h.M.ckpt_every - 1) / h.M.ckpt_every);
    // (segments last first: the order must not matter)
    for (int sg = nseg - 1; ok && sg >= 0; --sg)
      for (const auto& tl : tiles)
        ok = ok && run_wave(L, tl.first, tl.second, false, false, nullptr,
                            [&](TeamLanes& t, Env& E, bool valid) { env_recompute(t, h.M, E, valid, ga, sg); });
  }
  for (const auto& tl : tiles)
    ok = ok && run_wave(L, tl.first, tl.second, true, false, nullptr, [&](TeamLanes& t, Env& E, bool valid) {
           if (h.M.dump != DUMP_REPLAY) env_rollout_grad<true>(t, h.M, E, valid, ga);
           else env_rollout_grad<false>(t, h.M, E, valid, ga);
         });
  if (!ok) {
    snprintf(err, err_cap, "%s", L.err.c_str());
    return -1;
  }
  if (h.M.ctrl) {
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
  return L.phases;
}

// Tolerance-mode forward rollout (plain or learned warm start) with counts and
// records, as kh_rollout_solve, on multi-lane waves.
long long kl_rollout_solve(const sim_model_desc* d, const double* x0, const double* u, double* loss, double* xf,
                           int* iters, int* fbs, double* rec, long long rec_cap, int rec_every, int sched,
                           unsigned seed, int min_team, int teams_per_wave, long long* n_rec, char* err,
                           int err_cap) {
  Host h;
  if (!make(d, h)) return -1;
  Launch L;
  L.h = &h;
  L.sched = sched;
  L.seed = seed;
  L.teams_per_wave = teams_per_wave;
  std::vector<double> lf(h.M.lam_tot), net(4867, 0.0);
  if (d->ws_kind)
    for (int p = 0; p < 4867; ++p) net[p] = bf16r(d->ws_net[p]);
  unsigned long long count = 0;
  RolloutArgs ra{x0, u, loss, xf, lf.data(), nullptr, nullptr, iters, fbs,
                 RecArgs{rec, rec_cap, &count, rec ? rec_every : 0}};
  bool ok = true;
  for (const auto& tl : make_tiles(L, d->n_envs, min_team))
    ok = ok && run_wave(L, tl.first, tl.second, false, true, net.data(),
                        [&](TeamLanes& t, Env& E, bool valid) { env_rollout<TeamLanes, true>(t, h.M, E, valid, ra); });
  if (!ok) {
    snprintf(err, err_cap, "%s", L.err.c_str());
    return -1;
  }
  *n_rec = (long long)count;
  return L.phases;
}
}
