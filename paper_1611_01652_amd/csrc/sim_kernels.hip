// gfx950 kernels of the batched rigid-body step: persistent grids of
// one-wave workgroups; each workgroup repeatedly takes a tile of envs from an
// atomic queue (tiles are pre-sorted longest first) and splits its 64 lanes
// into teams of TEAM lanes, one env per team, with the env's whole working
// set in LDS.
#include <hip/hip_runtime.h>

#include "drivers.h"
#include "sim_internal.h"
#include "wsn_core.h"

namespace sim {

struct TeamGPU {
  int tl, ts, lane;
  unsigned long long mask;
  int team, n_teams;
  // learned warm start: workgroup LDS base, per-team contact counts and the
  // wave's contact list (extras-slot offsets from lds0), network image, tiles
  float* lds0;
  int *cnt, *map;
  WsnNet net;
  uint16_t *H1, *H2;
  // controller: per team, the offsets (from lds0) of its env's forward and
  // adjoint controller regions
  int* coff;
  __device__ void sync() const { __syncthreads(); }
  __device__ float team_max(float v) const {
    for (int o = ts >> 1; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, ts));
    return v;
  }
  __device__ int* shared_cnt() const { return cnt; }
  __device__ int* shared_map() const { return map; }
  // The network on the wave's `total` listed contacts, 16 per tile: inputs at
  // lds0[map[i] + XF .. +6], outputs to lds0[map[i] + XY .. +2].  Every lane
  // of the wave calls it with the same total.
  __device__ void wsn_rows(int total, const int* mp) const {
    const int kq = 4 * (lane >> 4), c16 = lane & 15;
    for (int t0 = 0; t0 < total; t0 += 16) {
      const int i = t0 + c16;
      const float* xrow = i < total ? lds0 + mp[i] + XF : nullptr;
      const floatx4 y = wsn_forward_tile(net, xrow, H1, H2, lane);
      for (int r = 0; r < 4; ++r) {
        const int i2 = t0 + kq + r;
        if (i2 < total && c16 < WSN_OUT) lds0[mp[i2] + XY + c16] = y[r];
      }
    }
  }
  // n records reserved by the team's first lane; the base index is returned
  // to every lane of the team
  __device__ unsigned long long reserve(unsigned long long* ctr, int n) const {
    unsigned long long v = 0;
    if (tl == 0 && n > 0) v = atomicAdd(ctr, (unsigned long long)n);
    const int src = lane - tl;
    const unsigned lo = __shfl((unsigned)(v & 0xffffffffull), src);
    const unsigned hi = __shfl((unsigned)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
  }
  __device__ bool any(bool p) const { return __any((int)p) != 0; }
  // exclusive prefix count of p over the team's lanes, and the team total
  __device__ int prefix(bool p, int& total) const {
    const unsigned long long b = __ballot((int)p) & mask;
    total = __popcll(b);
    return __popcll(b & ((1ull << lane) - 1ull));
  }
  __device__ float team_sum(float v) const {
    for (int o = ts >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, ts);
    return v;
  }
  __device__ bool team_any(bool p) const { return (__ballot((int)p) & mask) != 0ull; }

  // ---- the controller's layers as matrix-core products over the wave's envs
  // One layer for the envs 4g .. 4g+3 of the wave (team indices; fewer when
  // the wave has fewer):
  //   Y_r[n] = f(c[n] + sum_k X_r[k] B[k][n]),  n < N, k < K,
  // with v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4): each instruction adds one
  // k for 4 envs x 64 outputs.  Lane l feeds A = X_(l%4)[k] (xa: the
  // lane's env row in LDS) and B = B[k][n] for n = 64 p + l, and receives
  // Y_r[64 p + l] for r = 0..3 in its 4 accumulators.  B: row-major [K][N]
  // in global memory; c: bias (global) or none.  Post-op f: 0 identity,
  // 1 tanh, 2 multiply by (1 - h^2) with h at lds0[hb[r] + n].  Output to
  // lds0[yb[r] + n] for the envs with yb[r] >= 0.
  __device__ void mfma_layer(const float* xa, int K, const float* B, int N, const float* c, const int* yb, int f,
                             const int* hb) const {
    for (int p0 = 0; p0 < N; p0 += 128) {
      const int na = p0 + lane, nb = p0 + 64 + lane;
      const bool va = na < N, vb = nb < N, two = p0 + 64 < N;
      const float ca = (c && va) ? c[na] : 0.f, cb = (c && vb) ? c[nb] : 0.f;
      floatx4 ya = {ca, ca, ca, ca}, yb2 = {cb, cb, cb, cb};
      for (int k = 0; k < K; ++k) {
        const float x = xa[k];
        const float* Bk = B + (size_t)k * N;
        ya = __builtin_amdgcn_mfma_f32_4x4x1f32(x, va ? Bk[na] : 0.f, ya, 0, 0, 0);
        if (two) yb2 = __builtin_amdgcn_mfma_f32_4x4x1f32(x, vb ? Bk[nb] : 0.f, yb2, 0, 0, 0);
      }
      for (int r = 0; r < 4; ++r) {
        if (yb[r] < 0) continue;
        float y0 = ya[r], y1 = yb2[r];
        if (f == 1) { y0 = tanhf(y0); y1 = tanhf(y1); }
        if (f == 2) {
          if (va) { const float h = lds0[hb[r] + na]; y0 *= 1.f - h * h; }
          if (vb) { const float h = lds0[hb[r] + nb]; y1 *= 1.f - h * h; }
        }
        if (va) lds0[yb[r] + na] = y0;
        if (two && vb) lds0[yb[r] + nb] = y1;
      }
    }
  }
  // the group's env offsets: region offset + o for envs present, -1 else
  __device__ void ctrl_group(int g, int which, int o, int* out) const {
    for (int r = 0; r < 4; ++r) {
      const int e = 4 * g + r;
      out[r] = e < n_teams ? coff[2 * e + which] + o : -1;
    }
  }
  __device__ const float* ctrl_row(int g, int which, int o) const {
    const int e = min(4 * g + (lane & 3), n_teams - 1);
    return lds0 + coff[2 * e + which] + o;
  }
  // h1 = tanh(W1 s + b1), h2 = tanh(W2 h1 + b2), u = W3 h2 + b3 for every
  // env of the wave; the forward products read the transposed weights
  __device__ void ctrl_forward(const DevModel& M, const Env& E) const {
    if (tl == 0) { coff[2 * team] = (int)(E.mlp() - lds0); coff[2 * team + 1] = (int)(E.mlpA() - lds0); }
    __syncthreads();
    const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
    const float* b1 = M.W + n1 * in;
    const float* b2 = b1 + n1 + n2 * n1;
    const float* b3 = b2 + n2 + no * n2;
    const float* Wt1 = M.Wt;
    const float* Wt2 = Wt1 + in * n1;
    const float* Wt3 = Wt2 + n1 * n2;
    int yb[4];
    for (int g = 0; 4 * g < n_teams; ++g) {
      ctrl_group(g, 0, mo_h1(M), yb);
      mfma_layer(ctrl_row(g, 0, 0), in, Wt1, n1, b1, yb, 1, nullptr);
      __syncthreads();
      ctrl_group(g, 0, mo_h2(M), yb);
      mfma_layer(ctrl_row(g, 0, mo_h1(M)), n1, Wt2, n2, b2, yb, 1, nullptr);
      __syncthreads();
      ctrl_group(g, 0, mo_u(M), yb);
      mfma_layer(ctrl_row(g, 0, mo_h2(M)), n2, Wt3, no, b3, yb, 0, nullptr);
    }
    __syncthreads();
  }
  // d2 = (W3^T du) (1 - h2^2), d1 = (W2^T d2) (1 - h1^2), sbar = W1^T d1 for
  // every env of the wave (W rows are the K index: row-major W is B)
  __device__ void ctrl_backward(const DevModel& M, const Env& E) const {
    if (tl == 0) { coff[2 * team] = (int)(E.mlp() - lds0); coff[2 * team + 1] = (int)(E.mlpA() - lds0); }
    __syncthreads();
    const int in = M.mlp_in, n1 = M.mlp_h1, n2 = M.mlp_h2, no = M.mlp_out;
    const float* W1 = M.W;
    const float* W2 = W1 + n1 * in + n1;
    const float* W3 = W2 + n2 * n1 + n2;
    int yb[4], hb[4];
    for (int g = 0; 4 * g < n_teams; ++g) {
      ctrl_group(g, 1, mo_d2(M), yb);
      ctrl_group(g, 0, mo_h2(M), hb);
      mfma_layer(ctrl_row(g, 1, 0), no, W3, n2, nullptr, yb, 2, hb);
      __syncthreads();
      ctrl_group(g, 1, mo_d1(M), yb);
      ctrl_group(g, 0, mo_h1(M), hb);
      mfma_layer(ctrl_row(g, 1, mo_d2(M)), n2, W2, n1, nullptr, yb, 2, hb);
      __syncthreads();
      ctrl_group(g, 1, mo_sb(M), yb);
      mfma_layer(ctrl_row(g, 1, mo_d1(M)), n1, W1, in, nullptr, yb, 0, nullptr);
    }
    __syncthreads();
  }
  // the value of the other lane of this lane's pair (2m, 2m+1): a DPP
  // quad permutation [1, 0, 3, 2]; both lanes must be active
  __device__ float pair_swap(float v) const {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  }
};

template <int TEAM>
__device__ __forceinline__ TeamGPU make_team() {
  TeamGPU t;
  t.lane = threadIdx.x;
  t.tl = threadIdx.x % TEAM;
  t.ts = TEAM;
  const int team = threadIdx.x / TEAM;
  t.mask = TEAM == 64 ? ~0ull : (((1ull << TEAM) - 1ull) << (team * TEAM));
  t.team = team;
  t.n_teams = 64 / TEAM;
  t.lds0 = nullptr;
  t.cnt = t.map = nullptr;
  t.H1 = t.H2 = nullptr;
  t.coff = nullptr;
  return t;
}

// Shared region after the env tiles: the controller's per-team offsets
// (CTRL_SHARED floats, with a controller), then for the learned warm start
// (forward kernels) the network image, two activation tiles, per-team
// counts and the contact list.
__device__ __forceinline__ void setup_shared(TeamGPU& tm, const DevModel& M, float* lds, int env_floats, bool ws) {
  tm.lds0 = lds;
  float* sh = lds + tm.n_teams * env_floats;
  if (M.ctrl) {
    tm.coff = reinterpret_cast<int*>(sh);
    sh += CTRL_SHARED;
  }
  if (!ws || !M.ws_kind) return;
  tm.net = wsn_net_at(sh);
  tm.H1 = reinterpret_cast<uint16_t*>(sh + WSN_NET_FLOATS);
  tm.H2 = tm.H1 + 16 * WSN_SH;
  tm.cnt = reinterpret_cast<int*>(sh + WSN_NET_FLOATS + WSN_TILE_FLOATS);
  tm.map = tm.cnt + 64;
  wsn_stage(M.wsn, tm.net, threadIdx.x, 64);
  __syncthreads();
}

// Take the next tile index; every lane of the wave gets the same value.
__device__ __forceinline__ int next_tile(int* queue) {
  int v = 0;
  if (threadIdx.x == 0) v = atomicAdd(queue, 1);
  return __shfl(v, 0);
}

template <int TEAM, int SOLVE>
__global__ __launch_bounds__(64) void k_rollout(DevModel M, TileSet ts, RolloutArgs a) {
  extern __shared__ float lds[];
  TeamGPU tm = make_team<TEAM>();
  setup_shared(tm, M, lds, ts.env_floats, SOLVE != 0);
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    // (a team without an env takes the layout of the tile's first env, which
    // the bucket's LDS stride covers, and does no work)
    Env E = make_env(M, valid ? ie : ts.envs[tile * EPW], lds + team * ts.env_floats, M.n_iters, false);
    env_rollout<TeamGPU, SOLVE != 0>(tm, M, E, valid, a);
    __syncthreads();
  }
}

// The fixed-sweep rollout that also writes every step's saved working set
// (trajectory mode), so that the reverse sweep needs no recompute.
template <int TEAM>
__global__ __launch_bounds__(64) void k_rollout_keep(DevModel M, TileSet ts, RolloutArgs a) {
  extern __shared__ float lds[];
  TeamGPU tm = make_team<TEAM>();
  setup_shared(tm, M, lds, ts.env_floats, false);
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : ts.envs[tile * EPW], lds + team * ts.env_floats, M.n_iters, false);
    env_rollout_keep(tm, M, E, valid, a);
    __syncthreads();
  }
}

template <int TEAM, int SOLVE>
__global__ __launch_bounds__(64) void k_step(DevModel M, TileSet ts, StepArgs a) {
  extern __shared__ float lds[];
  TeamGPU tm = make_team<TEAM>();
  setup_shared(tm, M, lds, ts.env_floats, SOLVE != 0);
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : ts.envs[tile * EPW], lds + team * ts.env_floats, M.n_iters, false);
    env_single_step<TeamGPU, SOLVE != 0>(tm, M, E, valid, a);
    __syncthreads();
  }
}

template <int TEAM, int SAVED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rollout_grad(DevModel M, TileSet ts, GradArgs a) {
  extern __shared__ float lds[];
  TeamGPU tm = make_team<TEAM>();
  setup_shared(tm, M, lds, ts.env_floats, false);
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : ts.envs[tile * EPW], lds + team * ts.env_floats, M.n_iters, true);
    env_rollout_grad<SAVED != 0>(tm, M, E, valid, a);
    __syncthreads();
  }
}

// Trajectory-mode recompute: the work units are (segment, tile) pairs, all
// segments of all tiles at once, each team recomputing one segment of one env
// from its checkpoint with the forward LDS layout.
template <int TEAM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_recompute(DevModel M, TileSet ts, GradArgs a) {
  extern __shared__ float lds[];
  TeamGPU tm = make_team<TEAM>();
  setup_shared(tm, M, lds, ts.env_floats, false);
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  const int n_units = ts.n_tiles * ts.n_seg;
  for (int u = next_tile(ts.queue); u < n_units; u = next_tile(ts.queue)) {
    const int sg = u / ts.n_tiles, tile = u - sg * ts.n_tiles;
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : ts.envs[tile * EPW], lds + team * ts.env_floats, M.n_iters, false);
    env_recompute(tm, M, E, valid, a, sg);
    __syncthreads();
  }
}

// Weight gradient of the controller as a contraction over env-steps:
//   dW_l[i][k] = sum_n delta_l[n][i] * act_l[n][k],  db_l[i] = sum_n delta_l[n][i]
// (act_1 = s, act_2 = h1, act_3 = h2; delta_1 = d1, delta_2 = d2, delta_3 = du).
// One wave computes one 32x32 output tile of one layer over one chunk of
// env-steps with v_mfma_f32_32x32x2f32 (A = delta rows, B = activations with
// an all-ones column for the bias), and writes the partial tile; the chunks
// are summed in a fixed order by k_wgrad_reduce (no atomics).
typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(64) void k_wgrad_mfma(const float* __restrict__ tape, int stride, int n_rows, int chunk,
                                                   const WgradTile* __restrict__ tiles, int n_tiles,
                                                   float* __restrict__ partial) {
  const int tile = blockIdx.x, c = blockIdx.y, lane = threadIdx.x;
  const WgradTile T = tiles[tile];
  const int li = lane & 31, lk = lane >> 5;
  const int i = T.i0 + li, j = T.k0 + li;
  const bool ia = i < T.M;
  const bool jb = j < T.K;
  const float one = (j == T.K) ? 1.f : 0.f;
  const int n0 = c * chunk;
  const int n1 = min(n_rows, n0 + chunk);
  floatx16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int n = n0; n < n1; n += 2) {
    const int row = n + lk;
    float a = 0.f, b = 0.f;
    if (row < n1) {
      const float* rp = tape + (size_t)row * stride;
      a = ia ? rp[T.a_off + i] : 0.f;
      b = jb ? rp[T.b_off + j] : one;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
  // D[row][col], col = lane % 32, row = 8 (r / 4) + 4 (lane / 32) + r % 4
  float* out = partial + ((size_t)c * n_tiles + tile) * 1024;
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r >> 2) + 4 * lk + (r & 3);
    out[row * 32 + li] = acc[r];
  }
}

__global__ void k_wgrad_reduce(const float* __restrict__ partial, int n_chunks, int n_tiles,
                               const int* __restrict__ map, int n_params, float* __restrict__ g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_params) return;
  const int m = map[p];
  float acc = 0.f, comp = 0.f;
  for (int c = 0; c < n_chunks; ++c) kahan_add(&acc, &comp, partial[(size_t)c * n_tiles * 1024 + m]);
  g[p] = acc;
}

hipError_t launch_wgrad(const float* tape, int stride, int n_rows, int chunk, const WgradTile* tiles, int n_tiles,
                        float* partial, const int* map, int n_params, float* g, hipStream_t st) {
  const int n_chunks = (n_rows + chunk - 1) / chunk;
  if (n_chunks > 0) {
    hipLaunchKernelGGL(k_wgrad_mfma, dim3(n_tiles, n_chunks), dim3(64), 0, st, tape, stride, n_rows, chunk, tiles,
                       n_tiles, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((n_params + 255) / 256), dim3(256), 0, st, partial, n_chunks, n_tiles,
                     map, n_params, g);
  return hipGetLastError();
}

// Transposed controller weights for the forward products: Wt_l[k][n] = W_l[n][k].
__global__ void k_ctrl_transpose(const float* W, float* Wt, int in, int n1, int n2, int no) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int s1 = n1 * in, s2 = n2 * n1, s3 = no * n2;
  if (p < s1) {
    const int k = p / n1, n = p - k * n1;           // Wt1[k][n], k < in
    Wt[p] = W[n * in + k];
  } else if (p < s1 + s2) {
    const int q = p - s1, k = q / n2, n = q - k * n2;   // Wt2[k][n], k < n1
    Wt[p] = W[s1 + n1 + n * n1 + k];
  } else if (p < s1 + s2 + s3) {
    const int q = p - s1 - s2, k = q / no, n = q - k * no;   // Wt3[k][n], k < n2
    Wt[p] = W[s1 + n1 + s2 + n2 + n * n2 + k];
  }
}
hipError_t launch_ctrl_transpose(const float* W, float* Wt, int in, int n1, int n2, int no, hipStream_t st) {
  const int n = n1 * in + n2 * n1 + no * n2;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctrl_transpose, dim3((n + 255) / 256), dim3(256), 0, st, W, Wt, in, n1, n2, no);
  return hipGetLastError();
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ launchers
template <int TEAM, class Args, class K>
static hipError_t launch_one(K kern, const DevModel& M, const TileSet& ts, const Args& a, int grid, size_t lds,
                             hipStream_t st) {
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, st, M, ts, a);
  return hipGetLastError();
}

#define SIM_DISPATCH(TEAMV, KNAME, ARGS)                                                        \
  switch (TEAMV) {                                                                              \
    case 1: return launch_one<1>(KNAME<1>, M, ts, ARGS, grid, lds, st);                         \
    case 2: return launch_one<2>(KNAME<2>, M, ts, ARGS, grid, lds, st);                         \
    case 4: return launch_one<4>(KNAME<4>, M, ts, ARGS, grid, lds, st);                         \
    case 8: return launch_one<8>(KNAME<8>, M, ts, ARGS, grid, lds, st);                         \
    case 16: return launch_one<16>(KNAME<16>, M, ts, ARGS, grid, lds, st);                      \
    case 32: return launch_one<32>(KNAME<32>, M, ts, ARGS, grid, lds, st);                      \
    case 64: return launch_one<64>(KNAME<64>, M, ts, ARGS, grid, lds, st);                      \
    default: return hipErrorInvalidValue;                                                       \
  }
// forward kernels: instantiated for the fixed-sweep (S = 0) and the tolerance (S = 1) solve
#define SIM_DISPATCH_S(TEAMV, KNAME, ARGS, S)                                                   \
  switch (TEAMV) {                                                                              \
    case 1: return launch_one<1>(KNAME<1, S>, M, ts, ARGS, grid, lds, st);                      \
    case 2: return launch_one<2>(KNAME<2, S>, M, ts, ARGS, grid, lds, st);                      \
    case 4: return launch_one<4>(KNAME<4, S>, M, ts, ARGS, grid, lds, st);                      \
    case 8: return launch_one<8>(KNAME<8, S>, M, ts, ARGS, grid, lds, st);                      \
    case 16: return launch_one<16>(KNAME<16, S>, M, ts, ARGS, grid, lds, st);                   \
    case 32: return launch_one<32>(KNAME<32, S>, M, ts, ARGS, grid, lds, st);                   \
    case 64: return launch_one<64>(KNAME<64, S>, M, ts, ARGS, grid, lds, st);                   \
    default: return hipErrorInvalidValue;                                                       \
  }

hipError_t launch_zero(int* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_rollout(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                          const RolloutArgs& a, hipStream_t st) {
  if (M.solve_mode) { SIM_DISPATCH_S(team, k_rollout, a, 1) }
  SIM_DISPATCH_S(team, k_rollout, a, 0)
}
hipError_t launch_step(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds, const StepArgs& a,
                       hipStream_t st) {
  if (M.solve_mode) { SIM_DISPATCH_S(team, k_step, a, 1) }
  SIM_DISPATCH_S(team, k_step, a, 0)
}
hipError_t launch_rollout_grad(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                               const GradArgs& a, hipStream_t st) {
  if (M.dump != DUMP_REPLAY) { SIM_DISPATCH_S(team, k_rollout_grad, a, 1) }
  SIM_DISPATCH_S(team, k_rollout_grad, a, 0)
}
hipError_t launch_recompute(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                            const GradArgs& a, hipStream_t st) {
  SIM_DISPATCH(team, k_recompute, a)
}
hipError_t launch_rollout_keep(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                               const RolloutArgs& a, hipStream_t st) {
  SIM_DISPATCH(team, k_rollout_keep, a)
}

template <class K>
static hipError_t allow_lds(K kern, int bytes) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
hipError_t allow_large_lds(int bytes) {
  hipError_t e = hipSuccess;
#define SIM_ALLOW(K)                                                                            \
  if ((e = allow_lds(K<1>, bytes)) != hipSuccess) return e;                                     \
  if ((e = allow_lds(K<2>, bytes)) != hipSuccess) return e;                                     \
  if ((e = allow_lds(K<4>, bytes)) != hipSuccess) return e;                                     \
  if ((e = allow_lds(K<8>, bytes)) != hipSuccess) return e;                                     \
  if ((e = allow_lds(K<16>, bytes)) != hipSuccess) return e;                                    \
  if ((e = allow_lds(K<32>, bytes)) != hipSuccess) return e;                                    \
  if ((e = allow_lds(K<64>, bytes)) != hipSuccess) return e;
#define SIM_ALLOW_S(K, S)                                                                       \
  if ((e = allow_lds(K<1, S>, bytes)) != hipSuccess) return e;                                  \
  if ((e = allow_lds(K<2, S>, bytes)) != hipSuccess) return e;                                  \
  if ((e = allow_lds(K<4, S>, bytes)) != hipSuccess) return e;                                  \
  if ((e = allow_lds(K<8, S>, bytes)) != hipSuccess) return e;                                  \
  if ((e = allow_lds(K<16, S>, bytes)) != hipSuccess) return e;                                 \
  if ((e = allow_lds(K<32, S>, bytes)) != hipSuccess) return e;                                 \
  if ((e = allow_lds(K<64, S>, bytes)) != hipSuccess) return e;
  SIM_ALLOW_S(k_rollout, 0)
  SIM_ALLOW_S(k_rollout, 1)
  SIM_ALLOW_S(k_step, 0)
  SIM_ALLOW_S(k_step, 1)
  SIM_ALLOW_S(k_rollout_grad, 0)
  SIM_ALLOW_S(k_rollout_grad, 1)
  SIM_ALLOW(k_recompute)
  SIM_ALLOW(k_rollout_keep)
#undef SIM_ALLOW
#undef SIM_ALLOW_S
  return e;
}

}  // namespace sim
