// gfx950 kernels of the batched rigid-body step: persistent grids of
// one-wave workgroups; each workgroup repeatedly takes a tile of envs from an
// atomic queue (tiles are pre-sorted longest first) and splits its 64 lanes
// into teams of TEAM lanes, one env per team, with the env's whole working
// set in LDS.
#include <hip/hip_runtime.h>

#include "drivers.h"
#include "sim_internal.h"

namespace sim {

struct TeamGPU {
  int tl, ts, lane;
  unsigned long long mask;
  __device__ void sync() const { __syncthreads(); }
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
};

template <int TEAM>
__device__ __forceinline__ TeamGPU make_team() {
  TeamGPU t;
  t.lane = threadIdx.x;
  t.tl = threadIdx.x % TEAM;
  t.ts = TEAM;
  const int team = threadIdx.x / TEAM;
  t.mask = TEAM == 64 ? ~0ull : (((1ull << TEAM) - 1ull) << (team * TEAM));
  return t;
}

// Take the next tile index; every lane of the wave gets the same value.
__device__ __forceinline__ int next_tile(int* queue) {
  int v = 0;
  if (threadIdx.x == 0) v = atomicAdd(queue, 1);
  return __shfl(v, 0);
}

template <int TEAM>
__global__ __launch_bounds__(64) void k_rollout(DevModel M, TileSet ts, RolloutArgs a) {
  extern __shared__ float lds[];
  const TeamGPU tm = make_team<TEAM>();
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : 0, lds + team * ts.env_floats, M.n_iters, false);
    env_rollout(tm, M, E, valid, a);
    __syncthreads();
  }
}

template <int TEAM>
__global__ __launch_bounds__(64) void k_step(DevModel M, TileSet ts, StepArgs a) {
  extern __shared__ float lds[];
  const TeamGPU tm = make_team<TEAM>();
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : 0, lds + team * ts.env_floats, M.n_iters, false);
    env_single_step(tm, M, E, valid, a);
    __syncthreads();
  }
}

template <int TEAM>
__global__ __launch_bounds__(64) void k_rollout_grad(DevModel M, TileSet ts, GradArgs a) {
  extern __shared__ float lds[];
  const TeamGPU tm = make_team<TEAM>();
  const int team = threadIdx.x / TEAM;
  constexpr int EPW = 64 / TEAM;
  for (int tile = next_tile(ts.queue); tile < ts.n_tiles; tile = next_tile(ts.queue)) {
    const int ie = ts.envs[tile * EPW + team];
    const bool valid = ie >= 0;
    Env E = make_env(M, valid ? ie : 0, lds + team * ts.env_floats, M.n_iters, true);
    env_rollout_grad(tm, M, E, valid, a);
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

hipError_t launch_zero(int* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_rollout(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                          const RolloutArgs& a, hipStream_t st) {
  SIM_DISPATCH(team, k_rollout, a)
}
hipError_t launch_step(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds, const StepArgs& a,
                       hipStream_t st) {
  SIM_DISPATCH(team, k_step, a)
}
hipError_t launch_rollout_grad(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                               const GradArgs& a, hipStream_t st) {
  SIM_DISPATCH(team, k_rollout_grad, a)
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
  SIM_ALLOW(k_rollout)
  SIM_ALLOW(k_step)
  SIM_ALLOW(k_rollout_grad)
#undef SIM_ALLOW
  return e;
}

}  // namespace sim
