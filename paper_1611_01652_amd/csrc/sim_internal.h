// Host <-> kernel interface inside the library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "drivers.h"

namespace sim {

// A bucket of env tiles that share one team size.
struct TileSet {
  const int* envs;   // [n_tiles * (64/TEAM)] env indices, -1 = idle team
  int n_tiles;
  int env_floats;    // LDS floats reserved per env
  int* queue;        // device counter of the persistent tile queue
  int n_seg;         // trajectory recompute: segments per tile (units = n_tiles * n_seg)
};

// One 32x32 output tile of the controller's weight-gradient contraction:
// rows i0.. of delta (M rows valid) against columns k0.. of the activations
// (K columns valid, column K is the bias).
struct WgradTile {
  int a_off, b_off, M, K, i0, k0;
};

// LDS floats after the env tiles for the controller's per-team offsets
constexpr int CTRL_SHARED = 128;

hipError_t launch_zero(int* p, int n, hipStream_t st);
hipError_t launch_ctrl_transpose(const float* W, float* Wt, int in, int n1, int n2, int no, hipStream_t st);
hipError_t launch_wgrad(const float* tape, int stride, int n_rows, int chunk, const WgradTile* tiles, int n_tiles,
                        float* partial, const int* map, int n_params, float* g, hipStream_t st);
hipError_t launch_rollout(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                          const RolloutArgs& a, hipStream_t st);
hipError_t launch_step(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds, const StepArgs& a,
                       hipStream_t st);
hipError_t launch_rollout_grad(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                               const GradArgs& a, hipStream_t st);
hipError_t launch_recompute(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                            const GradArgs& a, hipStream_t st);
hipError_t launch_rollout_keep(const DevModel& M, const TileSet& ts, int team, int grid, size_t lds,
                               const RolloutArgs& a, hipStream_t st);
hipError_t allow_large_lds(int bytes);

// the differentiable camera (render_kernels.hip)
constexpr int kRenderMaxSpheres = 16;   // spheres per env the gradient reduction holds
struct RenderScene {
  int E, B, ground;
  const int* env_sph;    // [E+1] first sphere of each env
  const int* env_body;   // [E+1] first body of each env
  const int* sph_body;   // [S] body (global index)
  const float4* sph;     // [S] offset in the body frame (x, y, z), radius (w)
};
struct RenderCam {
  float pos[3], axes[9], focal, pitch;
  int width, height;
};
struct RenderTex {
  const float* sphere;
  int snx, sny;
  const float* ground;
  int gnx, gny;
  float cell;
};
hipError_t launch_render(const RenderScene& sc, const float* x, const RenderCam& cam, const RenderTex& tex,
                         float* image, hipStream_t st);
hipError_t launch_render_grad(const RenderScene& sc, const float* x, const RenderCam& cam, const RenderTex& tex,
                              const float* w, float* g_x, hipStream_t st);

// warm-start network (wsn_kernels.hip)
int wsn_parts(long long n, int n_cu);
// LDS floats of the shared region a forward workgroup needs for the learned
// warm start with a contact list of n_list entries
int wsn_shared_floats(int n_list);
hipError_t launch_wsn_loss_grad(const uint16_t* w, const float* rec, long long stride, long long n, float huber,
                                int relative, float* partial, int n_parts, float* grad, float* loss, hipStream_t st);
hipError_t launch_wsn_forward(const uint16_t* w, const float* x, long long stride, long long n, float* y,
                              int n_cu, hipStream_t st);
hipError_t launch_wsn_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st);
hipError_t launch_wsn_to_bf16(const float* w, uint16_t* wb, hipStream_t st);
// Adam with gradient-norm clipping for any parameter vector
int adam_scratch_floats();
hipError_t launch_adam(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, float max_norm, float* scratch, float* norm_out,
                       hipStream_t st);

}  // namespace sim
