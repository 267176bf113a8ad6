// gfx950 kernels of the differentiable camera (paper section 3.4): one ray
// per pixel from a pinhole through the pixel's centre on the projection
// plane, the closest intersection in front of that plane among the env's
// spheres and the ground plane, and a bilinear sample of the object's
// texture; and the reverse of that map for the gradient of sum(w * image)
// with respect to every body's position and rotation.
//
// The ray of pixel (i, j) is C + s d, d = f e_z + u e_x + v e_y with (u, v)
// = ((i + 1/2 - W/2) p, (H/2 - j - 1/2) p), so the projection plane is s = 1.
// A sphere of centre c = p_b + R_b o and radius r is hit at the smallest root
// s >= 1 of |C + s d - c|^2 = r^2; the ground z = 0 at s = -C_z / d_z.  A
// sphere's texel coordinates are ((l_x + 1) (nx - 1) / 2, (l_y + 1) (ny - 1)
// / 2) for its body-frame direction l = R_b^T (h - c) / r, the ground's
// (h_x, h_y) / cell; texel (a, b) sits at integer coordinates, indices wrap.
//
// Reverse of a sphere hit, for the pixel's weight w: the bilinear piece's
// slopes give (u-bar, v-bar); l-bar = (u-bar kx, v-bar ky, 0); R-bar +=
// q l-bar^T / r and q-bar = R l-bar / r for q = h - c; h-bar = q-bar and
// c-bar = -q-bar; the root's derivative in the centre, ds/dc = q / (d . q)
// (implicit differentiation of the sphere equation), adds (d . h-bar) q /
// (d . q) to c-bar; c = p + R o gives p-bar += c-bar, R-bar += c-bar o^T.
// Which object a ray hits is decided on values: silhouettes carry no
// derivative.  The gradient is reduced per env in a fixed order (no float
// atomics), so it is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "sim_internal.h"

namespace sim {

namespace {

struct RHit {
  int k;       // -2 nothing, -1 ground, >= 0 sphere (index within the env)
  float s;     // ray parameter of the hit
};

__device__ __forceinline__ int wrapi(int k, int n) {
  const int m = k % n;
  return m < 0 ? m + n : m;
}

// bilinear sample and its slopes in the texel coordinates
__device__ __forceinline__ float bilinear(const float* T, int nx, int ny, float u, float v, float* du, float* dv) {
  const float fu0 = floorf(u), fv0 = floorf(v);
  const float fu = u - fu0, fv = v - fv0;
  const int a0 = wrapi((int)fu0, nx), a1 = wrapi((int)fu0 + 1, nx);
  const int b0 = wrapi((int)fv0, ny), b1 = wrapi((int)fv0 + 1, ny);
  const float t00 = T[b0 * nx + a0], t10 = T[b0 * nx + a1], t01 = T[b1 * nx + a0], t11 = T[b1 * nx + a1];
  if (du) *du = (1.f - fv) * (t10 - t00) + fv * (t11 - t01);
  if (dv) *dv = (1.f - fu) * (t01 - t00) + fu * (t11 - t10);
  return (1.f - fu) * (1.f - fv) * t00 + fu * (1.f - fv) * t10 + (1.f - fu) * fv * t01 + fu * fv * t11;
}

// an integral double's index in [0, n) (fmod is exact at any magnitude)
__device__ __forceinline__ int wrapd(double k, int n) {
  double m = fmod(k, (double)n);
  if (m < 0.0) m += (double)n;
  const int r = (int)m;
  return r >= n ? 0 : r;
}

// the ground's bilinear sample at FP64 texel coordinates (far from the
// camera they reach hundreds of texels): the floor and the fractions in FP64,
// the interpolation in FP32
__device__ __forceinline__ float ground_sample(const RenderTex& tex, double u, double v) {
  const double fu0 = floor(u), fv0 = floor(v);
  const float fu = (float)(u - fu0), fv = (float)(v - fv0);
  const int a0 = wrapd(fu0, tex.gnx), a1 = (a0 + 1) % tex.gnx;
  const int b0 = wrapd(fv0, tex.gny), b1 = (b0 + 1) % tex.gny;
  const float* T = tex.ground;
  const float t00 = T[b0 * tex.gnx + a0], t10 = T[b0 * tex.gnx + a1], t01 = T[b1 * tex.gnx + a0],
              t11 = T[b1 * tex.gnx + a1];
  return (1.f - fu) * (1.f - fv) * t00 + fu * (1.f - fv) * t10 + (1.f - fu) * fv * t01 + fu * fv * t11;
}

// The ray's direction is set up in FP64 and kept in both precisions: near the
// horizon the ground's hit point moves by s / |d_z| times any rounding of
// d_z, so the ground is intersected in FP64 (a few operations per pixel);
// the spheres take the direction rounded to FP32.
struct Ray {
  float c[3], d[3];
  double d64[3];
};

__device__ __forceinline__ Ray pixel_ray(const RenderCam& cam, int i, int j) {
  const double u = ((double)i + 0.5 - 0.5 * (double)cam.width) * (double)cam.pitch;
  const double v = (0.5 * (double)cam.height - (double)j - 0.5) * (double)cam.pitch;
  Ray r;
  for (int k = 0; k < 3; ++k) {
    r.c[k] = cam.pos[k];
    r.d64[k] = (double)cam.focal * (double)cam.axes[6 + k] + u * (double)cam.axes[k] + v * (double)cam.axes[3 + k];
    r.d[k] = (float)r.d64[k];
  }
  return r;
}

// the ground's hit parameter (FP64), or a negative value when the ray is
// parallel to the ground
__device__ __forceinline__ double ground_s(const Ray& ray) {
  return ray.d64[2] != 0.0 ? -(double)ray.c[2] / ray.d64[2] : -1.0;
}

// sphere k's centre from its body's state (x: [18][B], component-major)
__device__ __forceinline__ void sphere_centre(const float* x, int B, int b, const float* o, float* c) {
  for (int r = 0; r < 3; ++r)
    c[r] = x[r * B + b] + x[(3 + 3 * r) * B + b] * o[0] + x[(4 + 3 * r) * B + b] * o[1] +
           x[(5 + 3 * r) * B + b] * o[2];
}

// Spheres [g0, g1) of env order staged in LDS: centre p + R o and radius,
// one float4 each, made once per workgroup instead of once per pixel.
__device__ __forceinline__ void stage_spheres(const RenderScene& sc, const float* x, int g0, int g1, float4* cs) {
  for (int g = g0 + (int)threadIdx.x; g < g1; g += (int)blockDim.x) {
    const float4 so = sc.sph[g];
    const float o[3] = {so.x, so.y, so.z};
    float c[3];
    sphere_centre(x, sc.B, sc.sph_body[g], o, c);
    cs[g - g0] = make_float4(c[0], c[1], c[2], so.w);
  }
}

// The roots of |m + s d|^2 = r^2 (m = C - c) are s = t0 -/+ sqrt(D) with t0 =
// -(d . m) / a and D = (r^2 - |m + t0 d|^2) / a, a = |d|^2: the distance of
// the ray from the centre, m + t0 d, is formed first, so D does not come
// from the difference of two terms of the size |m|^2 |d|^2 (which loses
// every digit of a small D in FP32).  Both quotients by a use one
// reciprocal of a per pixel (ia).  The staged spheres are tested in env
// order (index k0 + k); the first of equal nearest roots is kept.
__device__ __forceinline__ void trace_spheres(const float4* cs, int n, int k0, const Ray& ray, float ia, RHit& h) {
  for (int k = 0; k < n; ++k) {
    const float4 cc = cs[k];
    const float m0 = ray.c[0] - cc.x, m1 = ray.c[1] - cc.y, m2 = ray.c[2] - cc.z;
    const float t0 = -(ray.d[0] * m0 + ray.d[1] * m1 + ray.d[2] * m2) * ia;
    const float p0 = m0 + t0 * ray.d[0], p1 = m1 + t0 * ray.d[1], p2 = m2 + t0 * ray.d[2];
    const float D = (cc.w * cc.w - (p0 * p0 + p1 * p1 + p2 * p2)) * ia;
    if (D < 0.f) continue;
    const float sq = sqrtf(D);
    const float s = t0 - sq >= 1.f ? t0 - sq : t0 + sq;
    if (s >= 1.f && s < h.s) { h.s = s; h.k = k0 + k; }
  }
}

__device__ __forceinline__ void trace_ground(const RenderScene& sc, const Ray& ray, RHit& h) {
  if (sc.ground) {
    const double s = ground_s(ray);
    if (s >= 1.0 && s < (double)h.s) { h.s = (float)s; h.k = -1; }
  }
}

// 1 / |d|^2 of the ray
__device__ __forceinline__ float ray_ia(const Ray& ray) {
  return 1.f / (ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2]);
}

constexpr int kStage = 64;   // spheres staged in LDS at a time by k_render

// One thread per pixel, a workgroup 256 pixels of one env; the env's spheres
// are staged kStage at a time (every thread of the workgroup takes part in
// the staging, so no thread leaves before the last chunk).
__global__ __launch_bounds__(256) void k_render(RenderScene sc, const float* x, RenderCam cam, RenderTex tex,
                                                float* image) {
  __shared__ float4 cs[kStage];
  const int e = blockIdx.y;
  const int n = cam.width * cam.height;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < n;
  const Ray ray = pixel_ray(cam, live ? p % cam.width : 0, live ? p / cam.width : 0);
  const float ia = ray_ia(ray);
  RHit h{-2, INFINITY};
  const int s0 = sc.env_sph[e], s1 = sc.env_sph[e + 1];
  for (int g0 = s0; g0 < s1; g0 += kStage) {
    const int g1 = g0 + kStage < s1 ? g0 + kStage : s1;
    __syncthreads();
    stage_spheres(sc, x, g0, g1, cs);
    __syncthreads();
    trace_spheres(cs, g1 - g0, g0 - s0, ray, ia, h);
  }
  if (!live) return;
  trace_ground(sc, ray, h);
  float col = 0.f;
  if (h.k == -1) {
    const double sg = ground_s(ray);
    const double gu = ((double)ray.c[0] + sg * ray.d64[0]) / (double)tex.cell;
    const double gv = ((double)ray.c[1] + sg * ray.d64[1]) / (double)tex.cell;
    col = ground_sample(tex, gu, gv);
  } else if (h.k >= 0) {
    const int g = s0 + h.k, b = sc.sph_body[g];
    const float4 so = sc.sph[g];
    const float o[3] = {so.x, so.y, so.z};
    float c[3], q[3];
    sphere_centre(x, sc.B, b, o, c);
    for (int k = 0; k < 3; ++k) q[k] = ray.c[k] + h.s * ray.d[k] - c[k];
    // l = R^T q / r (R row-major at x[3 + 3 r + i])
    const float lx = (x[3 * sc.B + b] * q[0] + x[6 * sc.B + b] * q[1] + x[9 * sc.B + b] * q[2]) / so.w;
    const float ly = (x[4 * sc.B + b] * q[0] + x[7 * sc.B + b] * q[1] + x[10 * sc.B + b] * q[2]) / so.w;
    col = bilinear(tex.sphere, tex.snx, tex.sny, (lx + 1.f) * (0.5f * (float)(tex.snx - 1)),
                   (ly + 1.f) * (0.5f * (float)(tex.sny - 1)), nullptr, nullptr);
  }
  image[(size_t)e * n + p] = col;
}

constexpr int kGradWaves = 4;
constexpr int kGradThreads = 64 * kGradWaves;

// One workgroup of four waves per env.  In each pass the workgroup takes 256
// consecutive pixels, wave v the v-th 64 of them, one per lane.  A lane whose
// pixel shows sphere k forms that pixel's 12 terms (the body's position 3,
// rotation 9); then, for each sphere that some lane of the wave shows (in
// the order of the lowest such lane), the wave adds those lanes' terms by a
// butterfly over the 64 lanes (a fixed tree) and lane 0 adds the sums to the
// wave's row for that sphere in LDS.  At the end the four waves' rows are
// added in wave order and each sphere's sums go to its body, spheres in env
// order.  Every sum runs in an order fixed by the inputs, so the gradient is
// bitwise reproducible.
__global__ __launch_bounds__(kGradThreads) void k_render_grad(RenderScene sc, const float* x, RenderCam cam,
                                                              RenderTex tex, const float* w, float* g_x) {
  __shared__ float4 cs[kRenderMaxSpheres];
  __shared__ float acc[kGradWaves][kRenderMaxSpheres][12];
  __shared__ float tot[kRenderMaxSpheres][12];
  const int e = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int n = cam.width * cam.height;
  const int s0 = sc.env_sph[e], ns = sc.env_sph[e + 1] - s0;
  for (int u = t; u < kGradWaves * kRenderMaxSpheres * 12; u += kGradThreads) (&acc[0][0][0])[u] = 0.f;
  stage_spheres(sc, x, s0, s0 + ns, cs);
  __syncthreads();
  const float kx = 0.5f * (float)(tex.snx - 1), ky = 0.5f * (float)(tex.sny - 1);
  for (int base = 0; base < n; base += kGradThreads) {
    const int p = base + t;
    int hk = -1;
    float v[12];
    for (int c = 0; c < 12; ++c) v[c] = 0.f;
    const float wt = p < n ? w[(size_t)e * n + p] : 0.f;
    if (wt != 0.f) {
      const Ray ray = pixel_ray(cam, p % cam.width, p / cam.width);
      RHit h{-2, INFINITY};
      trace_spheres(cs, ns, 0, ray, ray_ia(ray), h);
      trace_ground(sc, ray, h);
      // the ground and the background do not depend on the state
      if (h.k >= 0) {
        hk = h.k;
        const int g = s0 + h.k, b = sc.sph_body[g];
        const float4 so = sc.sph[g];
        const float o[3] = {so.x, so.y, so.z};
        const float r = so.w;
        const float4 cc = cs[h.k];
        const float c[3] = {cc.x, cc.y, cc.z};
        float q[3], R[9];
        for (int k = 0; k < 9; ++k) R[k] = x[(3 + k) * sc.B + b];
        for (int k = 0; k < 3; ++k) q[k] = ray.c[k] + h.s * ray.d[k] - c[k];
        const float lx = (R[0] * q[0] + R[3] * q[1] + R[6] * q[2]) / r;
        const float ly = (R[1] * q[0] + R[4] * q[1] + R[7] * q[2]) / r;
        float du, dv;
        (void)bilinear(tex.sphere, tex.snx, tex.sny, (lx + 1.f) * kx, (ly + 1.f) * ky, &du, &dv);
        const float lbx = wt * du * kx, lby = wt * dv * ky;
        // R-bar_{k i} = q_k l-bar_i / r (i = x, y); q-bar_k = (R_k0 l-bar_x + R_k1 l-bar_y) / r
        float qb[3];
        for (int k = 0; k < 3; ++k) {
          v[3 + 3 * k] = q[k] * lbx / r;
          v[4 + 3 * k] = q[k] * lby / r;
          qb[k] = (R[3 * k] * lbx + R[3 * k + 1] * lby) / r;
        }
        // h-bar = q-bar, c-bar = -q-bar + (d . h-bar) q / (d . q)
        const float dh = ray.d[0] * qb[0] + ray.d[1] * qb[1] + ray.d[2] * qb[2];
        const float dq = ray.d[0] * q[0] + ray.d[1] * q[1] + ray.d[2] * q[2];
        float cb[3];
        for (int k = 0; k < 3; ++k) cb[k] = -qb[k] + dh * q[k] / dq;
        // c = p + R o
        for (int k = 0; k < 3; ++k) {
          v[k] = cb[k];
          for (int m = 0; m < 3; ++m) v[3 + 3 * k + m] += cb[k] * o[m];
        }
      }
    }
    // (wave-uniform: the ballots are the same in every lane)
    unsigned long long todo = __ballot(hk >= 0);
    while (todo) {
      const int kk = __shfl(hk, __ffsll(todo) - 1);
      const bool mine = hk == kk;
      float r[12];
      for (int c = 0; c < 12; ++c) r[c] = mine ? v[c] : 0.f;
      for (int m = 32; m >= 1; m >>= 1)
        for (int c = 0; c < 12; ++c) r[c] += __shfl_xor(r[c], m);
      if (lane == 0)
        for (int c = 0; c < 12; ++c) acc[wv][kk][c] += r[c];
      todo &= ~__ballot(mine);
    }
  }
  __syncthreads();
  for (int u = t; u < ns * 12; u += kGradThreads) {
    const int k = u / 12, c = u % 12;
    float s = acc[0][k][c];
    for (int q = 1; q < kGradWaves; ++q) s += acc[q][k][c];
    tot[k][c] = s;
  }
  __syncthreads();
  // the env's bodies: each sphere's sums added to its body in sphere order
  // (one thread per value)
  const int b0 = sc.env_body[e], b1 = sc.env_body[e + 1];
  for (int u = t; u < (b1 - b0) * 18; u += kGradThreads) {
    const int b = b0 + u / 18, c = u % 18;
    float s = 0.f;
    if (c < 12)
      for (int k = 0; k < ns; ++k)
        if (sc.sph_body[s0 + k] == b) s += tot[k][c];
    g_x[(size_t)c * sc.B + b] = s;
  }
}

}  // namespace

hipError_t launch_render(const RenderScene& sc, const float* x, const RenderCam& cam, const RenderTex& tex,
                         float* image, hipStream_t st) {
  const int n = cam.width * cam.height;
  if (sc.E == 0 || n == 0) return hipSuccess;
  const dim3 grid((n + 255) / 256, sc.E);
  hipLaunchKernelGGL(k_render, grid, dim3(256), 0, st, sc, x, cam, tex, image);
  return hipGetLastError();
}

hipError_t launch_render_grad(const RenderScene& sc, const float* x, const RenderCam& cam, const RenderTex& tex,
                              const float* w, float* g_x, hipStream_t st) {
  if (sc.E == 0) return hipSuccess;
  hipLaunchKernelGGL(k_render_grad, dim3(sc.E), dim3(kGradThreads), 0, st, sc, x, cam, tex, w, g_x);
  return hipGetLastError();
}

}  // namespace sim
