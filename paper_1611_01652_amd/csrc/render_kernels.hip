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

// The roots of |m + s d|^2 = r^2 (m = C - c) are s = t0 -/+ sqrt(D) with t0 =
// -(d . m) / a and D = (r^2 - |m + t0 d|^2) / a, a = |d|^2: the distance of
// the ray from the centre, m + t0 d, is formed first, so D does not come
// from the difference of two terms of the size |m|^2 |d|^2 (which loses
// every digit of a small D in FP32).
__device__ RHit trace(const RenderScene& sc, const float* x, int e, const Ray& ray) {
  const float a = ray.d[0] * ray.d[0] + ray.d[1] * ray.d[1] + ray.d[2] * ray.d[2];
  RHit h{-2, INFINITY};
  const int s0 = sc.env_sph[e], s1 = sc.env_sph[e + 1];
  for (int g = s0; g < s1; ++g) {
    const float4 so = sc.sph[g];
    const float o[3] = {so.x, so.y, so.z};
    float c[3];
    sphere_centre(x, sc.B, sc.sph_body[g], o, c);
    const float m0 = ray.c[0] - c[0], m1 = ray.c[1] - c[1], m2 = ray.c[2] - c[2];
    const float t0 = -(ray.d[0] * m0 + ray.d[1] * m1 + ray.d[2] * m2) / a;
    const float p0 = m0 + t0 * ray.d[0], p1 = m1 + t0 * ray.d[1], p2 = m2 + t0 * ray.d[2];
    const float D = (so.w * so.w - (p0 * p0 + p1 * p1 + p2 * p2)) / a;
    if (D < 0.f) continue;
    const float sq = sqrtf(D);
    const float s = t0 - sq >= 1.f ? t0 - sq : t0 + sq;
    if (s >= 1.f && s < h.s) { h.s = s; h.k = g - s0; }
  }
  if (sc.ground) {
    const double s = ground_s(ray);
    if (s >= 1.0 && s < (double)h.s) { h.s = (float)s; h.k = -1; }
  }
  return h;
}

__global__ __launch_bounds__(256) void k_render(RenderScene sc, const float* x, RenderCam cam, RenderTex tex,
                                                float* image) {
  const int e = blockIdx.y;
  const int n = cam.width * cam.height;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = p % cam.width, j = p / cam.width;
  const Ray ray = pixel_ray(cam, i, j);
  const RHit h = trace(sc, x, e, ray);
  float col = 0.f;
  if (h.k == -1) {
    const double sg = ground_s(ray);
    const double gu = ((double)ray.c[0] + sg * ray.d64[0]) / (double)tex.cell;
    const double gv = ((double)ray.c[1] + sg * ray.d64[1]) / (double)tex.cell;
    col = ground_sample(tex, gu, gv);
  } else if (h.k >= 0) {
    const int g = sc.env_sph[e] + h.k, b = sc.sph_body[g];
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

constexpr int kGradThreads = 64;

// One workgroup per env: thread t takes pixels t, t + 64, ...; each keeps
// its sums per sphere (12 values: the body's position 3, rotation 9) in LDS,
// then the 64 rows are added in order and the spheres' sums go to their
// bodies in sphere order.
__global__ __launch_bounds__(kGradThreads) void k_render_grad(RenderScene sc, const float* x, RenderCam cam,
                                                              RenderTex tex, const float* w, float* g_x) {
  __shared__ float acc[kGradThreads][kRenderMaxSpheres][12];
  const int e = blockIdx.x, t = threadIdx.x;
  const int n = cam.width * cam.height;
  const int s0 = sc.env_sph[e], ns = sc.env_sph[e + 1] - s0;
  for (int k = 0; k < kRenderMaxSpheres; ++k)
    for (int c = 0; c < 12; ++c) acc[t][k][c] = 0.f;
  const float kx = 0.5f * (float)(tex.snx - 1), ky = 0.5f * (float)(tex.sny - 1);
  for (int p = t; p < n; p += kGradThreads) {
    const float wt = w[(size_t)e * n + p];
    if (wt == 0.f) continue;
    const int i = p % cam.width, j = p / cam.width;
    const Ray ray = pixel_ray(cam, i, j);
    const RHit h = trace(sc, x, e, ray);
    if (h.k < 0) continue;   // the ground and the background do not depend on the state
    const int g = s0 + h.k, b = sc.sph_body[g];
    const float4 so = sc.sph[g];
    const float o[3] = {so.x, so.y, so.z};
    const float r = so.w;
    float c[3], q[3], R[9];
    sphere_centre(x, sc.B, b, o, c);
    for (int k = 0; k < 9; ++k) R[k] = x[(3 + k) * sc.B + b];
    for (int k = 0; k < 3; ++k) q[k] = ray.c[k] + h.s * ray.d[k] - c[k];
    const float lx = (R[0] * q[0] + R[3] * q[1] + R[6] * q[2]) / r;
    const float ly = (R[1] * q[0] + R[4] * q[1] + R[7] * q[2]) / r;
    float du, dv;
    (void)bilinear(tex.sphere, tex.snx, tex.sny, (lx + 1.f) * kx, (ly + 1.f) * ky, &du, &dv);
    const float lbx = wt * du * kx, lby = wt * dv * ky;
    float* A = acc[t][h.k];
    // R-bar_{k i} += q_k l-bar_i / r (i = x, y); q-bar_k = (R_k0 l-bar_x + R_k1 l-bar_y) / r
    float qb[3];
    for (int k = 0; k < 3; ++k) {
      A[3 + 3 * k] += q[k] * lbx / r;
      A[4 + 3 * k] += q[k] * lby / r;
      qb[k] = (R[3 * k] * lbx + R[3 * k + 1] * lby) / r;
    }
    // h-bar = q-bar, c-bar = -q-bar + (d . h-bar) q / (d . q)
    const float dh = ray.d[0] * qb[0] + ray.d[1] * qb[1] + ray.d[2] * qb[2];
    const float dq = ray.d[0] * q[0] + ray.d[1] * q[1] + ray.d[2] * q[2];
    float cb[3];
    for (int k = 0; k < 3; ++k) cb[k] = -qb[k] + dh * q[k] / dq;
    // c = p + R o
    for (int k = 0; k < 3; ++k) {
      A[k] += cb[k];
      for (int m = 0; m < 3; ++m) A[3 + 3 * k + m] += cb[k] * o[m];
    }
  }
  __syncthreads();
  // sums over the threads in order, per (sphere, value)
  for (int u = t; u < ns * 12; u += kGradThreads) {
    const int k = u / 12, c = u % 12;
    float s = 0.f;
    for (int r = 0; r < kGradThreads; ++r) s += acc[r][k][c];
    acc[0][k][c] = s;
  }
  __syncthreads();
  // the env's bodies: zero, then each sphere's sums added to its body in
  // sphere order (one thread per value)
  const int b0 = sc.env_body[e], b1 = sc.env_body[e + 1];
  for (int u = t; u < (b1 - b0) * 18; u += kGradThreads) {
    const int b = b0 + u / 18, c = u % 18;
    float s = 0.f;
    if (c < 12)
      for (int k = 0; k < ns; ++k)
        if (sc.sph_body[s0 + k] == b) s += acc[0][k][c];
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
