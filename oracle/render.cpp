// FP64 oracle of the differentiable camera (paper section 3.4).
//
// TEST INFRASTRUCTURE ONLY, like oracle.cpp: tests call it; the product
// library never includes, links or runs it.
//
// What it computes: a pinhole camera at C with axes (e_x right, e_y up, e_z
// the optical axis) and its projection plane at distance f.  The ray of
// pixel (i, j) of a W x H image goes from C through the pixel's centre on that
// plane, at (u, v) = ((i + 1/2 - W/2) p, (H/2 - j - 1/2) p) for a pixel pitch
// p: points C + s d with d = f e_z + u e_x + v e_y, so the plane is s = 1.
// The ray is intersected with every sphere of the env and, when the model
// has one, the ground plane z = 0; of all intersections the one closest in
// front of the projection plane (the smallest s >= 1) is kept.  Its colour
// is a bilinear sample of the object's texture (section 3.4: bilinear so that
// the image has non-zero derivatives with respect to the state): a sphere of
// centre c and radius r hit at h reads its texture at the body-frame
// direction l = R^T (h - c) / r as texel coordinates ((l_x + 1) (nx - 1) / 2,
// (l_y + 1) (ny - 1) / 2); the ground reads its texture at (h_x, h_y) / cell.
// Texel (a, b) sits at integer coordinates; indices wrap around.  A ray that
// hits nothing is 0.
//
// The gradient of L = sum over pixels of w * colour with respect to every
// body's position and rotation matrix comes from the operator-overloading
// tape of scalar.hpp through this same code; the floor of a texel
// coordinate is a constant of the tape (each bilinear piece is smooth), and
// which object a ray hits is decided on the values (the silhouettes carry no
// derivative).
#include <cmath>
#include <vector>

#include "oracle.h"
#include "scalar.hpp"

namespace orc {
namespace {

template <class S> struct P3 { S x, y, z; };
template <class S> P3<S> add(const P3<S>& a, const P3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> P3<S> sub(const P3<S>& a, const P3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> P3<S> scl(const S& s, const P3<S>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> S dotp(const P3<S>& a, const P3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// bilinear sample of an nx x ny texture (row-major, texel (a, b) at
// T[b * nx + a]) at texel coordinates (u, v), indices wrapped
template <class S>
S bilinear(const double* T, int nx, int ny, const S& u, const S& v) {
  const double fu0 = std::floor(val(u)), fv0 = std::floor(val(v));
  const S fu = u - S(fu0), fv = v - S(fv0);
  auto wrap = [](long long k, int n) { return (int)(((k % n) + n) % n); };
  const int a0 = wrap((long long)fu0, nx), a1 = wrap((long long)fu0 + 1, nx);
  const int b0 = wrap((long long)fv0, ny), b1 = wrap((long long)fv0 + 1, ny);
  const S one(1.0);
  return (one - fu) * (one - fv) * S(T[b0 * nx + a0]) + fu * (one - fv) * S(T[b0 * nx + a1]) +
         (one - fu) * fv * S(T[b1 * nx + a0]) + fu * fv * S(T[b1 * nx + a1]);
}

// The colour of one pixel of one env.  xs: the env's body states (18 per
// body: position, rotation row-major, ...); spheres of the env given by
// their body (local index), offset in the body frame and radius.
template <class S>
S pixel(const oracle_camera& cam, const std::vector<S>& xs, const std::vector<int>& sb, const double* so,
        const double* sr, int ground, const oracle_textures& tex, int i, int j) {
  const double u = (i + 0.5 - 0.5 * cam.width) * cam.pitch, v = (0.5 * cam.height - j - 0.5) * cam.pitch;
  const P3<S> C{S(cam.pos[0]), S(cam.pos[1]), S(cam.pos[2])};
  P3<S> d;
  d.x = S(cam.focal * cam.axes[6] + u * cam.axes[0] + v * cam.axes[3]);
  d.y = S(cam.focal * cam.axes[7] + u * cam.axes[1] + v * cam.axes[4]);
  d.z = S(cam.focal * cam.axes[8] + u * cam.axes[2] + v * cam.axes[5]);
  double best = INFINITY;
  int hit = -2;   // -2 nothing, -1 ground, k >= 0 sphere k
  // (which object is hit, and where its root lies, are decided on values)
  const double a = val(dotp(d, d));
  for (size_t k = 0; k < sb.size(); ++k) {
    const S* B = xs.data() + 18 * sb[k];
    const P3<S> o{S(so[3 * k]), S(so[3 * k + 1]), S(so[3 * k + 2])};
    const P3<S> c{B[0] + B[3] * o.x + B[4] * o.y + B[5] * o.z, B[1] + B[6] * o.x + B[7] * o.y + B[8] * o.z,
                  B[2] + B[9] * o.x + B[10] * o.y + B[11] * o.z};
    const P3<S> m = sub(C, c);
    const double b = val(dotp(d, m)), cc = val(dotp(m, m)) - sr[k] * sr[k];
    const double disc = b * b - a * cc;
    if (disc < 0.0) continue;
    const double s1 = (-b - std::sqrt(disc)) / a, s2 = (-b + std::sqrt(disc)) / a;
    const double s = s1 >= 1.0 ? s1 : s2;
    if (s >= 1.0 && s < best) { best = s; hit = (int)k; }
  }
  if (ground && val(d.z) != 0.0) {
    const double s = -val(C.z) / val(d.z);
    if (s >= 1.0 && s < best) { best = s; hit = -1; }
  }
  if (hit == -2) return S(0.0);
  if (hit == -1) {
    const S s = -C.z / d.z;
    const P3<S> h = add(C, scl(s, d));
    return bilinear(tex.ground, tex.ground_nx, tex.ground_ny, h.x / S(tex.ground_cell), h.y / S(tex.ground_cell));
  }
  // the sphere's root as a function of its centre: |C + s d - c|^2 = r^2
  const int k = hit;
  const S* B = xs.data() + 18 * sb[k];
  const P3<S> o{S(so[3 * k]), S(so[3 * k + 1]), S(so[3 * k + 2])};
  const P3<S> c{B[0] + B[3] * o.x + B[4] * o.y + B[5] * o.z, B[1] + B[6] * o.x + B[7] * o.y + B[8] * o.z,
                B[2] + B[9] * o.x + B[10] * o.y + B[11] * o.z};
  const P3<S> m = sub(C, c);
  const S A = dotp(d, d), Bq = dotp(d, m), Cq = dotp(m, m) - S(sr[k] * sr[k]);
  const S root = sqrt(Bq * Bq - A * Cq);
  const double s1v = (-val(Bq) - val(root)) / val(A);
  const S s = s1v >= 1.0 ? (S(0.0) - Bq - root) / A : (S(0.0) - Bq + root) / A;
  const P3<S> h = add(C, scl(s, d));
  const P3<S> q = sub(h, c);
  const S rr(sr[k]);
  // l = R^T q / r
  const S lx = (B[3] * q.x + B[6] * q.y + B[9] * q.z) / rr;
  const S ly = (B[4] * q.x + B[7] * q.y + B[10] * q.z) / rr;
  const S one(1.0);
  return bilinear(tex.sphere, tex.sphere_nx, tex.sphere_ny, (lx + one) * S(0.5 * (tex.sphere_nx - 1)),
                  (ly + one) * S(0.5 * (tex.sphere_ny - 1)));
}

struct EnvSpheres {
  std::vector<int> body;   // local body index
  std::vector<double> off, rad;
  int b0 = 0, nb = 0;
};

EnvSpheres env_spheres(const oracle_model* m, int e) {
  EnvSpheres s;
  s.b0 = m->env_body_off[e];
  s.nb = m->env_body_off[e + 1] - s.b0;
  for (int g = m->env_sphere_off[e]; g < m->env_sphere_off[e + 1]; ++g) {
    s.body.push_back(m->sphere_body[g] - s.b0);
    for (int k = 0; k < 3; ++k) s.off.push_back(m->sphere_offset[3 * g + k]);
    s.rad.push_back(m->sphere_radius[g]);
  }
  return s;
}

}  // namespace
}  // namespace orc

using namespace orc;

extern "C" {

int oracle_render(const oracle_model* m, const double* x, const oracle_camera* cam, const oracle_textures* tex,
                  double* image) {
  const int W = cam->width, H = cam->height;
  for (int e = 0; e < m->n_envs; ++e) {
    const EnvSpheres es = env_spheres(m, e);
    std::vector<double> xs(x + 18 * es.b0, x + 18 * (es.b0 + es.nb));
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i)
        image[((size_t)e * H + j) * W + i] =
            pixel<double>(*cam, xs, es.body, es.off.data(), es.rad.data(), m->ground, *tex, i, j);
  }
  return 0;
}

// g_x [B][18] (host, overwritten): dL/dx of every body's position (0..2) and
// rotation (3..11) for L = sum of w * image; the velocity entries are zero.
int oracle_render_grad(const oracle_model* m, const double* x, const oracle_camera* cam, const oracle_textures* tex,
                       const double* w, double* g_x) {
  const int W = cam->width, H = cam->height;
  Tape tp;
  tape() = &tp;
  for (int e = 0; e < m->n_envs; ++e) {
    const EnvSpheres es = env_spheres(m, e);
    for (int b = 0; b < es.nb; ++b)
      for (int k = 0; k < 18; ++k) g_x[18 * (es.b0 + b) + k] = 0.0;
    for (int j = 0; j < H; ++j)
      for (int i = 0; i < W; ++i) {
        const double wt = w[((size_t)e * H + j) * W + i];
        if (wt == 0.0) continue;
        tp.clear();
        std::vector<Var> xs(18 * es.nb);
        for (int k = 0; k < 18 * es.nb; ++k) xs[k] = Var::input(x[18 * es.b0 + k]);
        const Var col = pixel<Var>(*cam, xs, es.body, es.off.data(), es.rad.data(), m->ground, *tex, i, j);
        if (col.id < 0) continue;
        tp.adj.assign(tp.nodes.size(), 0.0);
        tp.adj[col.id] = wt;
        tp.sweep();
        for (int k = 0; k < 18 * es.nb; ++k)
          if (xs[k].id >= 0) g_x[18 * es.b0 + k] += tp.adj[xs[k].id];
      }
  }
  tape() = nullptr;
  return 0;
}

}  // extern "C"
