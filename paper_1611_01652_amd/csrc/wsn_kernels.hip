// Training and batch inference of the per-contact warm-start network on
// matrix cores (bfloat16 operands, FP32 accumulation).
//
// k_wsn_loss_grad: each one-wave workgroup takes 16-record tiles, runs the
// forward pass, the adjoint of the mean (Huber) loss and the backward pass,
// and accumulates its share of the weight gradient in registers:
//   dY  = 2 clamp(Y - T, -h, h) / N          (T: converged impulses over their
//                                             masses, optionally minus the carried ones)
//   gW3 = dY^T H2,  dZ2 = (dY W3) . [H2 > 0]
//   gW2 = dZ2^T H1, dZ1 = (dZ2 W2) . [H1 > 0]
//   gW1 = dZ1^T [X 1]                         (the ones column gives gb1)
//   gb2, gb3: column sums of dZ2, dY
// Every product is a 16x16x16 bf16 MFMA; the operands whose k index runs over
// the records of the tile are kept transposed in LDS so that each lane reads
// four consecutive k.  Each workgroup writes its partial gradient and loss;
// k_wsn_reduce sums the partials in a fixed order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sim_internal.h"
#include "wsn_core.h"

namespace sim {

enum { WSN_ST = 20 };   // row stride of [*][16] bf16 tiles (16 used)

struct WsnTrainLds {
  WsnNet net;
  uint16_t* W3T;   // [64][WSN_ST]: W3T[h][o] = W3[o][h], o < 3
  uint16_t* W2T;   // [64][WSN_SH]: W2T[i][o] = W2[o][i]
  uint16_t* XT;    // [16][WSN_ST]: input k (7 = ones) x record
  uint16_t *H1, *H2, *DZ2;            // [16][WSN_SH]: record x unit
  uint16_t *H1T, *H2T, *DZ2T, *DZ1T;  // [64][WSN_ST]: unit x record
  uint16_t *DY, *DYT;                 // [16][WSN_ST]
};
enum { WSN_TRAIN_FLOATS = WSN_NET_FLOATS + (64 * WSN_ST + 64 * WSN_SH + 16 * WSN_ST + 3 * 16 * WSN_SH +
                                            4 * 64 * WSN_ST + 2 * 16 * WSN_ST) / 2 };

__device__ inline WsnTrainLds wsn_train_at(float* p) {
  WsnTrainLds L;
  L.net = wsn_net_at(p);
  uint16_t* q = reinterpret_cast<uint16_t*>(p + WSN_NET_FLOATS);
  L.W3T = q; q += 64 * WSN_ST;
  L.W2T = q; q += 64 * WSN_SH;
  L.XT = q; q += 16 * WSN_ST;
  L.H1 = q; q += 16 * WSN_SH;
  L.H2 = q; q += 16 * WSN_SH;
  L.DZ2 = q; q += 16 * WSN_SH;
  L.H1T = q; q += 64 * WSN_ST;
  L.H2T = q; q += 64 * WSN_ST;
  L.DZ2T = q; q += 64 * WSN_ST;
  L.DZ1T = q; q += 64 * WSN_ST;
  L.DY = q; q += 16 * WSN_ST;
  L.DYT = q;
  return L;
}

// column sum over the 16 rows of a D fragment (result valid in lanes 0..15)
__device__ __forceinline__ float col_sum(floatx4 d) {
  float s = (d[0] + d[1]) + (d[2] + d[3]);
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

__global__ __launch_bounds__(64) void k_wsn_loss_grad(const uint16_t* __restrict__ w, const float* __restrict__ rec,
                                                      long long stride, long long n, float inv_n, float huber,
                                                      int relative, float* __restrict__ partial) {
  extern __shared__ float lds[];
  const WsnTrainLds L = wsn_train_at(lds);
  const int lane = threadIdx.x, kq = 4 * (lane >> 4), c16 = lane & 15;
  wsn_stage(w, L.net, lane, 64);
  for (int i = lane; i < 64 * WSN_ST; i += 64) {
    const int h = i / WSN_ST, o = i % WSN_ST;
    L.W3T[i] = o < WSN_OUT ? w[WSN_W3 + o * 64 + h] : (uint16_t)0;
  }
  for (int i = lane; i < 64 * WSN_SH; i += 64) {
    const int a = i / WSN_SH, b = i % WSN_SH;
    L.W2T[i] = b < 64 ? w[WSN_W2 + b * 64 + a] : (uint16_t)0;
  }
  __syncthreads();
  floatx4 g1[4], g2[4][4], g3[4];
  for (int i = 0; i < 4; ++i) {
    g1[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    g3[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 4; ++j) g2[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  float gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f, loss = 0.f;
  const long long n_tiles = (n + 15) / 16;
  for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const long long r0 = tile * 16;
    // inputs: A operand of row l % 16, and the transposed copy with the ones column
    const long long my = r0 + c16;
    const float* xrow = my < n ? rec + my * stride : nullptr;
    bf16x4 a0[1] = {wsn_input_operand(xrow, lane)};
    {
      const int k = lane & 15, s0 = 4 * (lane >> 4);   // input k, records s0..s0+3
      for (int j = 0; j < 4; ++j) {
        const long long s = r0 + s0 + j;
        float v = 0.f;
        if (s < n) v = k < WSN_IN ? rec[s * stride + k] : (k == WSN_IN ? 1.f : 0.f);
        L.XT[k * WSN_ST + s0 + j] = f2bf(v);
      }
    }
    // forward
    wsn_hidden<1>(a0, L.net.W1, WSN_S1, L.net.b1, L.H1, lane);
    __syncthreads();
    bf16x4 a[4];
    wsn_tile_operands(L.H1, lane, a);
    wsn_hidden<4>(a, L.net.W2, WSN_SH, L.net.b2, L.H2, lane);
    __syncthreads();
    for (int i = lane; i < 16 * 64; i += 64) {   // transposed hidden tiles
      const int s = i / 64, h = i % 64;
      L.H1T[h * WSN_ST + s] = L.H1[s * WSN_SH + h];
      L.H2T[h * WSN_ST + s] = L.H2[s * WSN_SH + h];
    }
    wsn_tile_operands(L.H2, lane, a);
    floatx4 y = {0.f, 0.f, 0.f, 0.f};
    {
      const uint16_t* wr = L.net.W3 + c16 * WSN_SH + kq;
      for (int ks = 0; ks < 4; ++ks) y = mfma16(a[ks], ld_bf4(wr + 16 * ks), y);
    }
    // loss and output adjoint (rows kq + r, column c16)
    floatx4 dy;
    for (int r = 0; r < 4; ++r) {
      const long long s = r0 + kq + r;
      float d = 0.f;
      if (s < n && c16 < WSN_OUT) {
        const float* q = rec + s * stride;
        const float t = q[WSN_IN + c16] - (relative ? q[4 + c16] : 0.f);
        const float e = y[r] + L.net.b3[c16] - t;
        if (huber > 0.f && fabsf(e) > huber) {
          loss += 2.f * huber * fabsf(e) - huber * huber;
          d = 2.f * copysignf(huber, e) * inv_n;
        } else {
          loss += e * e;
          d = 2.f * e * inv_n;
        }
      }
      dy[r] = d;
      const uint16_t hb = f2bf(d);
      L.DY[(kq + r) * WSN_ST + c16] = hb;
      L.DYT[c16 * WSN_ST + kq + r] = hb;
    }
    gb3 += col_sum(dy);
    __syncthreads();
    // gW3 += dY^T H2 (rows: outputs, columns: hidden units, k: records)
    {
      const bf16x4 at = ld_bf4(L.DYT + c16 * WSN_ST + kq);
      for (int ct = 0; ct < 4; ++ct) g3[ct] = mfma16(at, ld_bf4(L.H2T + (16 * ct + c16) * WSN_ST + kq), g3[ct]);
    }
    // dZ2 = (dY W3) . [H2 > 0]
    {
      const bf16x4 ad = ld_bf4(L.DY + c16 * WSN_ST + kq);
      for (int ct = 0; ct < 4; ++ct) {
        floatx4 z = {0.f, 0.f, 0.f, 0.f};
        z = mfma16(ad, ld_bf4(L.W3T + (16 * ct + c16) * WSN_ST + kq), z);
        const int col = 16 * ct + c16;
        for (int r = 0; r < 4; ++r) {
          if (!(bf2f(L.H2[(kq + r) * WSN_SH + col]) > 0.f)) z[r] = 0.f;
          const uint16_t hb = f2bf(z[r]);
          L.DZ2[(kq + r) * WSN_SH + col] = hb;
          L.DZ2T[col * WSN_ST + kq + r] = hb;
        }
        gb2[ct] += col_sum(z);
      }
    }
    __syncthreads();
    // gW2 += dZ2^T H1
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x4 at = ld_bf4(L.DZ2T + (16 * mt + c16) * WSN_ST + kq);
      for (int nt = 0; nt < 4; ++nt)
        g2[mt][nt] = mfma16(at, ld_bf4(L.H1T + (16 * nt + c16) * WSN_ST + kq), g2[mt][nt]);
    }
    // dZ1 = (dZ2 W2) . [H1 > 0]
    wsn_tile_operands(L.DZ2, lane, a);
    for (int ct = 0; ct < 4; ++ct) {
      floatx4 z = {0.f, 0.f, 0.f, 0.f};
      const uint16_t* wr = L.W2T + (16 * ct + c16) * WSN_SH + kq;
      for (int ks = 0; ks < 4; ++ks) z = mfma16(a[ks], ld_bf4(wr + 16 * ks), z);
      const int col = 16 * ct + c16;
      for (int r = 0; r < 4; ++r) {
        if (!(bf2f(L.H1[(kq + r) * WSN_SH + col]) > 0.f)) z[r] = 0.f;
        L.DZ1T[col * WSN_ST + kq + r] = f2bf(z[r]);
      }
    }
    __syncthreads();
    // gW1 (+ gb1 in input column 7) += dZ1^T [X 1]
    {
      const bf16x4 bx = ld_bf4(L.XT + c16 * WSN_ST + kq);
      for (int mt = 0; mt < 4; ++mt) g1[mt] = mfma16(ld_bf4(L.DZ1T + (16 * mt + c16) * WSN_ST + kq), bx, g1[mt]);
    }
    __syncthreads();
  }
  // partial gradient in the packed parameter order, then the loss
  float* out = partial + (size_t)blockIdx.x * (WSN_PARAMS + 1);
  for (int mt = 0; mt < 4; ++mt)
    for (int r = 0; r < 4; ++r) {
      const int h = 16 * mt + kq + r;
      if (c16 < WSN_IN) out[WSN_W1 + h * WSN_IN + c16] = g1[mt][r];
      else if (c16 == WSN_IN) out[WSN_B1 + h] = g1[mt][r];
      for (int nt = 0; nt < 4; ++nt) out[WSN_W2 + h * 64 + 16 * nt + c16] = g2[mt][nt][r];
    }
  for (int ct = 0; ct < 4; ++ct)
    for (int r = 0; r < 4; ++r)
      if (kq + r < WSN_OUT) out[WSN_W3 + (kq + r) * 64 + 16 * ct + c16] = g3[ct][r];
  if (lane < 16)
    for (int ct = 0; ct < 4; ++ct) out[WSN_B2 + 16 * ct + lane] = gb2[ct];
  if (lane < WSN_OUT) out[WSN_B3 + lane] = gb3;
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o);
  if (lane == 0) out[WSN_PARAMS] = loss * inv_n;
}

__global__ void k_wsn_reduce(const float* __restrict__ partial, int n_parts, float* __restrict__ grad,
                             float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > WSN_PARAMS) return;
  float s = 0.f;
  for (int i = 0; i < n_parts; ++i) s += partial[(size_t)i * (WSN_PARAMS + 1) + p];
  if (p < WSN_PARAMS) {
    if (grad) grad[p] = s;
  } else if (loss) {
    *loss = s;
  }
}

__global__ __launch_bounds__(64) void k_wsn_forward(const uint16_t* __restrict__ w, const float* __restrict__ x,
                                                    long long stride, long long n, float* __restrict__ y) {
  extern __shared__ float lds[];
  const WsnNet net = wsn_net_at(lds);
  uint16_t* H1 = reinterpret_cast<uint16_t*>(lds + WSN_NET_FLOATS);
  uint16_t* H2 = H1 + 16 * WSN_SH;
  const int lane = threadIdx.x, kq = 4 * (lane >> 4), c16 = lane & 15;
  wsn_stage(w, net, lane, 64);
  __syncthreads();
  const long long n_tiles = (n + 15) / 16;
  for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const long long r0 = tile * 16, my = r0 + c16;
    const floatx4 o = wsn_forward_tile(net, my < n ? x + my * stride : nullptr, H1, H2, lane);
    for (int r = 0; r < 4; ++r) {
      const long long s = r0 + kq + r;
      if (s < n && c16 < WSN_OUT) y[s * WSN_OUT + c16] = o[r];
    }
  }
}

__global__ void k_wsn_adam(float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= WSN_PARAMS) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float wp = w[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
  w[p] = wp;
  wb[p] = f2bf(wp);
}

__global__ void k_wsn_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) wb[p] = f2bf(w[p]);
}

// ------------------------------------------------------------------ Adam for any parameter vector
// |g| in two fixed-order passes that cannot overflow: per block the largest
// |g_i| (m_b) and the sum of (g_i / m_b)^2 (s_b); then one thread combines
// |g| = M sqrt(sum_b s_b (m_b / M)^2), M = max_b m_b, and writes the clip scale
// min(1, max_norm / |g|) (0 for a non-finite gradient: the step is skipped).
__global__ void k_sq_partial(const float* __restrict__ g, long long n, float* __restrict__ part) {
  __shared__ float sh[256];
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    m = fmaxf(m, fabsf(g[i]) <= 3.0e38f ? fabsf(g[i]) : __builtin_inff());
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const float mb = sh[0];
  __syncthreads();
  float s = 0.f;
  if (mb > 0.f && mb <= 3.0e38f)
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
      const float q = g[i] / mb;
      s += q * q;
    }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = mb;
    part[2 * blockIdx.x + 1] = sh[0];
  }
}

__global__ void k_clip_scale(float* __restrict__ part, int n_part, float max_norm, float* __restrict__ norm_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float M = 0.f;
  for (int i = 0; i < n_part; ++i) M = fmaxf(M, part[2 * i]);
  float s = 0.f;
  if (M > 0.f && M <= 3.0e38f)
    for (int i = 0; i < n_part; ++i) {
      const float r = part[2 * i] / M;
      s += part[2 * i + 1] * r * r;
    }
  const float nrm = M <= 3.0e38f ? M * sqrtf(s) : M;
  float sc = 1.f;
  if (!(nrm <= 3.0e38f)) sc = 0.f;
  else if (max_norm > 0.f && nrm > max_norm) sc = max_norm / nrm;
  part[2 * n_part] = sc;
  if (norm_out) *norm_out = nrm;
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, const float* __restrict__ scale, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float sc = scale ? *scale : 1.f;
  if (sc == 0.f) return;
  const float gp = g[p] * sc;
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  w[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

// ------------------------------------------------------------------ launchers
int wsn_parts(long long n, int n_cu) {
  const long long tiles = (n + 15) / 16;
  return (int)std::max<long long>(1, std::min<long long>(tiles, 2LL * n_cu));
}

hipError_t launch_wsn_loss_grad(const uint16_t* w, const float* rec, long long stride, long long n, float huber,
                                int relative, float* partial, int n_parts, float* grad, float* loss, hipStream_t st) {
  const size_t lds = WSN_TRAIN_FLOATS * sizeof(float);
  if (n > 0) {
    hipLaunchKernelGGL(k_wsn_loss_grad, dim3(n_parts), dim3(64), lds, st, w, rec, stride, n, 1.f / (float)n, huber,
                       relative, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_wsn_reduce, dim3((WSN_PARAMS + 1 + 255) / 256), dim3(256), 0, st, partial,
                     n > 0 ? n_parts : 0, grad, loss);
  return hipGetLastError();
}

hipError_t launch_wsn_forward(const uint16_t* w, const float* x, long long stride, long long n, float* y,
                              int n_cu, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = (WSN_NET_FLOATS + WSN_TILE_FLOATS) * sizeof(float);
  hipLaunchKernelGGL(k_wsn_forward, dim3(wsn_parts(n, n_cu)), dim3(64), lds, st, w, x, stride, n, y);
  return hipGetLastError();
}

hipError_t launch_wsn_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_wsn_adam, dim3((WSN_PARAMS + 255) / 256), dim3(256), 0, st, w, wb, g, m, v, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_wsn_to_bf16(const float* w, uint16_t* wb, hipStream_t st) {
  hipLaunchKernelGGL(k_wsn_to_bf16, dim3((WSN_PARAMS + 255) / 256), dim3(256), 0, st, w, wb, (int)WSN_PARAMS);
  return hipGetLastError();
}

size_t wsn_train_lds_bytes() { return WSN_TRAIN_FLOATS * sizeof(float); }

int wsn_shared_floats(int n_list) { return WSN_NET_FLOATS + WSN_TILE_FLOATS + 64 + ((n_list + 3) & ~3); }

int adam_scratch_floats() { return 2 * 256 + 1; }

hipError_t launch_adam(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, float max_norm, float* scratch, float* norm_out,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nb = (int)std::min<long long>(256, (n + 255) / 256);
  hipLaunchKernelGGL(k_sq_partial, dim3(nb), dim3(256), 0, st, g, n, scratch);
  hipLaunchKernelGGL(k_clip_scale, dim3(1), dim3(64), 0, st, scratch, nb, max_norm, norm_out);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, g, m, v, n, scratch + 2 * nb,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace sim
