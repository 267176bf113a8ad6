// Per-contact warm-start network on matrix cores: 7 -> 64 ReLU -> 64 ReLU ->
// 3, bfloat16 weights, inputs and hidden activations, FP32 accumulation
// (v_mfma_f32_16x16x16bf16_1k).  One wave evaluates 16 rows at a time.
//
// Operand layout of the 16x16x16 instruction (lane l, element j = 0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + j
//   B[k][n]: n = l % 16, k = 4 (l / 16) + j
//   D[i][n]: i = 4 (l / 16) + j, n = l % 16
// so a lane's A or B operand is four consecutive k of one row of a matrix
// stored with k contiguous: the weights are kept in LDS as W[out][in]
// (= B^T), padded to multiples of 16 and with rows spaced to avoid bank
// conflicts between the 16 rows one load touches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sim {

enum {
  WSN_IN = 7, WSN_HID = 64, WSN_OUT = 3, WSN_PARAMS = 4867,
  // packed parameter offsets: W1[64][7] b1[64] W2[64][64] b2[64] W3[3][64] b3[3]
  WSN_W1 = 0, WSN_B1 = 448, WSN_W2 = 512, WSN_B2 = 4608, WSN_W3 = 4672, WSN_B3 = 4864,
  // LDS row strides (bf16 elements)
  WSN_S1 = 20,   // W1 rows: 16 inputs (7 used) + spacing
  WSN_SH = 72,   // 64-wide rows + spacing
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16, nearest with ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 ld_bf4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

// LDS image of the network used by the forward pass.
struct WsnNet {
  uint16_t* W1;  // [64][WSN_S1]: W1[h][k], k < 7, zero beyond
  uint16_t* W2;  // [64][WSN_SH]
  uint16_t* W3;  // [16][WSN_SH]: rows >= 3 zero
  float* b1;     // [64]
  float* b2;     // [64]
  float* b3;     // [16]: entries >= 3 zero
};
// floats of LDS taken by the network image
enum { WSN_NET_FLOATS = (64 * WSN_S1 + 64 * WSN_SH + 16 * WSN_SH) / 2 + 64 + 64 + 16 };
// floats of LDS taken by the two hidden-activation tiles [16][WSN_SH]
enum { WSN_TILE_FLOATS = 16 * WSN_SH };

__device__ __forceinline__ WsnNet wsn_net_at(float* p) {
  WsnNet n;
  n.W1 = reinterpret_cast<uint16_t*>(p);
  n.W2 = n.W1 + 64 * WSN_S1;
  n.W3 = n.W2 + 64 * WSN_SH;
  n.b1 = reinterpret_cast<float*>(n.W3 + 16 * WSN_SH);
  n.b2 = n.b1 + 64;
  n.b3 = n.b2 + 64;
  return n;
}

// Copy the packed bfloat16 parameters (global) into the LDS image; threads
// tid = 0..nt-1 of the workgroup share the work.  Caller synchronises.
__device__ inline void wsn_stage(const uint16_t* __restrict__ g, const WsnNet& n, int tid, int nt) {
  for (int i = tid; i < 64 * WSN_S1; i += nt) {
    const int h = i / WSN_S1, k = i % WSN_S1;
    n.W1[i] = k < WSN_IN ? g[WSN_W1 + h * WSN_IN + k] : (uint16_t)0;
  }
  for (int i = tid; i < 64 * WSN_SH; i += nt) {
    const int h = i / WSN_SH, k = i % WSN_SH;
    n.W2[i] = k < 64 ? g[WSN_W2 + h * 64 + k] : (uint16_t)0;
  }
  for (int i = tid; i < 16 * WSN_SH; i += nt) {
    const int o = i / WSN_SH, k = i % WSN_SH;
    n.W3[i] = (o < WSN_OUT && k < 64) ? g[WSN_W3 + o * 64 + k] : (uint16_t)0;
  }
  for (int i = tid; i < 64; i += nt) {
    n.b1[i] = bf2f(g[WSN_B1 + i]);
    n.b2[i] = bf2f(g[WSN_B2 + i]);
  }
  for (int i = tid; i < 16; i += nt) n.b3[i] = i < WSN_OUT ? bf2f(g[WSN_B3 + i]) : 0.f;
}

// A operand of the input layer: this lane's row (row l % 16) as bfloat16,
// features 4 (l / 16) .. +3, zero beyond 7 or for a missing row.
__device__ __forceinline__ bf16x4 wsn_input_operand(const float* xrow, int lane) {
  const int kq = 4 * (lane >> 4);
  bf16x4 a;
  for (int j = 0; j < 4; ++j) {
    const int k = kq + j;
    a[j] = (short)((xrow && k < WSN_IN) ? f2bf(xrow[k]) : (uint16_t)0);
  }
  return a;
}

// Hidden layer: H[16][64] (bf16, row stride WSN_SH) = relu(A W^T + b), with
// the A operand fragments given for the 16-wide k blocks.
template <int KB>
__device__ __forceinline__ void wsn_hidden(const bf16x4 (&a)[KB], const uint16_t* W, int wstride, const float* b,
                                           uint16_t* H, int lane) {
  const int kq = 4 * (lane >> 4), c16 = lane & 15;
  for (int ct = 0; ct < 4; ++ct) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const uint16_t* wr = W + (16 * ct + c16) * wstride + kq;
    for (int ks = 0; ks < KB; ++ks) acc = mfma16(a[ks], ld_bf4(wr + 16 * ks), acc);
    const int col = 16 * ct + c16;
    const float bb = b[col];
    for (int r = 0; r < 4; ++r) H[(kq + r) * WSN_SH + col] = f2bf(fmaxf(acc[r] + bb, 0.f));
  }
}

// A operand fragments of a [16][64] bf16 tile (row l % 16).
__device__ __forceinline__ void wsn_tile_operands(const uint16_t* H, int lane, bf16x4 (&a)[4]) {
  const uint16_t* hr = H + (lane & 15) * WSN_SH + 4 * (lane >> 4);
  for (int ks = 0; ks < 4; ++ks) a[ks] = ld_bf4(hr + 16 * ks);
}

// Forward of one 16-row tile.  xrow: this lane's input row (row l % 16; NULL
// for a missing row).  H1, H2: LDS tiles.  Returns this lane's outputs
// y[4 (l / 16) + r][l % 16], r = 0..3 (columns >= 3 are zero).  Every lane of
// the wave must call it (wave-uniform control flow).
__device__ inline floatx4 wsn_forward_tile(const WsnNet& n, const float* xrow, uint16_t* H1, uint16_t* H2,
                                           int lane) {
  bf16x4 a0[1] = {wsn_input_operand(xrow, lane)};
  wsn_hidden<1>(a0, n.W1, WSN_S1, n.b1, H1, lane);
  __syncthreads();
  bf16x4 a[4];
  wsn_tile_operands(H1, lane, a);
  wsn_hidden<4>(a, n.W2, WSN_SH, n.b2, H2, lane);
  __syncthreads();
  wsn_tile_operands(H2, lane, a);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const uint16_t* wr = n.W3 + (lane & 15) * WSN_SH + 4 * (lane >> 4);
  for (int ks = 0; ks < 4; ++ks) acc = mfma16(a[ks], ld_bf4(wr + 16 * ks), acc);
  const float bb = n.b3[lane & 15];
  for (int r = 0; r < 4; ++r) acc[r] += bb;
  __syncthreads();   // H1/H2 may be reused by the next tile
  return acc;
}

}  // namespace sim
