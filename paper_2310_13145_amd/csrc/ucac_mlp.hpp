// Wavefront-level BF16 MFMA building blocks of the learned line warm start:
// a 20 -> 64 -> 64 -> 4 perceptron with SiLU activations.  One 64-lane
// wavefront evaluates 64 samples (one per lane) with v_mfma_f32_32x32x16_bf16
// (BF16 operands, FP32 accumulation); activations move between layers through
// LDS as BF16 rows.
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (checked on gfx950 by a probe):
//   lane l, r = l & 31, h = l >> 5, j = 0..7 of the 8-element operands:
//   A[m = r][k = 8h + j], B[k = 8h + j][n = r];
//   result j = 0..15: D[m = 8(j/4) + 4h + (j%4)][n = r].
#pragma once
#include "ucac_dev.hpp"

namespace ucac {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MLP_IN = 20, MLP_H = 64, MLP_OUT = 4;
constexpr int MLP_KIN = 32;  // input width padded to the MFMA K step
constexpr int MLP_LD = 72;   // LDS row stride (BF16 elements) of an activation tile
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 5764
// offsets in the FP32 parameter vector: W1 [64][20], b1, W2 [64][64], b2, W3 [4][64], b3
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_OUT * MLP_H;
constexpr int MLP_WAVE_LDS = 64 * MLP_LD;  // BF16 elements of LDS per wavefront for inference

using Mlp = MlpView;

__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ inline bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ inline f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }

__device__ inline int d_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

// In place: X [64][K] (LDS rows, stride MLP_LD) becomes act(X W^T + b) [64][NOUT]
// with W [NOUT][K] BF16 in global memory.  Each 32-row tile's products are all
// formed before the tile is overwritten; the block barriers order the LDS reads
// of every lane before the writes, so every lane of the block must call this.
template <int K, int NOUT>
__device__ inline void layer_silu_inplace(__bf16* X, const __bf16* W, const float* bias) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
    f32x16 acc[NOUT / 32];
#pragma unroll
    for (int tn = 0; tn < NOUT / 32; ++tn) {
      acc[tn] = f32x16{};
#pragma unroll
      for (int ks = 0; ks < K / 16; ++ks)
        acc[tn] = mfma(ld8(X + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), ld8(W + (tn * 32 + r) * K + ks * 16 + h * 8), acc[tn]);
    }
    __syncthreads();
#pragma unroll
    for (int tn = 0; tn < NOUT / 32; ++tn) {
      const int n = tn * 32 + r;
      const float bn = bias[n];
#pragma unroll
      for (int j = 0; j < 16; ++j) X[(tm * 32 + d_row(j, h)) * MLP_LD + n] = (__bf16)silu_f(acc[tn][j] + bn);
    }
    __syncthreads();
  }
}

// Forward pass of the 64 samples of one wavefront.  feat: this lane's 20 inputs;
// buf: MLP_WAVE_LDS BF16 of LDS private to the wavefront.  Every lane of the
// block must call this (block barriers inside).  out: this lane's 4 outputs.
__device__ inline void mlp_forward_wave(const Mlp& w, const float (&feat)[MLP_IN], __bf16* buf, float (&out)[MLP_OUT]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int k = 0; k < MLP_KIN; ++k) buf[lane * MLP_LD + k] = (__bf16)(k < MLP_IN ? feat[k] : 0.0f);
  __syncthreads();
  layer_silu_inplace<MLP_KIN, MLP_H>(buf, w.W1b, w.b1);
  layer_silu_inplace<MLP_H, MLP_H>(buf, w.W2b, w.b2);
  f32x16 acc[2];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
    acc[tm] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < MLP_H / 16; ++ks)
      acc[tm] = mfma(ld8(buf + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), ld8(w.W3b + r * MLP_H + ks * 16 + h * 8), acc[tm]);
  }
  __syncthreads();
  float* Yf = reinterpret_cast<float*>(buf);  // [64][4] FP32 over the consumed activations
  if (r < MLP_OUT) {
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
      for (int j = 0; j < 16; ++j) Yf[(tm * 32 + d_row(j, h)) * MLP_OUT + r] = acc[tm][j] + w.b3[r];
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) out[o] = Yf[lane * MLP_OUT + o];
  __syncthreads();
}

}  // namespace ucac
