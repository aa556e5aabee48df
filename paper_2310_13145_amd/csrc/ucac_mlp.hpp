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

// Orders a wavefront's LDS accesses across its lanes where the buffer is private to the
// wavefront: the hardware performs a wavefront's LDS operations in program order, so
// only the compiler has to be kept from moving them across this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The barrier of the forward pass: the block's (every lane of the block calls the
// pass) or, with WAVE, the wavefront's (every lane of the wavefront calls it).
template <bool WAVE>
__device__ inline void mlp_sync() {
  if (WAVE) wave_sync();
  else __syncthreads();
}

__device__ inline f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }

__device__ inline int d_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

// SiLU from the hardware exponential and reciprocal (inference only; relative
// error ~1e-6 before the result is rounded to BF16).
__device__ inline float silu_fast(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// A lane's operands of the three layers: its weight fragments (the A operands of its
// MFMAs) and the biases of the outputs it finishes.  Loaded before any other work, so
// that their latency overlaps the inputs' loads instead of following each layer's
// barrier.
struct MlpFrags {
  bf16x8 a1[MLP_H / 32][MLP_KIN / 16], a2[MLP_H / 32][MLP_H / 16], a3[MLP_H / 16];
  float b1[MLP_H / 32][4][4], b2[MLP_H / 32][4][4];
};

__device__ inline void mlp_load_frags(const Mlp& w, MlpFrags& f) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int to = 0; to < MLP_H / 32; ++to) {
#pragma unroll
    for (int ks = 0; ks < MLP_KIN / 16; ++ks) f.a1[to][ks] = ld8(w.W1b + (to * 32 + r) * MLP_KIN + ks * 16 + h * 8);
#pragma unroll
    for (int ks = 0; ks < MLP_H / 16; ++ks) f.a2[to][ks] = ld8(w.W2b + (to * 32 + r) * MLP_H + ks * 16 + h * 8);
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f.b1[to][jb][q] = w.b1[to * 32 + 8 * jb + 4 * h + q];
        f.b2[to][jb][q] = w.b2[to * 32 + 8 * jb + 4 * h + q];
      }
  }
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks) f.a3[ks] = ld8(w.W3b + r * MLP_H + ks * 16 + h * 8);
}

// In place: X [64 samples][K] (LDS rows, stride MLP_LD) becomes
// silu(X W^T + b) [64][NOUT], computed as the product W X^T so that the MFMA
// result of a lane is four consecutive outputs of one sample (one 8-byte LDS
// store): A = W rows (this lane's fragments), B = X rows (LDS), D[out][sample].
// Each 32-sample tile is read completely before it is overwritten; the block
// barriers order the reads of every lane before the writes, so every lane of the
// block calls this.
template <int K, int NOUT, bool WAVE = false>
__device__ inline void layer_silu_inplace(__bf16* X, const bf16x8 (&A)[NOUT / 32][K / 16],
                                          const float (&bias)[NOUT / 32][4][4]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int ts = 0; ts < 2; ++ts) {  // sample tile
    f32x16 acc[NOUT / 32];
#pragma unroll
    for (int to = 0; to < NOUT / 32; ++to) {
      acc[to] = f32x16{};
#pragma unroll
      for (int ks = 0; ks < K / 16; ++ks) acc[to] = mfma(A[to][ks], ld8(X + (ts * 32 + r) * MLP_LD + ks * 16 + h * 8), acc[to]);
    }
    mlp_sync<WAVE>();
    __bf16* row = X + (ts * 32 + r) * MLP_LD;
#pragma unroll
    for (int to = 0; to < NOUT / 32; ++to)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        const int o = to * 32 + 8 * jb + 4 * h;  // outputs o .. o+3 of sample ts*32 + r
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (__bf16)silu_fast(acc[to][4 * jb + q] + bias[to][jb][q]);
        *reinterpret_cast<bf16x4*>(row + o) = v;
      }
    mlp_sync<WAVE>();
  }
}

// Forward pass of the 64 samples of one wavefront with the operands in fr.  feat:
// this lane's 20 inputs; buf: MLP_WAVE_LDS BF16 of LDS private to the wavefront.
// Every lane of the block must call this (block barriers inside).  out: this lane's
// 4 outputs.
__device__ inline void mlp_forward_frags(const MlpFrags& fr, const float* b3, const float (&feat)[MLP_IN], __bf16* buf,
                                         float (&out)[MLP_OUT]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
  {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    __bf16* row = buf + lane * MLP_LD;
#pragma unroll
    for (int k = 0; k < MLP_KIN; k += 4) {
      bf16x4 v;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (__bf16)(k + q < MLP_IN ? feat[k + q] : 0.0f);
      *reinterpret_cast<bf16x4*>(row + k) = v;
    }
  }
  __syncthreads();
  layer_silu_inplace<MLP_KIN, MLP_H>(buf, fr.a1, fr.b1);
  layer_silu_inplace<MLP_H, MLP_H>(buf, fr.a2, fr.b2);
  // output layer, W3 padded to 32 rows: outputs 0..3 of sample ts*32 + r sit in
  // acc[0..3] of lane r (h = 0)
  f32x16 acc[2];
#pragma unroll
  for (int ts = 0; ts < 2; ++ts) {
    acc[ts] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < MLP_H / 16; ++ks) acc[ts] = mfma(fr.a3[ks], ld8(buf + (ts * 32 + r) * MLP_LD + ks * 16 + h * 8), acc[ts]);
  }
  __syncthreads();
  float* Yf = reinterpret_cast<float*>(buf);  // [64][4] FP32 over the consumed activations
  if (h == 0) {
#pragma unroll
    for (int ts = 0; ts < 2; ++ts)
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) Yf[(ts * 32 + r) * MLP_OUT + o] = acc[ts][o] + b3[o];
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) out[o] = Yf[lane * MLP_OUT + o];
  __syncthreads();
}

// The same arithmetic for a caller that keeps other work live (the fused line lanes):
// each layer's operands loaded just before the layer (a third of the registers of
// mlp_forward_frags) and wavefront barriers (the buffer is the wavefront's own), so
// that every lane of the wavefront calls it.
__device__ inline void mlp_forward_layers(const Mlp& w, const float (&feat)[MLP_IN], __bf16* buf, float (&out)[MLP_OUT]) {
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
  {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    __bf16* row = buf + lane * MLP_LD;
#pragma unroll
    for (int k = 0; k < MLP_KIN; k += 4) {
      bf16x4 v;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (__bf16)(k + q < MLP_IN ? feat[k + q] : 0.0f);
      *reinterpret_cast<bf16x4*>(row + k) = v;
    }
  }
  wave_sync();
  {
    bf16x8 a[MLP_H / 32][MLP_KIN / 16];
    float b[MLP_H / 32][4][4];
#pragma unroll
    for (int to = 0; to < MLP_H / 32; ++to) {
#pragma unroll
      for (int ks = 0; ks < MLP_KIN / 16; ++ks) a[to][ks] = ld8(w.W1b + (to * 32 + r) * MLP_KIN + ks * 16 + h * 8);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) b[to][jb][q] = w.b1[to * 32 + 8 * jb + 4 * h + q];
    }
    layer_silu_inplace<MLP_KIN, MLP_H, true>(buf, a, b);
  }
  {
    bf16x8 a[MLP_H / 32][MLP_H / 16];
    float b[MLP_H / 32][4][4];
#pragma unroll
    for (int to = 0; to < MLP_H / 32; ++to) {
#pragma unroll
      for (int ks = 0; ks < MLP_H / 16; ++ks) a[to][ks] = ld8(w.W2b + (to * 32 + r) * MLP_H + ks * 16 + h * 8);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) b[to][jb][q] = w.b2[to * 32 + 8 * jb + 4 * h + q];
    }
    layer_silu_inplace<MLP_H, MLP_H, true>(buf, a, b);
  }
  bf16x8 a3[MLP_H / 16];
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks) a3[ks] = ld8(w.W3b + r * MLP_H + ks * 16 + h * 8);
  // output layer as in mlp_forward_frags
  f32x16 acc[2];
#pragma unroll
  for (int ts = 0; ts < 2; ++ts) {
    acc[ts] = f32x16{};
#pragma unroll
    for (int ks = 0; ks < MLP_H / 16; ++ks) acc[ts] = mfma(a3[ks], ld8(buf + (ts * 32 + r) * MLP_LD + ks * 16 + h * 8), acc[ts]);
  }
  wave_sync();
  float* Yf = reinterpret_cast<float*>(buf);
  if (h == 0) {
#pragma unroll
    for (int ts = 0; ts < 2; ++ts)
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) Yf[(ts * 32 + r) * MLP_OUT + o] = acc[ts][o] + w.b3[o];
  }
  wave_sync();
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) out[o] = Yf[lane * MLP_OUT + o];
  wave_sync();
}

__device__ inline void mlp_forward_wave(const Mlp& w, const float (&feat)[MLP_IN], __bf16* buf, float (&out)[MLP_OUT]) {
  MlpFrags fr;
  mlp_load_frags(w, fr);
  mlp_forward_frags(fr, w.b3, feat, buf, out);
}

}  // namespace ucac
