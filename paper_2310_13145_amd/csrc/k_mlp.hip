// Training and batch inference of the learned line warm start (BF16 MFMA, FP32
// accumulation).
//
// k_mlp_train: one 64-lane wavefront per 64 samples: forward pass (pre-activations
//   kept in registers), mean-squared-error output error, backward pass, and the
//   wavefront's partial weight and bias gradients (every product a BF16 MFMA over
//   the samples), written to its own slot.  The BF16 rounding points are those of
//   the FP64 oracle in oracle/mlp.py: input, weights, hidden activations, output
//   error and pre-activation errors.
// k_mlp_reduce: sums the slots in wavefront order (deterministic) and optionally
//   takes one Adam step on the FP32 master weights, refreshing the BF16 copies.
// k_mlp_forward: batch inference through mlp_forward_wave.
#include "ucac_mlp.hpp"

namespace ucac {

constexpr int SLOT = MLP_NPARAM + 4;  // per-wavefront gradient slot: parameters, then the loss sum

// B operand from a row-major BF16 LDS matrix M[k][n] (stride ld): elements M[k0 + 8h + j][n]
__device__ inline bf16x8 col8(const __bf16* M, int ld, int k0, int n) {
  const int h = (threadIdx.x & 63) >> 5;
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = M[(k0 + 8 * h + j) * ld + n];
  return v;
}

// B operand from a row-major BF16 global matrix W[k][n] (row length ld), rows >= kmax read as zero
__device__ inline bf16x8 gcol8(const __bf16* W, int ld, int k0, int n, int kmax) {
  const int h = (threadIdx.x & 63) >> 5;
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = k0 + 8 * h + j;
    v[j] = k < kmax ? W[k * ld + n] : (__bf16)0.0f;
  }
  return v;
}

__global__ void __launch_bounds__(64) k_mlp_train(Mlp w, const float* __restrict__ X, const float* __restrict__ Yt,
                                                  const int* __restrict__ idx, int nb, float inv_norm, float* slots) {
  __shared__ __bf16 Xs[64 * MLP_LD], H1[64 * MLP_LD], H2[64 * MLP_LD], Gs[64 * MLP_LD];
  __shared__ __bf16 Ys[64 * 16];
  const int lane = threadIdx.x, r = lane & 31, h = lane >> 5;
  const int sample = blockIdx.x * 64 + lane;
  const bool valid = sample < nb;
  const int s = valid ? idx[sample] : 0;
  float* slot = slots + (size_t)blockIdx.x * SLOT;

  for (int k = 0; k < MLP_KIN; ++k) Xs[lane * MLP_LD + k] = (__bf16)(valid && k < MLP_IN ? X[(size_t)s * MLP_IN + k] : 0.0f);
  for (int k = 0; k < 16; ++k) Ys[lane * 16 + k] = (__bf16)0.0f;
  __syncthreads();

  // forward, keeping the pre-activations
  f32x16 z1[2][2], z2[2][2];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
        acc = mfma(ld8(Xs + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), ld8(w.W1b + (tn * 32 + r) * MLP_KIN + ks * 16 + h * 8), acc);
      const int n = tn * 32 + r;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[j] += w.b1[n];
        H1[(tm * 32 + d_row(j, h)) * MLP_LD + n] = (__bf16)silu_f(acc[j]);
      }
      z1[tm][tn] = acc;
    }
  __syncthreads();
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc = mfma(ld8(H1 + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), ld8(w.W2b + (tn * 32 + r) * MLP_H + ks * 16 + h * 8), acc);
      const int n = tn * 32 + r;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[j] += w.b2[n];
        H2[(tm * 32 + d_row(j, h)) * MLP_LD + n] = (__bf16)silu_f(acc[j]);
      }
      z2[tm][tn] = acc;
    }
  __syncthreads();

  // output, error and its bias gradient
  float lsum = 0.0f, db3 = 0.0f;
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
    f32x16 acc = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      acc = mfma(ld8(H2 + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), ld8(w.W3b + r * MLP_H + ks * 16 + h * 8), acc);
    if (r < MLP_OUT) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int m = tm * 32 + d_row(j, h);
        const int sm = blockIdx.x * 64 + m;
        float e = 0.0f;
        if (sm < nb) {
          e = acc[j] + w.b3[r] - Yt[(size_t)idx[sm] * MLP_OUT + r];
          lsum += e * e;
        }
        const float dy = e * inv_norm;
        db3 += dy;
        Ys[m * 16 + r] = (__bf16)dy;
      }
    }
  }
  __syncthreads();

  // dW3[o][k] = sum_m dY[m][o] H2[m][k]
#pragma unroll
  for (int tn = 0; tn < 2; ++tn) {
    f32x16 acc = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      bf16x8 a;
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = r < 16 ? Ys[(ks * 16 + 8 * h + j) * 16 + r] : (__bf16)0.0f;
      acc = mfma(a, col8(H2, MLP_LD, ks * 16, tn * 32 + r), acc);
    }
    if (h == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) slot[OFF_W3 + j * MLP_H + tn * 32 + r] = acc[j];  // rows 0..3
    }
  }

  // dA2 = dY W3, dZ2 = dA2 * silu'(Z2)
  float db2[2] = {0.0f, 0.0f};
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      f32x16 acc = {};
      acc = mfma(ld8(Ys + (tm * 32 + r) * 16 + h * 8), gcol8(w.W3b, MLP_H, 0, tn * 32 + r, MLP_OUT), acc);
      const int n = tn * 32 + r;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float g = acc[j] * dsilu_f(z2[tm][tn][j]);
        db2[tn] += g;
        Gs[(tm * 32 + d_row(j, h)) * MLP_LD + n] = (__bf16)g;
      }
    }
  __syncthreads();

  // dW2[n][k] = sum_m dZ2[m][n] H1[m][k]
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = Gs[(ks * 16 + 8 * h + j) * MLP_LD + tm * 32 + r];
        acc = mfma(a, col8(H1, MLP_LD, ks * 16, tn * 32 + r), acc);
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) slot[OFF_W2 + (tm * 32 + d_row(j, h)) * MLP_H + tn * 32 + r] = acc[j];
    }

  // dA1 = dZ2 W2, dZ1 = dA1 * silu'(Z1)
  f32x16 g1[2][2];
  float db1[2] = {0.0f, 0.0f};
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc = mfma(ld8(Gs + (tm * 32 + r) * MLP_LD + ks * 16 + h * 8), gcol8(w.W2b, MLP_H, ks * 16, tn * 32 + r, MLP_H), acc);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[j] *= dsilu_f(z1[tm][tn][j]);
        db1[tn] += acc[j];
      }
      g1[tm][tn] = acc;
    }
  __syncthreads();
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int j = 0; j < 16; ++j) Gs[(tm * 32 + d_row(j, h)) * MLP_LD + tn * 32 + r] = (__bf16)g1[tm][tn][j];
  __syncthreads();

  // dW1[n][k] = sum_m dZ1[m][n] X[m][k]
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
    f32x16 acc = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      bf16x8 a;
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = Gs[(ks * 16 + 8 * h + j) * MLP_LD + tm * 32 + r];
      acc = mfma(a, col8(Xs, MLP_LD, ks * 16, r), acc);
    }
    if (r < MLP_IN) {
#pragma unroll
      for (int j = 0; j < 16; ++j) slot[OFF_W1 + (tm * 32 + d_row(j, h)) * MLP_IN + r] = acc[j];
    }
  }

  // bias gradients: lanes r and r + 32 hold the two row halves of column r
#pragma unroll
  for (int tn = 0; tn < 2; ++tn) {
    const float b2s = db2[tn] + __shfl_xor(db2[tn], 32, 64);
    const float b1s = db1[tn] + __shfl_xor(db1[tn], 32, 64);
    if (h == 0) {
      slot[OFF_B2 + tn * 32 + r] = b2s;
      slot[OFF_B1 + tn * 32 + r] = b1s;
    }
  }
  const float b3s = db3 + __shfl_xor(db3, 32, 64);
  if (h == 0 && r < MLP_OUT) slot[OFF_B3 + r] = b3s;
  // loss sum of the wavefront
  float ls = lsum;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 64);
  if (lane == 0) slot[MLP_NPARAM] = ls;
}

// Pack FP32 master weights into the BF16 MFMA operand layouts.
__device__ inline void pack_one(int p, const float* P, __bf16* W1b, __bf16* W2b, __bf16* W3b) {
  if (p < OFF_B1) { const int n = p / MLP_IN, k = p - n * MLP_IN; W1b[n * MLP_KIN + k] = (__bf16)P[p]; }
  else if (p >= OFF_W2 && p < OFF_B2) { const int q = p - OFF_W2; W2b[q] = (__bf16)P[p]; }
  else if (p >= OFF_W3 && p < OFF_B3) { const int q = p - OFF_W3; W3b[q] = (__bf16)P[p]; }
}

__global__ void k_mlp_reduce(const float* __restrict__ slots, int n_slots, float* grad, double* loss, float* P,
                             float* m1, float* m2, int step, float lr, __bf16* W1b, __bf16* W2b, __bf16* W3b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > MLP_NPARAM) return;
  float g = 0.0f;
  for (int s = 0; s < n_slots; ++s) g += slots[(size_t)s * SLOT + p];
  if (p == MLP_NPARAM) {
    *loss = (double)g;
    return;
  }
  if (grad) grad[p] = g;
  if (step > 0) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float v = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    const float ah = a / (1.0f - powf(b1, (float)step));
    const float vh = v / (1.0f - powf(b2, (float)step));
    P[p] -= lr * ah / (sqrtf(vh) + eps);
    pack_one(p, P, W1b, W2b, W3b);
  }
}

__global__ void k_mlp_pack(const float* P, __bf16* W1b, __bf16* W2b, __bf16* W3b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_NPARAM) pack_one(p, P, W1b, W2b, W3b);
}

__global__ void __launch_bounds__(BLOCK) k_mlp_forward(Mlp w, const float* __restrict__ X, int n, float* Y) {
  extern __shared__ __bf16 lds_mlp[];
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  float f[MLP_IN], o[MLP_OUT];
#pragma unroll
  for (int k = 0; k < MLP_IN; ++k) f[k] = i < n ? X[(size_t)i * MLP_IN + k] : 0.0f;
  mlp_forward_wave(w, f, lds_mlp + (threadIdx.x >> 6) * MLP_WAVE_LDS, o);
  if (i < n) {
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) Y[(size_t)i * MLP_OUT + k] = o[k];
  }
}

// ---- host launchers (used by ucac_api.hip) ------------------------------------

void mlp_launch_train(const Mlp& w, const float* X, const float* Yt, const int* idx, int nb, float inv_norm, float* slots,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_train, dim3((nb + 63) / 64), dim3(64), 0, st, w, X, Yt, idx, nb, inv_norm, slots);
}

void mlp_launch_reduce(const float* slots, int n_slots, float* grad, double* loss, float* P, float* m1, float* m2, int step,
                       float lr, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, slots, n_slots, grad, loss, P, m1,
                     m2, step, lr, W1b, W2b, W3b);
}

void mlp_launch_pack(const float* P, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, P, W1b, W2b, W3b);
}

void mlp_launch_forward(const Mlp& w, const float* X, int n, float* Y, hipStream_t st) {
  const size_t lds = sizeof(__bf16) * MLP_WAVE_LDS * (BLOCK / 64);
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), lds, st, w, X, n, Y);
}

}  // namespace ucac
