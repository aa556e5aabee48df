// Host-side launchers of the iteration kernels (one translation unit each).
#pragma once
#include "ucac_dev.hpp"

namespace ucac {
void launch_uc_dp(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_gen(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_branch(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_ubar(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_bus(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_gen_dual(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_finalize(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_lambda(const Net& n, const State& s, const Par& p, hipStream_t st);

// learned warm start (k_mlp.hip)
void mlp_launch_train(const MlpView& w, const float* X, const float* Yt, const int* idx, int nb, float inv_norm,
                      float* slots, hipStream_t st);
void mlp_launch_reduce(const float* slots, int n_slots, float* grad, double* loss, float* P, float* m1, float* m2, int step,
                       float lr, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st);
void mlp_launch_pack(const float* P, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st);
void mlp_launch_forward(const MlpView& w, const float* X, int n, float* Y, hipStream_t st);
constexpr int MLP_PARAMS = 5764;   // 64*20 + 64 + 64*64 + 64 + 4*64 + 4
constexpr int MLP_SLOT = MLP_PARAMS + 4;
}  // namespace ucac
