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
void launch_init(const Net& n, const State& s, const Par& p, double beta0, hipStream_t st);
}  // namespace ucac
