// The control step of an inner iteration (ucac_ctl.hpp) as a one-block kernel, and
// the step:outer multiplier update applied to every row for a call that ends with
// it pending (within an iteration the row owners apply it).
#include "ucac_ctl.hpp"
#include <hip/hip_ext.h>
#include "ucac_launch.hpp"

namespace ucac {

__global__ void __launch_bounds__(FIN_BLOCK) k_finalize(Net n, State s, Par p) { finalize_body(s, p, s.red_u); }

__global__ void __launch_bounds__(FIN_BLOCK) k_finalize_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  finalize_body(M.s, M.p, M.s.red_u);
}

__global__ void __launch_bounds__(FIN_BLOCK) k_finalize_ranges(State s, Par p, SlotRanges R) { finalize_ranges(s, p, R); }

void launch_finalize(const Net& n, const State& s, const Par& p, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_BLOCK), 0, st, n, s, p);
}

bool launch_finalize_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  hipExtLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_BLOCK), 0, st, e0, e1, 0u, n, s, p);
  return true;
}

void launch_finalize_ranges(const State& s, const Par& p, const SlotRanges& R, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_ranges, dim3(1), dim3(FIN_BLOCK), 0, st, s, p, R);
}

void launch_finalize_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_group, dim3(grid), dim3(FIN_BLOCK), 0, st, g);
}

__device__ __forceinline__ void lambda_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  const Ctl* c = s.ctl;
  if (c->halt || !c->pending) return;
  const int TL = n.T * n.L, TG = n.T * n.G;
  const int nb = NRB * TL, total = nb + NRG * TG;
  const double b = c->beta_for_lambda, lm = p.lambda_max;
  for (int k = blk * BLOCK + threadIdx.x; k < total; k += nblk * BLOCK) {
    if (k < nb) s.lB[k] = clampd(s.lB[k] + b * s.zB[k], -lm, lm);
    else s.lG[k - nb] = clampd(s.lG[k - nb] + b * s.zG[k - nb], -lm, lm);
  }
}

__global__ void __launch_bounds__(BLOCK) k_lambda(Net n, State s, Par p) { lambda_body(n, s, p, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(BLOCK) k_lambda_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  lambda_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}


int lambda_blocks(const Net& n) {
  const long total = (long)NRB * n.T * n.L + (long)NRG * n.T * n.G;
  long blocks = (total + BLOCK - 1) / BLOCK;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

void launch_lambda(const Net& n, const State& s, const Par& p, hipStream_t st) {
  hipLaunchKernelGGL(k_lambda, dim3(lambda_blocks(n)), dim3(BLOCK), 0, st, n, s, p);
}

void launch_lambda_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_lambda_group, dim3(grid), dim3(BLOCK), 0, st, g);
}

}  // namespace ucac
