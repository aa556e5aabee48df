// step:opf, generator part -- one lane per (generator, period).
//
// Minimises the generation cost k2 p^2 + k1 p plus the augmented-Lagrangian terms
// of rows G1, G2 (generator consensus) and C1..C6 (the slack forms of
// eq:coupling) over p in [0, P-bar], q in the reactive box and the slacks s >= 0.
// The slacks are eliminated in closed form (a "-s" row contributes
// rho/2 min(0, m)^2, a "+s" row rho/2 max(0, m)^2), leaving two independent 1-D
// convex piecewise quadratics.  The ramp rows use the previous period's bus-side
// duplicate pbar_{t-1}, which keeps every (g, t) independent.
// HBM-bound: 21 doubles in, 8 out per lane, all coalesced.
#include "ucac_launch.hpp"
#include "ucac_pwl.hpp"

namespace ucac {

__device__ __forceinline__ void gen_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int TG = n.T * n.G;
  const int i = blk * UBLOCK + threadIdx.x;
  if (i >= TG) return;
  const int t = i / n.G, g = i - t * n.G;
  const double rp = p.rho_pq, rc = p.rho_cpl;
  const double pb = s.pb[i], qb = s.qb[i];
  const double pbp = t == 0 ? n.p0[g] : s.pb[i - n.G];
  const double uon = s.ubon[i];
  const double uonp = t == 0 ? (double)n.u0[g] : s.ubon[i - n.G];
  const double usu = s.ubsu[i], usd = s.ubsd[i];
  double z[8], y[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) { z[r] = s.zG[r * TG + i]; y[r] = s.yG[r * TG + i]; }

  const double eG1 = -pb + z[RG_G1] + y[RG_G1] / rp;
  const double e1 = -n.pmin[g] * uon + z[RG_C1] + y[RG_C1] / rc;
  const double e2 = -n.pmax[g] * uon + z[RG_C2] + y[RG_C2] / rc;
  const double e5 = -pbp + n.rd[g] * uon + n.sd[g] * usd + z[RG_C5] + y[RG_C5] / rc;
  const double e6 = -pbp - n.ru[g] * uonp - n.su[g] * usu + z[RG_C6] + y[RG_C6] / rc;
  Pwl<4> fp;
  fp.A = 2.0 * n.k2[g] + rp;
  fp.B = n.k1[g] + rp * eG1;
  fp.w[0] = rc; fp.w[1] = rc; fp.w[2] = rc; fp.w[3] = rc;
  fp.e[0] = e1; fp.e[1] = e2; fp.e[2] = e5; fp.e[3] = e6;
  fp.neg[0] = true; fp.neg[1] = false; fp.neg[2] = true; fp.neg[3] = false;
  const double pv = fp.argmin(0.0, n.pmax[g]);

  const double eG2 = -qb + z[RG_G2] + y[RG_G2] / rp;
  const double e3 = -n.qmin[g] * uon + z[RG_C3] + y[RG_C3] / rc;
  const double e4 = -n.qmax[g] * uon + z[RG_C4] + y[RG_C4] / rc;
  Pwl<2> fq;
  fq.A = rp;
  fq.B = rp * eG2;
  fq.w[0] = rc; fq.w[1] = rc;
  fq.e[0] = e3; fq.e[1] = e4;
  fq.neg[0] = true; fq.neg[1] = false;
  const double qv = fq.argmin(fmin(0.0, n.qmin[g]), fmax(0.0, n.qmax[g]));

  s.p[i] = pv;
  s.q[i] = qv;
  s.s[0 * TG + i] = fmax(0.0, pv + e1);
  s.s[1 * TG + i] = fmax(0.0, -(pv + e2));
  s.s[2 * TG + i] = fmax(0.0, qv + e3);
  s.s[3 * TG + i] = fmax(0.0, -(qv + e4));
  s.s[4 * TG + i] = fmax(0.0, pv + e5);
  s.s[5 * TG + i] = fmax(0.0, -(pv + e6));
}

__global__ void __launch_bounds__(UBLOCK) k_gen(Net n, State s, Par p) { gen_body(n, s, p, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(UBLOCK) k_gen_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  gen_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}

int gen_blocks(const Net& n) { return (n.T * n.G + UBLOCK - 1) / UBLOCK; }

void launch_gen_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_group, dim3(grid), dim3(UBLOCK), 0, st, g);
}

void launch_gen(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const int TG = n.T * n.G;
  if (TG == 0) return;
  hipLaunchKernelGGL(k_gen, dim3(gen_blocks(n)), dim3(UBLOCK), 0, st, n, s, p);
}

}  // namespace ucac
