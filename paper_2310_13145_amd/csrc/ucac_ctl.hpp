// Inner/outer control of the two-level ADMM, decided on the device at the end of
// every inner iteration.
//
// The control step reduces the four residual maxima from the per-block slots,
// advances the counters and decides: converged (solve mode: r_p <= tol and
// r_d <= tol, then every later kernel of the instance returns at entry), or end of
// the inner loop (max(r_in, r_d) <= max(tol/2, eps_in0 2^-k), or max_inner
// iterations), in which case beta follows step:outer (times tau if
// ||z^k|| > theta ||z^{k-1}||) and the multiplier update
// lambda <- clamp(lambda + beta z) is left pending: the kernels that own the rows
// apply it in the next iteration just before their z update, and k_lambda applies
// it to every row when a call ends with it pending.
//
// It runs as its own one-block kernel after the iteration's last kernel (the
// line-end finish and generator-row multipliers).  Running it in the last block to
// finish of that work instead (a completion count per iteration) saved 1 % at 2,000
// buses and cost 25 % at 10,000: one block pulling every slot across the XCDs is
// slow.
#pragma once
#include "ucac_dev.hpp"

namespace ucac {

constexpr int FIN_BLOCK = 256;  // largest block that runs the control step

// The control step of one iteration, run by one whole block: reduce every per-block
// residual slot of the iteration, advance the counters and decide (see above).
__device__ inline void finalize_body(const State& s, const Par& p) {
  Ctl* c = s.ctl;
  if (c->halt) return;
  // reduce the per-block maxima of this iteration's kernels
  // up to 8 slots per thread per round, all loads issued before the first use
  double m[NACC] = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 8;
  for (int b0 = threadIdx.x; b0 < s.red_n; b0 += U * (int)blockDim.x) {
    double v[U][NACC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * (int)blockDim.x;
#pragma unroll
      for (int k = 0; k < NACC; ++k) v[u][k] = b < s.red_n ? s.red[(size_t)b * NACC + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NACC; ++k) m[k] = nmax(m[k], v[u][k]);
  }
  __shared__ double part[NACC][FIN_BLOCK / 64];
#pragma unroll
  for (int k = 0; k < NACC; ++k) m[k] = wave_max(m[k]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NACC; ++k) part[k][threadIdx.x >> 6] = m[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m[k] = nmax(m[k], part[k][w]);
    m[k] = nmax(m[k], part[k][0]);
  }
  double* sc = s.sc;
  const double rp = m[ACC_RP], rin = m[ACC_RIN], rd = m[ACC_RD], zinf = m[ACC_ZINF];
  sc[SC_RP] = rp;
  sc[SC_RIN] = rin;
  sc[SC_RD] = rd;
  sc[SC_ZINF] = zinf;
  sc[SC_ITER] += 1.0;
  sc[SC_LIN] += 1.0;
  c->pending = 0;
  if (rp != rp || rin != rin || rd != rd || zinf != zinf) c->bad = 1;
  c->ms_count += 1;
  for (int m = 0; m < 3; ++m)
    if (c->ms_iter[m] < 0 && rp <= c->ms_tol[m] && rd <= c->ms_tol[m]) c->ms_iter[m] = c->ms_count;
  if (c->stop_at_tol && rp <= c->tol && rd <= c->tol) {
    sc[SC_CONV] = 1.0;
    c->halt = 1;
    return;
  }
  const double eps = fmax(0.5 * c->tol, p.eps_in0 * ldexp(1.0, -(int)sc[SC_KOUT]));
  if (fmax(rin, rd) <= eps || sc[SC_LIN] >= (double)p.max_inner) {
    const double beta = sc[SC_BETA];
    c->pending = 1;
    c->beta_for_lambda = beta;
    if (zinf > p.theta * sc[SC_ZPREV]) sc[SC_BETA] = fmin(p.tau * beta, p.beta_max);
    sc[SC_ZPREV] = zinf;
    sc[SC_KOUT] += 1.0;
    sc[SC_LIN] = 0.0;
  }
}


}  // namespace ucac
