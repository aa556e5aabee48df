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
// residual slot of the iteration (the unit side's from slot units_slot on), advance the
// counters and decide (see above).
__device__ inline void finalize_body(const State& s, const Par& p, const int units_slot) {
#pragma clang fp contract(off)
  Ctl* c = s.ctl;
  double* sc = s.sc;
  // The control fields and counters are loaded first (uniform addresses), so that
  // their latency overlaps the slot loads; a halted instance is checked only
  // before the stores (the reduction itself only reads).
  const int halt = c->halt, stop = c->stop_at_tol, ms_count = c->ms_count, conv_iter = c->conv_iter;
  const double tol = c->tol;
  int ms_iter[3];
  double ms_tol[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { ms_iter[k] = c->ms_iter[k]; ms_tol[k] = c->ms_tol[k]; }
  const double it = sc[SC_ITER], lin = sc[SC_LIN], kout = sc[SC_KOUT], beta = sc[SC_BETA], zprev = sc[SC_ZPREV];
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
      for (int k = 0; k < NACC; ++k) {
        const int slot = b < s.red_bus ? units_slot + b : b;
        v[u][k] = b < s.red_n ? s.red[(size_t)slot * NACC + k] : 0.0;
      }
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
  if (threadIdx.x != 0 || halt) return;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m[k] = nmax(m[k], part[k][w]);
    m[k] = nmax(m[k], part[k][0]);
  }
  const double rp = m[ACC_RP], rin = m[ACC_RIN], rd = m[ACC_RD], zinf = m[ACC_ZINF];
  sc[SC_RP] = rp;
  sc[SC_RIN] = rin;
  sc[SC_RD] = rd;
  sc[SC_ZINF] = zinf;
  sc[SC_ITER] = it + 1.0;
  c->pending = 0;
  if (rp != rp || rin != rin || rd != rd || zinf != zinf) c->bad = 1;
  c->ms_count = ms_count + 1;
  for (int k = 0; k < 3; ++k)
    if (ms_iter[k] < 0 && rp <= ms_tol[k] && rd <= ms_tol[k]) c->ms_iter[k] = ms_count + 1;
  if (conv_iter < 0 && rp <= tol && rd <= tol) c->conv_iter = ms_count + 1;
  if (stop && rp <= tol && rd <= tol) {
    sc[SC_LIN] = lin + 1.0;
    sc[SC_CONV] = 1.0;
    c->halt = 1;
    return;
  }
  const double eps = fmax(0.5 * tol, p.eps_in0 * ldexp(1.0, -(int)kout));
  if (fmax(rin, rd) <= eps || lin + 1.0 >= (double)p.max_inner) {
    c->pending = 1;
    c->beta_for_lambda = beta;
    if (zinf > p.theta * zprev) sc[SC_BETA] = fmin(p.tau * beta, p.beta_max);
    sc[SC_ZPREV] = zinf;
    sc[SC_KOUT] = kout + 1.0;
    sc[SC_LIN] = 0.0;
  } else {
    sc[SC_LIN] = lin + 1.0;
  }
}


}  // namespace ucac
