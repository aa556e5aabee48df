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

// Residual balancing of the penalty classes (the paper's conclusion names the
// penalty choice as the method's main limitation).  Per class c, from this
// iteration's class maxima: r_c = max |a + z| over its rows, s_c = rho_c max
// |xbar change| over the duplicates in its rows / max |y| over its rows (both
// relative); rho_c times tau when r_c > mu s_c, divided by tau when s_c > mu r_c,
// within [rho0_c / span, rho0_c span], at most adapt_max times per class; not for a
// class whose multipliers are all zero, nor for one whose two residuals are both at
// or below ADAPT_NOISE (rows satisfied to the rounding level, e.g. commitments equal
// to their binary duplicates: the ratio of two rounding errors decides nothing).  The
// new penalties live in the iterate's scalars, which every kernel of the next
// iteration reads.
constexpr double ADAPT_NOISE = 1e-9;
__device__ inline void adapt_penalties(double* sc, const Par& p, const double (&mc)[NCS]) {
#pragma clang fp contract(off)
  const int rho_slot[NCL] = {SC_RHO_PQ, SC_RHO_VA, SC_RHO_CPL, SC_RHO_UC};
  const int cnt_slot[NCL] = {SC_NCHG_PQ, SC_NCHG_VA, SC_NCHG_CPL, SC_NCHG_UC};
#pragma unroll
  for (int c = 0; c < NCL; ++c) {
    if (sc[cnt_slot[c]] >= (double)p.adapt_max || !(mc[CS_Y + c] > 0.0)) continue;
    const double rho = sc[rho_slot[c]];
    const double sd = rho * mc[CS_DX + c] / mc[CS_Y + c];
    if (!(mc[CS_RIN + c] > ADAPT_NOISE || sd > ADAPT_NOISE)) continue;  // both at the rounding level
    if (mc[CS_RIN + c] > p.adapt_mu * sd && rho * p.adapt_tau <= p.rho0[c] * p.adapt_span) {
      sc[rho_slot[c]] = rho * p.adapt_tau;
      sc[cnt_slot[c]] = sc[cnt_slot[c]] + 1.0;
    } else if (sd > p.adapt_mu * mc[CS_RIN + c] && rho / p.adapt_tau >= p.rho0[c] / p.adapt_span) {
      sc[rho_slot[c]] = rho / p.adapt_tau;
      sc[cnt_slot[c]] = sc[cnt_slot[c]] + 1.0;
    }
  }
}

// The residual slots of one iteration as up to four contiguous ranges of s.red: flat
// index b < end[k] (and >= end[k-1]) is slot b + off[k].
struct SlotRanges {
  int end[4];
  int off[4];
};

__host__ __device__ inline SlotRanges slot_ranges(const int (&first)[4], const int (&count)[4]) {
  SlotRanges r;
  int e = 0;
  for (int k = 0; k < 4; ++k) {
    r.off[k] = first[k] - e;
    e += count[k];
    r.end[k] = e;
  }
  return r;
}

// The kernel-by-kernel and pipelined iterations: the unit side's slots (G of them, from
// units_slot on, one of its two copies), then every slot from the bus kernel's on.
__host__ __device__ inline SlotRanges standard_ranges(const State& s, const int units_slot) {
  const int first[4] = {units_slot, s.red_bus, 0, 0};
  const int count[4] = {s.red_bus - s.red_units, s.red_n - s.red_bus, 0, 0};
  return slot_ranges(first, count);
}

__device__ inline int range_slot(const SlotRanges& R, const int b) {
  return b + (b < R.end[0] ? R.off[0] : b < R.end[1] ? R.off[1] : b < R.end[2] ? R.off[2] : R.off[3]);
}

// The control step of one iteration, run by one whole block: reduce every per-block
// residual slot of the iteration (the ranges R), advance the counters and decide (see
// above).
__device__ inline void finalize_ranges(const State& s, const Par& p, const SlotRanges& R) {
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
  const int nslots = R.end[3];
  for (int b0 = threadIdx.x; b0 < nslots; b0 += U * (int)blockDim.x) {
    double v[U][NACC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * (int)blockDim.x;
      const int slot = range_slot(R, b);
#pragma unroll
      for (int k = 0; k < NACC; ++k) v[u][k] = b < nslots ? s.red[(size_t)slot * NACC + k] : 0.0;
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
  // residual balancing after every adapt_every-th iteration: the per-class maxima of
  // the same slots (a uniform condition: every thread read the same counter)
  const bool adapt_now = p.adapt_every > 0 && fmod(it + 1.0, (double)p.adapt_every) == 0.0;
  __shared__ double partc[NCS][FIN_BLOCK / 64];
  double mc[NCS];
#pragma unroll
  for (int k = 0; k < NCS; ++k) mc[k] = 0.0;
  if (adapt_now) {
    for (int b = threadIdx.x; b < nslots; b += (int)blockDim.x) {
      const int slot = range_slot(R, b);
#pragma unroll
      for (int k = 0; k < NCS; ++k) mc[k] = nmax(mc[k], s.redc[(size_t)slot * NCS + k]);
    }
#pragma unroll
    for (int k = 0; k < NCS; ++k) mc[k] = wave_max(mc[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < NCS; ++k) partc[k][threadIdx.x >> 6] = mc[k];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0 || halt) return;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m[k] = nmax(m[k], part[k][w]);
    m[k] = nmax(m[k], part[k][0]);
  }
  if (adapt_now) {
#pragma unroll
    for (int k = 0; k < NCS; ++k) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mc[k] = nmax(mc[k], partc[k][w]);
      mc[k] = nmax(mc[k], partc[k][0]);
    }
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
  if (adapt_now) adapt_penalties(sc, p, mc);
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

__device__ inline void finalize_body(const State& s, const Par& p, const int units_slot) {
  finalize_ranges(s, p, standard_ranges(s, units_slot));
}

}  // namespace ucac
