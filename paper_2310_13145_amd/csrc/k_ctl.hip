// Inner/outer control of the two-level ADMM, decided on the device.
//
// k_finalize reads the four residual maxima, clears the accumulators, advances
// the counters and decides: converged (solve mode: r_p <= tol and r_d <= tol,
// then every later kernel of the handle returns at entry), or end of the inner
// loop (max(r_in, r_d) <= max(tol/2, eps_in0 2^-k), or max_inner iterations),
// in which case beta follows step:outer (times tau if ||z^k|| > theta ||z^{k-1}||)
// and k_lambda applies lambda <- clamp(lambda + beta z) to every row.
#include "ucac_launch.hpp"

namespace ucac {

__global__ void k_finalize(Net n, State s, Par p) {
  Ctl* c = s.ctl;
  if (c->halt) return;
  if (threadIdx.x != 0) return;
  double* sc = s.sc;
  const double rp = __longlong_as_double((long long)c->acc[ACC_RP]);
  const double rin = __longlong_as_double((long long)c->acc[ACC_RIN]);
  const double rd = __longlong_as_double((long long)c->acc[ACC_RD]);
  const double zinf = __longlong_as_double((long long)c->acc[ACC_ZINF]);
  for (int k = 0; k < NACC; ++k) c->acc[k] = 0ull;
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

__global__ void __launch_bounds__(BLOCK) k_lambda(Net n, State s, Par p) {
  const Ctl* c = s.ctl;
  if (c->halt || !c->pending) return;
  const int TL = n.T * n.L, TG = n.T * n.G;
  const int nb = NRB * TL, total = nb + NRG * TG;
  const double b = c->beta_for_lambda, lm = p.lambda_max;
  for (int k = blockIdx.x * BLOCK + threadIdx.x; k < total; k += gridDim.x * BLOCK) {
    if (k < nb) s.lB[k] = clampd(s.lB[k] + b * s.zB[k], -lm, lm);
    else s.lG[k - nb] = clampd(s.lG[k - nb] + b * s.zG[k - nb], -lm, lm);
  }
}

void launch_finalize(const Net& n, const State& s, const Par& p, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, n, s, p);
}

void launch_lambda(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const long total = (long)NRB * n.T * n.L + (long)NRG * n.T * n.G;
  long blocks = (total + BLOCK - 1) / BLOCK;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_lambda, dim3((unsigned)blocks), dim3(BLOCK), 0, st, n, s, p);
}

}  // namespace ucac
