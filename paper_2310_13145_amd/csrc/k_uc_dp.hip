// step:uc -- one dynamic program per generator (Sec. III-B, Alg. dp_algo).
//
// A group of 64 or 16 lanes per generator (one wavefront per generator, or four
// generators per wavefront).  The group's lanes build the cost table
// L^UC_{g,t}(s', s) for all periods in parallel into LDS (4 doubles per period),
// then the group's first lane runs the backward stay/switch induction
// (keep_formula, switch_formula) and the forward reconstruction from one decision
// bit per (period, state) -- O(T) extra space instead of the paper's stored O(T^2)
// trajectories -- and the lanes write u_on/u_su/u_sd back, one period each.
//
// This file is compiled with -ffp-contract=off: the table entries and the
// stay/switch sums are plain IEEE additions and products in a fixed order, so a
// commitment is decided on exactly the same numbers as in any other plain FP64
// evaluation of the same expressions.
#include "ucac_launch.hpp"

namespace ucac {

// L^UC(s', s): commitment costs plus y (u - ubar + z) + rho/2 (u - ubar + z)^2
// over (on, su, sd), with su = max(0, s - s'), sd = max(0, s' - s).
__device__ inline double uc_table_entry(double cnl, double csu, double csd, double rho, int sp, int s,
                                        const double* ub, const double* z, const double* y) {
  const int usu = s > sp ? 1 : 0;
  const int usd = sp > s ? 1 : 0;
  double L = cnl * (double)s + csu * (double)usu + csd * (double)usd;
  const double u[3] = {(double)s, (double)usu, (double)usd};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double r = (u[k] - ub[k]) + z[k];
    L += y[k] * r + 0.5 * rho * r * r;
  }
  return L;
}

// LDS bytes of one generator's DP at horizon T: cost table [T][2][2], cost-to-go
// [T+2][2], decision bits [T+2][2], schedule [T]; padded to 8 bytes.
__host__ __device__ inline size_t dp_slot_bytes(int T) {
  const size_t b = sizeof(double) * (4 * (size_t)T + 2 * ((size_t)T + 2)) + 2 * ((size_t)T + 2) + (size_t)T;
  return (b + 7) & ~(size_t)7;
}

// The stay/switch backward induction over the LDS table Lt (1-based period t at
// Lt[(t-1)*4 + s'*2 + s]), the initial hold (L_g periods on or F_g off), and the
// forward reconstruction of the schedule u[0..T).  Returns the optimal cost,
// summed in the order of the recursion.  Minimum up/down times below 1 act as 1.
__device__ inline double dp_recursion(int T, const double* Lt, double* c, unsigned char* dec, signed char* u, int u0,
                                      int lon, int loff, int tu, int td) {
  const int TU = tu < 1 ? 1 : tu, TD = td < 1 ? 1 : td;
  int hold = u0 ? lon : loff;
  hold = hold > T ? T : (hold < 0 ? 0 : hold);
  c[(T + 1) * 2 + 0] = 0.0;
  c[(T + 1) * 2 + 1] = 0.0;
  for (int t = T; t >= 1 && t > hold; --t) {
    for (int ss = 0; ss < 2; ++ss) {
      const double stay = Lt[((t - 1) * 2 + ss) * 2 + ss] + c[(t + 1) * 2 + ss];
      const int ns = 1 - ss;
      const int Tm = ns ? TU : TD;
      double sw = Lt[((t - 1) * 2 + ss) * 2 + ns];
      const int last = (t + Tm - 1) < T ? (t + Tm - 1) : T;
      for (int tp = t + 1; tp <= last; ++tp) sw += Lt[((tp - 1) * 2 + ns) * 2 + ns];
      const int nxt = t + Tm;
      sw += (nxt <= T) ? c[nxt * 2 + ns] : 0.0;
      const bool keep = stay <= sw;
      c[t * 2 + ss] = keep ? stay : sw;
      dec[t * 2 + ss] = keep ? 0 : 1;
    }
  }
  double cost;
  int st = u0;
  if (hold > 0) {
    cost = 0.0;
    for (int k = 1; k <= hold; ++k) cost += Lt[((k - 1) * 2 + u0) * 2 + u0];
    cost += c[(hold + 1) * 2 + u0];
  } else {
    cost = c[1 * 2 + u0];
  }
  for (int k = 1; k <= hold; ++k) u[k - 1] = (signed char)u0;
  int t = hold + 1;
  while (t <= T) {
    if (dec[t * 2 + st] == 0) {
      u[t - 1] = (signed char)st;
      ++t;
    } else {
      const int ns = 1 - st;
      const int Tm = ns ? TU : TD;
      for (int k = t; k <= t + Tm - 1 && k <= T; ++k) u[k - 1] = (signed char)ns;
      t += Tm;
      st = ns;
    }
  }
  return cost;
}

// LPG lanes per generator (64: one wavefront; 16: four generators per wavefront).
// The LPG lanes of a generator build its table; the group's first lane runs the
// recursion and the reconstruction.  slotT: horizon the LDS slots are sized for.
template <int LPG>
__device__ __forceinline__ void uc_dp_body(const Net& n, const State& s, const Par& p, int blk, int slotT) {
  if (s.ctl->halt) return;
  constexpr int GPB = 64 / LPG;  // generators per block
  const int T = n.T, G = n.G;
  const int sub = threadIdx.x / LPG, lane = threadIdx.x - sub * LPG;
  const int g = blk * GPB + sub;
  const bool act = g < G;
  extern __shared__ double lds[];
  char* base = (char*)lds + dp_slot_bytes(slotT) * sub;
  double* Lt = (double*)base;              // [T][2][2]
  double* c = Lt + 4 * T;                  // [T+2][2], c[T+1][*] = 0
  unsigned char* dec = (unsigned char*)(c + 2 * (T + 2));  // [T+2][2]
  signed char* u = (signed char*)(dec + 2 * (T + 2));      // [T]

  const double rho = p.rho_uc;
  const int TGs = T * G;
  if (act) {
    const double cnl = n.cnl[g], csu = n.csu[g], csd = n.csd[g];
    for (int t = lane; t < T; t += LPG) {
      const int k = t * G + g;
      const double ub[3] = {s.ubon[k], s.ubsu[k], s.ubsd[k]};
      const double z[3] = {s.zG[RG_U1 * TGs + k], s.zG[RG_U2 * TGs + k], s.zG[RG_U3 * TGs + k]};
      const double y[3] = {s.yG[RG_U1 * TGs + k], s.yG[RG_U2 * TGs + k], s.yG[RG_U3 * TGs + k]};
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int ss = 0; ss < 2; ++ss) Lt[(t * 2 + sp) * 2 + ss] = uc_table_entry(cnl, csu, csd, rho, sp, ss, ub, z, y);
    }
  }
  __syncthreads();

  if (act && lane == 0) dp_recursion(T, Lt, c, dec, u, n.u0[g], n.lon[g], n.loff[g], n.tu[g], n.td[g]);
  __syncthreads();

  if (act) {
    const int u0 = n.u0[g];
    for (int t = lane; t < T; t += LPG) {
      const int k = t * G + g;
      const int cur = u[t];
      const int prev = t == 0 ? u0 : u[t - 1];
      s.uon[k] = (double)cur;
      s.usu[k] = cur > prev ? 1.0 : 0.0;
      s.usd[k] = prev > cur ? 1.0 : 0.0;
    }
  }
}

template <int LPG>
__global__ void __launch_bounds__(64) k_uc_dp(Net n, State s, Par p) {
  uc_dp_body<LPG>(n, s, p, blockIdx.x, n.T);
}

template <int LPG>
__global__ void __launch_bounds__(64) k_uc_dp_group(Group gr, int slotT) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  uc_dp_body<LPG>(M.n, M.s, M.p, blockIdx.x - gr.blk_first[mk], slotT);
}

// Standalone batch of dynamic programs on given tables tab [G][T][2][2]: the same
// recursion, with the table loaded instead of built from the ADMM rows.
template <int LPG>
__global__ void __launch_bounds__(64) k_dp_tables(const double* __restrict__ tab, int G, int T, const int* tu,
                                                  const int* td, const int* u0, const int* lon, const int* loff,
                                                  signed char* u_out, double* cost_out) {
  constexpr int GPB = 64 / LPG;
  const int sub = threadIdx.x / LPG, lane = threadIdx.x - sub * LPG;
  const int g = blockIdx.x * GPB + sub;
  const bool act = g < G;
  extern __shared__ double lds[];
  char* base = (char*)lds + dp_slot_bytes(T) * sub;
  double* Lt = (double*)base;
  double* c = Lt + 4 * T;
  unsigned char* dec = (unsigned char*)(c + 2 * (T + 2));
  signed char* u = (signed char*)(dec + 2 * (T + 2));
  if (act) {
    const double* src = tab + (size_t)g * T * 4;
    for (int k = lane; k < 4 * T; k += LPG) Lt[k] = src[k];
  }
  __syncthreads();
  if (act && lane == 0) cost_out[g] = dp_recursion(T, Lt, c, dec, u, u0[g], lon[g], loff[g], tu[g], td[g]);
  __syncthreads();
  if (act)
    for (int t = lane; t < T; t += LPG) u_out[(size_t)g * T + t] = u[t];
}

size_t dp_tables_lds(int T, int lanes) { return dp_slot_bytes(T) * (64 / lanes); }

void launch_dp_tables(const double* tab, int G, int T, const int* tu, const int* td, const int* u0, const int* lon,
                      const int* loff, signed char* u_out, double* cost_out, int lanes, hipStream_t st) {
  const int gpb = 64 / lanes;
  const dim3 grid((G + gpb - 1) / gpb);
  const size_t lds = dp_tables_lds(T, lanes);
  if (lanes == 16) hipLaunchKernelGGL(k_dp_tables<16>, grid, dim3(64), lds, st, tab, G, T, tu, td, u0, lon, loff, u_out, cost_out);
  else hipLaunchKernelGGL(k_dp_tables<64>, grid, dim3(64), lds, st, tab, G, T, tu, td, u0, lon, loff, u_out, cost_out);
}

int uc_dp_blocks(const Net& n, int dp_lanes) {
  const int gpb = 64 / dp_lanes;
  return (n.G + gpb - 1) / gpb;
}

void launch_uc_dp_lanes(const Net& n, const State& s, const Par& p, hipStream_t st, int dp_lanes) {
  if (n.G == 0) return;
  const int nb = uc_dp_blocks(n, dp_lanes);
  const size_t lds = dp_slot_bytes(n.T) * (64 / dp_lanes);
  if (dp_lanes == 16) hipLaunchKernelGGL(k_uc_dp<16>, dim3(nb), dim3(64), lds, st, n, s, p);
  else hipLaunchKernelGGL(k_uc_dp<64>, dim3(nb), dim3(64), lds, st, n, s, p);
}

void launch_uc_dp(const Net& n, const State& s, const Par& p, hipStream_t st) { launch_uc_dp_lanes(n, s, p, st, 64); }

void launch_uc_dp_grouped(const Group& g, int grid, int dp_lanes, int max_T, hipStream_t st) {
  const size_t lds = dp_slot_bytes(max_T) * (64 / dp_lanes);
  if (dp_lanes == 16) hipLaunchKernelGGL(k_uc_dp_group<16>, dim3(grid), dim3(64), lds, st, g, max_T);
  else hipLaunchKernelGGL(k_uc_dp_group<64>, dim3(grid), dim3(64), lds, st, g, max_T);
}

}  // namespace ucac
