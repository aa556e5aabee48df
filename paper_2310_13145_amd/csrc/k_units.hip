// The unit side of the inner iteration (ucac_units.hpp) as kernels of its own, and
// the standalone batch of dynamic programs on given cost tables.
//
// This file is compiled with -ffp-contract=off.
#include <hip/hip_ext.h>
#include "ucac_launch.hpp"
#include "ucac_units.hpp"

namespace ucac {

// Unit blocks of their own launch are UNIT_BLOCK threads.
constexpr int UNIT_BLOCK = 256;

__global__ void __launch_bounds__(UNIT_BLOCK) k_units(Net n, State s, Par p, int gpb) {
  unit_body<UNIT_BLOCK>(n, s, p, blockIdx.x, n.T, gpb);
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
  double* P = Lt + 4 * T;
  double* c = P + 2 * T;
  unsigned char* dec = (unsigned char*)(c + 2 * (T + 2));
  signed char* u = (signed char*)(dec + 2 * (T + 2));
  if (act) {
    const double* src = tab + (size_t)g * T * 4;
    for (int k = lane; k < 4 * T; k += LPG) Lt[k] = src[k];
  }
  __syncthreads();
  if (act) dp_switch_sums(T, Lt, P, tu[g], td[g], lane, LPG);
  __syncthreads();
  if (act && lane == 0) cost_out[g] = dp_recursion(T, Lt, P, c, dec, u, u0[g], lon[g], loff[g], tu[g], td[g]);
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

// Generators per unit block: 256 / dp_lanes (dp_lanes: threads per generator, 16 or
// 64), reduced (16 -> 4 -> 1) while the DP slots for horizon T exceed the LDS one
// block of bs threads may take when it shares a launch with the line kernel: at the
// line kernel's two wavefronts per SIMD a compute unit holds 512 / bs blocks, each
// with the line kernel's 11 * 8 * bs bytes of static LDS.
int units_gpb(int T, int dp_lanes, int bs) {
  const size_t budget = (size_t)160 * 1024 * bs / 512 - (size_t)11 * 8 * bs - 256;
  int g = 256 / dp_lanes;
  while (g > 1 && dp_slot_bytes(T) * (size_t)g > budget) g = g == 16 ? 4 : 1;
  return g;
}

size_t units_lds(int T, int gpb) { return dp_slot_bytes(T) * (size_t)gpb; }

int units_blocks(const Net& n, int gpb) { return unit_blocks(n.G, gpb); }

void launch_units_lanes(const Net& n, const State& s, const Par& p, hipStream_t st, int dp_lanes) {
  if (n.G == 0 || n.T == 0) return;
  const int gpb = units_gpb(n.T, dp_lanes, 256);
  hipLaunchKernelGGL(k_units, dim3(units_blocks(n, gpb)), dim3(UNIT_BLOCK), units_lds(n.T, gpb), st, n, s, p, gpb);
}

void launch_units(const Net& n, const State& s, const Par& p, hipStream_t st) { launch_units_lanes(n, s, p, st, 16); }

bool launch_units_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (n.G == 0 || n.T == 0) return false;
  const int gpb = units_gpb(n.T, 16, 256);
  hipExtLaunchKernelGGL(k_units, dim3(units_blocks(n, gpb)), dim3(UNIT_BLOCK), units_lds(n.T, gpb), st, e0, e1, 0u, n, s,
                        p, gpb);
  return true;
}

}  // namespace ucac
