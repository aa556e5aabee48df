// Internal device-side layout of the UC-ACOPF ADMM library (gfx950).
//
// Every per-(item, period) array is stored period-major, [t][item], so a
// wavefront of consecutive lanes walks consecutive items of one period and every
// SoA load/store of the generator, line and bus kernels is coalesced.  The
// iterate lives in one flat FP64 buffer whose order is the state format of the
// C-ABI (ucac_get_state); the kernels receive raw pointers into it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ucac {

constexpr int NRB = 8;   // line rows: Pf Qf Pt Qt Wf Wt Thf Tht
constexpr int NRG = 11;  // generator rows: G1 G2 C1..C6 U1 U2 U3
enum { RB_PF, RB_QF, RB_PT, RB_QT, RB_WF, RB_WT, RB_TF, RB_TT };
enum { RG_G1, RG_G2, RG_C1, RG_C2, RG_C3, RG_C4, RG_C5, RG_C6, RG_U1, RG_U2, RG_U3 };
// Iterate scalars.  The penalties in force are part of the iterate: residual
// balancing (optional) changes them between iterations; every kernel reads them
// here.
enum { SC_BETA, SC_ZPREV, SC_KOUT, SC_LIN, SC_ITER, SC_RP, SC_RIN, SC_RD, SC_ZINF, SC_CONV,
       SC_RHO_PQ, SC_RHO_VA, SC_RHO_CPL, SC_RHO_UC, SC_NCHG_PQ, SC_NCHG_VA, SC_NCHG_CPL, SC_NCHG_UC, NSC };
enum { ACC_RP, ACC_RIN, ACC_RD, ACC_ZINF, NACC };
// Penalty classes: power rows (B1-B4, G1-G2), voltage and angle rows (B5-B8),
// coupling rows (C1-C6), commitment rows (U1-U3); and the per-class maxima the
// residual balancing needs (written only when it is on): |a + z| over the class's
// rows, the change of the duplicates they contain, |y| after the update.
enum { CL_PQ, CL_VA, CL_CPL, CL_UC, NCL };
enum { CS_RIN = 0, CS_DX = NCL, CS_Y = 2 * NCL, NCS = 3 * NCL };

constexpr int BLOCK = 256;
// Line-kernel work counters per wavefront: evaluations, rejected trials, CG
// iterations, Newton iterations, learned-start fallbacks, direct Newton steps,
// projected searches.
constexpr int NBRC = 7;
// Block size of the generator and relaxed-commitment kernels: they have few items
// (12,000 unit-periods at 2,000 buses), so smaller blocks spread the loads over more
// CUs.  The others keep 256-thread blocks, which also keeps the number of residual
// slots the control step reduces small.
constexpr int UBLOCK = 64;
constexpr double TWO_PI = 6.283185307179586;

// Device-resident control block of the iteration (written by the host between
// calls, never by a memset inside the captured graph).
struct Ctl {
  int halt;                      // set once converged in solve mode: every kernel returns at entry
  int stop_at_tol;               // solve mode
  int pending;                   // this iteration ended an inner loop: lambda kernel applies step:outer
  int bad;                       // a NaN was seen in the residuals
  double tol;
  double beta_for_lambda;        // beta of the inner loop that just ended
  double ms_tol[3];              // residual milestones 1e-2, 1e-3, 1e-4 of a solve
  int ms_iter[3];                // first iteration (counted from the solve start) with r_p, r_d <= ms_tol; -1 if not yet
  int ms_count;                  // iterations since the solve started
  int conv_iter;                 // first iteration (counted like ms_iter) with r_p, r_d <= tol; -1 if not yet
};

struct Net {
  int N, L, G, T, ref;
  // lines [L]
  const int* from;
  const int* to;
  const double* adm;  // [8][L]: G_ii B_ii G_ij B_ij G_jj B_jj G_ji B_ji
  const double* rate;
  // buses [N], loads [T][N]
  const double *gs, *bs, *vmin, *vmax, *Pd, *Qd;
  const int* inc_start;  // [N+1] incidence of line ends per bus
  const int* inc_code;   // [2L] line*2 + side (0: from end, 1: to end)
  const int* end_pos;    // [2L] position of line end line*2 + side in the incidence list
  const int* gen_start;  // [N+1]
  const int* gen_list;   // [G]
  const int* unit_first;  // [N] gen_list[gen_start[i]], the bus's first unit (0 for a bus without one)
  // generators [G]
  const double *pmin, *pmax, *qmin, *qmax, *k2, *k1, *cnl, *csu, *csd, *ru, *rd, *su, *sd, *p0;
  const int *tu, *td, *u0, *lon, *loff;
};

// Blocks of BLOCK threads over the (line, t) and (generator, t) items.
__host__ __device__ inline int line_blocks(const Net& n) { return (n.T * n.L + BLOCK - 1) / BLOCK; }
__host__ __device__ inline int gen_dual_blocks(const Net& n) { return (n.T * n.G + BLOCK - 1) / BLOCK; }

struct State {
  double *vf, *vt, *thf, *tht, *pf, *qf, *pt, *qt, *nuf, *nut;  // [T][L]
  double *p, *q, *s;                                           // s: [6][T][G]
  double *uon, *usu, *usd;                                     // [T][G] as 0.0 / 1.0
  double *wb, *thb;                                            // [T][N]
  double *Pbf, *Qbf, *Pbt, *Qbt;                               // [T][L]
  double *pb, *qb, *ubon, *ubsu, *ubsd;                        // [T][G]
  double *zB, *yB, *lB;                                        // [8][T][L]
  double *zG, *yG, *lG;                                        // [11][T][G]
  double* sc;                                                  // [NSC]
  double* ub_nxt;                                              // [3][T][G] new relaxed commitments
  int* br_iters;                                               // [T][L]
  unsigned long long* br_count;  // [waves][NBRC] running totals per wavefront of the line kernel (global lane / 64):
                                 // evaluations, rejected trials, CG its, Newton its, learned-start fallbacks,
                                 // direct Newton steps, projected searches
  double* red;                   // [red_total][NACC] per-block residual maxima of the unit side, bus and post (line ends, then generator rows)
  double* redc;                  // [red_total][NCS] the same slots' per-class maxima (residual balancing)
  int red_units, red_bus, red_bpost, red_gdual, red_n;  // first slot of each kernel's blocks; total slots
  // The unit side's slots have a second copy at red_n (G slots), so that an iteration's
  // control step can run beside the next iteration's unit blocks: red_u is where this
  // launch's unit blocks write (red_units or red_n).
  int red_u;
  // The fused iteration's slots: a second copy of the bus kernel's (red_bus2, so that
  // its control step can run beside the next bus solve; a launch's bus blocks write
  // from red_bus on, set to either copy) and the unit blocks' finish of the generator
  // rows (red_ugen, G slots); red_total slots in all.
  int red_bus2, red_ugen, red_total;
  double* ebuf;                  // [T][2L][4] per line end, in incidence order: P, Q targets, v^2, angle centres
  double* bmu;                   // [2][T][N] balance multipliers of the bus QP
  float* x0;                     // [4][T][L] start points of the learned Newton start (FP32)
  float* log_feat;               // null, or [log_cap][20] logged inputs of the learned start
  float* log_targ;               // [log_cap][4] logged solutions
  int* log_count;
  int log_cap, log_stride, log_phase;
  Ctl* ctl;
};

// Device view of the learned warm-start network: BF16 weights packed for the
// MFMA B operand (W1 [64][32] with zero columns >= 20, W2 [64][64], W3 [32][64]
// with zero rows >= 4) and FP32 biases.
struct MlpView {
  const __bf16* W1b;
  const __bf16* W2b;
  const __bf16* W3b;
  const float* b1;
  const float* b2;
  const float* b3;
};

struct Par {
  double rho_pq, rho_va, rho_uc, rho_cpl, mu;  // rho_*: the penalties in force (see live_par)
  double gtol;       // absolute projected-gradient tolerance: gtol_base * max(1, rho_pq, rho_va)
  double gtol_base;
  double tau, theta, lambda_max, beta_max, eps_in0;
  int newton_max_iter, max_inner, warm_start;  // warm_start 2: learned start from mlp
  // residual balancing: every adapt_every-th iteration (0: off), factors mu and tau,
  // at most adapt_max changes per class, within [rho0 / span, rho0 * span]
  int adapt_every, adapt_max;
  double adapt_mu, adapt_tau, adapt_span;
  // 1: the multiperiod ACOPF of the UC warm start (commitments held at their cold
  // start, no dynamic program, no commitment rows U1-U3, no minimum-generation row C1)
  int relax_uc;
  double rho0[NCL];  // the configured penalties (pq, va, cpl, uc)
  MlpView mlp;
};

// The parameters with the penalties in force, which live in the iterate's scalars
// (uniform loads).  Every kernel body starts from these.
__device__ inline Par live_par(const Par& p0, const State& s) {
  Par p = p0;
  p.rho_pq = s.sc[SC_RHO_PQ];
  p.rho_va = s.sc[SC_RHO_VA];
  p.rho_cpl = s.sc[SC_RHO_CPL];
  p.rho_uc = s.sc[SC_RHO_UC];
  p.gtol = p0.gtol_base * fmax(1.0, fmax(p.rho_pq, p.rho_va));
  return p;
}

// ---- batched (grouped) launches ----------------------------------------------
//
// Many independent instances run through one launch per kernel: the grid is the
// concatenation of every member's own grid (block ranges contiguous per member, in
// the order the tuner chose), and each block finds its member and its block index
// inside that member's grid from two small tables.  The kernel bodies are the
// single-instance ones, unchanged.
struct Member {
  Net n;
  State s;
  Par p;
};

struct Group {
  const Member* m;        // [members]
  const int* blk_member;  // [grid] member of each block
  const int* blk_first;   // [members] first block of each member's range
  const int* blk_count;   // [members] blocks of each member's range
};

// ---- reductions -------------------------------------------------------------

// max that keeps a NaN visible (fmax alone would drop it)
__device__ inline double nmax(double a, double b) { return (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000LL) : fmax(a, b); }

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide maxima of NV non-negative values, stored without atomics into this
// block's slot of NACC doubles (slot[which[k]] = max of value k; the other entries
// 0).  The control step reduces the slots of every block.  One slot per block
// instead of device-scope atomics on a few shared addresses: those serialize at
// the memory side of the chip, across its XCDs' separate L2 caches.
template <int NV, int W = NACC>
__device__ inline void block_max_store(const double (&v)[NV], const int (&which)[NV], double* slot) {
  __shared__ double red[NV][BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double w[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) w[k] = wave_max(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = w[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double out[W];
#pragma unroll
    for (int k = 0; k < W; ++k) out[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double m = red[k][0];
      for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = nmax(m, red[k][i]);
      out[which[k]] = m;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) slot[k] = out[k];
  }
}

__device__ inline double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

}  // namespace ucac
