// step:opf_bar and the multiplier updates (step:z, step:y).
//
// step:opf_bar -- the diagonal QP of every bus-side duplicate subject to the P and Q
//            balance equations (2x2 KKT system per bus; thetabar a weighted mean,
//            zero at the reference bus) -- in coalesced passes:
//            (the line kernel, one lane per (line, t), ends by storing per line end
//            the four quantities the bus sums need -- P and Q targets, v^2 and angle
//            centres -- in the bus incidence (CSR) order, so that each bus reads
//            one contiguous range)
// k_bus      one lane per (bus, t): sums its ends' quantities in incidence order,
//            solves the KKT system, writes wbar, thetabar and the two balance
//            multipliers, and updates its generators' duplicates and rows G1, G2;
//            it reads the previous relaxed commitments (the Jacobi pair
//            uc_bar || opf_bar: the new ones wait in ub_nxt);
// k_post     one launch of two block ranges: one lane per (line, t) for Pbar, Qbar
//            of both ends from the end buses' multipliers and z, y of the line's
//            eight rows (the arithmetic is the one-pass gather's, in the same
//            order); then one lane per (g, t) for z and y of rows C1..C6 and
//            U1..U3, which also commits the new relaxed commitments.
// Each kernel stores its blocks' residual maxima into per-block slots.
#include <hip/hip_ext.h>
#include "ucac_launch.hpp"
#include "ucac_rows.hpp"
#include "ucac_ctl.hpp"

namespace ucac {

// The consensus and next-period ramp terms of unit g at bus-side item k = t * G + g
// (the previous relaxed commitments): weight Wp and weighted centre Sp of pbar_t,
// and the centre tq of qbar_t.
__device__ inline void unit_terms(const Net& n, const State& s, const Par& p, int t, int k, int g, double& Wp,
                                  double& Sp, double& tq) {
  const int T = n.T, G = n.G, TG = T * G;
  const double rpq = p.rho_pq, rc = p.rho_cpl;
  Wp = rpq;
  Sp = rpq * (s.p[k] + s.zG[RG_G1 * TG + k] + s.yG[RG_G1 * TG + k] / rpq);
  if (t + 1 < T) {
    const int kn = k + G;
    const double t5 = s.p[kn] - s.s[4 * TG + kn] + n.rd[g] * s.ubon[kn] + n.sd[g] * s.ubsd[kn] +
                      s.zG[RG_C5 * TG + kn] + s.yG[RG_C5 * TG + kn] / rc;
    const double t6 = s.p[kn] + s.s[5 * TG + kn] - n.ru[g] * s.ubon[k] - n.su[g] * s.ubsu[kn] +
                      s.zG[RG_C6 * TG + kn] + s.yG[RG_C6 * TG + kn] / rc;
    Wp += 2.0 * rc;
    Sp += rc * t5 + rc * t6;
  }
  tq = s.q[k] + s.zG[RG_G2 * TG + k] + s.yG[RG_G2 * TG + k] / rpq;
}

// A unit's data as the bus solve and its update need them: the consensus and ramp
// terms, the previous bus-side values, its own p and q, and its two coupling rows.
struct UnitPre {
  int k;
  double Wp, Sp, tq, pold, qold, pv, qv;
  RowZY r1, r2;
};

// The values unit g at item k = t * G + g contributes, loaded without arithmetic so
// that the loads stay in flight while other work proceeds (the next-period values
// come from k itself in the last period, and are then unused).
struct UnitRaw {
  int k;
  double p, q, pb, qb, rd, sd, ru, su, ubon;
  RowZY r1, r2;
  double pn, s4n, s5n, ubonn, ubsdn, ubsun, z5n, y5n, z6n, y6n;
};

__device__ inline UnitRaw unit_raw(const Net& n, const State& s, int t, int g) {
  const int T = n.T, G = n.G, TG = T * G;
  UnitRaw r;
  const int k = t * G + g, kn = t + 1 < T ? k + G : k;
  r.k = k;
  r.p = s.p[k]; r.q = s.q[k]; r.pb = s.pb[k]; r.qb = s.qb[k];
  r.rd = n.rd[g]; r.sd = n.sd[g]; r.ru = n.ru[g]; r.su = n.su[g];
  r.ubon = s.ubon[k];
  r.r1 = row_load(s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, k);
  r.r2 = row_load(s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, k);
  r.pn = s.p[kn]; r.s4n = s.s[4 * TG + kn]; r.s5n = s.s[5 * TG + kn];
  r.ubonn = s.ubon[kn]; r.ubsdn = s.ubsd[kn]; r.ubsun = s.ubsu[kn];
  r.z5n = s.zG[RG_C5 * TG + kn]; r.y5n = s.yG[RG_C5 * TG + kn];
  r.z6n = s.zG[RG_C6 * TG + kn]; r.y6n = s.yG[RG_C6 * TG + kn];
  return r;
}

// unit_terms on loaded values: the same operations in the same order.
__device__ inline UnitPre unit_pre(const UnitRaw& r, const Par& p, int t, int T) {
  const double rpq = p.rho_pq, rc = p.rho_cpl;
  UnitPre u;
  u.k = r.k;
  u.Wp = rpq;
  u.Sp = rpq * (r.p + r.r1.z + r.r1.y / rpq);
  if (t + 1 < T) {
    const double t5 = r.pn - r.s4n + r.rd * r.ubonn + r.sd * r.ubsdn + r.z5n + r.y5n / rc;
    const double t6 = r.pn + r.s5n - r.ru * r.ubon - r.su * r.ubsun + r.z6n + r.y6n / rc;
    u.Wp += 2.0 * rc;
    u.Sp += rc * t5 + rc * t6;
  }
  u.tq = r.q + r.r2.z + r.r2.y / rpq;
  u.pold = r.pb; u.qold = r.qb; u.pv = r.p; u.qv = r.q;
  u.r1 = r.r1; u.r2 = r.r2;
  return u;
}

// One lane per (bus, t).  The loads form two dependent rounds: (1) the bus's own
// values, its incidence ranges and its first unit (a static per-bus index); (2) that
// unit's terms, rows and previous values (kept in registers through the solve and the
// update) together with the sums of up to eight line ends.  The end loads are
// unconditional (clamped indices; the contributions of unused slots are selected away
// as +0.0, which leaves every sum exactly as if they were skipped), so that none of
// them waits behind another; the sums keep the incidence order.
// ROWS = false: the bus solve alone (the fused iteration: rows G1, G2 are updated by
// the next launch's unit blocks, from the duplicates stored here).
template <bool ROWS>
__device__ __forceinline__ void bus_body_t(const Net& n, const State& s, const Par& p0, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const int N = n.N, G = n.G, T = n.T;
  const int TG = T * G;
  const int idx = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0;
  double rin_pq = 0.0, y_pq = 0.0, dx_va = 0.0, dx_pq = 0.0, dx_pb = 0.0;  // class maxima
  if (idx < T * N) {
    const int t = idx / N, i = idx - t * N;
    const double rpq = p.rho_pq, rva = p.rho_va;
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    // first load round
    const int e0 = n.inc_start[i], e1 = n.inc_start[i + 1];
    const int g0 = n.gen_start[i], g1 = n.gen_start[i + 1];
    const double wold = s.wb[idx], thold = s.thb[idx];
    const double gsh = n.gs[i], bsh = n.bs[i], Pd = n.Pd[idx], Qd = n.Qd[idx];
    const int gfirst = n.unit_first[i];
    // second load round: the first unit's data, issued before the end sums' loads so
    // that both travel together
    const int nu = g1 - g0;
    UnitRaw u0raw;
    if (nu > 0) u0raw = unit_raw(n, s, t, gfirst);
    double Ww = 0.0, Sw = 0.0, Wt = 0.0, St = 0.0;
    double M11 = 0.0, M12 = 0.0, M22 = 0.0, aT = 0.0, bT = 0.0;
    const double* eb = s.ebuf + (size_t)t * 2 * n.L * 4;
    constexpr int ER = 8;  // ends per round: every bus of the benchmark meshes in one
    for (int e = e0; e < e1; e += ER) {
      double q[ER][4];
#pragma unroll
      for (int j = 0; j < ER; ++j) {
        const double* src = eb + (size_t)(e + j < e1 ? e + j : e0) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) q[j][c] = src[c];
      }
#pragma unroll
      for (int j = 0; j < ER; ++j) {
        const bool on = e + j < e1;
        M11 += on ? 1.0 / rpq : 0.0;
        aT -= on ? q[j][0] : 0.0;
        M22 += on ? 1.0 / rpq : 0.0;
        bT -= on ? q[j][1] : 0.0;
        Ww += on ? rva : 0.0;
        Sw += on ? rva * q[j][2] : 0.0;
        Wt += on ? rva : 0.0;
        St += on ? rva * q[j][3] : 0.0;
      }
    }
    UnitPre u0;
    if (nu > 0) u0 = unit_pre(u0raw, p, t, T);
    for (int e = g0; e < g1; ++e) {
      double Wp, Sp, tq;
      if (e == g0) { Wp = u0.Wp; Sp = u0.Sp; tq = u0.tq; }
      else {
        const int g = n.gen_list[e];
        unit_terms(n, s, p, t, t * G + g, g, Wp, Sp, tq);
      }
      M11 += 1.0 / Wp;
      aT += Sp / Wp;
      M22 += 1.0 / rpq;
      bT += tq;
    }
    const bool has_w = Ww > 0.0;
    const double tauw = has_w ? Sw / Ww : wold;
    const double aw = has_w ? -gsh : 0.0, bw = has_w ? bsh : 0.0;
    if (has_w) { M11 += aw * aw / Ww; M12 += aw * bw / Ww; M22 += bw * bw / Ww; }
    aT += aw * tauw;
    bT += bw * tauw;
    const double r1 = Pd - aT, r2 = Qd - bT;
    const double det = M11 * M22 - M12 * M12;
    const double mu1 = (M22 * r1 - M12 * r2) / det;
    const double mu2 = (M11 * r2 - M12 * r1) / det;
    const double wnew = has_w ? tauw + (aw * mu1 + bw * mu2) / Ww : wold;
    const double thnew = (i == n.ref) ? 0.0 : (Wt > 0.0 ? St / Wt : thold);
    rd = nmax(fabs(wnew - wold), fabs(thnew - thold));
    dx_va = rd;
    for (int e = g0; e < g1; ++e) {
      UnitPre v = e == g0 ? u0 : unit_pre(unit_raw(n, s, t, n.gen_list[e]), p, t, T);
      const double pn = v.Sp / v.Wp + mu1 / v.Wp, qn = v.tq + mu2 / rpq;
      rd = nmax(rd, nmax(fabs(pn - v.pold), fabs(qn - v.qold)));
      dx_pb = nmax(dx_pb, fabs(pn - v.pold));
      dx_pq = nmax(dx_pq, nmax(fabs(pn - v.pold), fabs(qn - v.qold)));
      if (ROWS) {
        row_update_c(v.r1, v.pv - pn, rpq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
        row_update_c(v.r2, v.qv - qn, rpq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
      }
      s.pb[v.k] = pn;
      s.qb[v.k] = qn;
      if (ROWS) {
        row_store(v.r1, s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, v.k, lu);
        row_store(v.r2, s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, v.k, lu);
      }
    }
    s.wb[idx] = wnew;
    s.thb[idx] = thnew;
    s.bmu[idx] = mu1;
    s.bmu[T * N + idx] = mu2;
  }
  const double v[4] = {rp, rin, rd, zinf};
  const int which[4] = {ACC_RP, ACC_RIN, ACC_RD, ACC_ZINF};
  block_max_store<4>(v, which, s.red + (size_t)(s.red_bus + blk) * NACC);
  if (p.adapt_every > 0) {
    // (without the rows G1, G2 their class maxima come from the unit blocks' finish)
    const double vc[5] = {rin_pq, y_pq, dx_va, dx_pq, dx_pb};
    const int wc[5] = {CS_RIN + CL_PQ, CS_Y + CL_PQ, CS_DX + CL_VA, CS_DX + CL_PQ, CS_DX + CL_CPL};
    block_max_store<5, NCS>(vc, wc, s.redc + (size_t)(s.red_bus + blk) * NCS);
  }
}

__device__ __forceinline__ void bus_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  bus_body_t<true>(n, s, p, blk, nblk);
}

__global__ void __launch_bounds__(BLOCK) k_bus(Net n, State s, Par p) { bus_body(n, s, p, blockIdx.x, gridDim.x); }

// The second launch of the fused iteration: the bus solve without rows G1, G2 (its
// blocks write their residual slots from s.red_bus on, the copy the caller chose), and
// with has_fin set, a first block that runs the previous iteration's control step over
// the slot ranges fin.  That step writes nothing the bus solve reads: the penalties
// stay fixed (no residual balancing), the stop flag is never set (step mode), and the
// multiplier step and beta it may decide are read only by the next launch's row updates.
__global__ void __launch_bounds__(BLOCK) k_bus_fused(Net n, State s, Par p, SlotRanges fin, int has_fin) {
  static_assert(BLOCK == FIN_BLOCK, "the control step runs as one block of this launch");
  int b = blockIdx.x;
  if (has_fin) {
    if (b == 0) { finalize_ranges(s, p, fin); return; }
    --b;
  }
  bus_body_t<false>(n, s, p, b, (int)gridDim.x - has_fin);
}

__global__ void __launch_bounds__(BLOCK) k_bus_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  bus_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}

__device__ __forceinline__ void gen_dual_body(const Net& n, const State& s, const Par& p0, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const int G = n.G, TG = n.T * G;
  const int i = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, zinf = 0.0;
  double rin_c = 0.0, rin_u = 0.0, y_c = 0.0, y_u = 0.0;  // class maxima (coupling, commitment rows)
  if (i < TG) {
    const int t = i / G, g = i - t * G;
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    cu_rows_item(n, s, p, t, g, i, beta, lu, rp, rin, zinf, rin_c, rin_u, y_c, y_u);
  }
  const double v[3] = {rp, rin, zinf};
  const int which[3] = {ACC_RP, ACC_RIN, ACC_ZINF};
  block_max_store<3>(v, which, s.red + (size_t)(s.red_gdual + blk) * NACC);
  if (p.adapt_every > 0) {
    const double vc[4] = {rin_c, rin_u, y_c, y_u};
    const int wc[4] = {CS_RIN + CL_CPL, CS_RIN + CL_UC, CS_Y + CL_CPL, CS_Y + CL_UC};
    block_max_store<4, NCS>(vc, wc, s.redc + (size_t)(s.red_gdual + blk) * NCS);
  }
}

// step:opf_bar's line-end finish and the generator rows' multipliers in one launch:
// the first line_blocks blocks finish the line ends (bus_post_body), the rest update
// the coupling and commitment rows (gen_dual_body).  Both need only the bus solve,
// touch disjoint rows and write their own residual slots; one launch costs one
// kernel boundary on the iteration's critical path instead of a fork and a join.
__device__ __forceinline__ void post_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  const int nbp = line_blocks(n);
  if (blk < nbp) bus_post_body(n, s, p, blk, nbp);
  else gen_dual_body(n, s, p, blk - nbp, nblk - nbp);
}

__global__ void __launch_bounds__(BLOCK) k_post(Net n, State s, Par p) { post_body(n, s, p, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(BLOCK) k_post_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  post_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}

int bus_blocks(const Net& n) { return (n.T * n.N + BLOCK - 1) / BLOCK; }
int post_blocks(const Net& n) { return line_blocks(n) + gen_dual_blocks(n); }

void launch_bus_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_bus_group, dim3(grid), dim3(BLOCK), 0, st, g);
}
void launch_post_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_post_group, dim3(grid), dim3(BLOCK), 0, st, g);
}


void launch_bus(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const int TN = n.T * n.N;
  if (TN == 0) return;
  hipLaunchKernelGGL(k_bus, dim3(bus_blocks(n)), dim3(BLOCK), 0, st, n, s, p);
}

void launch_bus_fused(const Net& n, const State& s, const Par& p, hipStream_t st, const SlotRanges* fin) {
  const int nb = n.T * n.N ? bus_blocks(n) : 0;
  const int nf = fin ? 1 : 0;
  if (nb + nf == 0) return;
  const SlotRanges none{};
  hipLaunchKernelGGL(k_bus_fused, dim3(nf + nb), dim3(BLOCK), 0, st, n, s, p, fin ? *fin : none, nf);
}

void launch_post(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const int nb = post_blocks(n);
  if (nb == 0) return;
  hipLaunchKernelGGL(k_post, dim3(nb), dim3(BLOCK), 0, st, n, s, p);
}

bool launch_bus_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (n.T * n.N == 0) return false;
  hipExtLaunchKernelGGL(k_bus, dim3(bus_blocks(n)), dim3(BLOCK), 0, st, e0, e1, 0u, n, s, p);
  return true;
}

bool launch_post_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int nb = post_blocks(n);
  if (nb == 0) return false;
  hipExtLaunchKernelGGL(k_post, dim3(nb), dim3(BLOCK), 0, st, e0, e1, 0u, n, s, p);
  return true;
}

}  // namespace ucac
