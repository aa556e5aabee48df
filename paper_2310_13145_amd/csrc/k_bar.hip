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
#include "ucac_launch.hpp"

namespace ucac {

// A step:outer multiplier update decided by the previous iteration's control is
// applied here, by the kernel that owns the row, just before the row's z update
// (the multiplier is read nowhere else): lambda <- clamp(lambda + beta_prev z_prev).
struct LamUpd {
  bool on;
  double b, lm;
};

__device__ inline LamUpd lambda_pending(const State& s, const Par& p) {
  LamUpd u;
  u.on = s.ctl->pending != 0;
  u.b = s.ctl->beta_for_lambda;
  u.lm = p.lambda_max;
  return u;
}

// step:z and step:y of one row with value a = (Ax + Bxbar)_r, in three parts so that
// a lane issues the loads of all its rows before its first store (a store may
// alias any later load, so interleaving them costs one memory round trip per row):
//   z <- -(lambda + y + rho a) / (beta + rho),  y <- y + rho (a + z),
// with a pending step:outer update lambda <- clamp(lambda + beta_prev z_prev) first.
// The residual maxima r_p = |a|, r_in = |a + z| and ||z|| are accumulated.
struct RowZY {
  double z, y, l;
};

__device__ inline RowZY row_load(const double* zr, const double* yr, const double* lr, int k) {
  return RowZY{zr[k], yr[k], lr[k]};
}

__device__ inline void row_update(RowZY& r, double a, double rho, double beta, const LamUpd& lu, double& rp, double& rin,
                                  double& zinf) {
  if (lu.on) r.l = clampd(r.l + lu.b * r.z, -lu.lm, lu.lm);
  const double z = -(r.l + r.y + rho * a) / (beta + rho);
  r.y = r.y + rho * (a + z);
  r.z = z;
  rp = nmax(rp, fabs(a));
  rin = nmax(rin, fabs(a + z));
  zinf = nmax(zinf, fabs(z));
}

__device__ inline void row_store(const RowZY& r, double* zr, double* yr, double* lr, int k, const LamUpd& lu) {
  zr[k] = r.z;
  yr[k] = r.y;
  if (lu.on) lr[k] = r.l;
}



struct EndData {
  int k, rP, rQ, rW, rT;
  double fP, fQ, v, th, tP, tQ;
};

__device__ inline EndData load_end(const Net& n, const State& s, int t, int TL, int code, double rpq) {
  EndData d;
  const int l = code >> 1, side = code & 1;
  d.k = t * n.L + l;
  d.rP = side ? RB_PT : RB_PF; d.rQ = side ? RB_QT : RB_QF; d.rW = side ? RB_WT : RB_WF; d.rT = side ? RB_TT : RB_TF;
  d.fP = side ? s.pt[d.k] : s.pf[d.k];
  d.fQ = side ? s.qt[d.k] : s.qf[d.k];
  d.v = side ? s.vt[d.k] : s.vf[d.k];
  d.th = side ? s.tht[d.k] : s.thf[d.k];
  d.tP = d.fP + s.zB[d.rP * TL + d.k] + s.yB[d.rP * TL + d.k] / rpq;
  d.tQ = d.fQ + s.zB[d.rQ * TL + d.k] + s.yB[d.rQ * TL + d.k] / rpq;
  return d;
}

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

__device__ __forceinline__ void bus_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int N = n.N, G = n.G, T = n.T;
  const int TG = T * G;
  const int idx = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0;
  if (idx < T * N) {
    const int t = idx / N, i = idx - t * N;
    const double rpq = p.rho_pq, rva = p.rho_va;
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    const int e0 = n.inc_start[i], e1 = n.inc_start[i + 1];
    double Ww = 0.0, Sw = 0.0, Wt = 0.0, St = 0.0;
    double M11 = 0.0, M12 = 0.0, M22 = 0.0, aT = 0.0, bT = 0.0;
    const double* eb = s.ebuf + (size_t)t * 2 * n.L * 4;
    // four ends' sums loaded per round (all loads in flight), then added in order
    for (int e = e0; e < e1; e += 4) {
      double q[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double* src = eb + (size_t)(e + j < e1 ? e + j : e0) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) q[j][c] = src[c];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (e + j >= e1) break;
        M11 += 1.0 / rpq;
        aT -= q[j][0];
        M22 += 1.0 / rpq;
        bT -= q[j][1];
        Ww += rva;
        Sw += rva * q[j][2];
        Wt += rva;
        St += rva * q[j][3];
      }
    }
    const int g0 = n.gen_start[i], g1 = n.gen_start[i + 1];
    // the first two units' terms stay in registers for their updates after the solve
    double cW[2] = {0.0, 0.0}, cS[2] = {0.0, 0.0}, cq[2] = {0.0, 0.0};
    for (int e = g0; e < g1; ++e) {
      const int g = n.gen_list[e], k = t * G + g;
      double Wp, Sp, tq;
      unit_terms(n, s, p, t, k, g, Wp, Sp, tq);
      if (e == g0) { cW[0] = Wp; cS[0] = Sp; cq[0] = tq; }
      if (e == g0 + 1) { cW[1] = Wp; cS[1] = Sp; cq[1] = tq; }
      M11 += 1.0 / Wp;
      aT += Sp / Wp;
      M22 += 1.0 / rpq;
      bT += tq;
    }
    const double wold = s.wb[idx], thold = s.thb[idx];
    const bool has_w = Ww > 0.0;
    const double tauw = has_w ? Sw / Ww : wold;
    const double aw = has_w ? -n.gs[i] : 0.0, bw = has_w ? n.bs[i] : 0.0;
    if (has_w) { M11 += aw * aw / Ww; M12 += aw * bw / Ww; M22 += bw * bw / Ww; }
    aT += aw * tauw;
    bT += bw * tauw;
    const double r1 = n.Pd[idx] - aT, r2 = n.Qd[idx] - bT;
    const double det = M11 * M22 - M12 * M12;
    const double mu1 = (M22 * r1 - M12 * r2) / det;
    const double mu2 = (M11 * r2 - M12 * r1) / det;
    const double wnew = has_w ? tauw + (aw * mu1 + bw * mu2) / Ww : wold;
    const double thnew = (i == n.ref) ? 0.0 : (Wt > 0.0 ? St / Wt : thold);
    rd = nmax(fabs(wnew - wold), fabs(thnew - thold));
    for (int e = g0; e < g1; ++e) {
      const int g = n.gen_list[e], k = t * G + g;
      double Wp, Sp, tq;
      if (e == g0) { Wp = cW[0]; Sp = cS[0]; tq = cq[0]; }
      else if (e == g0 + 1) { Wp = cW[1]; Sp = cS[1]; tq = cq[1]; }
      else unit_terms(n, s, p, t, k, g, Wp, Sp, tq);
      const double pn = Sp / Wp + mu1 / Wp, qn = tq + mu2 / rpq;
      const double pold = s.pb[k], qold = s.qb[k], pv = s.p[k], qv = s.q[k];
      RowZY r1 = row_load(s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, k);
      RowZY r2 = row_load(s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, k);
      rd = nmax(rd, nmax(fabs(pn - pold), fabs(qn - qold)));
      row_update(r1, pv - pn, rpq, beta, lu, rp, rin, zinf);
      row_update(r2, qv - qn, rpq, beta, lu, rp, rin, zinf);
      s.pb[k] = pn;
      s.qb[k] = qn;
      row_store(r1, s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, k, lu);
      row_store(r2, s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, k, lu);
    }
    s.wb[idx] = wnew;
    s.thb[idx] = thnew;
    s.bmu[idx] = mu1;
    s.bmu[T * N + idx] = mu2;
  }
  const double v[4] = {rp, rin, rd, zinf};
  const int which[4] = {ACC_RP, ACC_RIN, ACC_RD, ACC_ZINF};
  block_max_store<4>(v, which, s.red + (size_t)(s.red_bus + blk) * NACC);
}

__device__ __forceinline__ void bus_post_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int TL = n.T * n.L, TN = n.T * n.N;
  const int idx = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0;
  if (idx < TL) {
    const int t = idx / n.L, l = idx - t * n.L;
    const double rpq = p.rho_pq, rva = p.rho_va;
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    // every load of both ends first, then the updates, then the stores
    EndData d[2];
    double mu1[2], mu2[2], wnew[2], thnew[2], Pold[2], Qold[2];
    RowZY r[2][4];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      d[side] = load_end(n, s, t, TL, 2 * l + side, rpq);
      const int b = t * n.N + (side ? n.to[l] : n.from[l]);
      mu1[side] = s.bmu[b]; mu2[side] = s.bmu[TN + b]; wnew[side] = s.wb[b]; thnew[side] = s.thb[b];
      const int k = d[side].k;
      Pold[side] = side ? s.Pbt[k] : s.Pbf[k];
      Qold[side] = side ? s.Qbt[k] : s.Qbf[k];
      const int rows[4] = {d[side].rP, d[side].rQ, d[side].rW, d[side].rT};
#pragma unroll
      for (int q = 0; q < 4; ++q) r[side][q] = row_load(s.zB + rows[q] * TL, s.yB + rows[q] * TL, s.lB + rows[q] * TL, k);
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const EndData& q = d[side];
      const double Pn = q.tP - mu1[side] / rpq, Qn = q.tQ - mu2[side] / rpq;
      rd = nmax(rd, nmax(fabs(Pn - Pold[side]), fabs(Qn - Qold[side])));
      row_update(r[side][0], q.fP - Pn, rpq, beta, lu, rp, rin, zinf);
      row_update(r[side][1], q.fQ - Qn, rpq, beta, lu, rp, rin, zinf);
      row_update(r[side][2], q.v * q.v - wnew[side], rva, beta, lu, rp, rin, zinf);
      row_update(r[side][3], q.th - thnew[side], rva, beta, lu, rp, rin, zinf);
      double* Pdup = side ? s.Pbt : s.Pbf;
      double* Qdup = side ? s.Qbt : s.Qbf;
      Pdup[q.k] = Pn;
      Qdup[q.k] = Qn;
      const int rows[4] = {q.rP, q.rQ, q.rW, q.rT};
#pragma unroll
      for (int w = 0; w < 4; ++w) row_store(r[side][w], s.zB + rows[w] * TL, s.yB + rows[w] * TL, s.lB + rows[w] * TL, q.k, lu);
    }
  }
  const double v[4] = {rp, rin, rd, zinf};
  const int which[4] = {ACC_RP, ACC_RIN, ACC_RD, ACC_ZINF};
  block_max_store<4>(v, which, s.red + (size_t)(s.red_bpost + blk) * NACC);
}

__global__ void __launch_bounds__(BLOCK) k_bus(Net n, State s, Par p) { bus_body(n, s, p, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(BLOCK) k_bus_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  bus_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}

__device__ __forceinline__ void gen_dual_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int G = n.G, TG = n.T * G;
  const int i = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, zinf = 0.0;
  if (i < TG) {
    const int t = i / G, g = i - t * G;
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    const double* nx_on = s.ub_nxt;
    const double* nx_su = s.ub_nxt + TG;
    const double* nx_sd = s.ub_nxt + 2 * TG;
    const double uon = nx_on[i], usu = nx_su[i], usd = nx_sd[i];
    const double uonp = t == 0 ? (double)n.u0[g] : nx_on[i - G];
    const double pbp = t == 0 ? n.p0[g] : s.pb[i - G];
    const double pv = s.p[i], qv = s.q[i];
    double a[9];
    a[0] = pv - s.s[0 * TG + i] - n.pmin[g] * uon;
    a[1] = pv + s.s[1 * TG + i] - n.pmax[g] * uon;
    a[2] = qv - s.s[2 * TG + i] - n.qmin[g] * uon;
    a[3] = qv + s.s[3 * TG + i] - n.qmax[g] * uon;
    a[4] = pv - pbp - s.s[4 * TG + i] + n.rd[g] * uon + n.sd[g] * usd;
    a[5] = pv - pbp + s.s[5 * TG + i] - n.ru[g] * uonp - n.su[g] * usu;
    a[6] = s.uon[i] - uon;
    a[7] = s.usu[i] - usu;
    a[8] = s.usd[i] - usd;
    RowZY rz[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) rz[r] = row_load(s.zG + (RG_C1 + r) * TG, s.yG + (RG_C1 + r) * TG, s.lG + (RG_C1 + r) * TG, i);
#pragma unroll
    for (int r = 0; r < 9; ++r) row_update(rz[r], a[r], r < 6 ? p.rho_cpl : p.rho_uc, beta, lu, rp, rin, zinf);
#pragma unroll
    for (int r = 0; r < 9; ++r) row_store(rz[r], s.zG + (RG_C1 + r) * TG, s.yG + (RG_C1 + r) * TG, s.lG + (RG_C1 + r) * TG, i, lu);
    s.ubon[i] = uon;
    s.ubsu[i] = usu;
    s.ubsd[i] = usd;
  }
  const double v[3] = {rp, rin, zinf};
  const int which[3] = {ACC_RP, ACC_RIN, ACC_ZINF};
  block_max_store<3>(v, which, s.red + (size_t)(s.red_gdual + blk) * NACC);
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

void launch_post(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const int nb = post_blocks(n);
  if (nb == 0) return;
  hipLaunchKernelGGL(k_post, dim3(nb), dim3(BLOCK), 0, st, n, s, p);
}

}  // namespace ucac
