// Row updates (step:z, step:y) shared by the bus-side kernels and the fused
// iteration, whose unit and line blocks finish the previous iteration's rows before
// their own work.  Every function here declares contraction off: the same
// arithmetic, rounded as plain IEEE FP64, in whichever translation unit runs it.
#pragma once
#include "ucac_dev.hpp"

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
#pragma clang fp contract(off)
  if (lu.on) r.l = clampd(r.l + lu.b * r.z, -lu.lm, lu.lm);
  const double z = -(r.l + r.y + rho * a) / (beta + rho);
  r.y = r.y + rho * (a + z);
  r.z = z;
  rp = nmax(rp, fabs(a));
  rin = nmax(rin, fabs(a + z));
  zinf = nmax(zinf, fabs(z));
}

// row_update that also accumulates the row's class maxima |a + z| and |y| (residual
// balancing); the row's own arithmetic is row_update's.
__device__ inline void row_update_c(RowZY& r, double a, double rho, double beta, const LamUpd& lu, double& rp,
                                    double& rin, double& zinf, double& rin_c, double& y_c) {
#pragma clang fp contract(off)
  row_update(r, a, rho, beta, lu, rp, rin, zinf);
  rin_c = nmax(rin_c, fabs(a + r.z));
  y_c = nmax(y_c, fabs(r.y));
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
#pragma clang fp contract(off)
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

// The coupling and commitment rows (C1-C6, U1-U3) of item i = t * G + g with the
// relaxed commitments that wait in ub_nxt, which are then committed.
__device__ inline void cu_rows_item(const Net& n, const State& s, const Par& p, const int t, const int g, const int i,
                                    const double beta, const LamUpd& lu, double& rp, double& rin, double& zinf,
                                    double& rin_c, double& rin_u, double& y_c, double& y_u) {
#pragma clang fp contract(off)
  const int G = n.G, TG = n.T * G;
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
  for (int r = 0; r < 9; ++r) {
    // the multiperiod ACOPF has no minimum-generation row (C1) and no commitment
    // rows (U1-U3): their z, y stay as they are and they count in no residual
    if (p.relax_uc && (r == 0 || r >= 6)) continue;
    if (r < 6) row_update_c(rz[r], a[r], p.rho_cpl, beta, lu, rp, rin, zinf, rin_c, y_c);
    else row_update_c(rz[r], a[r], p.rho_uc, beta, lu, rp, rin, zinf, rin_u, y_u);
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) row_store(rz[r], s.zG + (RG_C1 + r) * TG, s.yG + (RG_C1 + r) * TG, s.lG + (RG_C1 + r) * TG, i, lu);
  s.ubon[i] = uon;
  s.ubsu[i] = usu;
  s.ubsd[i] = usd;
}

// Rows G1, G2 of item i from the bus solve's duplicates pbar, qbar once they are
// stored: a = p - pbar and q - qbar (the bus kernel's own update of these rows takes
// the same values from its registers).
__device__ inline void g12_rows_item(const State& s, const Par& p, const int TG, const int i, const double beta,
                                     const LamUpd& lu, double& rp, double& rin, double& zinf, double& rin_pq,
                                     double& y_pq) {
#pragma clang fp contract(off)
  RowZY r1 = row_load(s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, i);
  RowZY r2 = row_load(s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, i);
  const double a1 = s.p[i] - s.pb[i], a2 = s.q[i] - s.qb[i];
  row_update_c(r1, a1, p.rho_pq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
  row_update_c(r2, a2, p.rho_pq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
  row_store(r1, s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, i, lu);
  row_store(r2, s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, i, lu);
}

// What the line-end finish of one item computes, for a caller that goes on with the
// item (the fused iteration's line lane), by line row (Pf Qf Pt Qt Wf Wt Thf Tht):
// the bus-side values the rows compare with (the new Pbar, Qbar of both ends, the end
// buses' wbar and thetabar) and the rows' new z and y.
struct LineFinish {
  double xb[NRB], z[NRB], y[NRB];
};

// The line-end finish of line item idx = t * L + l (step:opf_bar's Pbar, Qbar of both
// ends from the end buses' balance multipliers, then z, y of the line's eight rows),
// accumulating the residual maxima; with out set, also what LineFinish holds.
__device__ inline void line_finish_item(const Net& n, const State& s, const Par& p, const int idx, const double beta,
                                        const LamUpd& lu, double& rp, double& rin, double& rd, double& zinf,
                                        double& rin_pq, double& rin_va, double& y_pq, double& y_va,
                                        LineFinish* out) {
#pragma clang fp contract(off)
  const int TL = n.T * n.L, TN = n.T * n.N;
  const int t = idx / n.L, l = idx - t * n.L;
  const double rpq = p.rho_pq, rva = p.rho_va;
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
    row_update_c(r[side][0], q.fP - Pn, rpq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
    row_update_c(r[side][1], q.fQ - Qn, rpq, beta, lu, rp, rin, zinf, rin_pq, y_pq);
    row_update_c(r[side][2], q.v * q.v - wnew[side], rva, beta, lu, rp, rin, zinf, rin_va, y_va);
    row_update_c(r[side][3], q.th - thnew[side], rva, beta, lu, rp, rin, zinf, rin_va, y_va);
    double* Pdup = side ? s.Pbt : s.Pbf;
    double* Qdup = side ? s.Qbt : s.Qbf;
    Pdup[q.k] = Pn;
    Qdup[q.k] = Qn;
    const int rows[4] = {q.rP, q.rQ, q.rW, q.rT};
#pragma unroll
    for (int w = 0; w < 4; ++w) row_store(r[side][w], s.zB + rows[w] * TL, s.yB + rows[w] * TL, s.lB + rows[w] * TL, q.k, lu);
    if (out) {
      const double xb[4] = {Pn, Qn, wnew[side], thnew[side]};
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        out->xb[rows[w]] = xb[w];
        out->z[rows[w]] = r[side][w].z;
        out->y[rows[w]] = r[side][w].y;
      }
    }
  }
}

// Residual maxima of a block's line-end finish to slot red_bpost + blk (every thread
// of the block calls it).
__device__ inline void line_finish_store(const State& s, const Par& p, const int blk, const double rp, const double rin,
                                         const double rd, const double zinf, const double rin_pq, const double rin_va,
                                         const double y_pq, const double y_va) {
  const double v[4] = {rp, rin, rd, zinf};
  const int which[4] = {ACC_RP, ACC_RIN, ACC_RD, ACC_ZINF};
  block_max_store<4>(v, which, s.red + (size_t)(s.red_bpost + blk) * NACC);
  if (p.adapt_every > 0) {
    // the line-end duplicates' change is this block's rd
    const double vc[5] = {rin_pq, rin_va, y_pq, y_va, rd};
    const int wc[5] = {CS_RIN + CL_PQ, CS_RIN + CL_VA, CS_Y + CL_PQ, CS_Y + CL_VA, CS_DX + CL_PQ};
    block_max_store<5, NCS>(vc, wc, s.redc + (size_t)(s.red_bpost + blk) * NCS);
  }
}

// The line-end finish of the items of block blk (one lane per (line, t)).
__device__ __forceinline__ void bus_post_body(const Net& n, const State& s, const Par& p0, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const int idx = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0;
  double rin_pq = 0.0, rin_va = 0.0, y_pq = 0.0, y_va = 0.0;  // class maxima
  if (idx < n.T * n.L) {
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    line_finish_item(n, s, p, idx, beta, lu, rp, rin, rd, zinf, rin_pq, rin_va, y_pq, y_va, nullptr);
  }
  line_finish_store(s, p, blk, rp, rin, rd, zinf, rin_pq, rin_va, y_pq, y_va);
}

// The previous iteration's generator rows, finished by the unit block that owns the
// generators before its own work (the fused iteration): for each of the block's gpb
// generators (the unit side's lane mapping) and every period, rows G1, G2 and then the
// coupling and commitment rows; residual maxima to slot red_ugen + blk, and with
// residual balancing the rows' class maxima to the same slot of redc (what the bus
// kernel and the generator-row kernel store for these rows in the four-launch form).
// The caller synchronises the block before the generators' update reads these rows.
template <int BS>
__device__ __forceinline__ void unit_rows_body(const Net& n, const State& s, const Par& p0, const int blk, const int gpb) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const int TPAR = BS / gpb, T = n.T, G = n.G, TG = T * G;
  const int gsub = threadIdx.x % gpb, tb = threadIdx.x / gpb;
  const int g = blk * gpb + gsub;
  double rp = 0.0, rin = 0.0, zinf = 0.0;
  double rin_pq = 0.0, y_pq = 0.0, rin_c = 0.0, rin_u = 0.0, y_c = 0.0, y_u = 0.0;  // class maxima
  if (g < G) {
    const double beta = s.sc[SC_BETA];
    const LamUpd lu = lambda_pending(s, p);
    for (int t = tb; t < T; t += TPAR) {
      const int i = t * G + g;
      g12_rows_item(s, p, TG, i, beta, lu, rp, rin, zinf, rin_pq, y_pq);
      cu_rows_item(n, s, p, t, g, i, beta, lu, rp, rin, zinf, rin_c, rin_u, y_c, y_u);
    }
  }
  const double v[3] = {rp, rin, zinf};
  const int which[3] = {ACC_RP, ACC_RIN, ACC_ZINF};
  block_max_store<3>(v, which, s.red + (size_t)(s.red_ugen + blk) * NACC);
  if (p.adapt_every > 0) {
    const double vc[6] = {rin_pq, y_pq, rin_c, rin_u, y_c, y_u};
    const int wc[6] = {CS_RIN + CL_PQ, CS_Y + CL_PQ, CS_RIN + CL_CPL, CS_RIN + CL_UC, CS_Y + CL_CPL, CS_Y + CL_UC};
    block_max_store<6, NCS>(vc, wc, s.redc + (size_t)(s.red_ugen + blk) * NCS);
  }
}

}  // namespace ucac
