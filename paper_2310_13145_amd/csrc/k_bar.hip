// step:uc_bar, step:opf_bar and the multiplier updates (step:z, step:y).
//
// k_ubar     one lane per (g, t): exact minimiser of the star {ubar_on_t,
//            ubar_sd_t, ubar_su_{t+1}} in [0,1]^3 (rows U1(t), U3(t), C1..C5(t),
//            C6(t+1), U2(t+1)); the first period also solves ubar_su_1.  Writes
//            the new values to a side buffer so that the bus kernel still reads
//            the previous ones (the Jacobi pair uc_bar || opf_bar).
// step:opf_bar -- the diagonal QP of every bus-side duplicate subject to the P and Q
//            balance equations (2x2 KKT system per bus; thetabar a weighted mean,
//            zero at the reference bus) -- in three coalesced passes:
//            (the line kernel, one lane per (line, t), ends by storing per line end
//            the four quantities the bus sums need -- P and Q targets, v^2 and angle
//            centres -- in the bus incidence (CSR) order, so that each bus reads
//            one contiguous range)
// k_bus      one lane per (bus, t): sums its ends' quantities in incidence order,
//            solves the KKT system, writes wbar, thetabar and the two balance
//            multipliers, and updates its generators' duplicates and rows G1, G2;
// k_bus_post one lane per (line, t): Pbar, Qbar of both ends from the end buses'
//            multipliers, and z, y of the line's eight rows.
// The arithmetic is the one-pass gather's, in the same order.
// k_gen_dual one lane per (g, t): z and y of rows C1..C6 and U1..U3, and commits
//            the new relaxed commitments.
// Each kernel stores its blocks' residual maxima into per-block slots.
#include "ucac_launch.hpp"

namespace ucac {

__device__ __forceinline__ void ubar_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int G = n.G, T = n.T, TG = T * G;
  const int i = blk * UBLOCK + threadIdx.x;
  double dmax = 0.0;
  if (i < TG) {
    const int t = i / G, g = i - t * G;
    const double ruc = p.rho_uc, rc = p.rho_cpl;
    auto zy = [&](int r, int k, double rho) { return s.zG[r * TG + k] + s.yG[r * TG + k] / rho; };
    const double h1 = s.uon[i] + zy(RG_U1, i, ruc);
    const double h3 = s.usd[i] + zy(RG_U3, i, ruc);
    const double pv = s.p[i], qv = s.q[i];
    const double hc0 = pv - s.s[0 * TG + i] + zy(RG_C1, i, rc), k0 = n.pmin[g];
    const double hc1 = pv + s.s[1 * TG + i] + zy(RG_C2, i, rc), k1 = n.pmax[g];
    const double hc2 = qv - s.s[2 * TG + i] + zy(RG_C3, i, rc), k2 = n.qmin[g];
    const double hc3 = qv + s.s[3 * TG + i] + zy(RG_C4, i, rc), k3 = n.qmax[g];
    const double pbp = t == 0 ? n.p0[g] : s.pb[i - G];  // previous duplicate (Jacobi)
    const double h5 = pv - pbp - s.s[4 * TG + i] + zy(RG_C5, i, rc);
    const double RD = n.rd[g], SD = n.sd[g], RU = n.ru[g], SU = n.su[g];
    const bool nxt = t + 1 < T;
    double h6 = 0.0, h2 = 0.0;
    if (nxt) {
      const int kn = i + G;
      h6 = s.p[kn] - s.pb[i] + s.s[5 * TG + kn] + zy(RG_C6, kn, rc);
      h2 = s.usu[kn] + zy(RG_U2, kn, ruc);
    }
    // b*(a) = clamp(pb + qb a), c*(a) = clamp(pc + qc a)
    const double den_b = ruc + rc * SD * SD;
    const double pbv = (ruc * h3 - rc * SD * h5) / den_b, qbv = -(rc * SD * RD) / den_b;
    const double den_c = ruc + rc * SU * SU;
    const double pcv = nxt ? (ruc * h2 + rc * SU * h6) / den_c : 0.0;
    const double qcv = nxt ? -(rc * SU * RU) / den_c : 0.0;
    // phi'(a) = al a + ga + wb b*(a) + wc c*(a)
    const double al = ruc + rc * (k0 * k0 + k1 * k1 + k2 * k2 + k3 * k3) + rc * RD * RD + (nxt ? rc * RU * RU : 0.0);
    const double ga = -ruc * h1 - rc * (k0 * hc0 + k1 * hc1 + k2 * hc2 + k3 * hc3) + rc * RD * h5 - (nxt ? rc * RU * h6 : 0.0);
    const double wb = rc * RD * SD, wc = nxt ? rc * RU * SU : 0.0;
    auto dphi = [&](double a) {
      return al * a + ga + wb * clampd(pbv + qbv * a, 0.0, 1.0) + wc * clampd(pcv + qcv * a, 0.0, 1.0);
    };
    double a;
    if (dphi(0.0) >= 0.0) {
      a = 0.0;
    } else if (dphi(1.0) <= 0.0) {
      a = 1.0;
    } else {
      double lo = 0.0, hi = 1.0;
      double kink[4] = {-1.0, -1.0, -1.0, -1.0};
      if (qbv != 0.0) { kink[0] = -pbv / qbv; kink[1] = (1.0 - pbv) / qbv; }
      if (qcv != 0.0) { kink[2] = -pcv / qcv; kink[3] = (1.0 - pcv) / qcv; }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double k = kink[r];
        if (k > lo && k < hi) {
          if (dphi(k) < 0.0) lo = k; else hi = k;
        }
      }
      const double m = 0.5 * (lo + hi);
      const double bm = pbv + qbv * m, cm = pcv + qcv * m;
      const double B0 = bm <= 0.0 ? 0.0 : (bm >= 1.0 ? 1.0 : pbv), B1 = (bm <= 0.0 || bm >= 1.0) ? 0.0 : qbv;
      const double C0 = cm <= 0.0 ? 0.0 : (cm >= 1.0 ? 1.0 : pcv), C1 = (cm <= 0.0 || cm >= 1.0) ? 0.0 : qcv;
      a = clampd(-(ga + wb * B0 + wc * C0) / (al + wb * B1 + wc * C1), lo, hi);
    }
    const double b = clampd(pbv + qbv * a, 0.0, 1.0);
    const int TG3 = TG;
    double* nx_on = s.ub_nxt;
    double* nx_su = s.ub_nxt + TG3;
    double* nx_sd = s.ub_nxt + 2 * TG3;
    nx_on[i] = a;
    nx_sd[i] = b;
    dmax = fmax(fabs(a - s.ubon[i]), fabs(b - s.ubsd[i]));
    if (nxt) {
      const double c = clampd(pcv + qcv * a, 0.0, 1.0);
      nx_su[i + G] = c;
      dmax = nmax(dmax, fabs(c - s.ubsu[i + G]));
    }
    if (t == 0) {
      // ubar_su at the first period: rows U2(1), C6(1) with ubar_on_0 = u0
      const double h6f = pv - n.p0[g] + s.s[5 * TG + i] + zy(RG_C6, i, rc);
      const double h2f = s.usu[i] + zy(RG_U2, i, ruc);
      const double c0 = clampd((ruc * h2f + rc * SU * (h6f - RU * (double)n.u0[g])) / (ruc + rc * SU * SU), 0.0, 1.0);
      nx_su[i] = c0;
      dmax = nmax(dmax, fabs(c0 - s.ubsu[i]));
    }
  }
  const double v[1] = {dmax};
  const int which[1] = {ACC_RD};
  block_max_store<1>(v, which, s.red + (size_t)(s.red_ubar + blk) * NACC);
}

__global__ void __launch_bounds__(UBLOCK) k_ubar(Net n, State s, Par p) { ubar_body(n, s, p, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(UBLOCK) k_ubar_group(Group gr) {
  const int mk = gr.blk_member[blockIdx.x];
  const Member& M = gr.m[mk];
  const int b0 = gr.blk_first[mk];
  ubar_body(M.n, M.s, M.p, blockIdx.x - b0, gr.blk_count[mk]);
}

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

__device__ inline void zy_update(double* zr, double* yr, double* lr, int k, double a, double rho, double beta,
                                 const LamUpd& lu, double& rp, double& rin, double& zinf) {
  double lam = lr[k];
  if (lu.on) {
    lam = clampd(lam + lu.b * zr[k], -lu.lm, lu.lm);
    lr[k] = lam;
  }
  const double z = -(lam + yr[k] + rho * a) / (beta + rho);
  zr[k] = z;
  yr[k] = yr[k] + rho * (a + z);
  rp = nmax(rp, fabs(a));
  rin = nmax(rin, fabs(a + z));
  zinf = nmax(zinf, fabs(z));
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

__device__ __forceinline__ void bus_body(const Net& n, const State& s, const Par& p, const int blk, const int nblk) {
  if (s.ctl->halt) return;
  const int N = n.N, G = n.G, T = n.T;
  const int TG = T * G;
  const int idx = blk * BLOCK + threadIdx.x;
  double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0;
  if (idx < T * N) {
    const int t = idx / N, i = idx - t * N;
    const double rpq = p.rho_pq, rva = p.rho_va, rc = p.rho_cpl;
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
    for (int e = g0; e < g1; ++e) {
      const int g = n.gen_list[e], k = t * G + g;
      double Wp = rpq, Sp = rpq * (s.p[k] + s.zG[RG_G1 * TG + k] + s.yG[RG_G1 * TG + k] / rpq);
      if (t + 1 < T) {
        const int kn = k + G;
        const double t5 = s.p[kn] - s.s[4 * TG + kn] + n.rd[g] * s.ubon[kn] + n.sd[g] * s.ubsd[kn] +
                          s.zG[RG_C5 * TG + kn] + s.yG[RG_C5 * TG + kn] / rc;
        const double t6 = s.p[kn] + s.s[5 * TG + kn] - n.ru[g] * s.ubon[k] - n.su[g] * s.ubsu[kn] +
                          s.zG[RG_C6 * TG + kn] + s.yG[RG_C6 * TG + kn] / rc;
        Wp += 2.0 * rc;
        Sp += rc * t5 + rc * t6;
      }
      const double tq = s.q[k] + s.zG[RG_G2 * TG + k] + s.yG[RG_G2 * TG + k] / rpq;
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
    s.wb[idx] = wnew;
    s.thb[idx] = thnew;
    s.bmu[idx] = mu1;
    s.bmu[T * N + idx] = mu2;
    rd = nmax(fabs(wnew - wold), fabs(thnew - thold));
    for (int e = g0; e < g1; ++e) {
      const int g = n.gen_list[e], k = t * G + g;
      double Wp = rpq, Sp = rpq * (s.p[k] + s.zG[RG_G1 * TG + k] + s.yG[RG_G1 * TG + k] / rpq);
      if (t + 1 < T) {
        const int kn = k + G;
        const double t5 = s.p[kn] - s.s[4 * TG + kn] + n.rd[g] * s.ubon[kn] + n.sd[g] * s.ubsd[kn] +
                          s.zG[RG_C5 * TG + kn] + s.yG[RG_C5 * TG + kn] / rc;
        const double t6 = s.p[kn] + s.s[5 * TG + kn] - n.ru[g] * s.ubon[k] - n.su[g] * s.ubsu[kn] +
                          s.zG[RG_C6 * TG + kn] + s.yG[RG_C6 * TG + kn] / rc;
        Wp += 2.0 * rc;
        Sp += rc * t5 + rc * t6;
      }
      const double tq = s.q[k] + s.zG[RG_G2 * TG + k] + s.yG[RG_G2 * TG + k] / rpq;
      const double pn = Sp / Wp + mu1 / Wp, qn = tq + mu2 / rpq;
      rd = nmax(rd, nmax(fabs(pn - s.pb[k]), fabs(qn - s.qb[k])));
      s.pb[k] = pn;
      s.qb[k] = qn;
      zy_update(s.zG + RG_G1 * TG, s.yG + RG_G1 * TG, s.lG + RG_G1 * TG, k, s.p[k] - pn, rpq, beta, lu, rp, rin, zinf);
      zy_update(s.zG + RG_G2 * TG, s.yG + RG_G2 * TG, s.lG + RG_G2 * TG, k, s.q[k] - qn, rpq, beta, lu, rp, rin, zinf);
    }
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
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int code = 2 * l + side;
      const EndData d = load_end(n, s, t, TL, code, rpq);
      const int b = t * n.N + (side ? n.to[l] : n.from[l]);
      const double mu1 = s.bmu[b], mu2 = s.bmu[TN + b], wnew = s.wb[b], thnew = s.thb[b];
      double* Pdup = side ? s.Pbt : s.Pbf;
      double* Qdup = side ? s.Qbt : s.Qbf;
      const int k = d.k;
      const double Pn = d.tP - mu1 / rpq, Qn = d.tQ - mu2 / rpq;
      rd = nmax(rd, nmax(fabs(Pn - Pdup[k]), fabs(Qn - Qdup[k])));
      Pdup[k] = Pn;
      Qdup[k] = Qn;
      zy_update(s.zB + d.rP * TL, s.yB + d.rP * TL, s.lB + d.rP * TL, k, d.fP - Pn, rpq, beta, lu, rp, rin, zinf);
      zy_update(s.zB + d.rQ * TL, s.yB + d.rQ * TL, s.lB + d.rQ * TL, k, d.fQ - Qn, rpq, beta, lu, rp, rin, zinf);
      zy_update(s.zB + d.rW * TL, s.yB + d.rW * TL, s.lB + d.rW * TL, k, d.v * d.v - wnew, rva, beta, lu, rp, rin, zinf);
      zy_update(s.zB + d.rT * TL, s.yB + d.rT * TL, s.lB + d.rT * TL, k, d.th - thnew, rva, beta, lu, rp, rin, zinf);
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
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int row = RG_C1 + r;
      const double rho = r < 6 ? p.rho_cpl : p.rho_uc;
      zy_update(s.zG + row * TG, s.yG + row * TG, s.lG + row * TG, i, a[r], rho, beta, lu, rp, rin, zinf);
    }
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

int ubar_blocks(const Net& n) { return (n.T * n.G + UBLOCK - 1) / UBLOCK; }
int bus_blocks(const Net& n) { return (n.T * n.N + BLOCK - 1) / BLOCK; }
int post_blocks(const Net& n) { return line_blocks(n) + gen_dual_blocks(n); }

void launch_ubar_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_ubar_group, dim3(grid), dim3(UBLOCK), 0, st, g);
}
void launch_bus_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_bus_group, dim3(grid), dim3(BLOCK), 0, st, g);
}
void launch_post_grouped(const Group& g, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_post_group, dim3(grid), dim3(BLOCK), 0, st, g);
}

void launch_ubar(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const int TG = n.T * n.G;
  if (TG == 0) return;
  hipLaunchKernelGGL(k_ubar, dim3(ubar_blocks(n)), dim3(UBLOCK), 0, st, n, s, p);
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
