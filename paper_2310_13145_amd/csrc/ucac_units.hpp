// The unit side of an inner iteration, per generator: step:opf's generator part,
// step:uc (the dynamic program) and step:uc_bar.
//
// A block owns GPB consecutive generators for all T periods:
//   1. the generator update of every period (it reads only the previous iterate's
//      duplicates, multipliers and relaxed commitments, not this iteration's u);
//   2. the dynamic program (Sec. III-B, Alg. dp_algo): the block's lanes build the
//      cost tables L^UC_{g,t}(s', s) for all periods into LDS (4 doubles per period)
//      and the parts of the switch costs that do not depend on the cost-to-go (the
//      minimum up/down window sums); one lane per generator then runs the backward
//      stay/switch induction
//      (keep_formula, switch_formula) and the forward reconstruction from one
//      decision bit per (period, state) -- O(T) extra space instead of the paper's
//      stored O(T^2) trajectories -- and the lanes write u_on/u_su/u_sd;
//   3. after a block barrier (the block's own stores are then visible to it), the
//      relaxed-commitment star of every period, which needs the generator update
//      of periods t and t+1 and the new u.
// Nothing crosses generators, so the three steps need no grid-wide ordering and
// run in one launch.
//
// Every function here turns floating-point contraction off in its body: the table
// entries, stay/switch sums and closed-form updates are plain IEEE operations in a
// fixed order, so that a commitment is decided on exactly the same numbers as in
// any other plain FP64 evaluation of the same expressions, whatever the
// translation unit's own contraction setting (the line kernel's is fast, with
// pragmas honoured).
#pragma once
#include "ucac_dev.hpp"
#include "ucac_pwl.hpp"

namespace ucac {

// L^UC(s', s): commitment costs plus y (u - ubar + z) + rho/2 (u - ubar + z)^2
// over (on, su, sd), with su = max(0, s - s'), sd = max(0, s' - s).
__device__ inline double uc_table_entry(double cnl, double csu, double csd, double rho, int sp, int s,
                                        const double* ub, const double* z, const double* y) {
#pragma clang fp contract(off)
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

// LDS bytes of one generator's DP at horizon T: cost table [T][2][2], switch sums
// [T][2], cost-to-go [T+2][2], decision bits [T+2][2], schedule [T]; padded to 8
// bytes.
__host__ __device__ inline size_t dp_slot_bytes(int T) {
  const size_t b = sizeof(double) * (6 * (size_t)T + 2 * ((size_t)T + 2)) + 2 * ((size_t)T + 2) + (size_t)T;
  return (b + 7) & ~(size_t)7;
}

// The part of each switch cost that does not depend on the cost-to-go: for 1-based
// period t and state s, P[(t-1)*2 + s] = the table entry of switching from s to
// s' = 1 - s at t plus the entries of staying in s' through the rest of the
// minimum up (s' = 1) or down (s' = 0) time, added left to right -- the first
// operations of the switch formula, in its order.  Items k = first, first + step, ...
// of the 2T, so a group of lanes fills P in parallel.
__device__ inline void dp_switch_sums(int T, const double* Lt, double* P, int tu, int td, int first, int step) {
#pragma clang fp contract(off)
  const int TU = tu < 1 ? 1 : tu, TD = td < 1 ? 1 : td;
  for (int k = first; k < 2 * T; k += step) {
    const int t = k / 2 + 1, ss = k - (k / 2) * 2, ns = 1 - ss;
    const int Tm = ns ? TU : TD;
    double sw = Lt[((t - 1) * 2 + ss) * 2 + ns];
    const int last = (t + Tm - 1) < T ? (t + Tm - 1) : T;
    for (int tp = t + 1; tp <= last; ++tp) sw += Lt[((tp - 1) * 2 + ns) * 2 + ns];
    P[k] = sw;
  }
}

// The stay/switch backward induction over the LDS table Lt (1-based period t at
// Lt[(t-1)*4 + s'*2 + s]) and the switch sums P, the initial hold (L_g periods on
// or F_g off), and the forward reconstruction of the schedule u[0..T).  Returns
// the optimal cost, summed in the order of the recursion.  Minimum up/down times
// below 1 act as 1.
__device__ inline double dp_recursion(int T, const double* Lt, const double* P, double* c, unsigned char* dec,
                                      signed char* u, int u0, int lon, int loff, int tu, int td) {
#pragma clang fp contract(off)
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
      double sw = P[(t - 1) * 2 + ss];
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

// step:opf, generator part, for item i = t * G + g.
__device__ inline void gen_item(const Net& n, const State& s, const Par& p, const int i) {
#pragma clang fp contract(off)
  const int TG = n.T * n.G;
  const int t = i / n.G, g = i - t * n.G;
  const double rp = p.rho_pq, rc = p.rho_cpl;
  const double pb = s.pb[i], qb = s.qb[i];
  const double pbp = t == 0 ? n.p0[g] : s.pb[i - n.G];
  const double uon = s.ubon[i];
  const double uonp = t == 0 ? (double)n.u0[g] : s.ubon[i - n.G];
  const double usu = s.ubsu[i], usd = s.ubsd[i];
  double z[8], y[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) { z[r] = s.zG[r * TG + i]; y[r] = s.yG[r * TG + i]; }

  const double eG1 = -pb + z[RG_G1] + y[RG_G1] / rp;
  const double e1 = -n.pmin[g] * uon + z[RG_C1] + y[RG_C1] / rc;
  const double e2 = -n.pmax[g] * uon + z[RG_C2] + y[RG_C2] / rc;
  const double e5 = -pbp + n.rd[g] * uon + n.sd[g] * usd + z[RG_C5] + y[RG_C5] / rc;
  const double e6 = -pbp - n.ru[g] * uonp - n.su[g] * usu + z[RG_C6] + y[RG_C6] / rc;
  Pwl<4> fp;
  fp.A = 2.0 * n.k2[g] + rp;
  fp.B = n.k1[g] + rp * eG1;
  fp.w[0] = p.relax_uc ? 0.0 : rc;  // the multiperiod ACOPF has no minimum-generation row
  fp.w[1] = rc; fp.w[2] = rc; fp.w[3] = rc;
  fp.e[0] = e1; fp.e[1] = e2; fp.e[2] = e5; fp.e[3] = e6;
  fp.neg[0] = true; fp.neg[1] = false; fp.neg[2] = true; fp.neg[3] = false;
  const double pv = fp.argmin(0.0, n.pmax[g]);

  const double eG2 = -qb + z[RG_G2] + y[RG_G2] / rp;
  const double e3 = -n.qmin[g] * uon + z[RG_C3] + y[RG_C3] / rc;
  const double e4 = -n.qmax[g] * uon + z[RG_C4] + y[RG_C4] / rc;
  Pwl<2> fq;
  fq.A = rp;
  fq.B = rp * eG2;
  fq.w[0] = rc; fq.w[1] = rc;
  fq.e[0] = e3; fq.e[1] = e4;
  fq.neg[0] = true; fq.neg[1] = false;
  const double qv = fq.argmin(fmin(0.0, n.qmin[g]), fmax(0.0, n.qmax[g]));

  s.p[i] = pv;
  s.q[i] = qv;
  s.s[0 * TG + i] = fmax(0.0, pv + e1);
  s.s[1 * TG + i] = fmax(0.0, -(pv + e2));
  s.s[2 * TG + i] = fmax(0.0, qv + e3);
  s.s[3 * TG + i] = fmax(0.0, -(qv + e4));
  s.s[4 * TG + i] = fmax(0.0, pv + e5);
  s.s[5 * TG + i] = fmax(0.0, -(pv + e6));
}


// step:uc_bar for item i = t * G + g: the star's new values go to ub_nxt; returns the
// largest change of the star's values (a dual-residual contribution).
__device__ inline double ubar_item(const Net& n, const State& s, const Par& p, const int i) {
#pragma clang fp contract(off)
  const int G = n.G, T = n.T, TG = T * G;
  double dmax = 0.0;
  {
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
  return dmax;
}


// The three steps for the gpb consecutive generators of block blk (BS threads; gpb
// is 1, 4 or 16).  Thread j works on generator blk * gpb + j % gpb and periods
// j / gpb, + BS / gpb, ...: consecutive lanes take consecutive generators, so every
// (g, t) load and store of a wavefront covers runs of gpb consecutive doubles of
// the [T][G] arrays.  The recursion runs on the first gpb threads, one generator
// each.
// slotT: the horizon the LDS slots are sized for.  The largest star change of the
// block goes to its residual slot.
template <int BS>
__device__ __forceinline__ void unit_body(const Net& n, const State& s, const Par& p0, int blk, int slotT, int gpb) {
#pragma clang fp contract(off)
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const int TPAR = BS / gpb;  // periods in flight per generator
  const int T = n.T, G = n.G;
  const int gsub = threadIdx.x % gpb, tb = threadIdx.x / gpb;
  const int g = blk * gpb + gsub;
  const bool act = g < G;

  if (act)
    for (int t = tb; t < T; t += TPAR) gen_item(n, s, p, t * G + g);
  if (p.relax_uc) {
    // the multiperiod ACOPF: no commitment decisions; the relaxed commitments keep
    // their values (copied to where the generator-row kernel commits them from)
    const int TG = T * G;
    if (act)
      for (int t = tb; t < T; t += TPAR) {
        const int k = t * G + g;
        s.ub_nxt[k] = s.ubon[k];
        s.ub_nxt[TG + k] = s.ubsu[k];
        s.ub_nxt[2 * TG + k] = s.ubsd[k];
      }
    const double v[1] = {0.0};
    const int which[1] = {ACC_RD};
    block_max_store<1>(v, which, s.red + (size_t)(s.red_u + blk) * NACC);
    if (p.adapt_every > 0) {
      const double vc[2] = {0.0, 0.0};
      const int wc[2] = {CS_DX + CL_CPL, CS_DX + CL_UC};
      block_max_store<2, NCS>(vc, wc, s.redc + (size_t)(s.red_u + blk) * NCS);
    }
    return;
  }

  extern __shared__ double lds_units[];
  char* base = (char*)lds_units + dp_slot_bytes(slotT) * gsub;
  double* Lt = (double*)base;                              // [T][2][2]
  double* P = Lt + 4 * T;                                  // [T][2] switch sums
  double* c = P + 2 * T;                                   // [T+2][2], c[T+1][*] = 0
  unsigned char* dec = (unsigned char*)(c + 2 * (T + 2));  // [T+2][2]
  signed char* u = (signed char*)(dec + 2 * (T + 2));      // [T]
  const double rho = p.rho_uc;
  const int TG = T * G;
  if (act) {
    const double cnl = n.cnl[g], csu = n.csu[g], csd = n.csd[g];
    for (int t = tb; t < T; t += TPAR) {
      const int k = t * G + g;
      const double ub[3] = {s.ubon[k], s.ubsu[k], s.ubsd[k]};
      const double z[3] = {s.zG[RG_U1 * TG + k], s.zG[RG_U2 * TG + k], s.zG[RG_U3 * TG + k]};
      const double y[3] = {s.yG[RG_U1 * TG + k], s.yG[RG_U2 * TG + k], s.yG[RG_U3 * TG + k]};
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int ss = 0; ss < 2; ++ss) Lt[(t * 2 + sp) * 2 + ss] = uc_table_entry(cnl, csu, csd, rho, sp, ss, ub, z, y);
    }
  }
  __syncthreads();
  if (act) dp_switch_sums(T, Lt, P, n.tu[g], n.td[g], tb, TPAR);
  __syncthreads();
  if (act && tb == 0) dp_recursion(T, Lt, P, c, dec, u, n.u0[g], n.lon[g], n.loff[g], n.tu[g], n.td[g]);
  __syncthreads();
  if (act) {
    const int u0 = n.u0[g];
    for (int t = tb; t < T; t += TPAR) {
      const int k = t * G + g;
      const int cur = u[t];
      const int prev = t == 0 ? u0 : u[t - 1];
      s.uon[k] = (double)cur;
      s.usu[k] = cur > prev ? 1.0 : 0.0;
      s.usd[k] = prev > cur ? 1.0 : 0.0;
    }
  }
  __syncthreads();  // this block's u and generator updates are visible to all its lanes

  double dmax = 0.0;
  if (act)
    for (int t = tb; t < T; t += TPAR) dmax = nmax(dmax, ubar_item(n, s, p, t * G + g));
  const double v[1] = {dmax};
  const int which[1] = {ACC_RD};
  block_max_store<1>(v, which, s.red + (size_t)(s.red_u + blk) * NACC);
  if (p.adapt_every > 0) {
    // the relaxed commitments are duplicates of both the coupling and the commitment rows
    const double vc[2] = {dmax, dmax};
    const int wc[2] = {CS_DX + CL_CPL, CS_DX + CL_UC};
    block_max_store<2, NCS>(vc, wc, s.redc + (size_t)(s.red_u + blk) * NCS);
  }
}

// Blocks for the unit side at gpb generators per block.
__host__ __device__ inline int unit_blocks(int G, int gpb) { return (G + gpb - 1) / gpb; }

}  // namespace ucac
