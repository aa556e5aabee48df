// step:opf, line part -- one lane per (line, period).
//
// Each lane minimises, over the four end variables x = (v_i, v_j, th_i, th_j) in
// the box v in [Vmin, Vmax], |th| <= 2 pi, the augmented-Lagrangian terms of the
// line's eight rows (the four flows of eq:acopf in polar form against their
// bus-side duplicates, v^2 against wbar and the angles against thetabar) plus a
// PHR term for each end's MVA limit, by a projected trust-region Newton method:
// basic trust-region iteration with a Steihaug-Toint truncated CG step on the free
// variables, projection onto the box and ratio-test acceptance.  The line-limit
// multipliers nu are then advanced once: nu <- max(0, nu + mu h(x*)).
//
// gfx950 mapping: FP64 vector ALU bound.  All Newton state (x, gradient, the 10
// distinct Hessian entries, CG vectors) lives in VGPRs; every loop over the four
// variables is unrolled so no array is indexed dynamically; one sincos per
// function evaluation.  The kernel is latency-bound (few wavefronts per SIMD, long
// dependent FP64 chains), so sums are formed as trees, the CG quotients use a
// refined hardware reciprocal, and sin/cos of the small angle difference come from
// a short polynomial chain.  The objective's Hessian is assembled from two per-end
// Gauss-Newton blocks and one weighted second-derivative block (all four flows
// share the form a v_i^2 + b v_j^2 + v_i v_j (al cos d + be sin d)), so a full
// evaluation costs about 200 flops.
#include <hip/hip_ext.h>
#include "ucac_launch.hpp"
#include "ucac_mlp.hpp"
#include "ucac_units.hpp"
#include "ucac_ctl.hpp"
#include "ucac_rows.hpp"

namespace ucac {

namespace {

struct Line {
  // flow k = a_k vi^2 + b_k vj^2 + vi vj (al_k cos d + be_k sin d).  Lines are pi-models
  // without taps or phase shifts, so the admittance blocks are symmetric:
  // G_ii = G_jj = G, G_ij = G_ji = -G, B_ii = B_jj = Bs, B_ij = B_ji = Bm.
  double G, Bs, Bm;
  double rate, rate2;
  double lo0, hi0, lo1, hi1;  // voltage boxes; angles are in [-2pi, 2pi]
  double c[8];
  double rpq, rva, mu, inv2mu, nu0, nu1;
};

// The line Hessian.  The flows depend on the two angles only through their
// difference, so every term except the angle rows' rho_va on the diagonal has
// h03 = -h02, h13 = -h12, h33 = h22 and h23 = -h22; the angle rows add rho_va to h22
// and h33 alike.  Seven values are kept; the other three are exact negations or
// copies.
struct Sym4 {
  double h00, h01, h02, h11, h12, h22, h23;
  __device__ double h03() const { return -h02; }
  __device__ double h13() const { return -h12; }
  __device__ double h33() const { return h22; }
};

// Quotient n / d for d > 0 from the hardware reciprocal refined by two Newton
// steps (relative error within a few ulp; a shorter dependency chain than the
// IEEE division sequence).  Used on the CG recurrences, where only the accuracy
// matters.
__device__ inline double qdiv(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return n * r;
}

// sin and cos of the angle difference.  For |x| <= pi/4 (the usual case: the two
// end angles of a line stay close) both come from their Taylor series to degree
// 17 / 16 (first omitted terms below 1e-17 relative), evaluated in x^2 by Estrin's
// scheme so the dependency chain is five operations deep; larger angles use the
// library routine.
__device__ inline void sincos_line(double x, double& S, double& C) {
  if (!(fabs(x) <= 0.78539816339744831)) {
    sincos(x, &S, &C);
    return;
  }
  const double y = x * x, y2 = y * y, y4 = y2 * y2;
  // coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!, k = 0..8
  double lo = fma(fma(-0.0001984126984126984, y, 0.008333333333333333), y2, fma(-0.16666666666666666, y, 1.0));
  double hi = fma(fma(-7.647163731819816e-13, y, 1.6059043836821613e-10), y2,
                  fma(-2.505210838544172e-08, y, 2.7557319223985893e-06));
  S = x * fma(fma(2.8114572543455206e-15, y4, hi), y4, lo);
  lo = fma(fma(-0.001388888888888889, y, 0.041666666666666664), y2, fma(-0.5, y, 1.0));
  hi = fma(fma(-1.1470745597729725e-11, y, 2.08767569878681e-09), y2, fma(-2.755731922398589e-07, y, 2.48015873015873e-05));
  C = fma(fma(4.779477332387385e-14, y4, hi), y4, lo);
}

__device__ inline void flows4(const Line& L, double vi, double vj, double C, double S, double& f0, double& f1,
                              double& f2, double& f3) {
  const double vv = vi * vj, vi2 = vi * vi, vj2 = vj * vj;
  f0 = L.G * vi2 + vv * (-L.G * C + L.Bm * S);
  f1 = -L.Bs * vi2 + vv * (-L.Bm * C - L.G * S);
  f2 = L.G * vj2 + vv * (-L.G * C - L.Bm * S);
  f3 = -L.Bs * vj2 + vv * (-L.Bm * C + L.G * S);
}

// H += w v v^T for v with v[3] = -v[2] (a flow gradient), on the independent entries;
// h23 is set from h22 once the flow terms are complete.
__device__ inline void rank1(Sym4& H, double w, const double (&v)[4]) {
  H.h00 += w * v[0] * v[0]; H.h01 += w * v[0] * v[1]; H.h02 += w * v[0] * v[2];
  H.h11 += w * v[1] * v[1]; H.h12 += w * v[1] * v[2];
  H.h22 += w * v[2] * v[2];
}

// value, gradient and Hessian
__device__ inline double evaluate(const Line& L, const double (&x)[4], double (&g)[4], Sym4& H) {
  const double vi = x[0], vj = x[1];
  double S, C;
  sincos_line(x[2] - x[3], S, C);
  const double vv = vi * vj;
  // per-flow (a, b, al, be)
  const double a[4] = {L.G, -L.Bs, 0.0, 0.0};
  const double b[4] = {0.0, 0.0, L.G, -L.Bs};
  const double al[4] = {-L.G, -L.Bm, -L.G, -L.Bm};
  const double be[4] = {L.Bm, -L.G, -L.Bm, L.G};
  double f[4], gf[4][4], T[4], Td[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T[k] = al[k] * C + be[k] * S;
    Td[k] = -al[k] * S + be[k] * C;
    f[k] = a[k] * vi * vi + b[k] * vj * vj + vv * T[k];
    gf[k][0] = 2.0 * a[k] * vi + vj * T[k];
    gf[k][1] = 2.0 * b[k] * vj + vi * T[k];
    gf[k][2] = vv * Td[k];
    gf[k][3] = -vv * Td[k];
  }
  double w[4];
  double F = 0.0;
  H = Sym4{0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int kp = 2 * m, kq = 2 * m + 1;
    const double nu = m == 0 ? L.nu0 : L.nu1;
    const double rP = f[kp] - L.c[kp], rQ = f[kq] - L.c[kq];
    const double h = f[kp] * f[kp] + f[kq] * f[kq] - L.rate2;
    const double tm = nu + L.mu * h;
    const double tp = tm > 0.0 ? tm : 0.0;
    F += 0.5 * L.rpq * (rP * rP + rQ * rQ) + (tp * tp - nu * nu) * L.inv2mu;
    w[kp] = L.rpq * rP + 2.0 * tp * f[kp];
    w[kq] = L.rpq * rQ + 2.0 * tp * f[kq];
    const double gn = L.rpq + 2.0 * tp;
    rank1(H, gn, gf[kp]);
    rank1(H, gn, gf[kq]);
    if (tm > 0.0) {
      double gh[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) gh[i] = 2.0 * f[kp] * gf[kp][i] + 2.0 * f[kq] * gf[kq][i];
      rank1(H, L.mu, gh);
    }
  }
  double Aw = 0.0, Bw = 0.0, Tw = 0.0, Tdw = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Aw += w[k] * a[k];
    Bw += w[k] * b[k];
    Tw += w[k] * T[k];
    Tdw += w[k] * Td[k];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) g[i] = (w[0] * gf[0][i] + w[1] * gf[1][i]) + (w[2] * gf[2][i] + w[3] * gf[3][i]);
  g[3] = -g[2];  // gf[k][3] = -gf[k][2]
  // weighted second derivatives of the flows
  H.h00 += 2.0 * Aw;      H.h01 += Tw;           H.h02 += vj * Tdw;
  H.h11 += 2.0 * Bw;      H.h12 += vi * Tdw;
  H.h22 -= vv * Tw;
  H.h23 = -H.h22;
  // voltage-square and angle rows
  const double r4 = vi * vi - L.c[4], r5 = vj * vj - L.c[5];
  const double r6 = x[2] - L.c[6], r7 = x[3] - L.c[7];
  F += 0.5 * L.rva * (r4 * r4 + r5 * r5 + r6 * r6 + r7 * r7);
  g[0] += L.rva * r4 * 2.0 * vi;
  g[1] += L.rva * r5 * 2.0 * vj;
  g[2] += L.rva * r6;
  g[3] += L.rva * r7;
  H.h00 += L.rva * (4.0 * vi * vi + 2.0 * r4);
  H.h11 += L.rva * (4.0 * vj * vj + 2.0 * r5);
  H.h22 += L.rva;  // and h33
  return F;
}

// 4-term sums are formed as two pairs (a tree): a shorter dependency chain.
__device__ inline void symv(const Sym4& H, const double (&v)[4], double (&out)[4]) {
  out[0] = (H.h00 * v[0] + H.h01 * v[1]) + (H.h02 * v[2] + H.h03() * v[3]);
  out[1] = (H.h01 * v[0] + H.h11 * v[1]) + (H.h12 * v[2] + H.h13() * v[3]);
  out[2] = (H.h02 * v[0] + H.h12 * v[1]) + (H.h22 * v[2] + H.h23 * v[3]);
  out[3] = (H.h03() * v[0] + H.h13() * v[1]) + (H.h23 * v[2] + H.h33() * v[3]);
}

__device__ inline double dot(const double (&a)[4], const double (&b)[4]) {
  return (a[0] * b[0] + a[1] * b[1]) + (a[2] * b[2] + a[3] * b[3]);
}

// Refined reciprocal of d > 0: the hardware estimate plus two Newton steps.
__device__ inline double qrcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// The step length tau >= 0 with ||z + tau d|| = delta (||z|| < delta).  The reciprocal
// of d.d is formed beside the square root rather than after it.
__device__ inline double to_boundary(const double (&z)[4], const double (&d)[4], double delta2) {
  const double zd = dot(z, d), dd = dot(d, d), zz = dot(z, z);
  const double inv = qrcp(dd);
  return (-zd + sqrt(zd * zd + dd * (delta2 - zz))) * inv;
}

// Steihaug-Toint CG on the free variables (mask fr), radius delta.
__device__ inline void steihaug(const Sym4& H, const double (&g)[4], const double (&fr)[4], int nf, double delta,
                                double (&out)[4], int& cg_its) {
  double z[4] = {0.0, 0.0, 0.0, 0.0}, r[4], d[4], Hd[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { r[i] = fr[i] * g[i]; d[i] = -r[i]; }
  double rr = dot(r, r);
  const double tol2 = 1e-24 * rr, delta2 = delta * delta;  // ||r|| <= 1e-12 ||r0||, ||z|| >= delta
  for (int j = 0; j < nf; ++j) {
    ++cg_its;
    symv(H, d, Hd);
#pragma unroll
    for (int i = 0; i < 4; ++i) Hd[i] *= fr[i];
    const double dHd = dot(d, Hd);
    double zn[4];
    const double alpha = qdiv(rr, dHd);  // used only when dHd > 0
#pragma unroll
    for (int i = 0; i < 4; ++i) zn[i] = z[i] + alpha * d[i];
    if (dHd <= 0.0 || dot(zn, zn) >= delta2) {
      // to the boundary along d
      const double tau = to_boundary(z, d, delta2);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[i] = z[i] + tau * d[i];
      return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) { r[i] += alpha * Hd[i]; z[i] = zn[i]; }
    const double rr_new = dot(r, r);
    if (rr_new <= tol2) break;
    const double beta = qdiv(rr_new, rr);
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = -r[i] + beta * d[i];
    rr = rr_new;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = z[i];
}

// The Newton step of the free subspace by a 4x4 LDL^T factorization, when it is what
// Steihaug-Toint CG returns: if H restricted to the free variables is positive
// definite, CG's iterates grow monotonically in norm and it ends (in at most nf
// iterations, in exact arithmetic) at the solution of H_ff s = -g_f; if that
// solution lies strictly inside the trust region, no iterate reached the boundary
// and CG returns it.  Returns true with that step in d; false (indefinite H_ff or a
// step of length >= delta) leaves the step to CG.  The fixed variables get identity
// rows, so their step is zero.  About 70 operations against about 120 per CG
// iteration for the 4x4 form; the usual reduced 3x3 form needs about 50.
__device__ inline bool newton_step_direct(const Sym4& H, const double (&g)[4], const double (&fr)[4], double delta,
                                          double inv_rva, double (&d)[4]) {
  if (fr[2] != 0.0 && fr[3] != 0.0) {
    // Both angles free (their bounds are +-2 pi): in the coordinates D = th_i - th_j,
    // S = th_i + th_j the flows depend on D alone, so S decouples (its curvature is
    // rho_va / 2, its coupling to v_i, v_j and D is zero) and the system is 3x3 in
    // (v_i, v_j, D): H_DD = (h22 - h23) / 2, H_vD = h02, h12, g_D = (g2 - g3) / 2.
    const double a00 = fr[0] * H.h00 + (1.0 - fr[0]), a11 = fr[1] * H.h11 + (1.0 - fr[1]);
    const double a01 = fr[0] * fr[1] * H.h01, a02 = fr[0] * H.h02, a12 = fr[1] * H.h12;
    const double a22 = 0.5 * (H.h22 - H.h23);
    const double d0 = a00, i0 = qrcp(d0);
    const double l10 = a01 * i0, l20 = a02 * i0;
    const double d1 = a11 - a01 * l10, i1 = qrcp(d1);
    const double b12 = a12 - a02 * l10;
    const double l21 = b12 * i1;
    const double d2 = (a22 - a02 * l20) - b12 * l21;
    const bool pd = d0 > 0.0 && d1 > 0.0 && d2 > 0.0;
    const double i2 = qrcp(d2);
    const double y0 = -fr[0] * g[0];
    const double y1 = -fr[1] * g[1] - l10 * y0;
    const double y2 = (-0.5 * (g[2] - g[3]) - l20 * y0) - l21 * y1;
    const double sD = y2 * i2;
    const double s1 = y1 * i1 - l21 * sD;
    const double s0 = (y0 * i0 - l10 * s1) - l20 * sD;
    const double sS = -(g[2] + g[3]) * inv_rva;  // -g_S / (rho_va / 2), g_S = (g2 + g3) / 2
    const double s2 = 0.5 * (sS + sD), s3 = 0.5 * (sS - sD);
    d[0] = s0; d[1] = s1; d[2] = s2; d[3] = s3;
    return pd && (s0 * s0 + s1 * s1) + (s2 * s2 + s3 * s3) < delta * delta;
  }
  const double a00 = fr[0] * H.h00 + (1.0 - fr[0]), a11 = fr[1] * H.h11 + (1.0 - fr[1]);
  const double a22 = fr[2] * H.h22 + (1.0 - fr[2]), a33 = fr[3] * H.h33() + (1.0 - fr[3]);
  const double a01 = fr[0] * fr[1] * H.h01, a02 = fr[0] * fr[2] * H.h02, a03 = fr[0] * fr[3] * H.h03();
  const double a12 = fr[1] * fr[2] * H.h12, a13 = fr[1] * fr[3] * H.h13(), a23 = fr[2] * fr[3] * H.h23;
  // A = L D L^T, unit lower L
  const double d0 = a00, i0 = qrcp(d0);
  const double l10 = a01 * i0, l20 = a02 * i0, l30 = a03 * i0;
  const double d1 = a11 - a01 * l10, i1 = qrcp(d1);
  const double b12 = a12 - a02 * l10, b13 = a13 - a03 * l10;
  const double l21 = b12 * i1, l31 = b13 * i1;
  const double d2 = (a22 - a02 * l20) - b12 * l21, i2 = qrcp(d2);
  const double b23 = (a23 - a03 * l20) - b13 * l21;
  const double l32 = b23 * i2;
  const double d3 = ((a33 - a03 * l30) - b13 * l31) - b23 * l32;
  const bool pd = d0 > 0.0 && d1 > 0.0 && d2 > 0.0 && d3 > 0.0;
  const double i3 = qrcp(d3);
  // L y = -g_f, then D w = y, then L^T s = w
  const double y0 = -fr[0] * g[0];
  const double y1 = -fr[1] * g[1] - l10 * y0;
  const double y2 = (-fr[2] * g[2] - l20 * y0) - l21 * y1;
  const double y3 = ((-fr[3] * g[3] - l30 * y0) - l31 * y1) - l32 * y2;
  const double s3 = y3 * i3;
  const double s2 = y2 * i2 - l32 * s3;
  const double s1 = (y1 * i1 - l21 * s2) - l31 * s3;
  const double s0 = ((y0 * i0 - l10 * s1) - l20 * s2) - l30 * s3;
  d[0] = s0; d[1] = s1; d[2] = s2; d[3] = s3;
  return pd && (s0 * s0 + s1 * s1) + (s2 * s2 + s3 * s3) < delta * delta;
}

// Gradient and Hessian at the current iterate, kept in LDS so that a rejected trial
// (whose own gradient and Hessian were formed with its value) costs no second
// evaluation: slot k of the lane's 11 values at gh[k][lane] (conflict-free).
template <int BS>
struct GHSave {
  double (*gh)[BS];
  __device__ void store(const double (&g)[4], const Sym4& H) const {
    const int t = threadIdx.x;
    gh[0][t] = g[0]; gh[1][t] = g[1]; gh[2][t] = g[2]; gh[3][t] = g[3];
    gh[4][t] = H.h00; gh[5][t] = H.h01; gh[6][t] = H.h02; gh[7][t] = H.h11;
    gh[8][t] = H.h12; gh[9][t] = H.h22; gh[10][t] = H.h23;
  }
  __device__ void load(double (&g)[4], Sym4& H) const {
    const int t = threadIdx.x;
    g[0] = gh[0][t]; g[1] = gh[1][t]; g[2] = gh[2][t]; g[3] = gh[3][t];
    H.h00 = gh[4][t]; H.h01 = gh[5][t]; H.h02 = gh[6][t]; H.h11 = gh[7][t];
    H.h12 = gh[8][t]; H.h22 = gh[9][t]; H.h23 = gh[10][t];
  }
};

// The projected search of TRON (Lin and More), the solver the paper hands the line
// subproblem to, taken where the full step d leaves the box and its projection fails
// the model's sufficient-decrease test: the step stops at the first break point of
// the ray x + alpha d, alpha <= 1, over the variables moving towards a bound they
// are not on; the variable that sets alpha is placed on its bound.  Rare (a few lanes
// per launch), so the quotients are plain IEEE divisions.
__device__ inline void projected_search(const double (&x)[4], const double (&d)[4], const double (&lo)[4],
                                        const double (&hi)[4], double (&xe)[4], double (&sv)[4]) {
  double alpha = 1.0;
  int first = -1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool up = d[i] > 0.0 && x[i] < hi[i], down = d[i] < 0.0 && x[i] > lo[i];
    if (!(up || down)) continue;
    const double brk = ((up ? hi[i] : lo[i]) - x[i]) / d[i];
    if (brk < alpha) { alpha = brk; first = i; }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    xe[i] = i == first ? (d[i] > 0.0 ? hi[i] : lo[i]) : clampd(x[i] + alpha * d[i], lo[i], hi[i]);
    sv[i] = xe[i] - x[i];
  }
}

// Projected trust-region Newton from x (in place), with the hold step (below) from
// every start: lanes that begin on a voltage bound (warm starts often do) would
// otherwise be pushed out of the box by steps whose projection the ratio test then
// rejects.  Returns the iterations taken;
// conv is set when it stopped at the projected-gradient tolerance.  There is one
// evaluation site: value, gradient and Hessian are formed at every trial point in
// one pass (nearly every trial is accepted); after a rejection the gradient and
// Hessian at x come back from LDS.  The ratio tests compare the actual decrease
// with multiples of the predicted one (pred > 0), which decides as the quotient
// does without a division on the dependency chain.
template <int BS>
__device__ inline int newton(const Line& L, const double (&lo)[4], const double (&hi)[4], double (&x)[4], const Par& p,
                             const GHSave<BS>& save, int& n_eval, int& n_rej, int& n_cg, int& n_dir, int& n_srch,
                             bool& conv) {
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = clampd(x[i], lo[i], hi[i]);
  double g[4], xe[4];
  Sym4 H;
#pragma unroll
  for (int i = 0; i < 4; ++i) xe[i] = x[i];
  double F = 0.0, pred = 0.0, snorm = 0.0;
  // initial radius 0.1: the half-width of the per-unit voltage box.  From the flat start
  // a radius of 1 let the first step carry the voltages to their bound, and the slowest
  // lanes then spent three or four iterations there before the quadratic phase.
  double delta = 0.1;
  const double inv_rva = 1.0 / L.rva;
  bool trial = false;
  conv = false;
  int it = 0;
  for (;;) {
    const double Fe = evaluate(L, xe, g, H);
    ++n_eval;
    bool accept = true;
    if (trial) {
      // ratio = (F - Fe) / pred if pred > 0 (1 if pred is at the rounding level of F), else -1
      const double ared = F - Fe;
      const bool pos = pred > 0.0, noise = pred <= 1e-12 * fabs(F);
      const bool lt_quarter = !pos || (!noise && ared < 0.25 * pred);
      const bool gt_3quarter = pos && (noise || ared > 0.75 * pred);
      accept = pos && (noise || ared >= 1e-4 * pred);
      if (lt_quarter) delta = 0.25 * snorm;
      else if (gt_3quarter && snorm >= 0.99 * delta) delta = fmin(4.0 * delta, 10.0);
      trial = false;
    }
    if (accept) {
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = xe[i];
      F = Fe;
      save.store(g, H);
    } else {
      ++n_rej;
      save.load(g, H);
    }
    if (it >= p.newton_max_iter) break;
    double fr[4];
    int nf = 0;
    double pg = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool out = (x[i] <= lo[i] && g[i] > 0.0) || (x[i] >= hi[i] && g[i] < 0.0);
      fr[i] = out ? 0.0 : 1.0;
      nf += out ? 0 : 1;
      pg = out ? pg : fmax(pg, fabs(g[i]));
    }
    if (pg <= p.gtol) { conv = true; break; }
    // The step on the free set; then the hold step: a free variable on a bound (its
    // gradient points inwards) that the step pushes outwards is held on it and the
    // step solved once more without it, as TRON's subspace step holds every variable
    // that is on a bound.  One call site for the two passes keeps the code (and the
    // register allocation) of a single step solve.
    double d[4];
    double fs[4] = {fr[0], fr[1], fr[2], fr[3]};
    int nfs = nf;
    for (int pass = 0;; ++pass) {
      if (newton_step_direct(H, g, fs, delta, inv_rva, d)) ++n_dir;
      else steihaug(H, g, fs, nfs, delta, d, n_cg);
      if (pass) break;
      bool held = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool out = fs[i] != 0.0 && ((x[i] <= lo[i] && d[i] < 0.0) || (x[i] >= hi[i] && d[i] > 0.0));
        fs[i] = out ? 0.0 : fs[i];
        nfs -= out ? 1 : 0;
        held = held || out;
      }
      if (!held) break;
    }
    double sv[4];
    bool left_box = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double xd = x[i] + d[i];
      left_box = left_box || xd < lo[i] || xd > hi[i];
      xe[i] = clampd(xd, lo[i], hi[i]);
      sv[i] = xe[i] - x[i];
    }
    double Hs[4];
    symv(H, sv, Hs);
    double gs = dot(g, sv);
    double q = gs + 0.5 * dot(sv, Hs);
    if (left_box && q > 0.01 * gs) {
      ++n_srch;
      projected_search(x, d, lo, hi, xe, sv);
      symv(H, sv, Hs);
      gs = dot(g, sv);
      q = gs + 0.5 * dot(sv, Hs);
    }
    double sinf = 0.0, xinf = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sinf = fmax(sinf, fabs(sv[i]));
      xinf = fmax(xinf, fabs(x[i]));
    }
    if (sinf <= 1e-15 * (1.0 + xinf)) break;
    pred = -q;
    snorm = sqrt(dot(sv, sv));
    trial = true;
    ++it;
  }
  return it;
}

// The 20 inputs of the learned start: series conductance and susceptance, line
// charging, rating, the eight targets (flows, v^2 - 1, angle difference), the
// line-limit multipliers, voltage bounds, penalties, and the target loading.
__device__ inline void line_features(const Line& L, float (&f)[MLP_IN]) {
  f[0] = (float)(0.1 * L.G);
  f[1] = (float)(0.05 * L.Bm);
  f[2] = (float)(10.0 * (L.Bs + L.Bm));
  f[3] = (float)(L.rate / 3.0);
  f[4] = (float)L.c[0];
  f[5] = (float)L.c[1];
  f[6] = (float)L.c[2];
  f[7] = (float)L.c[3];
  f[8] = (float)(L.c[4] - 1.0);
  f[9] = (float)(L.c[5] - 1.0);
  f[10] = (float)(5.0 * (L.c[6] - L.c[7]));
  f[11] = (float)(L.nu0 / L.mu);
  f[12] = (float)(L.nu1 / L.mu);
  f[13] = (float)(L.lo0 - 1.0);
  f[14] = (float)(L.hi0 - 1.0);
  f[15] = (float)(L.lo1 - 1.0);
  f[16] = (float)(L.hi1 - 1.0);
  f[17] = (float)(log10(L.rpq) - 4.0);
  f[18] = (float)(log10(L.rva) - 4.0);
  f[19] = (float)((L.c[0] * L.c[0] + L.c[1] * L.c[1] - L.rate2) / L.rate2);
}

// The 4 outputs: v_i - 1, v_j - 1, 10 (th_i - c6), 10 (th_j - c7).
__device__ inline void encode_solution(const Line& L, const double (&x)[4], float (&y)[MLP_OUT]) {
  y[0] = (float)(x[0] - 1.0);
  y[1] = (float)(x[1] - 1.0);
  y[2] = (float)(10.0 * (x[2] - L.c[6]));
  y[3] = (float)(10.0 * (x[3] - L.c[7]));
}

}  // namespace

// The line subproblem of lane idx without its targets: admittances, rating, voltage
// boxes and line-limit multipliers.  Inactive lanes get a harmless unit line.
__device__ __forceinline__ Line load_line_static(const Net& n, const State& s, const Par& p, int idx, bool active) {
  Line L = {};
  L.rate = 1.0; L.rate2 = 1.0;
  L.rpq = p.rho_pq; L.rva = p.rho_va; L.mu = p.mu; L.inv2mu = 0.5 / p.mu;  // uniform: scalar registers
  if (active) {
    const int l = idx % n.L;
    L.G = n.adm[0 * n.L + l]; L.Bs = n.adm[1 * n.L + l]; L.Bm = n.adm[3 * n.L + l];
    L.rate = n.rate[l];
    L.rate2 = L.rate * L.rate;
    L.lo0 = n.vmin[n.from[l]]; L.hi0 = n.vmax[n.from[l]];
    L.lo1 = n.vmin[n.to[l]]; L.hi1 = n.vmax[n.to[l]];
    L.nu0 = s.nuf[idx]; L.nu1 = s.nut[idx];
  }
  return L;
}

// ... and with the completed-square targets c_r = xbar_r - z_r - y_r / rho_r of its
// eight rows, read from the iterate.
__device__ __forceinline__ Line load_line(const Net& n, const State& s, const Par& p, int idx, bool active) {
  Line L = load_line_static(n, s, p, idx, active);
  if (active) {
    const int TL = n.T * n.L;
    const int t = idx / n.L, l = idx - t * n.L;
    const int bi = t * n.N + n.from[l], bj = t * n.N + n.to[l];
    const double xb[8] = {s.Pbf[idx], s.Qbf[idx], s.Pbt[idx], s.Qbt[idx], s.wb[bi], s.wb[bj], s.thb[bi], s.thb[bj]};
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double rho = r < 4 ? p.rho_pq : p.rho_va;
      L.c[r] = xb[r] - s.zB[r * TL + idx] - s.yB[r * TL + idx] / rho;
    }
  }
  return L;
}

// ... the targets from the values the line-end finish of the same lane just computed
// (the values load_line would read back, in the same arithmetic).
__device__ __forceinline__ void line_targets(Line& L, const LineFinish& f, const Par& p) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const double rho = r < 4 ? p.rho_pq : p.rho_va;
    L.c[r] = f.xb[r] - f.z[r] - f.y[r] / rho;
  }
}

// The learned start of a lane of the fused launch: the network on its line data
// (every lane of the wavefront calls it: wavefront barriers inside), decoded to
// (v_i, v_j, th_i, th_j) in FP32 as k_line_start stores them in x0.
__device__ inline void learned_start_point(const Line& L, const Par& p, __bf16* buf, float (&x0)[4]) {
  float f[MLP_IN], y[MLP_OUT];
  line_features(L, f);
  mlp_forward_layers(p.mlp, f, buf, y);
  x0[0] = 1.0f + y[0];
  x0[1] = 1.0f + y[1];
  x0[2] = (float)(L.c[6] + 0.1 * (double)y[2]);
  x0[3] = (float)(L.c[7] + 0.1 * (double)y[3]);
}

// Newton start: START_FLAT (mid-box voltages, zero angles), START_PREV (the line's
// previous solution) or START_LEARNED: the point k_line_start predicted; a lane whose
// Newton does not reach the tolerance from there restarts from the flat start (the
// plain method is the fallback).  One instantiation per start keeps the plain kernel
// free of the others' code and registers.
enum { START_FLAT = 0, START_PREV = 1, START_LEARNED = 2 };

// The LDS save area of a line block's lanes (one per block size, whichever line
// kernel body instantiation uses it).
template <int BS>
__device__ inline GHSave<BS> gh_save_area() {
  __shared__ double gh_lds[11][BS];
  return GHSave<BS>{gh_lds};
}

// FIN (the fused iteration, BS = BLOCK): the lane first finishes the previous
// iteration's line ends of its own item (line_finish_item, residual maxima to the
// block's slot red_bpost + blk) and takes its targets from that finish's registers.
template <int START, int BS, bool FIN = false>
__device__ __forceinline__ void branch_body(const Net& n, const State& s, const Par& p0, const int blk) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  const GHSave<BS> save = gh_save_area<BS>();
  const int TL = n.T * n.L;
  const int idx = blk * BS + threadIdx.x;
  const bool active = idx < TL;
  int n_eval = 0, n_rej = 0, n_cg = 0, it = 0, n_fb = 0, n_dir = 0, n_srch = 0;
  Line L;
  if (FIN) {
    static_assert(!FIN || BS == BLOCK, "the finish's block slots are per BLOCK items");
    L = load_line_static(n, s, p, idx, active);
    double rp = 0.0, rin = 0.0, rd = 0.0, zinf = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    if (active) {
      LineFinish f;
      line_finish_item(n, s, p, idx, s.sc[SC_BETA], lambda_pending(s, p), rp, rin, rd, zinf, c0, c1, c2, c3, &f);
      line_targets(L, f, p);
    }
    line_finish_store(s, p, blk, rp, rin, rd, zinf, c0, c1, c2, c3);
  } else {
    L = load_line(n, s, p, idx, active);
  }
  const double lo[4] = {L.lo0, L.lo1, -TWO_PI, -TWO_PI};
  const double hi[4] = {L.hi0, L.hi1, TWO_PI, TWO_PI};
  double x[4];
  if (START == START_LEARNED && FIN) {
    // the network on the targets the finish just formed (what k_line_start computes
    // from them after reading them back), its LDS in the launch's dynamic area
    extern __shared__ __bf16 lds_net[];
    float x0[4];
    learned_start_point(L, p, lds_net + (threadIdx.x >> 6) * MLP_WAVE_LDS, x0);
    if (active) {
#pragma unroll
      for (int k = 0; k < 4; ++k) s.x0[k * TL + idx] = x0[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = (double)x0[k];
    if (!(x[0] == x[0] && x[1] == x[1] && x[2] == x[2] && x[3] == x[3])) {
      x[0] = 0.5 * (L.lo0 + L.hi0); x[1] = 0.5 * (L.lo1 + L.hi1); x[2] = 0.0; x[3] = 0.0;
    }
  } else if (START == START_LEARNED && active) {
    // the point k_line_start predicted for this line (FP32), NaN-guarded
    x[0] = (double)s.x0[idx]; x[1] = (double)s.x0[TL + idx];
    x[2] = (double)s.x0[2 * TL + idx]; x[3] = (double)s.x0[3 * TL + idx];
    if (!(x[0] == x[0] && x[1] == x[1] && x[2] == x[2] && x[3] == x[3])) {
      x[0] = 0.5 * (L.lo0 + L.hi0); x[1] = 0.5 * (L.lo1 + L.hi1); x[2] = 0.0; x[3] = 0.0;
    }
  } else if (START == START_PREV && active) {
    x[0] = s.vf[idx]; x[1] = s.vt[idx]; x[2] = s.thf[idx]; x[3] = s.tht[idx];
  } else {
    x[0] = 0.5 * (L.lo0 + L.hi0); x[1] = 0.5 * (L.lo1 + L.hi1); x[2] = 0.0; x[3] = 0.0;
  }
  if (active) {
    bool conv;
    it = 0;
    for (int attempt = 0;; ++attempt) {
      it += newton<BS>(L, lo, hi, x, p, save, n_eval, n_rej, n_cg, n_dir, n_srch, conv);
      if (START != START_LEARNED || conv || attempt) break;
      ++n_fb;
      x[0] = 0.5 * (L.lo0 + L.hi0); x[1] = 0.5 * (L.lo1 + L.hi1); x[2] = 0.0; x[3] = 0.0;
    }
    // z, y of the eight rows for the per-end sums below, loaded before this lane's
    // first store so that their latency overlaps the final flows
    double zz[8], yy[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) { zz[r] = s.zB[r * TL + idx]; yy[r] = s.yB[r * TL + idx]; }
    const int epos0 = n.end_pos[2 * (idx % n.L)], epos1 = n.end_pos[2 * (idx % n.L) + 1];
    double S, C;
    sincos(x[2] - x[3], &S, &C);
    double f0, f1, f2, f3;
    flows4(L, x[0], x[1], C, S, f0, f1, f2, f3);
    s.vf[idx] = x[0]; s.vt[idx] = x[1]; s.thf[idx] = x[2]; s.tht[idx] = x[3];
    s.pf[idx] = f0; s.qf[idx] = f1; s.pt[idx] = f2; s.qt[idx] = f3;
    s.nuf[idx] = fmax(0.0, L.nu0 + L.mu * (f0 * f0 + f1 * f1 - L.rate2));
    s.nut[idx] = fmax(0.0, L.nu1 + L.mu * (f2 * f2 + f3 * f3 - L.rate2));
    s.br_iters[idx] = it;
    {
      // the per-end sums of the bus QP (step:opf_bar): P and Q targets and the v^2 and
      // angle centres of both ends, stored at each end's place in its bus's incidence
      // list, in plain IEEE arithmetic (no contraction) like the bus solve itself
#pragma clang fp contract(off)
      const int t = idx / n.L;
      double* eb = s.ebuf + (size_t)t * 2 * n.L * 4;
      const double fP[2] = {f0, f2}, fQ[2] = {f1, f3}, v[2] = {x[0], x[1]}, th[2] = {x[2], x[3]};
      const int epos[2] = {epos0, epos1};
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int rP = side ? RB_PT : RB_PF, rQ = side ? RB_QT : RB_QF;
        const int rW = side ? RB_WT : RB_WF, rT = side ? RB_TT : RB_TF;
        double* o = eb + (size_t)epos[side] * 4;
        o[0] = fP[side] + zz[rP] + yy[rP] / L.rpq;
        o[1] = fQ[side] + zz[rQ] + yy[rQ] / L.rpq;
        o[2] = v[side] * v[side] + zz[rW] + yy[rW] / L.rva;
        o[3] = th[side] + zz[rT] + yy[rT] / L.rva;
      }
    }
    if (s.log_feat && idx % s.log_stride == s.log_phase) {
      // (inputs, converged solution) pair for training the learned start
      const int slot = atomicAdd(s.log_count, 1);
      if (slot < s.log_cap) {
        float f[MLP_IN], y[MLP_OUT];
        line_features(L, f);
        encode_solution(L, x, y);
#pragma unroll
        for (int k = 0; k < MLP_IN; ++k) s.log_feat[(size_t)slot * MLP_IN + k] = f[k];
#pragma unroll
        for (int k = 0; k < MLP_OUT; ++k) s.log_targ[(size_t)slot * MLP_OUT + k] = y[k];
      }
    }
  }
  // work counters: one wave-level sum per counter, added to the wave's own slot
  unsigned long long c[NBRC] = {(unsigned long long)n_eval, (unsigned long long)n_rej, (unsigned long long)n_cg,
                                (unsigned long long)it, (unsigned long long)n_fb, (unsigned long long)n_dir,
                                (unsigned long long)n_srch};
#pragma unroll
  for (int k = 0; k < NBRC; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c[k] += __shfl_xor(c[k], off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    // this wavefront's own slot (no atomics: the same wave owns it in every launch)
    unsigned long long* slot = s.br_count + (size_t)((blk * BS + (int)threadIdx.x) >> 6) * NBRC;
#pragma unroll
    for (int k = 0; k < NBRC; ++k) slot[k] += c[k];
  }
}

template <int START, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2))) k_branch(Net n, State s, Par p) {
  branch_body<START, BS>(n, s, p, blockIdx.x);
}

// The unit side (ucac_units.hpp) and the lines in one launch: blocks [0, nb_units) run
// the unit side, the rest the line kernel.  Neither reads what the other writes in
// the same iteration, and one launch on one stream avoids the fork and join that two
// concurrent launches cost on the iteration's critical path.  The unit blocks come
// first, so that they start with the first wave of line blocks.
//
// With fin_units >= 0 the first block is instead the control step of the previous
// iteration (its unit side's residual slots from fin_units on).  Nothing else in this
// launch reads what the control step writes, except the stop flag, which it sets only
// in solve mode, where the step runs as a kernel of its own; the unit blocks write the
// other copy of their slots (s.red_u).
template <int START, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2)))
k_front(Net n, State s, Par p, int nb_units, int gpb, int fin_units) {
  static_assert(BS == FIN_BLOCK, "the control step runs as one block of this launch");
  int b = blockIdx.x;
  if (fin_units >= 0) {
    if (b == 0) { finalize_body(s, p, fin_units); return; }
    --b;
  }
  if (b < nb_units) unit_body<BS>(n, s, p, b, n.T, gpb);
  else branch_body<START, BS>(n, s, p, b - nb_units);
}

// The first launch of the fused iteration (two launches per iteration; the second,
// k_bus_fused, solves the bus QP and runs the control step of the iteration before).
// With FUSE_PRO every block first finishes the previous iteration's rows it owns: a
// line block the line ends of its own (line, t) items, each lane the item of its own
// Newton solve, whose targets it then takes from the finish's registers (branch_body
// with FIN); a unit block its generators' rows G1, G2, C1-C6 and U1-U3, with their
// relaxed commitments committed (unit_rows_body).  With FUSE_WORK it then runs this
// iteration's work.  A line lane reads, of what the finish writes, only its own
// item's rows and duplicates, which it wrote itself; a unit block synchronises between
// the two parts.  A graph's first launch runs the work alone, its last the finish
// alone (bus_post_body).  The learned start's instantiation has only the
// finish-and-work path: its lanes evaluate the network between the finish and Newton.
template <int START, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2)))
k_front_fused(Net n, State s, Par p, int nb_units, int gpb, int mode) {
  static_assert(BS == BLOCK, "a line block finishes the line ends of its own items");
  const int b = blockIdx.x;
  if (b < nb_units) {
    if (mode & FUSE_PRO) {
      unit_rows_body<BS>(n, s, p, b, gpb);
      __syncthreads();
    }
    if (mode & FUSE_WORK) unit_body<BS>(n, s, p, b, n.T, gpb);
  } else if (mode == (FUSE_PRO | FUSE_WORK)) {
    branch_body<START, BS, true>(n, s, p, b - nb_units);
  } else if constexpr (START != START_LEARNED) {
    // (the learned start's first and last launches of a graph use the other kernels:
    // its instantiation keeps only the finish-and-solve path, and its registers)
    if (mode == FUSE_PRO) bus_post_body(n, s, p, b - nb_units, line_blocks(n));
    else branch_body<START, BS>(n, s, p, b - nb_units);
  }
}

template <int START, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2)))
k_front_group(Group gu, Group gb, int grid_u, int slotT, int gpb) {
  const int b = blockIdx.x;
  if (b < grid_u) {
    const int mk = gu.blk_member[b];
    const Member& M = gu.m[mk];
    unit_body<BS>(M.n, M.s, M.p, b - gu.blk_first[mk], slotT, gpb);
  } else {
    const int mk = gb.blk_member[b - grid_u];
    const Member& M = gb.m[mk];
    branch_body<START, BS>(M.n, M.s, M.p, b - grid_u - gb.blk_first[mk]);
  }
}

// Learned start, run just before the line kernel: every wavefront evaluates the
// warm-start network on its 64 lines (20 local inputs each; BF16 MFMA, FP32
// accumulation, activations in LDS) and stores the decoded start point
// (v_i, v_j, th_i, th_j) as FP32 in x0 [4][T*L].  A kernel of its own so that the
// Newton kernel keeps its registers (no spills) and the network runs at the
// occupancy its small footprint allows.
// One wavefront per block, so that the launch spreads over every CU.
constexpr int START_BLOCK = 64;

__global__ void __launch_bounds__(START_BLOCK) k_line_start(Net n, State s, Par p0) {
  if (s.ctl->halt) return;
  const Par p = live_par(p0, s);
  extern __shared__ __bf16 lds_start[];
  const int TL = n.T * n.L;
  const int idx = blockIdx.x * START_BLOCK + threadIdx.x;
  const bool active = idx < TL;
  MlpFrags fr;
  mlp_load_frags(p.mlp, fr);  // in flight with the line's own loads
  const Line L = load_line(n, s, p, idx, active);
  float f[MLP_IN], y[MLP_OUT];
  line_features(L, f);
  mlp_forward_frags(fr, p.mlp.b3, f, lds_start + (threadIdx.x >> 6) * MLP_WAVE_LDS, y);
  if (active) {
    s.x0[idx] = 1.0f + y[0];
    s.x0[TL + idx] = 1.0f + y[1];
    s.x0[2 * TL + idx] = (float)(L.c[6] + 0.1 * (double)y[2]);
    s.x0[3 * TL + idx] = (float)(L.c[7] + 0.1 * (double)y[3]);
  }
}

int branch_blocks(const Net& n, int block) { return (n.T * n.L + block - 1) / block; }

static void launch_line_start(const Net& n, const State& s, const Par& p, hipStream_t st) {
  const size_t lds = sizeof(__bf16) * MLP_WAVE_LDS * (START_BLOCK / 64);
  hipLaunchKernelGGL(k_line_start, dim3(branch_blocks(n, START_BLOCK)), dim3(START_BLOCK), lds, st, n, s, p);
}

// With e0 set, the launch carries its own start and stop events, which take the
// dispatch's begin and end timestamps: the kernel's duration without the latency
// of separate event records around it.
template <int BS>
static void launch_branch_bs(const Net& n, const State& s, const Par& p, int grid, int start, hipStream_t st,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  void (*kern)(Net, State, Par) = start == START_LEARNED ? k_branch<START_LEARNED, BS>
                                  : start == START_PREV  ? k_branch<START_PREV, BS>
                                                         : k_branch<START_FLAT, BS>;
  if (e0) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(BS), 0, st, e0, e1, 0u, n, s, p);
  else hipLaunchKernelGGL(kern, dim3(grid), dim3(BS), 0, st, n, s, p);
}

static void launch_branch_impl(const Net& n, const State& s, const Par& p, hipStream_t st, int block, hipEvent_t e0,
                               hipEvent_t e1) {
  if (n.T * n.L == 0) return;
  if (p.warm_start == START_LEARNED) launch_line_start(n, s, p, st);
  const int grid = branch_blocks(n, block);
  if (block == 64) launch_branch_bs<64>(n, s, p, grid, p.warm_start, st, e0, e1);
  else launch_branch_bs<256>(n, s, p, grid, p.warm_start, st, e0, e1);
}

void launch_branch_block(const Net& n, const State& s, const Par& p, hipStream_t st, int block) {
  launch_branch_impl(n, s, p, st, block, nullptr, nullptr);
}

bool launch_branch_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  launch_branch_impl(n, s, p, st, 256, e0, e1);
  return n.T * n.L > 0;
}

void launch_branch(const Net& n, const State& s, const Par& p, hipStream_t st) { launch_branch_block(n, s, p, st, 256); }

void launch_front(const Net& n, const State& s, const Par& p, hipStream_t st, int fin_units) {
  const int TL = n.T * n.L;
  const int gpb = units_gpb(n.T, 16, 256);
  const int nu = n.G && n.T ? units_blocks(n, gpb) : 0;
  const int nb = TL ? branch_blocks(n, 256) : 0;
  const int nf = fin_units >= 0 ? 1 : 0;
  if (nu + nb + nf == 0) return;
  if (TL && p.warm_start == START_LEARNED) launch_line_start(n, s, p, st);
  const size_t lds = nu ? units_lds(n.T, gpb) : 0;
  const dim3 grid(nf + nu + nb), block(256);
  if (p.warm_start == START_LEARNED)
    hipLaunchKernelGGL((k_front<START_LEARNED, 256>), grid, block, lds, st, n, s, p, nu, gpb, fin_units);
  else if (p.warm_start == START_PREV)
    hipLaunchKernelGGL((k_front<START_PREV, 256>), grid, block, lds, st, n, s, p, nu, gpb, fin_units);
  else hipLaunchKernelGGL((k_front<START_FLAT, 256>), grid, block, lds, st, n, s, p, nu, gpb, fin_units);
}

void launch_front_fused(const Net& n, const State& s, const Par& p, hipStream_t st, int mode) {
  const int TL = n.T * n.L;
  const int gpb = units_gpb(n.T, 16, 256);
  const int nu = n.G && n.T ? units_blocks(n, gpb) : 0;
  const int nb = TL ? branch_blocks(n, 256) : 0;
  if (nu + nb == 0) return;
  size_t lds = nu && (mode & FUSE_WORK) ? units_lds(n.T, gpb) : 0;
  const dim3 grid(nu + nb), block(256);
  if (p.warm_start == START_LEARNED) {
    // with the finish, the line blocks evaluate the network in the launch's dynamic
    // LDS (beside the unit blocks' DP tables); without it (a graph's first launch),
    // the network kernel runs first, as in the other forms
    if (mode == (FUSE_PRO | FUSE_WORK)) {
      const size_t net = sizeof(__bf16) * MLP_WAVE_LDS * (256 / 64);
      lds = lds > net ? lds : net;
      hipLaunchKernelGGL((k_front_fused<START_LEARNED, 256>), grid, block, lds, st, n, s, p, nu, gpb, mode);
    } else if (mode == FUSE_WORK) {
      launch_front(n, s, p, st, -1);  // the network kernel, then the unit side and lines
    } else {
      hipLaunchKernelGGL((k_front_fused<START_FLAT, 256>), grid, block, lds, st, n, s, p, nu, gpb, mode);
    }
  } else if (p.warm_start == START_PREV)
    hipLaunchKernelGGL((k_front_fused<START_PREV, 256>), grid, block, lds, st, n, s, p, nu, gpb, mode);
  else hipLaunchKernelGGL((k_front_fused<START_FLAT, 256>), grid, block, lds, st, n, s, p, nu, gpb, mode);
}

template <int BS>
static void launch_front_bs(const Group& gu, int grid_u, const Group& gb, int grid_b, int warm_start, int gpb, int max_T,
                            hipStream_t st) {
  const size_t lds = grid_u ? units_lds(max_T, gpb) : 0;
  const dim3 grid(grid_u + grid_b), block(BS);
  if (warm_start == START_PREV) hipLaunchKernelGGL((k_front_group<START_PREV, BS>), grid, block, lds, st, gu, gb, grid_u, max_T, gpb);
  else hipLaunchKernelGGL((k_front_group<START_FLAT, BS>), grid, block, lds, st, gu, gb, grid_u, max_T, gpb);
}

void launch_front_grouped(const Group& gu, int grid_u, const Group& gb, int grid_b, int warm_start, int block,
                          int dp_lanes, int max_T, hipStream_t st) {
  if (grid_u + grid_b == 0) return;
  const int gpb = units_gpb(max_T, dp_lanes, block == 64 ? 64 : 256);
  if (block == 64) launch_front_bs<64>(gu, grid_u, gb, grid_b, warm_start, gpb, max_T, st);
  else launch_front_bs<256>(gu, grid_u, gb, grid_b, warm_start, gpb, max_T, st);
}

}  // namespace ucac
