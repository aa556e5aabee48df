/*
 * FP64 CPU ORACLE for the inner iteration of the two-level component-based ADMM
 * for unit commitment with AC optimal power flow (Zhang, Kim & Kim, "On Solving
 * Unit Commitment with Alternating Current Optimal Power Flow on GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the HIP library; the only thing both sides consume is
 * the seeded instance data.
 *
 * It is plain and slow on purpose: every block written out in the order the paper
 * states it, with no blocking, fusion or reordering.  The items of a block are
 * independent (that is the decomposition of Sec. III), so each block's loop over
 * them is an OpenMP parallel for; every item is computed by the same code whatever
 * thread runs it, and the only reductions are maxima, which are exact, so the
 * results do not depend on the thread count.
 *
 * What each part follows:
 *   - rows, costs and the augmented Lagrangian: Sec. II (eq:uc-acopf, eq:acopf,
 *     set:UC, eq:coupling) and Sec. III (eq:uc-acopf-ext with the slack rows
 *     eq:uc_duplicate .. eq:ramp_up, eq:outer, the Lagrangian L_{beta,rho});
 *   - inner iteration order and its Jacobi pairs: step:uc .. step:y and the
 *     remarks that uc || opf and uc_bar || opf_bar;
 *   - outer update: step:outer with tau = 6, theta = 0.8, Alg. alg:basic;
 *   - UC block: the DP of Sec. III-B (keep_formula, switch_formula, Alg. dp_algo);
 *   - generator / bus / line blocks: the component-based decomposition the paper
 *     adopts from its ExaAdmm.jl lineage, with the readings stated at each block
 *     (ramp rows on the bus-side duplicate of p_{t-1}, ramp-down row as in the
 *     inequality, line limits by a PHR term, projected trust-region Newton).
 *
 * Parity pins: see tests/test_oracle_*.py (brute-force DP, block optimality
 * against generic solvers, finite differences, closed forms, AC power-flow
 * residuals at convergence).
 *
 * Parity unpinned: which local minimiser and which commitments the non-convex
 * iteration reaches on the 118- and 2000-bus workloads.  The paper prints no worked
 * example and its Table 1 needs data that is not available, so those trajectories
 * are checked only against this oracle (their blocks and stopping point are pinned
 * as above).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* inputs                                                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t n_bus, n_line, n_gen, T, ref_bus;
  double base_mva;
  const int32_t *line_from, *line_to;
  const double *line_r, *line_x, *line_b, *line_rate;
  const double *bus_gs, *bus_bs, *bus_vmin, *bus_vmax;
  const double *load_p, *load_q; /* [T][n_bus] */
  const int32_t *gen_bus;
  const double *gen_pmin, *gen_pmax, *gen_qmin, *gen_qmax;
  const double *gen_c2, *gen_c1, *gen_cnl, *gen_csu, *gen_csd;
  const double *gen_ru, *gen_rd, *gen_su, *gen_sd;
  const int32_t *gen_min_up, *gen_min_dn, *gen_u0, *gen_init_on, *gen_init_off;
  const double *gen_p0;
} orc_net;

typedef struct {
  double rho_pq, rho_va, rho_uc, rho_cpl;
  double beta0, tau, theta, lambda_max, beta_max, mu_line;
  int32_t newton_max_iter;
  double newton_gtol;
  int32_t max_inner;
  double eps_in0, tol;
  int32_t warm_start; /* 0 flat start, 1 previous iterate */
  /* residual balancing of the four penalty classes (0 = fixed penalties) */
  int32_t adapt_every;   /* decide after every adapt_every-th inner iteration */
  double adapt_mu;       /* imbalance factor */
  double adapt_tau;      /* scaling factor of one change */
  int32_t adapt_max;     /* at most this many changes per class */
  double adapt_span;     /* a class's penalty stays within [rho0 / span, rho0 * span] */
  /* 1: the multiperiod ACOPF of the UC warm start (commitments fixed at their cold
   * start, no DP, no commitment rows, no minimum-generation row) */
  int32_t relax_uc;
} orc_params;

/* row indices */
enum { RB_PF, RB_QF, RB_PT, RB_QT, RB_WF, RB_WT, RB_TF, RB_TT, NRB };
enum { RG_G1, RG_G2, RG_C1, RG_C2, RG_C3, RG_C4, RG_C5, RG_C6, RG_U1, RG_U2, RG_U3, NRG };

#define TWO_PI 6.283185307179586

/* State: one flat array of doubles; the order below is the state format. */
typedef struct {
  double *vf, *vt, *thf, *tht, *pf, *qf, *pt, *qt, *nuf, *nut;   /* [T][L] line x-side */
  double *p, *q, *s[6], *uon, *usu, *usd;                         /* [T][G] generator x-side */
  double *wb, *thb;                                               /* [T][N] bus duplicates */
  double *Pbf, *Qbf, *Pbt, *Qbt;                                  /* [T][L] bus-side flows */
  double *pb, *qb, *ubon, *ubsu, *ubsd;                           /* [T][G] duplicates */
  double *zB[NRB], *yB[NRB], *lB[NRB];                            /* [T][L] line rows */
  double *zG[NRG], *yG[NRG], *lG[NRG];                            /* [T][G] generator rows */
  double *sc; /* scalars: see SC_* */
} orc_state;

enum { SC_BETA, SC_ZPREV, SC_KOUT, SC_LIN, SC_ITER, SC_RP, SC_RIN, SC_RD, SC_ZINF, SC_CONV,
       SC_RHO_PQ, SC_RHO_VA, SC_RHO_CPL, SC_RHO_UC, SC_NCHG_PQ, SC_NCHG_VA, SC_NCHG_CPL, SC_NCHG_UC, NSC };
/* penalty classes: power rows (line flows B1-B4, generator consensus G1-G2), voltage
 * and angle rows (B5-B8), bound and ramp coupling rows (C1-C6), commitment rows (U1-U3) */
enum { CL_PQ, CL_VA, CL_CPL, CL_UC, NCL };

typedef struct {
  int N, L, G, T, ref;
  orc_params par;
  /* lines */
  int *from, *to;
  double *adm; /* [L][8] G_ii B_ii G_ij B_ij G_jj B_jj G_ji B_ji */
  double *rate;
  /* buses */
  double *gs, *bs, *vmin, *vmax, *Pd, *Qd;
  int *inc_start, *inc_line, *inc_side; /* incidence lists: side 0 = from end, 1 = to end */
  int *gen_start, *gen_list;
  /* generators */
  int *gbus;
  double *pmin, *pmax, *qmin, *qmax, *k2, *k1, *cnl, *csu, *csd, *ru, *rd, *su, *sd, *p0;
  int *tu, *td, *u0, *lon, *loff;
  /* state */
  size_t n_state;
  double *buf;
  orc_state st;
  double *xb_old; /* copy of the duplicates at the start of an iteration */
  int *br_iters;  /* Newton iterations of the last branch solve, per (t, line) */
} orc_problem;

/* ------------------------------------------------------------------------- */
/* line model (Sec. II-A, eq:acopf; polar form of the W-variables)           */
/* ------------------------------------------------------------------------- */

/* pi-model admittances of a line without transformer */
static void line_admittance(double r, double x, double b, double *adm) {
  double den = r * r + x * x;
  double gs = r / den;
  double bs = -x / den;
  adm[0] = gs;            /* G_ii */
  adm[1] = bs + 0.5 * b;  /* B_ii */
  adm[2] = -gs;           /* G_ij */
  adm[3] = -bs;           /* B_ij */
  adm[4] = gs;            /* G_jj */
  adm[5] = bs + 0.5 * b;  /* B_jj */
  adm[6] = -gs;           /* G_ji */
  adm[7] = -bs;           /* B_ji */
}

/* Each flow is a*v_i^2 + b*v_j^2 + v_i v_j (al cos d + be sin d), d = th_i - th_j.
 * With w_i = v_i^2, wR = v_i v_j cos d, wI = v_i v_j sin d these are the four
 * flow equations of eq:acopf (the third and fourth are the flows into j). */
static void flow_coefs(const double *adm, int k, double *a, double *b, double *al, double *be) {
  switch (k) {
    case 0: *a = adm[0];  *b = 0.0;     *al = adm[2];  *be = adm[3];  break; /* p_ij */
    case 1: *a = -adm[1]; *b = 0.0;     *al = -adm[3]; *be = adm[2];  break; /* q_ij */
    case 2: *a = 0.0;     *b = adm[4];  *al = adm[6];  *be = -adm[7]; break; /* p_ji */
    default:*a = 0.0;     *b = -adm[5]; *al = -adm[7]; *be = -adm[6]; break; /* q_ji */
  }
}

static void line_flows(const double *adm, const double *x, double *f) {
  double d = x[2] - x[3];
  double c = cos(d), s = sin(d);
  for (int k = 0; k < 4; ++k) {
    double a, b, al, be;
    flow_coefs(adm, k, &a, &b, &al, &be);
    f[k] = a * x[0] * x[0] + b * x[1] * x[1] + x[0] * x[1] * (al * c + be * s);
  }
}

/* value, gradient and Hessian of one flow */
static void flow_derivs(const double *adm, int k, const double *x, double *f, double *g, double H[4][4]) {
  double a, b, al, be;
  flow_coefs(adm, k, &a, &b, &al, &be);
  double vi = x[0], vj = x[1], d = x[2] - x[3];
  double c = cos(d), s = sin(d);
  double Tv = al * c + be * s;   /* T(d)   */
  double Td = -al * s + be * c;  /* T'(d)  */
  *f = a * vi * vi + b * vj * vj + vi * vj * Tv;
  g[0] = 2.0 * a * vi + vj * Tv;
  g[1] = 2.0 * b * vj + vi * Tv;
  g[2] = vi * vj * Td;
  g[3] = -vi * vj * Td;
  H[0][0] = 2.0 * a;   H[0][1] = Tv;        H[0][2] = vj * Td;        H[0][3] = -vj * Td;
  H[1][0] = Tv;        H[1][1] = 2.0 * b;   H[1][2] = vi * Td;        H[1][3] = -vi * Td;
  H[2][0] = vj * Td;   H[2][1] = vi * Td;   H[2][2] = -vi * vj * Tv;  H[2][3] = vi * vj * Tv;
  H[3][0] = -vj * Td;  H[3][1] = -vi * Td;  H[3][2] = vi * vj * Tv;   H[3][3] = -vi * vj * Tv;
}

/* One line subproblem of step:opf: the augmented Lagrangian terms of the eight
 * line rows (completed squares with targets c[k] = xbar_k - z_k - y_k/rho_k)
 * plus a PHR term for each end's MVA limit (uc_acopf_ij_limit / ji_limit). */
typedef struct {
  double adm[8];
  double rate;
  double lo[4], hi[4];
  double c[8];
  double rho_pq, rho_va, mu;
  double nu[2];
} branch_pb;

static double branch_F(const branch_pb *b, const double *x) {
  double f[4];
  line_flows(b->adm, x, f);
  double F = 0.0;
  for (int k = 0; k < 4; ++k) F += 0.5 * b->rho_pq * (f[k] - b->c[k]) * (f[k] - b->c[k]);
  double r4 = x[0] * x[0] - b->c[4], r5 = x[1] * x[1] - b->c[5];
  double r6 = x[2] - b->c[6], r7 = x[3] - b->c[7];
  F += 0.5 * b->rho_va * (r4 * r4 + r5 * r5 + r6 * r6 + r7 * r7);
  for (int m = 0; m < 2; ++m) {
    double h = f[2 * m] * f[2 * m] + f[2 * m + 1] * f[2 * m + 1] - b->rate * b->rate;
    double t = b->nu[m] + b->mu * h;
    double tp = t > 0.0 ? t : 0.0;
    F += (tp * tp - b->nu[m] * b->nu[m]) / (2.0 * b->mu);
  }
  return F;
}

static double branch_eval(const branch_pb *b, const double *x, double *g, double H[4][4]) {
  double f[4], gf[4][4], Hf[4][4][4];
  for (int k = 0; k < 4; ++k) flow_derivs(b->adm, k, x, &f[k], gf[k], Hf[k]);
  for (int i = 0; i < 4; ++i) {
    g[i] = 0.0;
    for (int j = 0; j < 4; ++j) H[i][j] = 0.0;
  }
  double F = 0.0;
  for (int k = 0; k < 4; ++k) {
    double r = f[k] - b->c[k];
    F += 0.5 * b->rho_pq * r * r;
    for (int i = 0; i < 4; ++i) {
      g[i] += b->rho_pq * r * gf[k][i];
      for (int j = 0; j < 4; ++j) H[i][j] += b->rho_pq * (gf[k][i] * gf[k][j] + r * Hf[k][i][j]);
    }
  }
  /* voltage-square and angle rows */
  double r4 = x[0] * x[0] - b->c[4], r5 = x[1] * x[1] - b->c[5];
  double r6 = x[2] - b->c[6], r7 = x[3] - b->c[7];
  F += 0.5 * b->rho_va * (r4 * r4 + r5 * r5 + r6 * r6 + r7 * r7);
  g[0] += b->rho_va * r4 * 2.0 * x[0];
  g[1] += b->rho_va * r5 * 2.0 * x[1];
  g[2] += b->rho_va * r6;
  g[3] += b->rho_va * r7;
  H[0][0] += b->rho_va * (4.0 * x[0] * x[0] + 2.0 * r4);
  H[1][1] += b->rho_va * (4.0 * x[1] * x[1] + 2.0 * r5);
  H[2][2] += b->rho_va;
  H[3][3] += b->rho_va;
  /* PHR line-limit terms */
  for (int m = 0; m < 2; ++m) {
    int kp = 2 * m, kq = 2 * m + 1;
    double h = f[kp] * f[kp] + f[kq] * f[kq] - b->rate * b->rate;
    double t = b->nu[m] + b->mu * h;
    double tp = t > 0.0 ? t : 0.0;
    F += (tp * tp - b->nu[m] * b->nu[m]) / (2.0 * b->mu);
    if (t > 0.0) {
      double gh[4], Hh[4][4];
      for (int i = 0; i < 4; ++i) gh[i] = 2.0 * f[kp] * gf[kp][i] + 2.0 * f[kq] * gf[kq][i];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
          Hh[i][j] = 2.0 * (gf[kp][i] * gf[kp][j] + f[kp] * Hf[kp][i][j] + gf[kq][i] * gf[kq][j] + f[kq] * Hf[kq][i][j]);
      for (int i = 0; i < 4; ++i) {
        g[i] += t * gh[i];
        for (int j = 0; j < 4; ++j) H[i][j] += b->mu * gh[i] * gh[j] + t * Hh[i][j];
      }
    }
  }
  return F;
}

static double dot4(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3]; }

/* Steihaug-Toint truncated CG on the free variables (Nocedal & Wright Alg. 7.2). */
static void steihaug(double H[4][4], const double *g, const int *fr, double delta, double *out, int *cg_its) {
  double z[4] = {0, 0, 0, 0}, r[4], d[4], Hd[4];
  for (int i = 0; i < 4; ++i) { r[i] = fr[i] ? g[i] : 0.0; d[i] = -r[i]; }
  int nf = fr[0] + fr[1] + fr[2] + fr[3];
  double rr = dot4(r, r);
  double tol = 1e-12 * sqrt(rr);
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  for (int j = 0; j < nf; ++j) {
    ++*cg_its;
    for (int i = 0; i < 4; ++i) {
      Hd[i] = 0.0;
      if (!fr[i]) continue;
      for (int k = 0; k < 4; ++k) if (fr[k]) Hd[i] += H[i][k] * d[k];
    }
    double dHd = dot4(d, Hd);
    if (dHd <= 0.0) {
      /* negative curvature: go to the boundary along d */
      double zd = dot4(z, d), dd = dot4(d, d), zz = dot4(z, z);
      double tau = (-zd + sqrt(zd * zd + dd * (delta * delta - zz))) / dd;
      for (int i = 0; i < 4; ++i) out[i] = z[i] + tau * d[i];
      return;
    }
    double alpha = rr / dHd;
    double zn[4];
    for (int i = 0; i < 4; ++i) zn[i] = z[i] + alpha * d[i];
    if (sqrt(dot4(zn, zn)) >= delta) {
      double zd = dot4(z, d), dd = dot4(d, d), zz = dot4(z, z);
      double tau = (-zd + sqrt(zd * zd + dd * (delta * delta - zz))) / dd;
      for (int i = 0; i < 4; ++i) out[i] = z[i] + tau * d[i];
      return;
    }
    for (int i = 0; i < 4; ++i) r[i] += alpha * Hd[i];
    double rr_new = dot4(r, r);
    for (int i = 0; i < 4; ++i) z[i] = zn[i];
    if (sqrt(rr_new) <= tol) break;
    double beta = rr_new / rr;
    for (int i = 0; i < 4; ++i) d[i] = -r[i] + beta * d[i];
    rr = rr_new;
  }
  for (int i = 0; i < 4; ++i) out[i] = z[i];
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* The trial point of one projected trust-region Newton iteration from x with
 * gradient g, Hessian H, free set fr and radius delta: the Steihaug step d of
 * Alg. 7.2 on the free set, projected onto the box.  Where the full step leaves the
 * box and its projection fails the sufficient-decrease test of the quadratic model,
 * q(s) <= mu0 g.s with mu0 = 0.01, the step instead stops at the first break point
 * of the ray x + alpha d (the projected search of Lin and More's TRON, the solver
 * the paper hands the line subproblem to): the model decreases along the ray up to
 * there, and the variable whose bound is reached first is placed on it.  Before that,
 * a free variable that lies on a bound but that the step pushes outwards is held on
 * its bound and the step solved again without it.  Writes the trial point xt and step
 * s = xt - x; returns the model value q(s). */
static double trial_point(const branch_pb *b, const double *x, const double *g, double H[4][4], const int *fr,
                          double delta, int hold, double *xt, double *s, int *cg_its) {
  double d[4];
  steihaug(H, g, fr, delta, d, cg_its);
  /* with hold set, a free variable on a bound (its gradient points inwards) that the
   * step pushes outwards is held on it, and the step is solved once more without it:
   * TRON's subspace step holds every variable that is on a bound */
  int fr2[4], held = 0;
  for (int i = 0; i < 4; ++i) {
    int out = hold && fr[i] && ((x[i] <= b->lo[i] && d[i] < 0.0) || (x[i] >= b->hi[i] && d[i] > 0.0));
    fr2[i] = out ? 0 : fr[i];
    held |= out;
  }
  if (held) steihaug(H, g, fr2, delta, d, cg_its);
  int left_box = 0;
  for (int i = 0; i < 4; ++i) {
    double xd = x[i] + d[i];
    if (xd < b->lo[i] || xd > b->hi[i]) left_box = 1;
    xt[i] = clampd(xd, b->lo[i], b->hi[i]);
    s[i] = xt[i] - x[i];
  }
  double Hs[4];
  for (int i = 0; i < 4; ++i) {
    Hs[i] = 0.0;
    for (int k = 0; k < 4; ++k) Hs[i] += H[i][k] * s[k];
  }
  double gs = dot4(g, s);
  double q = gs + 0.5 * dot4(s, Hs);
  if (left_box && q > 0.01 * gs) {
    /* projected search: the first break point, where a component moving towards a
     * bound it is not on reaches it (at most the full step) */
    double alpha = 1.0;
    int first = -1;
    for (int i = 0; i < 4; ++i) {
      double brk;
      if (d[i] > 0.0 && x[i] < b->hi[i]) brk = (b->hi[i] - x[i]) / d[i];
      else if (d[i] < 0.0 && x[i] > b->lo[i]) brk = (b->lo[i] - x[i]) / d[i];
      else continue;
      if (brk < alpha) { alpha = brk; first = i; }
    }
    for (int i = 0; i < 4; ++i) {
      if (i == first) xt[i] = d[i] > 0.0 ? b->hi[i] : b->lo[i];
      else xt[i] = clampd(x[i] + alpha * d[i], b->lo[i], b->hi[i]);
      s[i] = xt[i] - x[i];
    }
    for (int i = 0; i < 4; ++i) {
      Hs[i] = 0.0;
      for (int k = 0; k < 4; ++k) Hs[i] += H[i][k] * s[k];
    }
    gs = dot4(g, s);
    q = gs + 0.5 * dot4(s, Hs);
  }
  return q;
}

/* Projected trust-region Newton (Nocedal & Wright Alg. 4.1 with the trial point
 * above).  Returns the number of Newton iterations taken; x holds the start on entry
 * and the result on exit. */
static int branch_solve(const branch_pb *b, double *x, int max_iter, double gtol, int hold, int *cg_total) {
  double g[4], H[4][4];
  for (int i = 0; i < 4; ++i) x[i] = clampd(x[i], b->lo[i], b->hi[i]);
  double F = branch_eval(b, x, g, H);
  /* initial radius: the half-width of the per-unit voltage box, the scale on which the
   * voltages move (the paper leaves the radius to the solver it cites) */
  double delta = 0.1;
  int it;
  int cg_its = 0;
  for (it = 0; it < max_iter; ++it) {
    int fr[4];
    double pg = 0.0;
    for (int i = 0; i < 4; ++i) {
      int at_lo = x[i] <= b->lo[i] && g[i] > 0.0;
      int at_hi = x[i] >= b->hi[i] && g[i] < 0.0;
      fr[i] = !(at_lo || at_hi);
      if (fr[i] && fabs(g[i]) > pg) pg = fabs(g[i]);
    }
    if (pg <= gtol) break;
    double xt[4], s[4];
    double q = trial_point(b, x, g, H, fr, delta, hold, xt, s, &cg_its);
    double sinf = 0.0, xinf = 0.0;
    for (int i = 0; i < 4; ++i) {
      if (fabs(s[i]) > sinf) sinf = fabs(s[i]);
      if (fabs(x[i]) > xinf) xinf = fabs(x[i]);
    }
    if (sinf <= 1e-15 * (1.0 + xinf)) break;
    double pred = -q;
    double Ft = branch_F(b, xt);
    /* a predicted decrease below the rounding level of F cannot be judged by the
     * actual decrease (both are noise): take the Newton step as agreeing */
    double ratio = pred > 0.0 ? (pred <= 1e-12 * fabs(F) ? 1.0 : (F - Ft) / pred) : -1.0;
    double snorm = sqrt(dot4(s, s));
    if (ratio < 0.25) delta = 0.25 * snorm;
    else if (ratio > 0.75 && snorm >= 0.99 * delta) delta = fmin(4.0 * delta, 10.0);  /* TRON: up to 4x */
    if (ratio >= 1e-4) {
      for (int i = 0; i < 4; ++i) x[i] = xt[i];
      F = branch_eval(b, x, g, H);
    }
  }
  if (cg_total) *cg_total = cg_its;
  return it;
}

/* ------------------------------------------------------------------------- */
/* 1-D convex piecewise-quadratic minimisation by bracketing                 */
/* ------------------------------------------------------------------------- */

/* D(x) = A x + B + sum_r rho_r * (neg_r ? min(0, x + e_r) : max(0, x + e_r)) is
 * continuous, piecewise linear and increasing; return argmin over [lo, hi] of
 * the function whose derivative it is. */
typedef struct { double A, B; int n; double rho[4], e[4]; int neg[4]; } pwl;

static double pwl_D(const pwl *f, double x) {
  double D = f->A * x + f->B;
  for (int r = 0; r < f->n; ++r) {
    double m = x + f->e[r];
    D += f->rho[r] * (f->neg[r] ? (m < 0.0 ? m : 0.0) : (m > 0.0 ? m : 0.0));
  }
  return D;
}

static double bracket_root(double (*D)(const void *, double), const void *ctx, double lo, double hi,
                           const double *kinks, int nk) {
  double dlo = D(ctx, lo), dhi = D(ctx, hi);
  if (dlo >= 0.0) return lo;
  if (dhi <= 0.0) return hi;
  double pts[8];
  int np = 0;
  pts[np++] = lo;
  for (int k = 0; k < nk; ++k) if (kinks[k] > lo && kinks[k] < hi) pts[np++] = kinks[k];
  pts[np++] = hi;
  /* insertion sort */
  for (int i = 1; i < np; ++i) {
    double v = pts[i];
    int j = i - 1;
    while (j >= 0 && pts[j] > v) { pts[j + 1] = pts[j]; --j; }
    pts[j + 1] = v;
  }
  for (int i = 0; i + 1 < np; ++i) {
    double da = D(ctx, pts[i]), db = D(ctx, pts[i + 1]);
    if (da < 0.0 && db >= 0.0) return pts[i] - da * (pts[i + 1] - pts[i]) / (db - da);
  }
  return hi; /* not reached for a continuous increasing D */
}

static double pwl_D_cb(const void *ctx, double x) { return pwl_D((const pwl *)ctx, x); }

static double pwl_argmin(const pwl *f, double lo, double hi) {
  double kinks[4];
  for (int r = 0; r < f->n; ++r) kinks[r] = -f->e[r];
  return bracket_root(pwl_D_cb, f, lo, hi, kinks, f->n);
}

/* ------------------------------------------------------------------------- */
/* generator block of step:opf (rows G1, G2, C1..C6; slacks eliminated)      */
/* ------------------------------------------------------------------------- */

typedef struct {
  double k2, k1, pmax, qlo_box, qhi_box;
  double pmin, pmaxc, qmin, qmax, ru, rd, su, sd;
  double rho_pq, rho_c;
  int relax; /* the multiperiod ACOPF: no minimum-generation row C1 */
} gen_data;

/* in: pbar_t, qbar_t, pbar_{t-1}, ubar_on_t, ubar_on_{t-1}, ubar_su_t, ubar_sd_t,
 * z and y of rows G1, G2, C1..C6.  out: p, q, s1..s6. */
static void gen_solve(const gen_data *d, double pb, double qb, double pb_prev, double uon, double uon_prev,
                      double usu, double usd, const double *z, const double *y, double *out) {
  double rp = d->rho_pq, rc = d->rho_c;
  /* p part: rows G1, C1 (-s1), C2 (+s2), C5 (-s5), C6 (+s6) */
  double eG1 = -pb + z[RG_G1] + y[RG_G1] / rp;
  double e1 = -d->pmin * uon + z[RG_C1] + y[RG_C1] / rc;
  double e2 = -d->pmaxc * uon + z[RG_C2] + y[RG_C2] / rc;
  double e5 = -pb_prev + d->rd * uon + d->sd * usd + z[RG_C5] + y[RG_C5] / rc;
  double e6 = -pb_prev - d->ru * uon_prev - d->su * usu + z[RG_C6] + y[RG_C6] / rc;
  pwl fp = {2.0 * d->k2 + rp, d->k1 + rp * eG1, 4, {d->relax ? 0.0 : rc, rc, rc, rc}, {e1, e2, e5, e6}, {1, 0, 1, 0}};
  double p = pwl_argmin(&fp, 0.0, d->pmax);
  /* q part: rows G2, C3 (-s3), C4 (+s4) */
  double eG2 = -qb + z[RG_G2] + y[RG_G2] / rp;
  double e3 = -d->qmin * uon + z[RG_C3] + y[RG_C3] / rc;
  double e4 = -d->qmax * uon + z[RG_C4] + y[RG_C4] / rc;
  pwl fq = {rp, rp * eG2, 2, {rc, rc, 0, 0}, {e3, e4, 0, 0}, {1, 0, 0, 0}};
  double q = pwl_argmin(&fq, d->qlo_box, d->qhi_box);
  out[0] = p;
  out[1] = q;
  out[2] = fmax(0.0, p + e1);   /* s1 */
  out[3] = fmax(0.0, -(p + e2)); /* s2 */
  out[4] = fmax(0.0, q + e3);   /* s3 */
  out[5] = fmax(0.0, -(q + e4)); /* s4 */
  out[6] = fmax(0.0, p + e5);   /* s5 */
  out[7] = fmax(0.0, -(p + e6)); /* s6 */
}

/* ------------------------------------------------------------------------- */
/* relaxed-commitment block step:uc_bar on the star {on_t, sd_t, su_{t+1}}   */
/* ------------------------------------------------------------------------- */

typedef struct {
  double rho_uc, rho_c;
  double h1, h3, h2;     /* U1(t), U3(t), U2(t+1) targets */
  double hc[4], kc[4];   /* C1..C4: (h - k a) */
  double h5, RD, SD;     /* C5(t): (h5 + RD a + SD b) */
  double h6, RU, SU;     /* C6(t+1): (h6 - RU a - SU c) */
  int has_next;
} ubar_pb;

static double ubar_b(const ubar_pb *u, double a) {
  return clampd((u->rho_uc * u->h3 - u->rho_c * u->SD * (u->h5 + u->RD * a)) / (u->rho_uc + u->rho_c * u->SD * u->SD), 0.0, 1.0);
}
static double ubar_c(const ubar_pb *u, double a) {
  return clampd((u->rho_uc * u->h2 + u->rho_c * u->SU * (u->h6 - u->RU * a)) / (u->rho_uc + u->rho_c * u->SU * u->SU), 0.0, 1.0);
}
/* derivative of the reduced objective phi(a) = min_{b,c} (...) (Danskin) */
static double ubar_dphi(const void *ctx, double a) {
  const ubar_pb *u = (const ubar_pb *)ctx;
  double D = -u->rho_uc * (u->h1 - a);
  for (int r = 0; r < 4; ++r) D -= u->rho_c * u->kc[r] * (u->hc[r] - u->kc[r] * a);
  D += u->rho_c * u->RD * (u->h5 + u->RD * a + u->SD * ubar_b(u, a));
  if (u->has_next) D -= u->rho_c * u->RU * (u->h6 - u->RU * a - u->SU * ubar_c(u, a));
  return D;
}

static void ubar_solve(const ubar_pb *u, double *a_out, double *b_out, double *c_out) {
  double kinks[4];
  int nk = 0;
  double den_b = u->rho_uc + u->rho_c * u->SD * u->SD;
  double slope_b = u->rho_c * u->SD * u->RD;
  if (slope_b != 0.0) {
    for (int v = 0; v < 2; ++v)
      kinks[nk++] = (u->rho_uc * u->h3 - u->rho_c * u->SD * u->h5 - v * den_b) / slope_b;
  }
  if (u->has_next) {
    double den_c = u->rho_uc + u->rho_c * u->SU * u->SU;
    double slope_c = u->rho_c * u->SU * u->RU;
    if (slope_c != 0.0) {
      for (int v = 0; v < 2; ++v)
        kinks[nk++] = (u->rho_uc * u->h2 + u->rho_c * u->SU * u->h6 - v * den_c) / slope_c;
    }
  }
  double a = bracket_root(ubar_dphi, u, 0.0, 1.0, kinks, nk);
  *a_out = a;
  *b_out = ubar_b(u, a);
  *c_out = u->has_next ? ubar_c(u, a) : 0.0;
}

/* ------------------------------------------------------------------------- */
/* UC block step:uc: dynamic programming of Sec. III-B                      */
/* ------------------------------------------------------------------------- */

/* L^UC_{g,t}(s', s): commitment costs plus the terms of rows U1..U3
 * (y (u - ubar + z) + rho/2 (u - ubar + z)^2) with u_su, u_sd inferred from
 * (s', s).  Evaluated left to right in exactly this order. */
static double uc_cost(double cnl, double csu, double csd, double rho, int sp, int s,
                      const double *ub /*on,su,sd*/, const double *z, const double *y) {
  int u[3];
  u[0] = s;
  u[1] = (s - sp) > 0 ? (s - sp) : 0;
  u[2] = (sp - s) > 0 ? (sp - s) : 0;
  double L = cnl * s + csu * u[1] + csd * u[2];
  for (int k = 0; k < 3; ++k) {
    double r = ((double)u[k] - ub[k]) + z[k];
    L += y[k] * r + 0.5 * rho * r * r;
  }
  return L;
}

/* The UC subproblem of one generator (Sec. III-B) as a memoized recursion.
 * c(t, s) is the least cost of periods t..T when the state before period t is s.
 * It is the smaller of the two choices the paper defines, keep_formula (stay in s
 * for period t, then c(t+1, s)) and switch_formula (enter 1-s at t and hold it for
 * T^min periods, T^U when switching on and T^D when switching off, then
 * c(t + T^min, 1-s)); stay is taken on a tie.  The switch cost is summed left to
 * right from L(t, s, 1-s), with the continuation added last.  c is zero beyond the
 * horizon, so a switch near the end holds the new state only up to T (the windows
 * of set:UC end at T).  Each evaluated (t, s) also keeps its optimal trajectory
 * u_{t,s,t..T}, built from its successor's as the paper's u formulas state.
 * Ltab[(t*2 + sp)*2 + s], t = 0..T-1, is L^UC_t(sp, s). */
typedef struct {
  int T, TU, TD;
  const double *Ltab;
  double *c;           /* [(T + 2) * 2], index t*2 + s */
  unsigned char *done; /* whether c(t, s) has been evaluated */
  int8_t *traj;        /* [(T + 2) * 2][T]: u_{t,s,t'} at traj[(t*2 + s)*T + t' - 1] */
} uc_memo;

static double uc_L(const uc_memo *m, int t, int sp, int s) { return m->Ltab[((size_t)(t - 1) * 2 + sp) * 2 + s]; }
static int8_t *uc_traj(const uc_memo *m, int t, int s) { return m->traj + ((size_t)t * 2 + s) * m->T; }

static double uc_cost_to_go(uc_memo *m, int t, int s) {
  if (t > m->T) return 0.0;
  if (m->done[t * 2 + s]) return m->c[t * 2 + s];
  const int T = m->T, alt = 1 - s;
  const int hold = alt ? m->TU : m->TD;
  /* keep_formula */
  double c_stay = uc_L(m, t, s, s) + uc_cost_to_go(m, t + 1, s);
  /* switch_formula */
  double c_switch = uc_L(m, t, s, alt);
  int until = t + hold - 1 < T ? t + hold - 1 : T;
  for (int tp = t + 1; tp <= until; ++tp) c_switch += uc_L(m, tp, alt, alt);
  c_switch += uc_cost_to_go(m, t + hold, alt);
  int8_t *u = uc_traj(m, t, s);
  if (c_stay <= c_switch) {
    m->c[t * 2 + s] = c_stay;
    u[t - 1] = (int8_t)s;
    if (t + 1 <= T) memcpy(u + t, uc_traj(m, t + 1, s) + t, (size_t)(T - t));
  } else {
    m->c[t * 2 + s] = c_switch;
    for (int tp = t; tp <= until; ++tp) u[tp - 1] = (int8_t)alt;
    if (t + hold <= T) memcpy(u + t + hold - 1, uc_traj(m, t + hold, alt) + t + hold - 1, (size_t)(T - t - hold + 1));
  }
  m->done[t * 2 + s] = 1;
  return m->c[t * 2 + s];
}

/* Optimal schedule from the initial condition: a unit that starts in state u0 and
 * must keep it for its first L_g (u0 = 1) or F_g (u0 = 0) periods pays those periods
 * in state u0 and continues from c(hold + 1, u0) (the reading of the initial
 * condition of Alg. dp_algo: the hold, not T^U / T^D, bounds the forced periods).
 * Writes u_on[0..T-1]; returns the optimal cost. */
static double dp_solve(int T, const double *Ltab, int u0, int Lg, int Fg, int TU, int TD, int8_t *uon) {
  uc_memo m = {T, TU, TD, Ltab, NULL, NULL, NULL};
  m.c = (double *)calloc((size_t)(T + 2) * 2, sizeof(double));
  m.done = (unsigned char *)calloc((size_t)(T + 2) * 2, 1);
  m.traj = (int8_t *)calloc((size_t)(T + 2) * 2 * (size_t)(T > 0 ? T : 1), 1);
  int hold = u0 ? Lg : Fg;
  if (hold > T) hold = T;
  if (hold < 0) hold = 0;
  double cost = 0.0;
  for (int t = 1; t <= hold; ++t) {
    cost += uc_L(&m, t, u0, u0);
    uon[t - 1] = (int8_t)u0;
  }
  cost += uc_cost_to_go(&m, hold + 1, u0);
  if (hold < T) memcpy(uon + hold, uc_traj(&m, hold + 1, u0) + hold, (size_t)(T - hold));
  free(m.c);
  free(m.done);
  free(m.traj);
  return cost;
}

/* ------------------------------------------------------------------------- */
/* problem setup                                                             */
/* ------------------------------------------------------------------------- */

static double *take(double **cur, size_t n) { double *p = *cur; *cur += n; return p; }

static size_t layout_state(orc_problem *P, double *base) {
  size_t TL = (size_t)P->T * P->L, TG = (size_t)P->T * P->G, TN = (size_t)P->T * P->N;
  double *cur = base;
  orc_state *S = &P->st;
  S->vf = take(&cur, TL); S->vt = take(&cur, TL); S->thf = take(&cur, TL); S->tht = take(&cur, TL);
  S->pf = take(&cur, TL); S->qf = take(&cur, TL); S->pt = take(&cur, TL); S->qt = take(&cur, TL);
  S->nuf = take(&cur, TL); S->nut = take(&cur, TL);
  S->p = take(&cur, TG); S->q = take(&cur, TG);
  for (int k = 0; k < 6; ++k) S->s[k] = take(&cur, TG);
  S->uon = take(&cur, TG); S->usu = take(&cur, TG); S->usd = take(&cur, TG);
  S->wb = take(&cur, TN); S->thb = take(&cur, TN);
  S->Pbf = take(&cur, TL); S->Qbf = take(&cur, TL); S->Pbt = take(&cur, TL); S->Qbt = take(&cur, TL);
  S->pb = take(&cur, TG); S->qb = take(&cur, TG);
  S->ubon = take(&cur, TG); S->ubsu = take(&cur, TG); S->ubsd = take(&cur, TG);
  for (int r = 0; r < NRB; ++r) S->zB[r] = take(&cur, TL);
  for (int r = 0; r < NRB; ++r) S->yB[r] = take(&cur, TL);
  for (int r = 0; r < NRB; ++r) S->lB[r] = take(&cur, TL);
  for (int r = 0; r < NRG; ++r) S->zG[r] = take(&cur, TG);
  for (int r = 0; r < NRG; ++r) S->yG[r] = take(&cur, TG);
  for (int r = 0; r < NRG; ++r) S->lG[r] = take(&cur, TG);
  S->sc = take(&cur, NSC);
  return (size_t)(cur - base);
}

/* duplicates block inside the state: from wb to ubsd, contiguous */
static size_t xbar_count(const orc_problem *P) {
  return (size_t)P->T * (2 * (size_t)P->N + 4 * (size_t)P->L + 5 * (size_t)P->G);
}

void orc_params_default(orc_params *p) {
  p->rho_pq = 5e3; p->rho_va = 1e4; p->rho_uc = 1e5; p->rho_cpl = 5e3;
  p->beta0 = 1e5; p->tau = 6.0; p->theta = 0.8; p->lambda_max = 1e12; p->beta_max = 1e24;
  p->mu_line = 5e3;
  p->newton_max_iter = 50; p->newton_gtol = 1e-12;
  p->max_inner = 1000; p->eps_in0 = 1e-2; p->tol = 1e-4;
  p->warm_start = 0;
  p->adapt_every = 0; p->adapt_mu = 3.0; p->adapt_tau = 1.5; p->adapt_max = 20; p->adapt_span = 100.0;
  p->relax_uc = 0;
}

static void init_state_u(orc_problem *P, const int8_t *u);
static void init_state(orc_problem *P) { init_state_u(P, NULL); }

orc_problem *orc_create(const orc_net *net, const orc_params *par) {
  orc_problem *P = (orc_problem *)calloc(1, sizeof(orc_problem));
  int N = net->n_bus, L = net->n_line, G = net->n_gen, T = net->T;
  P->N = N; P->L = L; P->G = G; P->T = T; P->ref = net->ref_bus;
  P->par = *par;
  double base = net->base_mva;
  P->from = (int *)malloc(sizeof(int) * L); P->to = (int *)malloc(sizeof(int) * L);
  P->adm = (double *)malloc(sizeof(double) * 8 * L); P->rate = (double *)malloc(sizeof(double) * L);
  for (int l = 0; l < L; ++l) {
    P->from[l] = net->line_from[l]; P->to[l] = net->line_to[l];
    line_admittance(net->line_r[l], net->line_x[l], net->line_b[l], P->adm + 8 * l);
    P->rate[l] = net->line_rate[l];
  }
#define CP(dst, src, n) do { dst = (double *)malloc(sizeof(double) * (n)); memcpy(dst, src, sizeof(double) * (n)); } while (0)
#define CPI(dst, src, n) do { dst = (int *)malloc(sizeof(int) * (n)); for (int _i = 0; _i < (n); ++_i) dst[_i] = (src)[_i]; } while (0)
  CP(P->gs, net->bus_gs, N); CP(P->bs, net->bus_bs, N); CP(P->vmin, net->bus_vmin, N); CP(P->vmax, net->bus_vmax, N);
  CP(P->Pd, net->load_p, (size_t)T * N); CP(P->Qd, net->load_q, (size_t)T * N);
  CPI(P->gbus, net->gen_bus, G);
  CP(P->pmin, net->gen_pmin, G); CP(P->pmax, net->gen_pmax, G); CP(P->qmin, net->gen_qmin, G); CP(P->qmax, net->gen_qmax, G);
  P->k2 = (double *)malloc(sizeof(double) * G); P->k1 = (double *)malloc(sizeof(double) * G);
  for (int g = 0; g < G; ++g) { P->k2[g] = net->gen_c2[g] * base * base; P->k1[g] = net->gen_c1[g] * base; }
  CP(P->cnl, net->gen_cnl, G); CP(P->csu, net->gen_csu, G); CP(P->csd, net->gen_csd, G);
  CP(P->ru, net->gen_ru, G); CP(P->rd, net->gen_rd, G); CP(P->su, net->gen_su, G); CP(P->sd, net->gen_sd, G);
  CP(P->p0, net->gen_p0, G);
  CPI(P->tu, net->gen_min_up, G); CPI(P->td, net->gen_min_dn, G); CPI(P->u0, net->gen_u0, G);
  CPI(P->lon, net->gen_init_on, G); CPI(P->loff, net->gen_init_off, G);
#undef CP
#undef CPI
  /* incidence lists, built with plain counting */
  P->inc_start = (int *)calloc(N + 1, sizeof(int));
  for (int l = 0; l < L; ++l) { P->inc_start[P->from[l] + 1]++; P->inc_start[P->to[l] + 1]++; }
  for (int i = 0; i < N; ++i) P->inc_start[i + 1] += P->inc_start[i];
  P->inc_line = (int *)malloc(sizeof(int) * 2 * L); P->inc_side = (int *)malloc(sizeof(int) * 2 * L);
  int *fill = (int *)calloc(N, sizeof(int));
  for (int l = 0; l < L; ++l) {
    int i = P->from[l], j = P->to[l];
    int a = P->inc_start[i] + fill[i]++; P->inc_line[a] = l; P->inc_side[a] = 0;
    int b = P->inc_start[j] + fill[j]++; P->inc_line[b] = l; P->inc_side[b] = 1;
  }
  free(fill);
  P->gen_start = (int *)calloc(N + 1, sizeof(int));
  for (int g = 0; g < G; ++g) P->gen_start[P->gbus[g] + 1]++;
  for (int i = 0; i < N; ++i) P->gen_start[i + 1] += P->gen_start[i];
  P->gen_list = (int *)malloc(sizeof(int) * (G > 0 ? G : 1));
  fill = (int *)calloc(N, sizeof(int));
  for (int g = 0; g < G; ++g) { int i = P->gbus[g]; P->gen_list[P->gen_start[i] + fill[i]++] = g; }
  free(fill);
  /* state */
  P->n_state = layout_state(P, NULL);
  P->buf = (double *)calloc(P->n_state, sizeof(double));
  layout_state(P, P->buf);
  P->xb_old = (double *)malloc(sizeof(double) * xbar_count(P));
  P->br_iters = (int *)calloc((size_t)T * L, sizeof(int));
  init_state(P);
  return P;
}

void orc_destroy(orc_problem *P) {
  if (!P) return;
  free(P->from); free(P->to); free(P->adm); free(P->rate);
  free(P->gs); free(P->bs); free(P->vmin); free(P->vmax); free(P->Pd); free(P->Qd);
  free(P->inc_start); free(P->inc_line); free(P->inc_side); free(P->gen_start); free(P->gen_list);
  free(P->gbus); free(P->pmin); free(P->pmax); free(P->qmin); free(P->qmax); free(P->k2); free(P->k1);
  free(P->cnl); free(P->csu); free(P->csd); free(P->ru); free(P->rd); free(P->su); free(P->sd); free(P->p0);
  free(P->tu); free(P->td); free(P->u0); free(P->lon); free(P->loff);
  free(P->buf); free(P->xb_old); free(P->br_iters);
  free(P);
}

static double qbox_lo(const orc_problem *P, int g) { return fmin(0.0, P->qmin[g]); }
static double qbox_hi(const orc_problem *P, int g) { return fmax(0.0, P->qmax[g]); }

/* Cold start: p, q and v at the middle of their bounds, angles zero, flows from
 * the voltages, duplicates equal to their originals, the commitments u ([T][G],
 * or every unit committed when u is NULL) with start-ups and shut-downs from their
 * changes, slacks at their feasible values, multipliers zero, beta = beta0. */
static void init_state_u(orc_problem *P, const int8_t *u) {
  orc_state *S = &P->st;
  int N = P->N, L = P->L, G = P->G, T = P->T;
  memset(P->buf, 0, sizeof(double) * P->n_state);
  for (int t = 0; t < T; ++t) {
    for (int l = 0; l < L; ++l) {
      size_t k = (size_t)t * L + l;
      int i = P->from[l], j = P->to[l];
      double x[4] = {0.5 * (P->vmin[i] + P->vmax[i]), 0.5 * (P->vmin[j] + P->vmax[j]), 0.0, 0.0};
      double f[4];
      line_flows(P->adm + 8 * l, x, f);
      S->vf[k] = x[0]; S->vt[k] = x[1]; S->thf[k] = 0.0; S->tht[k] = 0.0;
      S->pf[k] = f[0]; S->qf[k] = f[1]; S->pt[k] = f[2]; S->qt[k] = f[3];
      S->Pbf[k] = f[0]; S->Qbf[k] = f[1]; S->Pbt[k] = f[2]; S->Qbt[k] = f[3];
    }
    for (int i = 0; i < N; ++i) {
      double v = 0.5 * (P->vmin[i] + P->vmax[i]);
      S->wb[(size_t)t * N + i] = v * v;
      S->thb[(size_t)t * N + i] = 0.0;
    }
    for (int g = 0; g < G; ++g) {
      size_t k = (size_t)t * G + g;
      S->p[k] = 0.5 * P->pmax[g];
      S->q[k] = 0.5 * (qbox_lo(P, g) + qbox_hi(P, g));
      S->pb[k] = S->p[k]; S->qb[k] = S->q[k];
      int on = u ? u[k] : 1;
      int prev = t == 0 ? P->u0[g] : (u ? u[k - G] : 1);
      S->uon[k] = (double)on; S->usu[k] = (on - prev) > 0 ? 1.0 : 0.0; S->usd[k] = (prev - on) > 0 ? 1.0 : 0.0;
      S->ubon[k] = S->uon[k]; S->ubsu[k] = S->usu[k]; S->ubsd[k] = S->usd[k];
    }
  }
  for (int t = 0; t < T; ++t) {
    for (int g = 0; g < G; ++g) {
      size_t k = (size_t)t * G + g;
      double pbp = t == 0 ? P->p0[g] : S->pb[k - G];
      double uonp = t == 0 ? (double)P->u0[g] : S->ubon[k - G];
      double p = S->p[k], q = S->q[k], u = S->ubon[k];
      S->s[0][k] = fmax(0.0, p - P->pmin[g] * u);
      S->s[1][k] = fmax(0.0, P->pmax[g] * u - p);
      S->s[2][k] = fmax(0.0, q - P->qmin[g] * u);
      S->s[3][k] = fmax(0.0, P->qmax[g] * u - q);
      S->s[4][k] = fmax(0.0, p - pbp + P->rd[g] * u + P->sd[g] * S->ubsd[k]);
      S->s[5][k] = fmax(0.0, -(p - pbp) + P->ru[g] * uonp + P->su[g] * S->ubsu[k]);
    }
  }
  S->sc[SC_BETA] = P->par.beta0;
  S->sc[SC_ZPREV] = INFINITY;
  S->sc[SC_RHO_PQ] = P->par.rho_pq; S->sc[SC_RHO_VA] = P->par.rho_va;
  S->sc[SC_RHO_CPL] = P->par.rho_cpl; S->sc[SC_RHO_UC] = P->par.rho_uc;
}

/* ------------------------------------------------------------------------- */
/* row values a_r = (A x + B xbar)_r  (eq:uc-acopf-ext with the slack rows)   */
/* ------------------------------------------------------------------------- */

static void rows_branch(const orc_problem *P, int t, int l, double *a) {
  const orc_state *S = &P->st;
  size_t k = (size_t)t * P->L + l;
  size_t bi = (size_t)t * P->N + P->from[l], bj = (size_t)t * P->N + P->to[l];
  a[RB_PF] = S->pf[k] - S->Pbf[k];
  a[RB_QF] = S->qf[k] - S->Qbf[k];
  a[RB_PT] = S->pt[k] - S->Pbt[k];
  a[RB_QT] = S->qt[k] - S->Qbt[k];
  a[RB_WF] = S->vf[k] * S->vf[k] - S->wb[bi];
  a[RB_WT] = S->vt[k] * S->vt[k] - S->wb[bj];
  a[RB_TF] = S->thf[k] - S->thb[bi];
  a[RB_TT] = S->tht[k] - S->thb[bj];
}

static void rows_gen(const orc_problem *P, int t, int g, double *a) {
  const orc_state *S = &P->st;
  size_t k = (size_t)t * P->G + g;
  double pbp = t == 0 ? P->p0[g] : S->pb[k - P->G];
  double uonp = t == 0 ? (double)P->u0[g] : S->ubon[k - P->G];
  double p = S->p[k], q = S->q[k], u = S->ubon[k];
  a[RG_G1] = p - S->pb[k];
  a[RG_G2] = q - S->qb[k];
  a[RG_C1] = p - S->s[0][k] - P->pmin[g] * u;
  a[RG_C2] = p + S->s[1][k] - P->pmax[g] * u;
  a[RG_C3] = q - S->s[2][k] - P->qmin[g] * u;
  a[RG_C4] = q + S->s[3][k] - P->qmax[g] * u;
  a[RG_C5] = p - pbp - S->s[4][k] + P->rd[g] * u + P->sd[g] * S->ubsd[k];
  a[RG_C6] = p - pbp + S->s[5][k] - P->ru[g] * uonp - P->su[g] * S->ubsu[k];
  a[RG_U1] = S->uon[k] - S->ubon[k];
  a[RG_U2] = S->usu[k] - S->ubsu[k];
  a[RG_U3] = S->usd[k] - S->ubsd[k];
}

/* the penalties in force: part of the iterate (residual balancing may change them) */
static double rho_pq(const orc_problem *P) { return P->st.sc[SC_RHO_PQ]; }
static double rho_va(const orc_problem *P) { return P->st.sc[SC_RHO_VA]; }
static double rho_cpl(const orc_problem *P) { return P->st.sc[SC_RHO_CPL]; }
static double rho_uc(const orc_problem *P) { return P->st.sc[SC_RHO_UC]; }
static double rho_branch(const orc_problem *P, int r) { return r < 4 ? rho_pq(P) : rho_va(P); }
static double rho_gen(const orc_problem *P, int r) {
  if (r <= RG_G2) return rho_pq(P);
  if (r <= RG_C6) return rho_cpl(P);
  return rho_uc(P);
}
static int class_branch(int r) { return r < 4 ? CL_PQ : CL_VA; }
static int class_gen(int r) { return r <= RG_G2 ? CL_PQ : (r <= RG_C6 ? CL_CPL : CL_UC); }

/* ------------------------------------------------------------------------- */
/* the six blocks of one inner iteration                                     */
/* ------------------------------------------------------------------------- */

/* old duplicates, indexed like the state's duplicate block */
typedef struct { const double *wb, *thb, *Pbf, *Qbf, *Pbt, *Qbt, *pb, *qb, *ubon, *ubsu, *ubsd; } xbar_view;

static xbar_view old_view(const orc_problem *P) {
  size_t TL = (size_t)P->T * P->L, TG = (size_t)P->T * P->G, TN = (size_t)P->T * P->N;
  const double *c = P->xb_old;
  xbar_view v;
  v.wb = c; c += TN; v.thb = c; c += TN;
  v.Pbf = c; c += TL; v.Qbf = c; c += TL; v.Pbt = c; c += TL; v.Qbt = c; c += TL;
  v.pb = c; c += TG; v.qb = c; c += TG; v.ubon = c; c += TG; v.ubsu = c; c += TG; v.ubsd = c;
  return v;
}

/* step:uc -- one DP per generator on L^UC built from the old ubar, z, y */
static void block_uc(orc_problem *P, const xbar_view *X) {
  orc_state *S = &P->st;
  int T = P->T, G = P->G;
  if (P->par.relax_uc) return; /* the multiperiod ACOPF has no commitment decisions */
#pragma omp parallel
  {
  double *Lt = (double *)malloc(sizeof(double) * 4 * (T > 0 ? T : 1));
  int8_t *u = (int8_t *)malloc((size_t)(T > 0 ? T : 1));
#pragma omp for schedule(static)
  for (int g = 0; g < G; ++g) {
    for (int t = 0; t < T; ++t) {
      size_t k = (size_t)t * G + g;
      double ub[3] = {X->ubon[k], X->ubsu[k], X->ubsd[k]};
      double z[3] = {S->zG[RG_U1][k], S->zG[RG_U2][k], S->zG[RG_U3][k]};
      double y[3] = {S->yG[RG_U1][k], S->yG[RG_U2][k], S->yG[RG_U3][k]};
      for (int sp = 0; sp < 2; ++sp)
        for (int s = 0; s < 2; ++s)
          Lt[((size_t)t * 2 + sp) * 2 + s] = uc_cost(P->cnl[g], P->csu[g], P->csd[g], rho_uc(P), sp, s, ub, z, y);
    }
    dp_solve(T, Lt, P->u0[g], P->lon[g], P->loff[g], P->tu[g], P->td[g], u);
    for (int t = 0; t < T; ++t) {
      size_t k = (size_t)t * G + g;
      int prev = t == 0 ? P->u0[g] : u[t - 1];
      S->uon[k] = u[t];
      S->usu[k] = (u[t] - prev) > 0 ? 1.0 : 0.0;
      S->usd[k] = (prev - u[t]) > 0 ? 1.0 : 0.0;
    }
  }
  free(Lt);
  free(u);
  }
}

static void gen_data_of(const orc_problem *P, int g, gen_data *d) {
  d->k2 = P->k2[g]; d->k1 = P->k1[g]; d->pmax = P->pmax[g];
  d->qlo_box = qbox_lo(P, g); d->qhi_box = qbox_hi(P, g);
  d->pmin = P->pmin[g]; d->pmaxc = P->pmax[g]; d->qmin = P->qmin[g]; d->qmax = P->qmax[g];
  d->ru = P->ru[g]; d->rd = P->rd[g]; d->su = P->su[g]; d->sd = P->sd[g];
  d->rho_pq = rho_pq(P); d->rho_c = rho_cpl(P);
  d->relax = P->par.relax_uc;
}

/* step:opf, generator part */
static void block_gen(orc_problem *P, const xbar_view *X) {
  orc_state *S = &P->st;
  int T = P->T, G = P->G;
#pragma omp parallel for collapse(2) schedule(static)
  for (int t = 0; t < T; ++t) {
    for (int g = 0; g < G; ++g) {
      size_t k = (size_t)t * G + g;
      gen_data d;
      gen_data_of(P, g, &d);
      double z[8], y[8], out[8];
      for (int r = 0; r < 8; ++r) { z[r] = S->zG[r][k]; y[r] = S->yG[r][k]; }
      double pbp = t == 0 ? P->p0[g] : X->pb[k - G];
      double uonp = t == 0 ? (double)P->u0[g] : X->ubon[k - G];
      gen_solve(&d, X->pb[k], X->qb[k], pbp, X->ubon[k], uonp, X->ubsu[k], X->ubsd[k], z, y, out);
      S->p[k] = out[0]; S->q[k] = out[1];
      for (int r = 0; r < 6; ++r) S->s[r][k] = out[2 + r];
    }
  }
}

/* step:opf, line part */
static void block_branch(orc_problem *P, const xbar_view *X) {
  orc_state *S = &P->st;
  int T = P->T, L = P->L, N = P->N;
  double gtol = P->par.newton_gtol * fmax(1.0, fmax(rho_pq(P), rho_va(P)));
#pragma omp parallel for collapse(2) schedule(dynamic, 64)
  for (int t = 0; t < T; ++t) {
    for (int l = 0; l < L; ++l) {
      size_t k = (size_t)t * L + l;
      int i = P->from[l], j = P->to[l];
      size_t bi = (size_t)t * N + i, bj = (size_t)t * N + j;
      branch_pb b;
      memcpy(b.adm, P->adm + 8 * l, sizeof(b.adm));
      b.rate = P->rate[l];
      b.lo[0] = P->vmin[i]; b.hi[0] = P->vmax[i];
      b.lo[1] = P->vmin[j]; b.hi[1] = P->vmax[j];
      b.lo[2] = -TWO_PI; b.hi[2] = TWO_PI; b.lo[3] = -TWO_PI; b.hi[3] = TWO_PI;
      double xb[8] = {X->Pbf[k], X->Qbf[k], X->Pbt[k], X->Qbt[k], X->wb[bi], X->wb[bj], X->thb[bi], X->thb[bj]};
      for (int r = 0; r < 8; ++r) {
        double rho = rho_branch(P, r);
        b.c[r] = xb[r] - S->zB[r][k] - S->yB[r][k] / rho;
      }
      b.rho_pq = rho_pq(P); b.rho_va = rho_va(P); b.mu = P->par.mu_line;
      b.nu[0] = S->nuf[k]; b.nu[1] = S->nut[k];
      double x[4];
      if (P->par.warm_start == 1) {
        x[0] = S->vf[k]; x[1] = S->vt[k]; x[2] = S->thf[k]; x[3] = S->tht[k];
      } else {
        x[0] = 0.5 * (P->vmin[i] + P->vmax[i]); x[1] = 0.5 * (P->vmin[j] + P->vmax[j]); x[2] = 0.0; x[3] = 0.0;
      }
      /* with the hold step of TRON's subspace step, from every start */
      P->br_iters[k] = branch_solve(&b, x, P->par.newton_max_iter, gtol, 1, NULL);
      double f[4];
      line_flows(b.adm, x, f);
      S->vf[k] = x[0]; S->vt[k] = x[1]; S->thf[k] = x[2]; S->tht[k] = x[3];
      S->pf[k] = f[0]; S->qf[k] = f[1]; S->pt[k] = f[2]; S->qt[k] = f[3];
      /* multiplier of the PHR line-limit term */
      double hf = f[0] * f[0] + f[1] * f[1] - b.rate * b.rate;
      double ht = f[2] * f[2] + f[3] * f[3] - b.rate * b.rate;
      S->nuf[k] = fmax(0.0, b.nu[0] + b.mu * hf);
      S->nut[k] = fmax(0.0, b.nu[1] + b.mu * ht);
    }
  }
}

/* step:uc_bar: new x, old pbar (Jacobi with step:opf_bar) */
static void block_ubar(orc_problem *P, const xbar_view *X) {
  orc_state *S = &P->st;
  int T = P->T, G = P->G;
  if (P->par.relax_uc) return; /* commitments fixed at their cold-start values */
  double ruc = rho_uc(P), rc = rho_cpl(P);
#pragma omp parallel for collapse(2) schedule(static)
  for (int t = 0; t < T; ++t) {
    for (int g = 0; g < G; ++g) {
      size_t k = (size_t)t * G + g;
      ubar_pb u;
      u.rho_uc = ruc; u.rho_c = rc;
      u.h1 = S->uon[k] + S->zG[RG_U1][k] + S->yG[RG_U1][k] / ruc;
      u.h3 = S->usd[k] + S->zG[RG_U3][k] + S->yG[RG_U3][k] / ruc;
      u.hc[0] = S->p[k] - S->s[0][k] + S->zG[RG_C1][k] + S->yG[RG_C1][k] / rc; u.kc[0] = P->pmin[g];
      u.hc[1] = S->p[k] + S->s[1][k] + S->zG[RG_C2][k] + S->yG[RG_C2][k] / rc; u.kc[1] = P->pmax[g];
      u.hc[2] = S->q[k] - S->s[2][k] + S->zG[RG_C3][k] + S->yG[RG_C3][k] / rc; u.kc[2] = P->qmin[g];
      u.hc[3] = S->q[k] + S->s[3][k] + S->zG[RG_C4][k] + S->yG[RG_C4][k] / rc; u.kc[3] = P->qmax[g];
      double pbp = t == 0 ? P->p0[g] : X->pb[k - G];
      u.h5 = S->p[k] - pbp - S->s[4][k] + S->zG[RG_C5][k] + S->yG[RG_C5][k] / rc;
      u.RD = P->rd[g]; u.SD = P->sd[g];
      u.RU = P->ru[g]; u.SU = P->su[g];
      u.has_next = t + 1 < T;
      if (u.has_next) {
        size_t kn = k + G;
        u.h6 = S->p[kn] - X->pb[k] + S->s[5][kn] + S->zG[RG_C6][kn] + S->yG[RG_C6][kn] / rc;
        u.h2 = S->usu[kn] + S->zG[RG_U2][kn] + S->yG[RG_U2][kn] / ruc;
      } else {
        u.h6 = 0.0; u.h2 = 0.0;
      }
      double a, b, c;
      ubar_solve(&u, &a, &b, &c);
      S->ubon[k] = a;
      S->ubsd[k] = b;
      if (u.has_next) S->ubsu[k + G] = c;
      if (t == 0) {
        /* ubar_su at the first period: rows U2(1) and C6(1), ubar_on_0 = u0 */
        double h6 = S->p[k] - P->p0[g] + S->s[5][k] + S->zG[RG_C6][k] + S->yG[RG_C6][k] / rc;
        double h2 = S->usu[k] + S->zG[RG_U2][k] + S->yG[RG_U2][k] / ruc;
        double SU = P->su[g];
        S->ubsu[k] = clampd((ruc * h2 + rc * SU * (h6 - P->ru[g] * (double)P->u0[g])) / (ruc + rc * SU * SU), 0.0, 1.0);
      }
    }
  }
}

/* step:opf_bar: one equality-constrained diagonal QP per (bus, t) */
static void block_bus(orc_problem *P, const xbar_view *X) {
  orc_state *S = &P->st;
  int T = P->T, L = P->L, N = P->N, G = P->G;
  double rpq = rho_pq(P), rva = rho_va(P), rc = rho_cpl(P);
#pragma omp parallel for collapse(2) schedule(static)
  for (int t = 0; t < T; ++t) {
    for (int i = 0; i < N; ++i) {
      size_t bi = (size_t)t * N + i;
      /* accumulate sum(rho*tau) and W for w and theta; the constraint sums */
      double Ww = 0.0, Sw = 0.0, Wt = 0.0, St = 0.0;
      double M11 = 0.0, M12 = 0.0, M22 = 0.0, aTt = 0.0, bTt = 0.0;
      for (int e = P->inc_start[i]; e < P->inc_start[i + 1]; ++e) {
        int l = P->inc_line[e], side = P->inc_side[e];
        size_t k = (size_t)t * L + l;
        int rP = side ? RB_PT : RB_PF, rQ = side ? RB_QT : RB_QF, rW = side ? RB_WT : RB_WF, rT = side ? RB_TT : RB_TF;
        double flowP = side ? S->pt[k] : S->pf[k];
        double flowQ = side ? S->qt[k] : S->qf[k];
        double v = side ? S->vt[k] : S->vf[k];
        double th = side ? S->tht[k] : S->thf[k];
        double tauP = flowP + S->zB[rP][k] + S->yB[rP][k] / rpq;  /* alpha = -1, W = rpq */
        double tauQ = flowQ + S->zB[rQ][k] + S->yB[rQ][k] / rpq;  /* beta = -1 */
        M11 += 1.0 / rpq; aTt += -tauP;
        M22 += 1.0 / rpq; bTt += -tauQ;
        Ww += rva; Sw += rva * (v * v + S->zB[rW][k] + S->yB[rW][k] / rva);
        Wt += rva; St += rva * (th + S->zB[rT][k] + S->yB[rT][k] / rva);
      }
      for (int e = P->gen_start[i]; e < P->gen_start[i + 1]; ++e) {
        int g = P->gen_list[e];
        size_t k = (size_t)t * G + g;
        double Wp = rpq, Sp = rpq * (S->p[k] + S->zG[RG_G1][k] + S->yG[RG_G1][k] / rpq);
        if (t + 1 < T) {
          size_t kn = k + G;
          double t5 = S->p[kn] - S->s[4][kn] + P->rd[g] * X->ubon[kn] + P->sd[g] * X->ubsd[kn] + S->zG[RG_C5][kn] + S->yG[RG_C5][kn] / rc;
          double t6 = S->p[kn] + S->s[5][kn] - P->ru[g] * X->ubon[k] - P->su[g] * X->ubsu[kn] + S->zG[RG_C6][kn] + S->yG[RG_C6][kn] / rc;
          Wp += 2.0 * rc;
          Sp += rc * t5 + rc * t6;
        }
        double tauq = S->q[k] + S->zG[RG_G2][k] + S->yG[RG_G2][k] / rpq;
        M11 += 1.0 / Wp; aTt += Sp / Wp;
        M22 += 1.0 / rpq; bTt += tauq;
      }
      /* a bus without lines has no row on w or theta: they keep their values */
      double tauw = Ww > 0.0 ? Sw / Ww : X->wb[bi];
      double aw = Ww > 0.0 ? -P->gs[i] : 0.0, bw = Ww > 0.0 ? P->bs[i] : 0.0;
      if (Ww > 0.0) { M11 += aw * aw / Ww; M12 += aw * bw / Ww; M22 += bw * bw / Ww; }
      aTt += aw * tauw; bTt += bw * tauw;
      double r1 = P->Pd[bi] - aTt, r2 = P->Qd[bi] - bTt;
      double det = M11 * M22 - M12 * M12;
      double mu1 = (M22 * r1 - M12 * r2) / det;
      double mu2 = (M11 * r2 - M12 * r1) / det;
      /* write the duplicates: x_k = tau_k + (alpha_k mu1 + beta_k mu2) / W_k */
      S->wb[bi] = Ww > 0.0 ? tauw + (aw * mu1 + bw * mu2) / Ww : X->wb[bi];
      S->thb[bi] = (i == P->ref || Wt == 0.0) ? ((i == P->ref) ? 0.0 : X->thb[bi]) : St / Wt;
      for (int e = P->inc_start[i]; e < P->inc_start[i + 1]; ++e) {
        int l = P->inc_line[e], side = P->inc_side[e];
        size_t k = (size_t)t * L + l;
        int rP = side ? RB_PT : RB_PF, rQ = side ? RB_QT : RB_QF;
        double flowP = side ? S->pt[k] : S->pf[k];
        double flowQ = side ? S->qt[k] : S->qf[k];
        double tauP = flowP + S->zB[rP][k] + S->yB[rP][k] / rpq;
        double tauQ = flowQ + S->zB[rQ][k] + S->yB[rQ][k] / rpq;
        double Pn = tauP - mu1 / rpq, Qn = tauQ - mu2 / rpq;
        if (side) { S->Pbt[k] = Pn; S->Qbt[k] = Qn; } else { S->Pbf[k] = Pn; S->Qbf[k] = Qn; }
      }
      for (int e = P->gen_start[i]; e < P->gen_start[i + 1]; ++e) {
        int g = P->gen_list[e];
        size_t k = (size_t)t * G + g;
        double Wp = rpq, Sp = rpq * (S->p[k] + S->zG[RG_G1][k] + S->yG[RG_G1][k] / rpq);
        if (t + 1 < T) {
          size_t kn = k + G;
          double t5 = S->p[kn] - S->s[4][kn] + P->rd[g] * X->ubon[kn] + P->sd[g] * X->ubsd[kn] + S->zG[RG_C5][kn] + S->yG[RG_C5][kn] / rc;
          double t6 = S->p[kn] + S->s[5][kn] - P->ru[g] * X->ubon[k] - P->su[g] * X->ubsu[kn] + S->zG[RG_C6][kn] + S->yG[RG_C6][kn] / rc;
          Wp += 2.0 * rc;
          Sp += rc * t5 + rc * t6;
        }
        double tauq = S->q[k] + S->zG[RG_G2][k] + S->yG[RG_G2][k] / rpq;
        S->pb[k] = Sp / Wp + mu1 / Wp;
        S->qb[k] = tauq + mu2 / rpq;
      }
    }
  }
}

/* step:z and step:y, then the residuals.  Fills the scalars and, per penalty class,
 * the largest |a_r + z_r| (rin_c) and the largest |y_r| after the update (y_c). */
static void block_duals(orc_problem *P, double *rin_c, double *y_c) {
  orc_state *S = &P->st;
  int T = P->T, L = P->L, G = P->G;
  double beta = S->sc[SC_BETA];
  double rp = 0.0, rin = 0.0, zinf = 0.0;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, y0 = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0;
  /* the line rows and the generator-side rows are two independent sets of items;
   * the residual maxima are exact whatever the order */
#pragma omp parallel for collapse(2) schedule(static) reduction(max : rp, rin, zinf, r0, r1, y0, y1)
  for (int t = 0; t < T; ++t) {
    for (int l = 0; l < L; ++l) {
      size_t k = (size_t)t * L + l;
      double a[NRB];
      rows_branch(P, t, l, a);
      for (int r = 0; r < NRB; ++r) {
        double rho = rho_branch(P, r);
        double z = -(S->lB[r][k] + S->yB[r][k] + rho * a[r]) / (beta + rho);
        S->zB[r][k] = z;
        S->yB[r][k] += rho * (a[r] + z);
        rp = fmax(rp, fabs(a[r])); rin = fmax(rin, fabs(a[r] + z)); zinf = fmax(zinf, fabs(z));
        if (class_branch(r) == CL_PQ) { r0 = fmax(r0, fabs(a[r] + z)); y0 = fmax(y0, fabs(S->yB[r][k])); }
        else { r1 = fmax(r1, fabs(a[r] + z)); y1 = fmax(y1, fabs(S->yB[r][k])); }
      }
    }
  }
#pragma omp parallel for collapse(2) schedule(static) reduction(max : rp, rin, zinf, r0, r2, r3, y0, y2, y3)
  for (int t = 0; t < T; ++t) {
    for (int g = 0; g < G; ++g) {
      size_t k = (size_t)t * G + g;
      double a[NRG];
      rows_gen(P, t, g, a);
      for (int r = 0; r < NRG; ++r) {
        /* the multiperiod ACOPF has no minimum-generation and no commitment rows */
        if (P->par.relax_uc && (r == RG_C1 || r >= RG_U1)) continue;
        double rho = rho_gen(P, r);
        double z = -(S->lG[r][k] + S->yG[r][k] + rho * a[r]) / (beta + rho);
        S->zG[r][k] = z;
        S->yG[r][k] += rho * (a[r] + z);
        rp = fmax(rp, fabs(a[r])); rin = fmax(rin, fabs(a[r] + z)); zinf = fmax(zinf, fabs(z));
        int c = class_gen(r);
        double ar = fabs(a[r] + z), yr = fabs(S->yG[r][k]);
        if (c == CL_PQ) { r0 = fmax(r0, ar); y0 = fmax(y0, yr); }
        else if (c == CL_CPL) { r2 = fmax(r2, ar); y2 = fmax(y2, yr); }
        else { r3 = fmax(r3, ar); y3 = fmax(y3, yr); }
      }
    }
  }
  S->sc[SC_RP] = rp; S->sc[SC_RIN] = rin; S->sc[SC_ZINF] = zinf;
  rin_c[CL_PQ] = r0; rin_c[CL_VA] = r1; rin_c[CL_CPL] = r2; rin_c[CL_UC] = r3;
  y_c[CL_PQ] = y0; y_c[CL_VA] = y1; y_c[CL_CPL] = y2; y_c[CL_UC] = y3;
}

/* Residual balancing of the penalty classes, the remedy the paper's conclusion
 * points to for its main limitation (convergence sensitive to rho_pq, rho_va, rho_uc).
 * For class c: the primal residual r_c = max |a_r + z_r| over its rows, the dual
 * residual s_c = rho_c max |xbar^{l+1} - xbar^l| over the duplicates its rows
 * contain, divided by the class's multiplier scale max |y_r| (so both are relative
 * and unit-free); rho_c doubles (times tau) when r_c > mu s_c and halves when
 * s_c > mu r_c, within [rho0_c / span, rho0_c span] and at most adapt_max times per
 * class.  A class whose multipliers are all zero carries no information and keeps
 * its penalty, and so does a class whose two residuals are both at or below
 * ADAPT_NOISE: rows satisfied to the rounding level (commitments equal to their
 * binary duplicates, say), whose ratio is rounding noise.  The new penalties hold from the next iteration on; the multipliers
 * are kept unscaled, so they stay valid. */
#define ADAPT_NOISE 1e-9
static void adapt_penalties(orc_problem *P, const double *rin_c, const double *dx_c, const double *y_c) {
  orc_state *S = &P->st;
  const int rho_slot[NCL] = {SC_RHO_PQ, SC_RHO_VA, SC_RHO_CPL, SC_RHO_UC};
  const int cnt_slot[NCL] = {SC_NCHG_PQ, SC_NCHG_VA, SC_NCHG_CPL, SC_NCHG_UC};
  const double rho0[NCL] = {P->par.rho_pq, P->par.rho_va, P->par.rho_cpl, P->par.rho_uc};
  const double mu = P->par.adapt_mu, tau = P->par.adapt_tau, span = P->par.adapt_span;
  for (int c = 0; c < NCL; ++c) {
    if (S->sc[cnt_slot[c]] >= (double)P->par.adapt_max || !(y_c[c] > 0.0)) continue;
    double rho = S->sc[rho_slot[c]];
    double sd = rho * dx_c[c] / y_c[c];
    if (!(rin_c[c] > ADAPT_NOISE || sd > ADAPT_NOISE)) continue; /* both at the rounding level */
    if (rin_c[c] > mu * sd && rho * tau <= rho0[c] * span) {
      S->sc[rho_slot[c]] = rho * tau;
      S->sc[cnt_slot[c]] += 1.0;
    } else if (sd > mu * rin_c[c] && rho / tau >= rho0[c] / span) {
      S->sc[rho_slot[c]] = rho / tau;
      S->sc[cnt_slot[c]] += 1.0;
    }
  }
}

/* step:outer */
static void outer_update(orc_problem *P) {
  orc_state *S = &P->st;
  size_t TL = (size_t)P->T * P->L, TG = (size_t)P->T * P->G;
  double beta = S->sc[SC_BETA], lm = P->par.lambda_max;
  for (int r = 0; r < NRB; ++r)
    for (size_t k = 0; k < TL; ++k) S->lB[r][k] = clampd(S->lB[r][k] + beta * S->zB[r][k], -lm, lm);
  for (int r = 0; r < NRG; ++r)
    for (size_t k = 0; k < TG; ++k) S->lG[r][k] = clampd(S->lG[r][k] + beta * S->zG[r][k], -lm, lm);
  if (S->sc[SC_ZINF] > P->par.theta * S->sc[SC_ZPREV]) S->sc[SC_BETA] = fmin(P->par.tau * beta, P->par.beta_max);
  S->sc[SC_ZPREV] = S->sc[SC_ZINF];
  S->sc[SC_KOUT] += 1.0;
  S->sc[SC_LIN] = 0.0;
}

/* inner tolerance of outer iteration k */
static double eps_inner(const orc_problem *P) {
  double k = P->st.sc[SC_KOUT];
  return fmax(0.5 * P->par.tol, P->par.eps_in0 * pow(2.0, -k));
}

/* One inner iteration (step:uc .. step:y) plus the control that follows it.
 * stop_at_tol: if nonzero and r_p, r_d <= tol, mark converged and skip the
 * outer update.  Returns 1 when converged. */
static int iterate(orc_problem *P, int stop_at_tol) {
  orc_state *S = &P->st;
  memcpy(P->xb_old, S->wb, sizeof(double) * xbar_count(P));
  xbar_view X = old_view(P);
  block_uc(P, &X);       /* step:uc     (uses old duplicates) */
  block_gen(P, &X);      /* step:opf    generators */
  block_branch(P, &X);   /* step:opf    lines */
  block_ubar(P, &X);     /* step:uc_bar (new x, old pbar) */
  block_bus(P, &X);      /* step:opf_bar (new x, old ubar) */
  /* dual residual: largest change of any duplicate; per penalty class, the largest
   * change of the duplicates its rows contain (power: line-end flows, pbar, qbar;
   * voltage/angle: wbar, thetabar; coupling: pbar and the relaxed commitments;
   * commitment: the relaxed commitments) */
  size_t TL = (size_t)P->T * P->L, TG = (size_t)P->T * P->G, TN = (size_t)P->T * P->N;
  double d_va = 0.0, d_fl = 0.0, d_pb = 0.0, d_qb = 0.0, d_ub = 0.0;
#pragma omp parallel for schedule(static) reduction(max : d_va)
  for (size_t k = 0; k < 2 * TN; ++k) d_va = fmax(d_va, fabs(S->wb[k] - P->xb_old[k]));
#pragma omp parallel for schedule(static) reduction(max : d_fl)
  for (size_t k = 2 * TN; k < 2 * TN + 4 * TL; ++k) d_fl = fmax(d_fl, fabs(S->wb[k] - P->xb_old[k]));
#pragma omp parallel for schedule(static) reduction(max : d_pb)
  for (size_t k = 2 * TN + 4 * TL; k < 2 * TN + 4 * TL + TG; ++k) d_pb = fmax(d_pb, fabs(S->wb[k] - P->xb_old[k]));
#pragma omp parallel for schedule(static) reduction(max : d_qb)
  for (size_t k = 2 * TN + 4 * TL + TG; k < 2 * TN + 4 * TL + 2 * TG; ++k) d_qb = fmax(d_qb, fabs(S->wb[k] - P->xb_old[k]));
#pragma omp parallel for schedule(static) reduction(max : d_ub)
  for (size_t k = 2 * TN + 4 * TL + 2 * TG; k < xbar_count(P); ++k) d_ub = fmax(d_ub, fabs(S->wb[k] - P->xb_old[k]));
  S->sc[SC_RD] = fmax(fmax(d_va, d_fl), fmax(fmax(d_pb, d_qb), d_ub));
  double dx_c[NCL] = {fmax(d_fl, fmax(d_pb, d_qb)), d_va, fmax(d_pb, d_ub), d_ub};
  double rin_c[NCL], y_c[NCL];
  block_duals(P, rin_c, y_c);  /* step:z, step:y */
  S->sc[SC_ITER] += 1.0;
  S->sc[SC_LIN] += 1.0;
  if (stop_at_tol && S->sc[SC_RP] <= P->par.tol && S->sc[SC_RD] <= P->par.tol) {
    S->sc[SC_CONV] = 1.0;
    return 1;
  }
  if (P->par.adapt_every > 0 && fmod(S->sc[SC_ITER], (double)P->par.adapt_every) == 0.0)
    adapt_penalties(P, rin_c, dx_c, y_c);
  if (fmax(S->sc[SC_RIN], S->sc[SC_RD]) <= eps_inner(P) || S->sc[SC_LIN] >= (double)P->par.max_inner)
    outer_update(P);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* exported API                                                              */
/* ------------------------------------------------------------------------- */

void orc_step(orc_problem *P, int n) {
  for (int i = 0; i < n; ++i) iterate(P, 0);
}

int orc_solve(orc_problem *P, double tol, int max_iters, int *iters_done) {
  P->par.tol = tol;
  int done = 0, i;
  for (i = 0; i < max_iters && !done; ++i) done = iterate(P, 1);
  if (iters_done) *iters_done = i;
  return done ? 0 : 1;
}

/* UC warm start (Sec. IV-A): solve the multiperiod ACOPF -- the same iteration with
 * the commitments held at their cold-start values, no dynamic program, no commitment
 * rows and no minimum-generation row, so that a unit's output may fall to zero --
 * from the cold start to tol (or max_iters iterations); then commit a unit in a
 * period when its generation there is at least half its minimum output, and start
 * the method from the cold start with those commitments.  Returns the relaxed
 * solve's status (0 converged, 1 not). */
int orc_uc_warmstart(orc_problem *P, double tol, int max_iters, int *iters_done) {
  orc_params saved = P->par;
  P->par.relax_uc = 1;
  init_state(P);
  int rc = orc_solve(P, tol, max_iters, iters_done);
  size_t TG = (size_t)P->T * P->G;
  int8_t *u = (int8_t *)malloc(TG > 0 ? TG : 1);
  for (int t = 0; t < P->T; ++t)
    for (int g = 0; g < P->G; ++g) {
      size_t k = (size_t)t * P->G + g;
      u[k] = P->st.p[k] >= 0.5 * P->pmin[g] ? 1 : 0;
    }
  P->par = saved;
  init_state_u(P, u);
  free(u);
  return rc;
}

size_t orc_state_size(const orc_problem *P) { return P->n_state; }
void orc_get_state(const orc_problem *P, double *out) { memcpy(out, P->buf, sizeof(double) * P->n_state); }
void orc_set_state(orc_problem *P, const double *in) { memcpy(P->buf, in, sizeof(double) * P->n_state); }
void orc_reset(orc_problem *P) { init_state(P); }
/* new parameters from the next iteration on; the penalties in force become the new
 * ones and their residual-balancing counts restart */
void orc_set_params(orc_problem *P, const orc_params *par) {
  P->par = *par;
  orc_state *S = &P->st;
  S->sc[SC_RHO_PQ] = par->rho_pq; S->sc[SC_RHO_VA] = par->rho_va;
  S->sc[SC_RHO_CPL] = par->rho_cpl; S->sc[SC_RHO_UC] = par->rho_uc;
  S->sc[SC_NCHG_PQ] = S->sc[SC_NCHG_VA] = S->sc[SC_NCHG_CPL] = S->sc[SC_NCHG_UC] = 0.0;
}
void orc_get_branch_iters(const orc_problem *P, int32_t *out) {
  for (size_t k = 0; k < (size_t)P->T * P->L; ++k) out[k] = P->br_iters[k];
}

/* threads of the parallel loops (0: the OpenMP default) and the default itself */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
int orc_max_threads(void) { return omp_get_max_threads(); }

double orc_objective(const orc_problem *P) {
  const orc_state *S = &P->st;
  double obj = 0.0;
  for (int t = 0; t < P->T; ++t)
    for (int g = 0; g < P->G; ++g) {
      size_t k = (size_t)t * P->G + g;
      double p = S->p[k];
      obj += P->k2[g] * p * p + P->k1[g] * p;
      obj += P->cnl[g] * S->uon[k] + P->csu[g] * S->usu[k] + P->csd[g] * S->usd[k];
    }
  return obj;
}

/* --- single-item entry points used by the pins --- */

double orc_dp(int T, const double *Ltab, int u0, int Lg, int Fg, int TU, int TD, int8_t *uon) {
  return dp_solve(T, Ltab, u0, Lg, Fg, TU, TD, uon);
}

double orc_uc_cost(double cnl, double csu, double csd, double rho, int sp, int s, const double *ub, const double *z, const double *y) {
  return uc_cost(cnl, csu, csd, rho, sp, s, ub, z, y);
}

/* data[13] = k2 k1 pmax qlo_box qhi_box pmin pmax qmin qmax ru rd su sd; rho[2] = rho_pq rho_c;
 * xin[7] = pbar qbar pbar_prev ubar_on ubar_on_prev ubar_su ubar_sd; z[8], y[8]: G1 G2 C1..C6 */
void orc_gen_solve(const double *data, const double *rho, const double *xin, const double *z, const double *y, double *out) {
  gen_data d = {data[0], data[1], data[2], data[3], data[4], data[5], data[6], data[7], data[8],
                data[9], data[10], data[11], data[12], rho[0], rho[1]};
  gen_solve(&d, xin[0], xin[1], xin[2], xin[3], xin[4], xin[5], xin[6], z, y, out);
}

/* pb[...]: see ubar_pb field order: rho_uc rho_c h1 h3 h2 hc[4] kc[4] h5 RD SD h6 RU SU has_next */
void orc_ubar_solve(const double *v, double *out) {
  ubar_pb u;
  u.rho_uc = v[0]; u.rho_c = v[1]; u.h1 = v[2]; u.h3 = v[3]; u.h2 = v[4];
  for (int r = 0; r < 4; ++r) { u.hc[r] = v[5 + r]; u.kc[r] = v[9 + r]; }
  u.h5 = v[13]; u.RD = v[14]; u.SD = v[15]; u.h6 = v[16]; u.RU = v[17]; u.SU = v[18]; u.has_next = v[19] != 0.0;
  ubar_solve(&u, &out[0], &out[1], &out[2]);
}

/* v[...] = adm[8] rate lo[4] hi[4] c[8] rho_pq rho_va mu nu[2] */
static void unpack_branch(const double *v, branch_pb *b) {
  memcpy(b->adm, v, 8 * sizeof(double));
  b->rate = v[8];
  memcpy(b->lo, v + 9, 4 * sizeof(double));
  memcpy(b->hi, v + 13, 4 * sizeof(double));
  memcpy(b->c, v + 17, 8 * sizeof(double));
  b->rho_pq = v[25]; b->rho_va = v[26]; b->mu = v[27]; b->nu[0] = v[28]; b->nu[1] = v[29];
}

double orc_branch_eval(const double *v, const double *x, double *g, double *H) {
  branch_pb b;
  unpack_branch(v, &b);
  double Hm[4][4];
  double F = branch_eval(&b, x, g, Hm);
  for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) H[4 * i + j] = Hm[i][j];
  return F;
}

double orc_branch_F(const double *v, const double *x) {
  branch_pb b;
  unpack_branch(v, &b);
  return branch_F(&b, x);
}

int orc_branch_solve(const double *v, double *x, int max_iter, double gtol, int hold, int *cg_its) {
  branch_pb b;
  unpack_branch(v, &b);
  return branch_solve(&b, x, max_iter, gtol, hold, cg_its);
}

/* One trial point from x with radius delta (evaluates g and H at x itself). */
double orc_branch_trial(const double *v, const double *x, double delta, int hold, double *xt) {
  branch_pb b;
  unpack_branch(v, &b);
  double g[4], H[4][4], s[4];
  int fr[4], cg = 0;
  branch_eval(&b, x, g, H);
  for (int i = 0; i < 4; ++i) fr[i] = !((x[i] <= b.lo[i] && g[i] > 0.0) || (x[i] >= b.hi[i] && g[i] < 0.0));
  return trial_point(&b, x, g, H, fr, delta, hold, xt, s, &cg);
}

void orc_line_admittance(double r, double x, double b, double *adm) { line_admittance(r, x, b, adm); }
void orc_line_flows(const double *adm, const double *x, double *f) { line_flows(adm, x, f); }
