// Host side of the C-ABI in include/ucac.h: input validation, device layout,
// cold start, the captured iteration graph and the control loop of ucac_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ucac.h"
#include "ucac_launch.hpp"
#include "ucac_solve_rule.hpp"

using namespace ucac;

namespace {

thread_local std::string g_create_error;

// ucac_solve examines the device-side status after every chunk of this many
// iterations.  (Queuing the next chunk before examining the previous one, with two
// snapshots, measured no faster: the host turnaround is not what solve mode pays.)
// Each chunk costs a snapshot and a status read; the stopping chunk is replayed up to
// its stop.  At 2,000 buses 64 was 1.8 % faster to 1e-4 than 32 and 128 0.6 %.
constexpr int SOLVE_CHUNK = 64;

// Iterations are captured in graphs of 64, 16, 4 and 1 iterations, and n
// iterations are enqueued largest graph first (500 = 7 x 64 + 3 x 16 + 4: 11
// launches).  Consecutive iterations inside a graph start without the per-graph
// launch gap (about 9 us at 2,000 buses; 16 iterations per graph measured 1.5 %
// faster per iteration than 4).  Iterations after convergence in solve mode return
// at kernel entry; a solve chunk (32) runs as two graphs of 16.
constexpr int N_GRAPHS = 4;
constexpr int GRAPH_SIZES[N_GRAPHS] = {64, 16, 4, 1};

struct GraphSet {
  hipGraph_t g[N_GRAPHS] = {};
  hipGraphExec_t x[N_GRAPHS] = {};
  void clear() {
    for (int j = 0; j < N_GRAPHS; ++j) {
      if (x[j]) (void)hipGraphExecDestroy(x[j]);
      if (g[j]) (void)hipGraphDestroy(g[j]);
      x[j] = nullptr;
      g[j] = nullptr;
    }
  }
  hipError_t launch(int n, hipStream_t st) const {
    hipError_t e = hipSuccess;
    for (int j = 0; j < N_GRAPHS && e == hipSuccess; ++j)
      for (; n >= GRAPH_SIZES[j] && e == hipSuccess; n -= GRAPH_SIZES[j]) e = hipGraphLaunch(x[j], st);
    return e;
  }
};

struct HostGen {
  std::vector<double> k2, k1, cnl, csu, csd;
  std::vector<int> u0;
  // for the UC warm start's restart (internal order)
  std::vector<double> pmin, pmax, qmin, qmax, ru, rd, su, sd, p0;
};

}  // namespace

struct ucac_handle {
  int N = 0, L = 0, G = 0, T = 0, ref = 0;
  ucac_params par{};
  hipStream_t own = nullptr, stream = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  Net net{};
  State st{};
  Par kp{};
  size_t n_state = 0;  // doubles
  double* d_state = nullptr;
  Ctl* d_ctl = nullptr;
  Ctl* h_ctl = nullptr;      // pinned staging of the control block
  double* h_sc = nullptr;    // pinned staging of the scalars
  GraphSet graphs;        // step mode: GRAPH_SIZES[j] iterations, control steps inside the next front launch
  GraphSet graphs_solve;  // solve mode: GRAPH_SIZES[j] iterations, each with its own control-step kernel
  // step mode with residual balancing: one period of adapt_every fused iterations
  // (the last one's control step decides), or null
  hipGraph_t g_period = nullptr;
  hipGraphExec_t x_period = nullptr;
  hipEvent_t ev_poll = nullptr;
  HostGen hg;
  int cus = 0;               // compute units of the device
  std::vector<double> cold;  // the cold-start iterate (internal layout)
  // learned warm start: FP32 parameters and BF16 operand copies
  void* mlp_mem = nullptr;
  // ucac_solve's snapshot at the start of each chunk: state, control block, work counters
  void* solve_save = nullptr;
  // locality ordering: internal index -> caller's index
  std::vector<int> perm_bus, perm_line, perm_gen;
  std::string err;
};

namespace {

int fail(ucac_handle* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf; else g_create_error = buf;
  return code;
}

#define HIP_OR(h, call)                                                                             \
  do {                                                                                              \
    hipError_t _e = (call);                                                                         \
    if (_e != hipSuccess) return fail(h, UCAC_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
  } while (0)

bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Wavefronts of the line kernel at either block size (64 or 256): one counter slot each.
size_t branch_waves_of(size_t TL) { return ((TL + 255) / 256) * 4; }

size_t state_doubles(size_t N, size_t L, size_t G, size_t T) {
  return T * L * (10 + 4 + 3 * NRB) + T * G * (11 + 5 + 3 * NRG) + T * N * 2 + NSC;
}

// residual balancing: adapt_every >= 0 (0 off), adapt_mu > 0, adapt_tau >= 1,
// adapt_max >= 0, adapt_span >= 1, all finite
bool adapt_params_ok(const ucac_params* p) {
  return p->adapt_every >= 0 && p->adapt_max >= 0 && p->adapt_mu > 0.0 && std::isfinite(p->adapt_mu) &&
         p->adapt_tau >= 1.0 && std::isfinite(p->adapt_tau) && p->adapt_span >= 1.0 && std::isfinite(p->adapt_span);
}

int validate(const ucac_network* n, const ucac_params* p) {
  if (!n || !p) return fail(nullptr, UCAC_E_INVAL, "null network or params");
  if (n->n_bus < 1 || n->n_line < 0 || n->n_gen < 0 || n->T < 1)
    return fail(nullptr, UCAC_E_INVAL, "bad sizes n_bus=%d n_line=%d n_gen=%d T=%d", n->n_bus, n->n_line, n->n_gen, n->T);
  const long long TL = (long long)n->T * n->n_line, TN = (long long)n->T * n->n_bus, TG = (long long)n->T * n->n_gen;
  if (TL * NRB > 0x7fffffffLL || TN > 0x7fffffffLL || TG * NRG > 0x7fffffffLL)
    return fail(nullptr, UCAC_E_INVAL, "instance too large for 32-bit item indices");
  if (n->ref_bus < 0 || n->ref_bus >= n->n_bus) return fail(nullptr, UCAC_E_INVAL, "ref_bus %d out of range", n->ref_bus);
  if (!(n->base_mva > 0.0) || !std::isfinite(n->base_mva)) return fail(nullptr, UCAC_E_INVAL, "base_mva must be positive");
  const int N = n->n_bus, L = n->n_line, G = n->n_gen;
  if (L > 0 && (!n->line_from || !n->line_to || !n->line_r || !n->line_x || !n->line_b || !n->line_rate))
    return fail(nullptr, UCAC_E_INVAL, "null line array");
  if (!n->bus_gs || !n->bus_bs || !n->bus_vmin || !n->bus_vmax || !n->load_p || !n->load_q)
    return fail(nullptr, UCAC_E_INVAL, "null bus array");
  if (G > 0 && (!n->gen_bus || !n->gen_pmin || !n->gen_pmax || !n->gen_qmin || !n->gen_qmax || !n->gen_c2 ||
                !n->gen_c1 || !n->gen_cnl || !n->gen_csu || !n->gen_csd || !n->gen_ru || !n->gen_rd || !n->gen_su ||
                !n->gen_sd || !n->gen_min_up || !n->gen_min_dn || !n->gen_u0 || !n->gen_init_on ||
                !n->gen_init_off || !n->gen_p0))
    return fail(nullptr, UCAC_E_INVAL, "null generator array");
  std::vector<int> deg(N, 0);
  for (int l = 0; l < L; ++l) {
    const int i = n->line_from[l], j = n->line_to[l];
    if (i < 0 || i >= N || j < 0 || j >= N || i == j) return fail(nullptr, UCAC_E_INVAL, "line %d has bad end buses (%d, %d)", l, i, j);
    if (!finite_all(&n->line_r[l], 1) || !finite_all(&n->line_x[l], 1) || !finite_all(&n->line_b[l], 1) ||
        !finite_all(&n->line_rate[l], 1))
      return fail(nullptr, UCAC_E_INVAL, "line %d has non-finite data", l);
    if (n->line_r[l] * n->line_r[l] + n->line_x[l] * n->line_x[l] <= 0.0) return fail(nullptr, UCAC_E_INVAL, "line %d has zero impedance", l);
    if (!(n->line_rate[l] > 0.0)) return fail(nullptr, UCAC_E_INVAL, "line %d has a non-positive rating", l);
    deg[i]++; deg[j]++;
  }
  if (!finite_all(n->bus_gs, N) || !finite_all(n->bus_bs, N) || !finite_all(n->bus_vmin, N) || !finite_all(n->bus_vmax, N))
    return fail(nullptr, UCAC_E_INVAL, "non-finite bus data");
  for (int i = 0; i < N; ++i)
    if (!(n->bus_vmin[i] > 0.0) || n->bus_vmin[i] > n->bus_vmax[i]) return fail(nullptr, UCAC_E_INVAL, "bus %d has bad voltage bounds", i);
  if (!finite_all(n->load_p, (size_t)TN) || !finite_all(n->load_q, (size_t)TN)) return fail(nullptr, UCAC_E_INVAL, "non-finite load");
  for (int g = 0; g < G; ++g) {
    const int b = n->gen_bus[g];
    if (b < 0 || b >= N) return fail(nullptr, UCAC_E_INVAL, "generator %d at bus %d out of range", g, b);
    const double* d[] = {&n->gen_pmin[g], &n->gen_pmax[g], &n->gen_qmin[g], &n->gen_qmax[g], &n->gen_c2[g], &n->gen_c1[g],
                         &n->gen_cnl[g], &n->gen_csu[g], &n->gen_csd[g], &n->gen_ru[g], &n->gen_rd[g], &n->gen_su[g],
                         &n->gen_sd[g], &n->gen_p0[g]};
    for (const double* v : d)
      if (!std::isfinite(*v)) return fail(nullptr, UCAC_E_INVAL, "generator %d has non-finite data", g);
    if (n->gen_pmin[g] > n->gen_pmax[g] || n->gen_pmax[g] < 0.0) return fail(nullptr, UCAC_E_INVAL, "generator %d: pmin > pmax or pmax < 0", g);
    if (n->gen_qmin[g] > n->gen_qmax[g]) return fail(nullptr, UCAC_E_INVAL, "generator %d: qmin > qmax", g);
    if (n->gen_c2[g] < 0.0) return fail(nullptr, UCAC_E_INVAL, "generator %d: c2 < 0 (non-convex cost)", g);
    if (n->gen_min_up[g] < 1 || n->gen_min_dn[g] < 1) return fail(nullptr, UCAC_E_INVAL, "generator %d: min up/down < 1", g);
    if (n->gen_u0[g] != 0 && n->gen_u0[g] != 1) return fail(nullptr, UCAC_E_INVAL, "generator %d: u0 not in {0,1}", g);
    if (n->gen_init_on[g] < 0 || n->gen_init_off[g] < 0) return fail(nullptr, UCAC_E_INVAL, "generator %d: negative initial hold", g);
    deg[b]++;
  }
  for (int i = 0; i < N; ++i)
    if (deg[i] == 0) return fail(nullptr, UCAC_E_INVAL, "bus %d has neither a line nor a generator", i);
  const double pos[] = {p->rho_pq, p->rho_va, p->rho_uc, p->rho_cpl, p->beta0, p->tau, p->lambda_max, p->beta_max, p->mu_line};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(nullptr, UCAC_E_INVAL, "penalty parameters must be positive and finite");
  if (!(p->theta > 0.0) || !(p->newton_gtol >= 0.0) || !(p->eps_in0 >= 0.0) || !(p->tol > 0.0) || p->newton_max_iter < 0 ||
      p->max_inner < 1 || p->warm_start < 0 || p->warm_start > 1)
    return fail(nullptr, UCAC_E_INVAL, "bad iteration parameters");
  if (!adapt_params_ok(p)) return fail(nullptr, UCAC_E_INVAL, "bad residual-balancing parameters");
  return UCAC_OK;
}

struct Arena {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * n;
    return p;
  }
};

// Carve every device array out of one allocation.  With base == nullptr only the
// size is computed.
size_t branch_waves(const ucac_handle* h) { return branch_waves_of((size_t)h->T * h->L); }

size_t carve(ucac_handle* h, char* base) {
  const size_t N = h->N, L = h->L, G = h->G, T = h->T;
  Arena a{base, 0};
  Net& n = h->net;
  State& s = h->st;
  n.N = h->N; n.L = h->L; n.G = h->G; n.T = h->T; n.ref = h->ref;
  n.from = a.take<int>(L); n.to = a.take<int>(L);
  n.adm = a.take<double>(8 * L); n.rate = a.take<double>(L);
  n.gs = a.take<double>(N); n.bs = a.take<double>(N); n.vmin = a.take<double>(N); n.vmax = a.take<double>(N);
  n.Pd = a.take<double>(T * N); n.Qd = a.take<double>(T * N);
  n.inc_start = a.take<int>(N + 1); n.inc_code = a.take<int>(2 * L); n.end_pos = a.take<int>(2 * L);
  n.gen_start = a.take<int>(N + 1); n.gen_list = a.take<int>(G); n.unit_first = a.take<int>(N);
  n.pmin = a.take<double>(G); n.pmax = a.take<double>(G); n.qmin = a.take<double>(G); n.qmax = a.take<double>(G);
  n.k2 = a.take<double>(G); n.k1 = a.take<double>(G); n.cnl = a.take<double>(G); n.csu = a.take<double>(G);
  n.csd = a.take<double>(G); n.ru = a.take<double>(G); n.rd = a.take<double>(G); n.su = a.take<double>(G);
  n.sd = a.take<double>(G); n.p0 = a.take<double>(G);
  n.tu = a.take<int>(G); n.td = a.take<int>(G); n.u0 = a.take<int>(G); n.lon = a.take<int>(G); n.loff = a.take<int>(G);
  h->d_state = a.take<double>(h->n_state);
  s.ub_nxt = a.take<double>(3 * T * G);
  s.br_iters = a.take<int>(T * L);
  s.x0 = a.take<float>(4 * T * L);
  s.br_count = a.take<unsigned long long>(branch_waves(h) * NBRC);
  s.red_units = 0;
  s.red_bus = s.red_units + n.G;  // one slot per unit block: at most one block per generator
  s.red_bpost = s.red_bus + bus_blocks(n);
  s.red_gdual = s.red_bpost + line_blocks(n);
  s.red_n = s.red_gdual + gen_dual_blocks(n);
  s.red_u = s.red_units;
  s.red_bus2 = s.red_n + n.G;
  s.red_ugen = s.red_bus2 + bus_blocks(n);
  s.red_total = s.red_ugen + n.G;
  s.red = a.take<double>((size_t)s.red_total * NACC);
  s.redc = a.take<double>((size_t)s.red_total * NCS);
  s.ebuf = a.take<double>(T * 2 * L * 4);
  s.bmu = a.take<double>(2 * T * N);
  s.log_feat = nullptr; s.log_targ = nullptr; s.log_count = nullptr;
  s.log_cap = 0; s.log_stride = 1; s.log_phase = 0;
  h->d_ctl = a.take<Ctl>(1);
  s.ctl = h->d_ctl;
  // state views (the state format of ucac_get_state)
  double* c = h->d_state;
  auto nx = [&](size_t k) { double* p = c; if (c) c += k; return p; };
  const size_t TL = T * L, TG = T * G, TN = T * N;
  s.vf = nx(TL); s.vt = nx(TL); s.thf = nx(TL); s.tht = nx(TL); s.pf = nx(TL); s.qf = nx(TL); s.pt = nx(TL); s.qt = nx(TL);
  s.nuf = nx(TL); s.nut = nx(TL);
  s.p = nx(TG); s.q = nx(TG); s.s = nx(6 * TG); s.uon = nx(TG); s.usu = nx(TG); s.usd = nx(TG);
  s.wb = nx(TN); s.thb = nx(TN);
  s.Pbf = nx(TL); s.Qbf = nx(TL); s.Pbt = nx(TL); s.Qbt = nx(TL);
  s.pb = nx(TG); s.qb = nx(TG); s.ubon = nx(TG); s.ubsu = nx(TG); s.ubsd = nx(TG);
  s.zB = nx(NRB * TL); s.yB = nx(NRB * TL); s.lB = nx(NRB * TL);
  s.zG = nx(NRG * TG); s.yG = nx(NRG * TG); s.lG = nx(NRG * TG);
  s.sc = nx(NSC);
  return a.off;
}

// Cold start (the initialisation of the ACOPF variables and an all-committed
// schedule): mid-range v, p, q; zero angles; flows of the flat voltages;
// duplicates equal to their originals; slacks at their feasible values;
// multipliers zero; beta = beta0.
void cold_start(const ucac_network* n, const std::vector<double>& adm, const ucac_params& par, std::vector<double>& S) {
  const size_t N = n->n_bus, L = n->n_line, G = n->n_gen, T = n->T;
  const size_t TL = T * L, TG = T * G, TN = T * N;
  S.assign(state_doubles(N, L, G, T), 0.0);
  double* c = S.data();
  auto nx = [&](size_t k) { double* p = c; c += k; return p; };
  double *vf = nx(TL), *vt = nx(TL), *thf = nx(TL), *tht = nx(TL), *pf = nx(TL), *qf = nx(TL), *pt = nx(TL), *qt = nx(TL);
  nx(2 * TL);  // nu
  double *p = nx(TG), *q = nx(TG), *s = nx(6 * TG), *uon = nx(TG), *usu = nx(TG), *usd = nx(TG);
  double *wb = nx(TN), *thb = nx(TN);
  double *Pbf = nx(TL), *Qbf = nx(TL), *Pbt = nx(TL), *Qbt = nx(TL);
  double *pb = nx(TG), *qb = nx(TG), *ubon = nx(TG), *ubsu = nx(TG), *ubsd = nx(TG);
  nx(3 * NRB * TL + 3 * NRG * TG);
  double* sc = nx(NSC);
  for (size_t t = 0; t < T; ++t) {
    for (size_t l = 0; l < L; ++l) {
      const size_t k = t * L + l;
      const int i = n->line_from[l], j = n->line_to[l];
      const double vi = 0.5 * (n->bus_vmin[i] + n->bus_vmax[i]), vj = 0.5 * (n->bus_vmin[j] + n->bus_vmax[j]);
      const double* A = &adm[0];
      const double Gii = A[0 * L + l], Bii = A[1 * L + l], Gij = A[2 * L + l], Bij = A[3 * L + l];
      const double Gjj = A[4 * L + l], Bjj = A[5 * L + l], Gji = A[6 * L + l], Bji = A[7 * L + l];
      // zero angle difference: cos = 1, sin = 0
      vf[k] = vi; vt[k] = vj; thf[k] = 0.0; tht[k] = 0.0;
      pf[k] = Gii * vi * vi + vi * vj * Gij;
      qf[k] = -Bii * vi * vi - vi * vj * Bij;
      pt[k] = Gjj * vj * vj + vi * vj * Gji;
      qt[k] = -Bjj * vj * vj - vi * vj * Bji;
      Pbf[k] = pf[k]; Qbf[k] = qf[k]; Pbt[k] = pt[k]; Qbt[k] = qt[k];
    }
    for (size_t i = 0; i < N; ++i) {
      const double v = 0.5 * (n->bus_vmin[i] + n->bus_vmax[i]);
      wb[t * N + i] = v * v;
      thb[t * N + i] = 0.0;
    }
    for (size_t g = 0; g < G; ++g) {
      const size_t k = t * G + g;
      const double qlo = std::fmin(0.0, n->gen_qmin[g]), qhi = std::fmax(0.0, n->gen_qmax[g]);
      p[k] = 0.5 * n->gen_pmax[g];
      q[k] = 0.5 * (qlo + qhi);
      pb[k] = p[k]; qb[k] = q[k];
      const int prev = t == 0 ? n->gen_u0[g] : 1;
      uon[k] = 1.0; usu[k] = prev == 0 ? 1.0 : 0.0; usd[k] = 0.0;
      ubon[k] = uon[k]; ubsu[k] = usu[k]; ubsd[k] = usd[k];
    }
  }
  for (size_t t = 0; t < T; ++t)
    for (size_t g = 0; g < G; ++g) {
      const size_t k = t * G + g;
      const double pbp = t == 0 ? n->gen_p0[g] : pb[k - G];
      const double uonp = t == 0 ? (double)n->gen_u0[g] : ubon[k - G];
      const double pv = p[k], qv = q[k], u = ubon[k];
      s[0 * TG + k] = std::fmax(0.0, pv - n->gen_pmin[g] * u);
      s[1 * TG + k] = std::fmax(0.0, n->gen_pmax[g] * u - pv);
      s[2 * TG + k] = std::fmax(0.0, qv - n->gen_qmin[g] * u);
      s[3 * TG + k] = std::fmax(0.0, n->gen_qmax[g] * u - qv);
      s[4 * TG + k] = std::fmax(0.0, pv - pbp + n->gen_rd[g] * u + n->gen_sd[g] * ubsd[k]);
      s[5 * TG + k] = std::fmax(0.0, -(pv - pbp) + n->gen_ru[g] * uonp + n->gen_su[g] * ubsu[k]);
    }
  sc[SC_BETA] = par.beta0;
  sc[SC_ZPREV] = INFINITY;
  sc[SC_RHO_PQ] = par.rho_pq; sc[SC_RHO_VA] = par.rho_va; sc[SC_RHO_CPL] = par.rho_cpl; sc[SC_RHO_UC] = par.rho_uc;
}

// A cold-start iterate S (internal layout) with the commitments u [T][G] (0/1)
// instead of every unit committed: start-ups and shut-downs from their changes (u0
// before the first period), relaxed commitments equal to them, and the slacks at
// their feasible values for them (the same expressions as the cold start).
void set_commitments(const HostGen& hg, size_t N, size_t L, size_t G, size_t T, std::vector<double>& S,
                     const std::vector<signed char>& u) {
  const size_t TL = T * L, TG = T * G, TN = T * N;
  double* c = S.data() + 10 * TL;  // after the line x-side
  double *p = c, *q = c + TG, *s = c + 2 * TG, *uon = c + 8 * TG, *usu = c + 9 * TG, *usd = c + 10 * TG;
  c += 11 * TG + 2 * TN + 4 * TL;  // the generator x-side, bus duplicates, line-end duplicates
  double *pb = c, *ubon = c + 2 * TG, *ubsu = c + 3 * TG, *ubsd = c + 4 * TG;
  for (size_t t = 0; t < T; ++t)
    for (size_t g = 0; g < G; ++g) {
      const size_t k = t * G + g;
      const int on = u[k], prev = t == 0 ? hg.u0[g] : u[k - G];
      uon[k] = (double)on;
      usu[k] = on > prev ? 1.0 : 0.0;
      usd[k] = prev > on ? 1.0 : 0.0;
      ubon[k] = uon[k]; ubsu[k] = usu[k]; ubsd[k] = usd[k];
    }
  for (size_t t = 0; t < T; ++t)
    for (size_t g = 0; g < G; ++g) {
      const size_t k = t * G + g;
      const double pbp = t == 0 ? hg.p0[g] : pb[k - G];
      const double uonp = t == 0 ? (double)hg.u0[g] : ubon[k - G];
      const double pv = p[k], qv = q[k], uu = ubon[k];
      s[0 * TG + k] = std::fmax(0.0, pv - hg.pmin[g] * uu);
      s[1 * TG + k] = std::fmax(0.0, hg.pmax[g] * uu - pv);
      s[2 * TG + k] = std::fmax(0.0, qv - hg.qmin[g] * uu);
      s[3 * TG + k] = std::fmax(0.0, hg.qmax[g] * uu - qv);
      s[4 * TG + k] = std::fmax(0.0, pv - pbp + hg.rd[g] * uu + hg.sd[g] * ubsd[k]);
      s[5 * TG + k] = std::fmax(0.0, -(pv - pbp) + hg.ru[g] * uonp + hg.su[g] * ubsu[k]);
    }
}

// ---- locality ordering ------------------------------------------------------
//
// The bus kernel gathers the x-side values of every incident line end and the line
// kernel gathers the duplicates of both end buses.  With the caller's numbering,
// consecutive lanes touch unrelated lines, so nearly every gather fetches a whole
// cache line for 8 useful bytes.  The library therefore renumbers buses by reverse
// Cuthill-McKee (neighbours get near indices), lines by their lower-numbered end,
// and units by their bus.  Everything the caller sees (state, solution, iteration
// counts) is converted back at the boundary.

void rcm_order(int N, const std::vector<std::vector<int>>& adj, std::vector<int>& order) {
  std::vector<int> idx(N);
  std::iota(idx.begin(), idx.end(), 0);
  auto by_deg = [&](int a, int b) { return adj[a].size() != adj[b].size() ? adj[a].size() < adj[b].size() : a < b; };
  std::stable_sort(idx.begin(), idx.end(), by_deg);
  std::vector<char> seen(N, 0);
  order.clear();
  order.reserve(N);
  for (int s0 : idx) {
    if (seen[s0]) continue;
    size_t head = order.size();
    order.push_back(s0);
    seen[s0] = 1;
    for (; head < order.size(); ++head) {
      std::vector<int> nb = adj[order[head]];
      std::stable_sort(nb.begin(), nb.end(), by_deg);
      for (int v : nb)
        if (!seen[v]) { seen[v] = 1; order.push_back(v); }
    }
  }
  std::reverse(order.begin(), order.end());
}

struct Permuted {
  ucac_network view;
  std::vector<int32_t> from, to, gbus, tu, td, u0, lon, loff;
  std::vector<double> r, x, b, rate, gs, bs, vmin, vmax, lp, lq;
  std::vector<double> pmin, pmax, qmin, qmax, c2, c1, cnl, csu, csd, ru, rd, su, sd, p0;
};

void make_order(const ucac_network* n, std::vector<int>& pb, std::vector<int>& pl, std::vector<int>& pg) {
  const int N = n->n_bus, L = n->n_line, G = n->n_gen;
  std::vector<std::vector<int>> adj(N);
  for (int l = 0; l < L; ++l) { adj[n->line_from[l]].push_back(n->line_to[l]); adj[n->line_to[l]].push_back(n->line_from[l]); }
  rcm_order(N, adj, pb);
  std::vector<int> inv(N);
  for (int i = 0; i < N; ++i) inv[pb[i]] = i;
  pl.resize(L);
  std::iota(pl.begin(), pl.end(), 0);
  std::stable_sort(pl.begin(), pl.end(), [&](int a, int c) {
    const int a0 = std::min(inv[n->line_from[a]], inv[n->line_to[a]]), c0 = std::min(inv[n->line_from[c]], inv[n->line_to[c]]);
    if (a0 != c0) return a0 < c0;
    return std::max(inv[n->line_from[a]], inv[n->line_to[a]]) < std::max(inv[n->line_from[c]], inv[n->line_to[c]]);
  });
  pg.resize(G);
  std::iota(pg.begin(), pg.end(), 0);
  std::stable_sort(pg.begin(), pg.end(), [&](int a, int c) { return inv[n->gen_bus[a]] < inv[n->gen_bus[c]]; });
}

void permute_network(const ucac_network* n, const std::vector<int>& pb, const std::vector<int>& pl,
                     const std::vector<int>& pg, Permuted& P) {
  const int N = n->n_bus, L = n->n_line, G = n->n_gen, T = n->T;
  std::vector<int> inv(N);
  for (int i = 0; i < N; ++i) inv[pb[i]] = i;
  auto bybus = [&](const double* a, std::vector<double>& out) { out.resize(N); for (int i = 0; i < N; ++i) out[i] = a[pb[i]]; };
  auto byline = [&](const double* a, std::vector<double>& out) { out.resize(L); for (int l = 0; l < L; ++l) out[l] = a[pl[l]]; };
  auto bygen = [&](const double* a, std::vector<double>& out) { out.resize(G); for (int g = 0; g < G; ++g) out[g] = a[pg[g]]; };
  auto bygeni = [&](const int32_t* a, std::vector<int32_t>& out) { out.resize(G); for (int g = 0; g < G; ++g) out[g] = a[pg[g]]; };
  P.from.resize(L); P.to.resize(L);
  for (int l = 0; l < L; ++l) { P.from[l] = inv[n->line_from[pl[l]]]; P.to[l] = inv[n->line_to[pl[l]]]; }
  byline(n->line_r, P.r); byline(n->line_x, P.x); byline(n->line_b, P.b); byline(n->line_rate, P.rate);
  bybus(n->bus_gs, P.gs); bybus(n->bus_bs, P.bs); bybus(n->bus_vmin, P.vmin); bybus(n->bus_vmax, P.vmax);
  P.lp.resize((size_t)T * N); P.lq.resize((size_t)T * N);
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < N; ++i) { P.lp[(size_t)t * N + i] = n->load_p[(size_t)t * N + pb[i]]; P.lq[(size_t)t * N + i] = n->load_q[(size_t)t * N + pb[i]]; }
  P.gbus.resize(G);
  for (int g = 0; g < G; ++g) P.gbus[g] = inv[n->gen_bus[pg[g]]];
  bygen(n->gen_pmin, P.pmin); bygen(n->gen_pmax, P.pmax); bygen(n->gen_qmin, P.qmin); bygen(n->gen_qmax, P.qmax);
  bygen(n->gen_c2, P.c2); bygen(n->gen_c1, P.c1); bygen(n->gen_cnl, P.cnl); bygen(n->gen_csu, P.csu); bygen(n->gen_csd, P.csd);
  bygen(n->gen_ru, P.ru); bygen(n->gen_rd, P.rd); bygen(n->gen_su, P.su); bygen(n->gen_sd, P.sd); bygen(n->gen_p0, P.p0);
  bygeni(n->gen_min_up, P.tu); bygeni(n->gen_min_dn, P.td); bygeni(n->gen_u0, P.u0);
  bygeni(n->gen_init_on, P.lon); bygeni(n->gen_init_off, P.loff);
  ucac_network& v = P.view;
  v = *n;
  v.ref_bus = inv[n->ref_bus];
  v.line_from = P.from.data(); v.line_to = P.to.data();
  v.line_r = P.r.data(); v.line_x = P.x.data(); v.line_b = P.b.data(); v.line_rate = P.rate.data();
  v.bus_gs = P.gs.data(); v.bus_bs = P.bs.data(); v.bus_vmin = P.vmin.data(); v.bus_vmax = P.vmax.data();
  v.load_p = P.lp.data(); v.load_q = P.lq.data();
  v.gen_bus = P.gbus.data();
  v.gen_pmin = P.pmin.data(); v.gen_pmax = P.pmax.data(); v.gen_qmin = P.qmin.data(); v.gen_qmax = P.qmax.data();
  v.gen_c2 = P.c2.data(); v.gen_c1 = P.c1.data(); v.gen_cnl = P.cnl.data(); v.gen_csu = P.csu.data(); v.gen_csd = P.csd.data();
  v.gen_ru = P.ru.data(); v.gen_rd = P.rd.data(); v.gen_su = P.su.data(); v.gen_sd = P.sd.data(); v.gen_p0 = P.p0.data();
  v.gen_min_up = P.tu.data(); v.gen_min_dn = P.td.data(); v.gen_u0 = P.u0.data();
  v.gen_init_on = P.lon.data(); v.gen_init_off = P.loff.data();
}

// Convert a flat state between the caller's numbering and the internal one.
void convert_state(const ucac_handle* h, const double* src, double* dst, bool to_internal) {
  const size_t T = h->T;
  struct Seg { const std::vector<int>* perm; int count; };
  const Seg segs[] = {{&h->perm_line, 10}, {&h->perm_gen, 11}, {&h->perm_bus, 2}, {&h->perm_line, 4},
                      {&h->perm_gen, 5}, {&h->perm_line, 3 * NRB}, {&h->perm_gen, 3 * NRG}};
  size_t off = 0;
  for (const Seg& sg : segs) {
    const size_t n = sg.perm->size();
    const int* pm = sg.perm->data();
    for (int a = 0; a < sg.count; ++a) {
      for (size_t t = 0; t < T; ++t) {
        const double* sr = src + off + t * n;
        double* ds = dst + off + t * n;
        if (to_internal) for (size_t i = 0; i < n; ++i) ds[i] = sr[pm[i]];
        else for (size_t i = 0; i < n; ++i) ds[pm[i]] = sr[i];
      }
      off += T * n;
    }
  }
  for (int k = 0; k < NSC; ++k) dst[off + k] = src[off + k];
}

// [T][n] array from internal to caller numbering
template <class V>
void unpermute_rows(const std::vector<int>& perm, size_t T, const V* src, V* dst) {
  const size_t n = perm.size();
  for (size_t t = 0; t < T; ++t)
    for (size_t i = 0; i < n; ++i) dst[t * n + perm[i]] = src[t * n + i];
}

Par kernel_params(const ucac_params& p) {
  Par k{};
  k.rho_pq = p.rho_pq; k.rho_va = p.rho_va; k.rho_uc = p.rho_uc; k.rho_cpl = p.rho_cpl; k.mu = p.mu_line;
  k.gtol = p.newton_gtol * std::fmax(1.0, std::fmax(p.rho_pq, p.rho_va));
  k.gtol_base = p.newton_gtol;
  k.adapt_every = p.adapt_every; k.adapt_max = p.adapt_max;
  k.adapt_mu = p.adapt_mu; k.adapt_tau = p.adapt_tau; k.adapt_span = p.adapt_span;
  k.rho0[CL_PQ] = p.rho_pq; k.rho0[CL_VA] = p.rho_va; k.rho0[CL_CPL] = p.rho_cpl; k.rho0[CL_UC] = p.rho_uc;
  k.relax_uc = 0;
  k.tau = p.tau; k.theta = p.theta; k.lambda_max = p.lambda_max; k.beta_max = p.beta_max; k.eps_in0 = p.eps_in0;
  k.newton_max_iter = p.newton_max_iter; k.max_inner = p.max_inner; k.warm_start = p.warm_start;
  return k;
}

// Enqueue one inner iteration for capture, on one stream:
//
//   front (unit side | lines) -> bus -> post -> finalize
//
// The unit side (generator update, step:uc, step:uc_bar; per generator) does not
// depend on the line kernel and vice versa, so both run in one launch of two block
// ranges; step:uc_bar reads the previous pbar, which the bus kernel then overwrites.
// After the bus QP, one launch finishes the line ends and updates the
// coupling/commitment multipliers.  Consecutive launches on one stream start back
// to back; a fork/join between two streams cost several microseconds per iteration.
//
// launch(k, stream) launches kernel k (K_FRONT or a K_* index) and returns
// hipGetLastError().
template <class F>
hipError_t enqueue_chain(F launch, hipStream_t st, const char** where) {
  static const char* names[] = {"front", "bus", "post", "finalize"};
  const int ks[] = {K_FRONT, K_BUS, K_POST, K_FINALIZE};
  for (int i = 0; i < 4; ++i) {
    const hipError_t e = launch(ks[i], st);
    if (e != hipSuccess) {
      if (where) *where = names[i];
      return e;
    }
  }
  return hipSuccess;
}

hipError_t enqueue_iteration(ucac_handle* h, hipStream_t st, const char** where) {
  auto launch = [&](int k, hipStream_t s) {
    switch (k) {
      case K_FRONT: launch_front(h->net, h->st, h->kp, s); break;
      case K_BUS: launch_bus(h->net, h->st, h->kp, s); break;
      case K_POST: launch_post(h->net, h->st, h->kp, s); break;
      default: launch_finalize(h->net, h->st, h->kp, s); break;
    }
    return hipGetLastError();
  };
  return enqueue_chain(launch, st, where);
}

// Iteration r of a step-mode graph of `size` iterations.  Its unit blocks write slot
// copy r & 1; from the second iteration on, its front launch also runs the previous
// iteration's control step (a block of its own, reading the other copy), which takes
// that kernel off the critical path; the graph's last iteration ends with its own
// control step.  Such a step cannot stop an instance (the next front launch already
// runs beside it); ucac_solve runs these graphs from a snapshot and replays the last
// chunk, ending in one solve-mode iteration, to stop at the right iteration.
hipError_t enqueue_step_iteration(ucac_handle* h, hipStream_t st, int r, int size, const char** where) {
  State sr = h->st;
  const int copy[2] = {h->st.red_units, h->st.red_n};
  sr.red_u = copy[r & 1];
  const int fin = r > 0 ? copy[(r - 1) & 1] : -1;
  launch_front(h->net, sr, h->kp, st, fin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { if (where) *where = "front"; return e; }
  launch_bus(h->net, h->st, h->kp, st);
  if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "bus"; return e; }
  launch_post(h->net, h->st, h->kp, st);
  if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "post"; return e; }
  if (r == size - 1) {
    launch_finalize(h->net, sr, h->kp, st);
    if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "finalize"; return e; }
  }
  return hipSuccess;
}

// Iteration r of a fused step graph of `size` iterations, two launches per iteration:
//
//   A(r) = finish of iteration r-1's rows (r > 0) | iteration r's unit side and lines
//   B(r) = iteration r's bus solve (without rows G1, G2) | iteration r-1's control step
//
// and after the last iteration one launch that finishes its rows, then its control
// step.  An iteration's residual slots: its unit blocks' (copy r & 1), its bus
// blocks' (bus copy r & 1), the line-end finish's (red_bpost) and the generator-row
// finish's (red_ugen), the last two written by the next A; the control step of r - 1
// thus runs beside the bus solve of r, which writes the other bus copy.  Every
// iterate is the kernel-by-kernel iteration's bit for bit: the same item arithmetic,
// each row updated once per iteration after the values it reads, and maxima whose
// grouping does not change them.  With residual balancing an iteration whose control
// step decides must end a graph (launch_balanced): that step changes penalties the
// next bus solve reads.  With the learned start the line lanes evaluate the network
// between the finish and the Newton solve.
hipError_t enqueue_fused_iteration(ucac_handle* h, hipStream_t st, int r, int size, const char** where) {
  const State& s0 = h->st;
  const int ucopy[2] = {s0.red_units, s0.red_n};
  const int bcopy[2] = {s0.red_bus, s0.red_bus2};
  auto ranges = [&](int k) {
    const int first[4] = {ucopy[k & 1], bcopy[k & 1], s0.red_bpost, s0.red_ugen};
    const int count[4] = {s0.red_bus - s0.red_units, bus_blocks(h->net), line_blocks(h->net), h->net.G};
    return slot_ranges(first, count);
  };
  State sr = s0;
  sr.red_u = ucopy[r & 1];
  sr.red_bus = bcopy[r & 1];
  launch_front_fused(h->net, sr, h->kp, st, r > 0 ? FUSE_PRO | FUSE_WORK : FUSE_WORK);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { if (where) *where = "front (fused)"; return e; }
  const SlotRanges prev = ranges(r - 1);
  launch_bus_fused(h->net, sr, h->kp, st, r > 0 ? &prev : nullptr);
  if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "bus (fused)"; return e; }
  if (r == size - 1) {
    launch_front_fused(h->net, sr, h->kp, st, FUSE_PRO);
    if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "finish (fused)"; return e; }
    launch_finalize_ranges(sr, h->kp, ranges(r), st);
    if ((e = hipGetLastError()) != hipSuccess) { if (where) *where = "finalize"; return e; }
  }
  return hipSuccess;
}

// Wavefronts of the launch that runs the unit side and the lines (256-thread blocks),
// against what the CUs hold at once (two such blocks per CU).
bool front_queues(const ucac_handle* h) {
  const long unit_blocks = h->G && h->T ? (h->G + units_gpb(h->T, 16, 256) - 1) / units_gpb(h->T, 16, 256) : 0;
  const long line_blocks = ((long)h->T * h->L + 255) / 256;
  return 4L * (unit_blocks + line_blocks) > 8L * h->cus;
}

// The step graphs' form: fused, unless the learned start's network would hold back a
// launch of several rounds of wavefronts; then the pipelined form.  Inside the fused
// launch the network saves a kernel and the reads of its inputs, which pays where the
// whole launch is resident at once (its time is the slowest lane's latency); its
// registers there lower what the line kernel's lanes may hold, which costs more where
// they queue for the CUs, and there the network kernel runs at its own occupancy
// (measured at 76,800 and 624,000 line solves: 0.96x and 0.92x of the plain iteration
// in the fused launch, 0.92x and 0.99x as a kernel of its own).
bool use_fused(const ucac_handle* h) { return h->kp.warm_start != 2 || !front_queues(h); }

// One kernel of the iteration by index (the order of enqueue_iteration).
hipError_t launch_one(ucac_handle* h, int k, hipStream_t st, const char** where, const State* sv = nullptr) {
  static const char* names[] = {"units", "branch", "bus", "post", "finalize"};
  static void (*const fns[])(const Net&, const State&, const Par&, hipStream_t) = {
      launch_units, launch_branch, launch_bus, launch_post, launch_finalize};
  fns[k](h->net, sv ? *sv : h->st, h->kp, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess && where) *where = names[k];
  return e;
}

void clear_period_graph(ucac_handle* h) {
  if (h->x_period) (void)hipGraphExecDestroy(h->x_period);
  if (h->g_period) (void)hipGraphDestroy(h->g_period);
  h->x_period = nullptr;
  h->g_period = nullptr;
}

// The longest balancing period captured as one graph; longer periods are split.
constexpr int MAX_PERIOD_GRAPH = 256;

int build_graph(ucac_handle* h) {
  h->graphs.clear();
  h->graphs_solve.clear();
  clear_period_graph(h);
  const int K = h->kp.adapt_every;
  if (K > 1 && K <= MAX_PERIOD_GRAPH && use_fused(h)) {
    (void)hipGetLastError();
    HIP_OR(h, hipStreamBeginCapture(h->own, hipStreamCaptureModeThreadLocal));
    const char* where = "";
    hipError_t le = hipSuccess;
    for (int r = 0; r < K && le == hipSuccess; ++r) le = enqueue_fused_iteration(h, h->own, r, K, &where);
    const hipError_t ce = hipStreamEndCapture(h->own, &h->g_period);
    if (le != hipSuccess) return fail(h, UCAC_E_DEVICE, "launch of kernel %s failed: %s", where, hipGetErrorString(le));
    if (ce != hipSuccess) return fail(h, UCAC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ce));
    HIP_OR(h, hipGraphInstantiate(&h->x_period, h->g_period, nullptr, nullptr, 0));
  }
  for (int solve = 0; solve < 2; ++solve) {
    GraphSet& gs = solve ? h->graphs_solve : h->graphs;
    for (int j = 0; j < N_GRAPHS; ++j) {
      (void)hipGetLastError();
      HIP_OR(h, hipStreamBeginCapture(h->own, hipStreamCaptureModeThreadLocal));
      const char* where = "";
      hipError_t le = hipSuccess;
      const int size = GRAPH_SIZES[j];
      const bool fused = !solve && use_fused(h);
      for (int r = 0; r < size && le == hipSuccess; ++r)
        le = solve   ? enqueue_iteration(h, h->own, &where)
             : fused ? enqueue_fused_iteration(h, h->own, r, size, &where)
                     : enqueue_step_iteration(h, h->own, r, size, &where);
      const hipError_t ce = hipStreamEndCapture(h->own, &gs.g[j]);
      if (le != hipSuccess) return fail(h, UCAC_E_DEVICE, "launch of kernel %s failed: %s", where, hipGetErrorString(le));
      if (ce != hipSuccess) return fail(h, UCAC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ce));
      HIP_OR(h, hipGraphInstantiate(&gs.x[j], gs.g[j], nullptr, nullptr, 0));
    }
  }
  return UCAC_OK;
}

// With residual balancing, a control step that decides (after every adapt_every-th
// iteration) may change the penalties, which the next iteration's kernels read, so it
// cannot run beside them.  In the fused step graphs only a graph's last iteration has
// its control step after its own rows and before the next launch: the n iterations
// are split at every deciding iteration (read the iterate's counter first), so that
// each deciding iteration ends a graph.  The pipelined form runs its control step
// beside the next front launch in every iteration: there the solve-mode graphs (a
// control-step kernel after every iteration, here without stopping) are used instead.
hipError_t launch_balanced(ucac_handle* h, int n) {
  hipError_t e = hipMemcpyAsync(&h->h_sc[SC_ITER], h->st.sc + SC_ITER, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  const long K = h->kp.adapt_every;
  long it = (long)h->h_sc[SC_ITER];
  while (e == hipSuccess && n > 0) {
    const long to_decision = K - it % K;
    const int seg = (long)n < to_decision ? n : (int)to_decision;
    // a whole period: its own graph where captured
    e = seg == K && h->x_period ? hipGraphLaunch(h->x_period, h->stream) : h->graphs.launch(seg, h->stream);
    it += seg;
    n -= seg;
  }
  return e;
}

// Enqueue n iterations, largest graph first (solve mode: with a control-step kernel
// after every iteration).
hipError_t launch_iterations(ucac_handle* h, int n, bool solve = false) {
  if (solve) return h->graphs_solve.launch(n, h->stream);
  if (h->kp.adapt_every > 0) return use_fused(h) ? launch_balanced(h, n) : h->graphs_solve.launch(n, h->stream);
  return h->graphs.launch(n, h->stream);
}

// Write the host-owned control fields (never inside a captured graph).
int set_ctl(ucac_handle* h, int stop_at_tol, double tol) {
  std::memset(h->h_ctl, 0, sizeof(Ctl));
  h->h_ctl->stop_at_tol = stop_at_tol;
  h->h_ctl->tol = tol;
  const double ms[3] = {1e-2, 1e-3, 1e-4};
  for (int m = 0; m < 3; ++m) { h->h_ctl->ms_tol[m] = ms[m]; h->h_ctl->ms_iter[m] = -1; }
  h->h_ctl->conv_iter = -1;
  HIP_OR(h, hipMemcpyAsync(h->d_ctl, h->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
  return UCAC_OK;
}

int read_status(ucac_handle* h) {
  HIP_OR(h, hipMemcpyAsync(h->h_sc, h->st.sc, sizeof(double) * NSC, hipMemcpyDeviceToHost, h->stream));
  HIP_OR(h, hipMemcpyAsync(h->h_ctl, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  return UCAC_OK;
}

// A call that ended right after an inner loop leaves the step:outer multiplier
// update pending (the row owners apply it at the start of the next iteration):
// apply it to every row now, so that the state a caller reads is complete.
// Requires h_ctl to be current (read_status).
int flush_lambda(ucac_handle* h) {
  if (!h->h_ctl->pending) return UCAC_OK;
  (void)hipGetLastError();
  launch_lambda(h->net, h->st, h->kp, h->stream);
  HIP_OR(h, hipGetLastError());
  h->h_ctl->pending = 0;
  HIP_OR(h, hipMemcpyAsync(&h->d_ctl->pending, &h->h_ctl->pending, sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  return UCAC_OK;
}

}  // namespace

extern "C" {

void ucac_params_default(ucac_params* p) {
  if (!p) return;
  p->rho_pq = 5e3; p->rho_va = 1e4; p->rho_uc = 1e5; p->rho_cpl = 5e3;
  p->beta0 = 1e5; p->tau = 6.0; p->theta = 0.8; p->lambda_max = 1e12; p->beta_max = 1e24; p->mu_line = 5e3;
  p->newton_max_iter = 50; p->newton_gtol = 1e-12;
  p->max_inner = 1000; p->eps_in0 = 1e-2; p->tol = 1e-4;
  p->warm_start = 0; p->device = 0;
  p->adapt_every = 0; p->adapt_mu = 3.0; p->adapt_tau = 1.5; p->adapt_max = 20; p->adapt_span = 100.0;
}

int ucac_create(const ucac_network* net, const ucac_params* params, ucac_handle** out) {
  if (!out) return fail(nullptr, UCAC_E_INVAL, "null output handle");
  *out = nullptr;
  int rc = validate(net, params);
  if (rc != UCAC_OK) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, UCAC_E_DEVICE, "no HIP device");
  if (params->device < 0 || params->device >= ndev) return fail(nullptr, UCAC_E_INVAL, "device %d out of range", params->device);
  if (hipSetDevice(params->device) != hipSuccess) return fail(nullptr, UCAC_E_DEVICE, "hipSetDevice failed");

  ucac_handle* h = new ucac_handle();
  Permuted perm;
  make_order(net, h->perm_bus, h->perm_line, h->perm_gen);
  permute_network(net, h->perm_bus, h->perm_line, h->perm_gen, perm);
  net = &perm.view;
  h->N = net->n_bus; h->L = net->n_line; h->G = net->n_gen; h->T = net->T; h->ref = net->ref_bus;
  h->par = *params;
  if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, params->device) != hipSuccess || h->cus < 1)
    h->cus = 1;
  const size_t N = h->N, L = h->L, G = h->G, T = h->T;
  h->n_state = state_doubles(N, L, G, T);

  // host copies in device layout
  std::vector<int> from(net->line_from, net->line_from + L), to(net->line_to, net->line_to + L);
  std::vector<double> adm(8 * L), rate(net->line_rate, net->line_rate + L);
  for (size_t l = 0; l < L; ++l) {
    const double r = net->line_r[l], x = net->line_x[l], b = net->line_b[l];
    const double den = r * r + x * x, gs = r / den, bs = -x / den;
    adm[0 * L + l] = gs; adm[1 * L + l] = bs + 0.5 * b; adm[2 * L + l] = -gs; adm[3 * L + l] = -bs;
    adm[4 * L + l] = gs; adm[5 * L + l] = bs + 0.5 * b; adm[6 * L + l] = -gs; adm[7 * L + l] = -bs;
  }
  std::vector<int> inc_start(N + 1, 0), inc_code(2 * L), gen_start(N + 1, 0), gen_list(G);
  for (size_t l = 0; l < L; ++l) { inc_start[from[l] + 1]++; inc_start[to[l] + 1]++; }
  for (size_t i = 0; i < N; ++i) inc_start[i + 1] += inc_start[i];
  {
    std::vector<int> fill(N, 0);
    for (size_t l = 0; l < L; ++l) {
      inc_code[inc_start[from[l]] + fill[from[l]]++] = (int)(2 * l);
      inc_code[inc_start[to[l]] + fill[to[l]]++] = (int)(2 * l + 1);
    }
  }
  std::vector<int> end_pos(2 * L);
  for (size_t e = 0; e < 2 * L; ++e) end_pos[inc_code[e]] = (int)e;
  for (size_t g = 0; g < G; ++g) gen_start[net->gen_bus[g] + 1]++;
  for (size_t i = 0; i < N; ++i) gen_start[i + 1] += gen_start[i];
  {
    std::vector<int> fill(N, 0);
    for (size_t g = 0; g < G; ++g) gen_list[gen_start[net->gen_bus[g]] + fill[net->gen_bus[g]]++] = (int)g;
  }
  std::vector<int> unit_first(N, 0);
  for (size_t i = 0; i < N; ++i)
    if (gen_start[i + 1] > gen_start[i]) unit_first[i] = gen_list[gen_start[i]];
  const double base = net->base_mva;
  h->hg.k2.resize(G); h->hg.k1.resize(G);
  for (size_t g = 0; g < G; ++g) { h->hg.k2[g] = net->gen_c2[g] * base * base; h->hg.k1[g] = net->gen_c1[g] * base; }
  h->hg.cnl.assign(net->gen_cnl, net->gen_cnl + G);
  h->hg.csu.assign(net->gen_csu, net->gen_csu + G);
  h->hg.csd.assign(net->gen_csd, net->gen_csd + G);
  h->hg.u0.assign(net->gen_u0, net->gen_u0 + G);
  h->hg.pmin.assign(net->gen_pmin, net->gen_pmin + G); h->hg.pmax.assign(net->gen_pmax, net->gen_pmax + G);
  h->hg.qmin.assign(net->gen_qmin, net->gen_qmin + G); h->hg.qmax.assign(net->gen_qmax, net->gen_qmax + G);
  h->hg.ru.assign(net->gen_ru, net->gen_ru + G); h->hg.rd.assign(net->gen_rd, net->gen_rd + G);
  h->hg.su.assign(net->gen_su, net->gen_su + G); h->hg.sd.assign(net->gen_sd, net->gen_sd + G);
  h->hg.p0.assign(net->gen_p0, net->gen_p0 + G);
  std::vector<double> S;
  cold_start(net, adm, *params, S);
  h->cold = S;

  h->arena_bytes = carve(h, nullptr);
  if (hipMalloc(&h->arena, h->arena_bytes) != hipSuccess) {
    const size_t bytes = h->arena_bytes;
    delete h;
    return fail(nullptr, UCAC_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  carve(h, (char*)h->arena);
  auto cleanup = [&](int code) {
    g_create_error = h->err;
    ucac_destroy(h);
    return code;
  };
  if (hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) != hipSuccess) return cleanup(fail(h, UCAC_E_DEVICE, "stream create failed"));
  h->stream = h->own;
  if (hipHostMalloc((void**)&h->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&h->h_sc, sizeof(double) * NSC, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(h, UCAC_E_NOMEM, "pinned host allocation failed"));
  bool ev_ok = hipEventCreateWithFlags(&h->ev_poll, hipEventDisableTiming) == hipSuccess;
  if (!ev_ok) return cleanup(fail(h, UCAC_E_DEVICE, "event create failed"));

  const Net& n = h->net;
  struct Up { void* dst; const void* src; size_t bytes; } ups[] = {
      {(void*)n.from, from.data(), sizeof(int) * L}, {(void*)n.to, to.data(), sizeof(int) * L},
      {(void*)n.adm, adm.data(), sizeof(double) * 8 * L}, {(void*)n.rate, rate.data(), sizeof(double) * L},
      {(void*)n.gs, net->bus_gs, sizeof(double) * N}, {(void*)n.bs, net->bus_bs, sizeof(double) * N},
      {(void*)n.vmin, net->bus_vmin, sizeof(double) * N}, {(void*)n.vmax, net->bus_vmax, sizeof(double) * N},
      {(void*)n.Pd, net->load_p, sizeof(double) * T * N}, {(void*)n.Qd, net->load_q, sizeof(double) * T * N},
      {(void*)n.inc_start, inc_start.data(), sizeof(int) * (N + 1)}, {(void*)n.inc_code, inc_code.data(), sizeof(int) * 2 * L},
      {(void*)n.end_pos, end_pos.data(), sizeof(int) * 2 * L},
      {(void*)n.gen_start, gen_start.data(), sizeof(int) * (N + 1)}, {(void*)n.gen_list, gen_list.data(), sizeof(int) * G},
      {(void*)n.unit_first, unit_first.data(), sizeof(int) * N},
      {(void*)n.pmin, net->gen_pmin, sizeof(double) * G}, {(void*)n.pmax, net->gen_pmax, sizeof(double) * G},
      {(void*)n.qmin, net->gen_qmin, sizeof(double) * G}, {(void*)n.qmax, net->gen_qmax, sizeof(double) * G},
      {(void*)n.k2, h->hg.k2.data(), sizeof(double) * G}, {(void*)n.k1, h->hg.k1.data(), sizeof(double) * G},
      {(void*)n.cnl, net->gen_cnl, sizeof(double) * G}, {(void*)n.csu, net->gen_csu, sizeof(double) * G},
      {(void*)n.csd, net->gen_csd, sizeof(double) * G}, {(void*)n.ru, net->gen_ru, sizeof(double) * G},
      {(void*)n.rd, net->gen_rd, sizeof(double) * G}, {(void*)n.su, net->gen_su, sizeof(double) * G},
      {(void*)n.sd, net->gen_sd, sizeof(double) * G}, {(void*)n.p0, net->gen_p0, sizeof(double) * G},
      {(void*)n.tu, net->gen_min_up, sizeof(int) * G}, {(void*)n.td, net->gen_min_dn, sizeof(int) * G},
      {(void*)n.u0, net->gen_u0, sizeof(int) * G}, {(void*)n.lon, net->gen_init_on, sizeof(int) * G},
      {(void*)n.loff, net->gen_init_off, sizeof(int) * G},
      {(void*)h->d_state, S.data(), sizeof(double) * h->n_state}};
  for (const Up& u : ups) {
    if (u.bytes == 0) continue;
    if (hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice) != hipSuccess) return cleanup(fail(h, UCAC_E_DEVICE, "upload failed"));
  }
  if (hipMemset(h->st.ub_nxt, 0, sizeof(double) * 3 * T * G) != hipSuccess ||
      hipMemset(h->st.br_iters, 0, sizeof(int) * T * L) != hipSuccess ||
      hipMemset(h->st.br_count, 0, sizeof(unsigned long long) * NBRC * branch_waves(h)) != hipSuccess ||
      hipMemset(h->st.red, 0, sizeof(double) * NACC * h->st.red_total) != hipSuccess ||
      hipMemset(h->st.redc, 0, sizeof(double) * NCS * h->st.red_total) != hipSuccess)
    return cleanup(fail(h, UCAC_E_DEVICE, "memset failed"));
  h->kp = kernel_params(*params);
  if (set_ctl(h, 0, params->tol) != UCAC_OK) return cleanup(UCAC_E_DEVICE);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return cleanup(fail(h, UCAC_E_DEVICE, "sync failed"));
  if (build_graph(h) != UCAC_OK) return cleanup(UCAC_E_DEVICE);
  *out = h;
  return UCAC_OK;
}

int ucac_set_stream(ucac_handle* h, void* hip_stream) {
  if (!h) return UCAC_E_INVAL;
  HIP_OR(h, hipStreamSynchronize(h->stream));
  h->stream = hip_stream ? (hipStream_t)hip_stream : h->own;
  return UCAC_OK;
}

static int check_bad(ucac_handle* h) {
  if (h->h_ctl->bad) return fail(h, UCAC_E_NUMERIC, "non-finite residual in the iterate");
  return UCAC_OK;
}

int ucac_step(ucac_handle* h, int32_t n_iters) {
  if (!h) return UCAC_E_INVAL;
  if (n_iters < 0) return fail(h, UCAC_E_INVAL, "negative iteration count");
  HIP_OR(h, hipSetDevice(h->par.device));
  int rc = set_ctl(h, 0, h->par.tol);
  if (rc) return rc;
  HIP_OR(h, launch_iterations(h, n_iters));
  rc = read_status(h);
  if (rc) return rc;
  rc = flush_lambda(h);
  if (rc) return rc;
  return check_bad(h);
}

int ucac_solve(ucac_handle* h, double tol, int32_t max_iters, int32_t* iters_done) {
  if (!h) return UCAC_E_INVAL;
  if (!(tol > 0.0) || max_iters < 0) return fail(h, UCAC_E_INVAL, "bad tol or max_iters");
  HIP_OR(h, hipSetDevice(h->par.device));
  h->par.tol = tol;
  int rc = read_status(h);
  if (rc) return rc;
  const double it0 = h->h_sc[SC_ITER];
  // clear the converged flag of a previous solve
  h->h_sc[SC_CONV] = 0.0;
  HIP_OR(h, hipMemcpyAsync(h->st.sc + SC_CONV, h->h_sc + SC_CONV, sizeof(double), hipMemcpyHostToDevice, h->stream));
  // The chunks run in step mode (each control step inside the next launch), which
  // cannot stop an instance; the control step records the first iteration at the
  // tolerance instead.  When a chunk reaches it, the chunk is replayed from its
  // snapshot up to the iteration before, and that iteration runs in solve mode, whose
  // control step stops the instance there: the same iterations and state as solve
  // mode throughout (the two forms compute the same iteration bit for bit).
  rc = set_ctl(h, 0, tol);
  if (rc) return rc;
  const size_t state_bytes = sizeof(double) * h->n_state;
  const size_t count_bytes = sizeof(unsigned long long) * NBRC * branch_waves(h);
  if (!h->solve_save && hipMalloc(&h->solve_save, state_bytes + sizeof(Ctl) + count_bytes) != hipSuccess) {
    h->solve_save = nullptr;
    return fail(h, UCAC_E_NOMEM, "solve snapshot allocation failed");
  }
  char* save = (char*)h->solve_save;
  auto snapshot = [&](bool restore) -> hipError_t {
    void* s0 = save;
    void* s1 = save + state_bytes;
    void* s2 = save + state_bytes + sizeof(Ctl);
    hipError_t e = hipMemcpyAsync(restore ? (void*)h->d_state : s0, restore ? s0 : (void*)h->d_state, state_bytes,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(restore ? (void*)h->d_ctl : s1, restore ? s1 : (void*)h->d_ctl, sizeof(Ctl),
                         hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && count_bytes)
      e = hipMemcpyAsync(restore ? (void*)h->st.br_count : s2, restore ? s2 : (void*)h->st.br_count, count_bytes,
                         hipMemcpyDeviceToDevice, h->stream);
    return e;
  };
  int launched = 0;
  bool done = false;
  while (!done && launched < max_iters) {
    const int k = (max_iters - launched) < SOLVE_CHUNK ? (max_iters - launched) : SOLVE_CHUNK;
    HIP_OR(h, snapshot(false));
    HIP_OR(h, launch_iterations(h, k));
    rc = read_status(h);
    if (rc) return rc;
    // the tolerance before the non-finite flag (ucac_solve_rule.hpp)
    const int conv_iter = h->h_ctl->conv_iter;
    const ChunkAction act = chunk_action(conv_iter, h->h_ctl->bad, launched);
    if (act.next == CHUNK_REPLAY) {
      HIP_OR(h, snapshot(true));
      HIP_OR(h, launch_iterations(h, act.replay));
      h->h_ctl->stop_at_tol = 1;  // pinned staging
      HIP_OR(h, hipMemcpyAsync(&h->d_ctl->stop_at_tol, &h->h_ctl->stop_at_tol, sizeof(int), hipMemcpyHostToDevice,
                               h->stream));
      HIP_OR(h, launch_iterations(h, 1, true));
      rc = read_status(h);
      if (rc) return rc;
      // the replay computes the chunk's iterations again bit for bit, so its stopping
      // iteration must stop the instance at the recorded iteration
      if (h->h_sc[SC_CONV] == 0.0 || h->h_ctl->conv_iter != conv_iter)
        return fail(h, UCAC_E_DEVICE, "solve replay diverged: the tolerance was recorded at iteration %d of the solve, "
                    "the replay stopped at %d (converged flag %g)", conv_iter, h->h_ctl->conv_iter, h->h_sc[SC_CONV]);
      done = true;
      break;
    }
    if (act.next == CHUNK_NONFINITE) break;
    launched += k;
  }
  rc = read_status(h);
  if (rc) return rc;
  rc = flush_lambda(h);
  if (rc) return rc;
  if (iters_done) *iters_done = (int32_t)(h->h_sc[SC_ITER] - it0);
  rc = check_bad(h);
  if (rc) return rc;
  return h->h_sc[SC_CONV] != 0.0 ? UCAC_OK : UCAC_NOT_CONVERGED;
}

int ucac_uc_warmstart(ucac_handle* h, double tol, int32_t max_iters, int32_t* iters_done) {
  if (!h) return UCAC_E_INVAL;
  if (!(tol > 0.0) || max_iters < 0) return fail(h, UCAC_E_INVAL, "bad tol or max_iters");
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  const Par kp_saved = h->kp;
  const ucac_params par_saved = h->par;
  // the multiperiod ACOPF, from the cold start
  h->kp.relax_uc = 1;
  int rc = build_graph(h);
  if (rc) { h->kp = kp_saved; return rc; }
  HIP_OR(h, hipMemcpy(h->d_state, h->cold.data(), sizeof(double) * h->n_state, hipMemcpyHostToDevice));
  int32_t it = 0;
  const int src = ucac_solve(h, tol, max_iters, &it);
  h->kp = kp_saved;
  h->par = par_saved;
  rc = build_graph(h);
  if (src < 0) return src;
  if (rc) return rc;
  // commitments from the generation levels: on where p >= P_lo / 2
  const size_t TG = (size_t)h->T * h->G, TL = (size_t)h->T * h->L;
  std::vector<double> p(TG);
  if (TG) HIP_OR(h, hipMemcpy(p.data(), h->d_state + 10 * TL, sizeof(double) * TG, hipMemcpyDeviceToHost));
  std::vector<signed char> u(TG);
  for (size_t k = 0; k < TG; ++k) u[k] = p[k] >= 0.5 * h->hg.pmin[k % h->G] ? 1 : 0;
  std::vector<double> S = h->cold;
  set_commitments(h->hg, h->N, h->L, h->G, h->T, S, u);
  HIP_OR(h, hipMemcpy(h->d_state, S.data(), sizeof(double) * h->n_state, hipMemcpyHostToDevice));
  rc = set_ctl(h, 0, h->par.tol);
  if (rc) return rc;
  if (iters_done) *iters_done = it;
  return src;
}

int ucac_residuals(const ucac_handle* hc, double* r_primal, double* r_dual, double* z_inf, double* objective) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h) return UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  int rc = read_status(h);
  if (rc) return rc;
  if (r_primal) *r_primal = h->h_sc[SC_RP];
  if (r_dual) *r_dual = h->h_sc[SC_RD];
  if (z_inf) *z_inf = h->h_sc[SC_ZINF];
  if (objective) {
    const size_t TG = (size_t)h->T * h->G;
    std::vector<double> buf(4 * TG);
    if (TG) {
      HIP_OR(h, hipMemcpy(buf.data(), h->st.p, sizeof(double) * TG, hipMemcpyDeviceToHost));
      HIP_OR(h, hipMemcpy(buf.data() + TG, h->st.uon, sizeof(double) * 3 * TG, hipMemcpyDeviceToHost));
    }
    double obj = 0.0;
    for (int t = 0; t < h->T; ++t)
      for (int g = 0; g < h->G; ++g) {
        const size_t k = (size_t)t * h->G + g;
        const double p = buf[k];
        obj += h->hg.k2[g] * p * p + h->hg.k1[g] * p;
        obj += h->hg.cnl[g] * buf[TG + k] + h->hg.csu[g] * buf[2 * TG + k] + h->hg.csd[g] * buf[3 * TG + k];
      }
    *objective = obj;
  }
  return UCAC_OK;
}

int ucac_get_solution(const ucac_handle* hc, double* p, double* q, int8_t* u_on, int8_t* u_su, int8_t* u_sd, double* vm,
                      double* va) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h) return UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  const size_t T = h->T, TG = T * h->G, TN = T * h->N;
  std::vector<double> tmp(TG > TN ? TG : TN), out(TG > TN ? TG : TN);
  double* dd[2] = {p, q};
  double* ds[2] = {h->st.p, h->st.q};
  for (int k = 0; k < 2; ++k) {
    if (!dd[k] || !TG) continue;
    HIP_OR(h, hipMemcpy(tmp.data(), ds[k], sizeof(double) * TG, hipMemcpyDeviceToHost));
    unpermute_rows(h->perm_gen, T, tmp.data(), dd[k]);
  }
  double* uu[3] = {h->st.uon, h->st.usu, h->st.usd};
  int8_t* uo[3] = {u_on, u_su, u_sd};
  for (int k = 0; k < 3; ++k) {
    if (!uo[k] || !TG) continue;
    HIP_OR(h, hipMemcpy(tmp.data(), uu[k], sizeof(double) * TG, hipMemcpyDeviceToHost));
    unpermute_rows(h->perm_gen, T, tmp.data(), out.data());
    for (size_t i = 0; i < TG; ++i) uo[k][i] = out[i] != 0.0 ? 1 : 0;
  }
  if (vm) {
    HIP_OR(h, hipMemcpy(tmp.data(), h->st.wb, sizeof(double) * TN, hipMemcpyDeviceToHost));
    unpermute_rows(h->perm_bus, T, tmp.data(), out.data());
    for (size_t i = 0; i < TN; ++i) vm[i] = std::sqrt(std::fmax(out[i], 0.0));
  }
  if (va) {
    HIP_OR(h, hipMemcpy(tmp.data(), h->st.thb, sizeof(double) * TN, hipMemcpyDeviceToHost));
    unpermute_rows(h->perm_bus, T, tmp.data(), va);
  }
  return UCAC_OK;
}

int ucac_get_state(const ucac_handle* hc, void* buf, size_t* bytes) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h || !bytes) return UCAC_E_INVAL;
  const size_t need = sizeof(double) * h->n_state;
  if (!buf) { *bytes = need; return UCAC_OK; }
  if (*bytes < need) return fail(h, UCAC_E_STATE, "state buffer holds %zu bytes, %zu needed", *bytes, need);
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  std::vector<double> tmp(h->n_state);
  HIP_OR(h, hipMemcpy(tmp.data(), h->d_state, need, hipMemcpyDeviceToHost));
  convert_state(h, tmp.data(), (double*)buf, false);
  *bytes = need;
  return UCAC_OK;
}

int ucac_set_state(ucac_handle* h, const void* buf, size_t bytes) {
  if (!h || !buf) return UCAC_E_INVAL;
  const size_t need = sizeof(double) * h->n_state;
  if (bytes != need) return fail(h, UCAC_E_STATE, "state of %zu bytes given, %zu expected", bytes, need);
  const double* d = (const double*)buf;
  // every entry finite except ||z^{k-1}||, which is +inf before the first outer update
  for (size_t i = 0; i < h->n_state; ++i)
    if (!std::isfinite(d[i]) && !(i == h->n_state - NSC + SC_ZPREV && d[i] == INFINITY))
      return fail(h, UCAC_E_STATE, "state entry %zu is not finite", i);
  // the penalties in force must be positive (every row divides by its penalty)
  for (int k = SC_RHO_PQ; k <= SC_RHO_UC; ++k)
    if (!(d[h->n_state - NSC + k] > 0.0)) return fail(h, UCAC_E_STATE, "state penalty scalar %d is not positive", k);
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  std::vector<double> tmp(h->n_state);
  convert_state(h, d, tmp.data(), true);
  HIP_OR(h, hipMemcpy(h->d_state, tmp.data(), need, hipMemcpyHostToDevice));
  return set_ctl(h, 0, h->par.tol);
}

int ucac_get_branch_iters(const ucac_handle* hc, int32_t* iters) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h || !iters) return UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  const size_t TL = (size_t)h->T * h->L;
  std::vector<int32_t> tmp(TL);
  if (TL) HIP_OR(h, hipMemcpy(tmp.data(), h->st.br_iters, sizeof(int) * TL, hipMemcpyDeviceToHost));
  unpermute_rows(h->perm_line, (size_t)h->T, tmp.data(), iters);
  return UCAC_OK;
}

int ucac_get_line_starts(const ucac_handle* hc, float* x0) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h || !x0) return h ? fail(h, UCAC_E_INVAL, "null output") : UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  const size_t TL = (size_t)h->T * h->L;
  std::vector<float> tmp(TL);
  for (int k = 0; k < 4; ++k) {
    if (TL) HIP_OR(h, hipMemcpy(tmp.data(), h->st.x0 + k * TL, sizeof(float) * TL, hipMemcpyDeviceToHost));
    unpermute_rows(h->perm_line, (size_t)h->T, tmp.data(), x0 + k * TL);
  }
  return UCAC_OK;
}

// Kernel k of the kernel-by-kernel iteration launched with its own start and stop
// events; false where it has no work (nothing launched).
static bool launch_timed(ucac_handle* h, int k, hipEvent_t e0, hipEvent_t e1) {
  static bool (*const fns[])(const Net&, const State&, const Par&, hipStream_t, hipEvent_t, hipEvent_t) = {
      launch_units_timed, launch_branch_timed, launch_bus_timed, launch_post_timed, launch_finalize_timed};
  return fns[k](h->net, h->st, h->kp, h->stream, e0, e1);
}

int ucac_kernel_times(ucac_handle* h, int32_t n_iters, double* avg_ms, int32_t n_slots) {
  if (!h || !avg_ms || n_iters < 1 || n_slots < UCAC_N_KERNELS) return h ? fail(h, UCAC_E_INVAL, "bad arguments") : UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  int rc = set_ctl(h, 0, h->par.tol);
  if (rc) return rc;
  const int K = UCAC_N_KERNELS;
  // kernels 0 .. nd-1 also carry their own dispatch events (slots K + k)
  const int nd = n_slots - K < K ? n_slots - K : K;
  // K + 1 markers per iteration, then a pair per dispatch-timed kernel
  const int E = K + 1 + 2 * nd;
  std::vector<hipEvent_t> ev((size_t)n_iters * E, nullptr);
  for (auto& e : ev) HIP_OR(h, hipEventCreate(&e));
  hipError_t err = hipSuccess;
  const char* where = "";
  static const char* names[] = {"units", "branch", "bus", "post", "finalize"};
  bool launched[UCAC_N_KERNELS] = {};
  for (int it = 0; it < n_iters && err == hipSuccess; ++it) {
    hipEvent_t* e = &ev[(size_t)it * E];
    err = hipEventRecord(e[0], h->stream);
    for (int k = 0; k < K && err == hipSuccess; ++k) {
      if (k < nd) {
        launched[k] = launch_timed(h, k, e[K + 1 + 2 * k], e[K + 2 + 2 * k]);
        err = hipGetLastError();
        if (err != hipSuccess) where = names[k];
      } else {
        err = launch_one(h, k, h->stream, &where);
      }
      if (err == hipSuccess) err = hipEventRecord(e[k + 1], h->stream);
    }
  }
  if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
  for (int k = 0; k < n_slots && k < K + nd; ++k) avg_ms[k] = 0.0;
  for (int it = 0; it < n_iters && err == hipSuccess; ++it) {
    const hipEvent_t* e = &ev[(size_t)it * E];
    for (int k = 0; k < K && err == hipSuccess; ++k) {
      float ms = 0.0f;
      err = hipEventElapsedTime(&ms, e[k], e[k + 1]);
      avg_ms[k] += ms / n_iters;
    }
    // a kernel without work launches nothing and leaves its pair unrecorded
    for (int k = 0; k < nd && err == hipSuccess; ++k) {
      if (!launched[k]) continue;
      float ms = 0.0f;
      err = hipEventElapsedTime(&ms, e[K + 1 + 2 * k], e[K + 2 + 2 * k]);
      avg_ms[K + k] += ms / n_iters;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(h, UCAC_E_DEVICE, "timed iteration failed at %s: %s", where, hipGetErrorString(err));
  rc = read_status(h);
  if (rc) return rc;
  rc = flush_lambda(h);
  if (rc) return rc;
  return check_bad(h);
}

int ucac_branch_counters(ucac_handle* h, uint64_t* out, int32_t reset) {
  if (!h || !out) return h ? fail(h, UCAC_E_INVAL, "null output") : UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  const size_t nw = branch_waves(h);
  std::vector<uint64_t> part(nw * NBRC);
  if (nw) HIP_OR(h, hipMemcpy(part.data(), h->st.br_count, sizeof(uint64_t) * NBRC * nw, hipMemcpyDeviceToHost));
  for (int k = 0; k < NBRC; ++k) out[k] = 0;
  for (size_t w = 0; w < nw; ++w)
    for (int k = 0; k < NBRC; ++k) out[k] += part[w * NBRC + k];
  if (reset && nw) HIP_OR(h, hipMemset(h->st.br_count, 0, sizeof(uint64_t) * NBRC * nw));
  return UCAC_OK;
}

int ucac_solve_milestones(const ucac_handle* hc, int32_t* first_iter) {
  ucac_handle* h = const_cast<ucac_handle*>(hc);
  if (!h || !first_iter) return h ? fail(h, UCAC_E_INVAL, "null output") : UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  int rc = read_status(h);
  if (rc) return rc;
  for (int m = 0; m < 3; ++m) first_iter[m] = h->h_ctl->ms_iter[m];
  return UCAC_OK;
}

// ---- learned warm start ---------------------------------------------------------

namespace {
struct MlpBufs {
  float* P;
  __bf16 *W1b, *W2b, *W3b;
};
size_t mlp_bytes() { return sizeof(float) * MLP_PARAMS + sizeof(__bf16) * (64 * 32 + 64 * 64 + 32 * 64) + 1024; }
MlpBufs mlp_carve(void* base) {
  char* c = (char*)base;
  MlpBufs b;
  b.P = (float*)c; c += ((sizeof(float) * MLP_PARAMS + 255) / 256) * 256;
  b.W1b = (__bf16*)c; c += sizeof(__bf16) * 64 * 32;
  b.W2b = (__bf16*)c; c += sizeof(__bf16) * 64 * 64;
  b.W3b = (__bf16*)c;
  return b;
}
MlpView mlp_view(const MlpBufs& b) {
  MlpView v;
  v.W1b = b.W1b; v.W2b = b.W2b; v.W3b = b.W3b;
  v.b1 = b.P + 64 * 20; v.b2 = b.P + 64 * 20 + 64 + 64 * 64; v.b3 = b.P + 64 * 20 + 64 + 64 * 64 + 64 + 4 * 64;
  return v;
}
}  // namespace

int ucac_set_params(ucac_handle* h, const ucac_params* params) {
  if (!h || !params) return h ? fail(h, UCAC_E_INVAL, "null params") : UCAC_E_INVAL;
  if (params->device != h->par.device) return fail(h, UCAC_E_INVAL, "params.device cannot change");
  if (!(params->rho_pq > 0.0) || !(params->rho_va > 0.0) || !(params->rho_uc > 0.0) || !(params->rho_cpl > 0.0) ||
      !(params->beta0 > 0.0) || !(params->tau > 0.0) || !(params->lambda_max > 0.0) || !(params->beta_max > 0.0) ||
      !(params->mu_line > 0.0) || !(params->theta > 0.0) || !(params->newton_gtol >= 0.0) || !(params->eps_in0 >= 0.0) ||
      !(params->tol > 0.0) || params->newton_max_iter < 0 || params->max_inner < 1 || params->warm_start < 0 ||
      params->warm_start > 1 || !std::isfinite(params->rho_pq) || !std::isfinite(params->rho_va) ||
      !std::isfinite(params->rho_uc) || !std::isfinite(params->rho_cpl) || !std::isfinite(params->mu_line) ||
      !adapt_params_ok(params))
    return fail(h, UCAC_E_INVAL, "invalid params");
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  // the penalties in force become the new ones; their residual-balancing counts restart
  const double rho_now[8] = {params->rho_pq, params->rho_va, params->rho_cpl, params->rho_uc, 0.0, 0.0, 0.0, 0.0};
  HIP_OR(h, hipMemcpy(h->st.sc + SC_RHO_PQ, rho_now, sizeof(rho_now), hipMemcpyHostToDevice));
  const bool learned = h->kp.warm_start == 2;
  const MlpView mlp = h->kp.mlp;
  h->par = *params;
  h->kp = kernel_params(*params);
  if (learned) { h->kp.warm_start = 2; h->kp.mlp = mlp; }
  return build_graph(h);
}

int ucac_set_warmstart(ucac_handle* h, const float* weights, size_t n) {
  if (!h) return UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  HIP_OR(h, hipStreamSynchronize(h->stream));
  if (!weights) {
    h->kp.warm_start = h->par.warm_start;
    return build_graph(h);
  }
  if (n != (size_t)MLP_PARAMS) return fail(h, UCAC_E_INVAL, "expected %d weights, got %zu", MLP_PARAMS, n);
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(weights[i])) return fail(h, UCAC_E_INVAL, "weight %zu is not finite", i);
  if (!h->mlp_mem) {
    HIP_OR(h, hipMalloc(&h->mlp_mem, mlp_bytes()));
    HIP_OR(h, hipMemset(h->mlp_mem, 0, mlp_bytes()));
  }
  const MlpBufs b = mlp_carve(h->mlp_mem);
  HIP_OR(h, hipMemcpy(b.P, weights, sizeof(float) * n, hipMemcpyHostToDevice));
  mlp_launch_pack(b.P, b.W1b, b.W2b, b.W3b, h->stream);
  HIP_OR(h, hipGetLastError());
  HIP_OR(h, hipStreamSynchronize(h->stream));
  h->kp.mlp = mlp_view(b);
  h->kp.warm_start = 2;
  return build_graph(h);
}

int ucac_log_pairs(ucac_handle* h, int32_t n_iters, int32_t stride, float* feats, float* targets, int64_t cap,
                   int64_t* n_logged) {
  if (!h || !feats || !targets || n_iters < 0 || stride < 1 || cap < 0 || cap > 0x7fffffff)
    return h ? fail(h, UCAC_E_INVAL, "bad arguments") : UCAC_E_INVAL;
  HIP_OR(h, hipSetDevice(h->par.device));
  int rc = set_ctl(h, 0, h->par.tol);
  if (rc) return rc;
  float* d = nullptr;
  int* cnt = nullptr;
  const size_t c = (size_t)(cap > 0 ? cap : 1);
  HIP_OR(h, hipMalloc(&d, sizeof(float) * c * 24));
  if (hipMalloc(&cnt, sizeof(int)) != hipSuccess) { (void)hipFree(d); return fail(h, UCAC_E_NOMEM, "log counter"); }
  hipError_t err = hipMemsetAsync(cnt, 0, sizeof(int), h->stream);
  State sv = h->st;
  sv.log_feat = d;
  sv.log_targ = d + c * 20;
  sv.log_count = cnt;
  sv.log_cap = (int)cap;
  sv.log_stride = stride;
  const char* where = "";
  for (int it = 0; it < n_iters && err == hipSuccess; ++it) {
    sv.log_phase = it % stride;
    for (int k = 0; k < UCAC_N_KERNELS && err == hipSuccess; ++k) err = launch_one(h, k, h->stream, &where, &sv);
  }
  int got = 0;
  if (err == hipSuccess) err = hipMemcpyAsync(&got, cnt, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
  const int64_t m = got < cap ? got : cap;
  if (err == hipSuccess && m > 0) err = hipMemcpy(feats, d, sizeof(float) * m * 20, hipMemcpyDeviceToHost);
  if (err == hipSuccess && m > 0) err = hipMemcpy(targets, d + c * 20, sizeof(float) * m * 4, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  (void)hipFree(cnt);
  if (err != hipSuccess) return fail(h, UCAC_E_DEVICE, "logging failed at %s: %s", where, hipGetErrorString(err));
  if (n_logged) *n_logged = m;
  rc = read_status(h);
  if (rc) return rc;
  rc = flush_lambda(h);
  if (rc) return rc;
  return check_bad(h);
}

// ---- the warm-start network on its own (training, inference, gradients) ---------

struct ucac_mlp {
  int device = 0;
  hipStream_t st = nullptr;
  void* mem = nullptr;  // P, BF16 copies
  float *m1 = nullptr, *m2 = nullptr;
  int step = 0;
  std::string err;
};

namespace {
int mfail(ucac_mlp* m, int code, const char* what, hipError_t e) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  if (m) m->err = buf; else g_create_error = buf;
  return code;
}
#define MLP_OR(m, call)                                                  \
  do {                                                                   \
    hipError_t _e = (call);                                              \
    if (_e != hipSuccess) return mfail(m, UCAC_E_DEVICE, #call, _e);     \
  } while (0)

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// device scratch of one call: inputs, targets, indices, gradient slots, gradient, loss
struct MlpCall {
  float *X = nullptr, *Y = nullptr, *slots = nullptr, *grad = nullptr;
  int* idx = nullptr;
  double* loss = nullptr;
  ~MlpCall() {
    for (void* p : {(void*)X, (void*)Y, (void*)slots, (void*)grad, (void*)idx, (void*)loss})
      if (p) (void)hipFree(p);
  }
};
}  // namespace

// ---- scratch of ucac_mlp_grad_noalloc ----------------------------------------------
// One fixed array per GPU (each device holds its own copy until the process ends):
// the sample indices of a call, then one gradient slot per wavefront of 64 samples.
// Host code never uses the array's name as an address: the device address of each
// GPU's copy is looked up once per device (hipGetSymbolAddress, with that device
// current) when the first network is created on it, and kept in g_scratch_ptr.
constexpr size_t NOALLOC_IDX_BYTES = sizeof(int) * UCAC_MLP_NOALLOC_MAX;
constexpr size_t NOALLOC_SLOT_OFF = (NOALLOC_IDX_BYTES + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_SLOT_OFF + sizeof(float) * (UCAC_MLP_NOALLOC_MAX / 64) * MLP_SLOT;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
bool g_scratch_done[MAX_DEVICES] = {};

// Once per device, with that device current: the address of its copy of the array.
void scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
  g_scratch_done[device] = true;
}

__global__ void k_iota(int* idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = i;
}
}  // namespace

int ucac_mlp_create(int32_t device, uint64_t seed, ucac_mlp** out) {
  if (!out) return UCAC_E_INVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, UCAC_E_DEVICE, "hipSetDevice failed");
  ucac_mlp* m = new ucac_mlp();
  m->device = device;
  std::vector<float> P(MLP_PARAMS, 0.0f);
  uint64_t s = seed;
  auto uni = [&](float bound) { return (float)((double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0) * bound; };
  for (int i = 0; i < 64 * 20; ++i) P[i] = uni(1.0f / std::sqrt(20.0f));
  for (int i = 0; i < 64 * 64; ++i) P[64 * 20 + 64 + i] = uni(1.0f / 8.0f);
  for (int i = 0; i < 4 * 64; ++i) P[64 * 20 + 64 + 64 * 64 + 64 + i] = uni(1.0f / 8.0f);
  auto bad = [&](hipError_t e, const char* what) { int rc = mfail(m, UCAC_E_DEVICE, what, e); g_create_error = m->err; ucac_mlp_destroy(m); return rc; };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking)) != hipSuccess) return bad(e, "stream");
  if ((e = hipMalloc(&m->mem, mlp_bytes())) != hipSuccess) return bad(e, "hipMalloc");
  if ((e = hipMemset(m->mem, 0, mlp_bytes())) != hipSuccess) return bad(e, "memset");
  if ((e = hipMalloc(&m->m1, sizeof(float) * MLP_PARAMS)) != hipSuccess) return bad(e, "hipMalloc");
  if ((e = hipMalloc(&m->m2, sizeof(float) * MLP_PARAMS)) != hipSuccess) return bad(e, "hipMalloc");
  if ((e = hipMemset(m->m1, 0, sizeof(float) * MLP_PARAMS)) != hipSuccess) return bad(e, "memset");
  if ((e = hipMemset(m->m2, 0, sizeof(float) * MLP_PARAMS)) != hipSuccess) return bad(e, "memset");
  scratch_setup(device);  // this device current (set above)
  const MlpBufs b = mlp_carve(m->mem);
  if ((e = hipMemcpy(b.P, P.data(), sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice)) != hipSuccess) return bad(e, "upload");
  mlp_launch_pack(b.P, b.W1b, b.W2b, b.W3b, m->st);
  if ((e = hipStreamSynchronize(m->st)) != hipSuccess) return bad(e, "pack");
  *out = m;
  return UCAC_OK;
}

int ucac_mlp_set_weights(ucac_mlp* m, const float* w, size_t n) {
  if (!m || !w || n != (size_t)MLP_PARAMS) return m ? (m->err = "bad weights", UCAC_E_INVAL) : UCAC_E_INVAL;
  MLP_OR(m, hipSetDevice(m->device));
  const MlpBufs b = mlp_carve(m->mem);
  MLP_OR(m, hipMemcpy(b.P, w, sizeof(float) * n, hipMemcpyHostToDevice));
  mlp_launch_pack(b.P, b.W1b, b.W2b, b.W3b, m->st);
  MLP_OR(m, hipStreamSynchronize(m->st));
  MLP_OR(m, hipMemset(m->m1, 0, sizeof(float) * MLP_PARAMS));
  MLP_OR(m, hipMemset(m->m2, 0, sizeof(float) * MLP_PARAMS));
  m->step = 0;
  return UCAC_OK;
}

int ucac_mlp_get_weights(const ucac_mlp* mc, float* w, size_t n) {
  ucac_mlp* m = const_cast<ucac_mlp*>(mc);
  if (!m || !w || n != (size_t)MLP_PARAMS) return m ? (m->err = "bad buffer", UCAC_E_INVAL) : UCAC_E_INVAL;
  MLP_OR(m, hipSetDevice(m->device));
  MLP_OR(m, hipStreamSynchronize(m->st));
  MLP_OR(m, hipMemcpy(w, mlp_carve(m->mem).P, sizeof(float) * n, hipMemcpyDeviceToHost));
  return UCAC_OK;
}

int ucac_mlp_forward(ucac_mlp* m, const float* x, int64_t n, float* y) {
  if (!m || !x || !y || n < 0 || n > 0x7fffffff) return m ? (m->err = "bad arguments", UCAC_E_INVAL) : UCAC_E_INVAL;
  if (n == 0) return UCAC_OK;
  MLP_OR(m, hipSetDevice(m->device));
  MlpCall c;
  MLP_OR(m, hipMalloc(&c.X, sizeof(float) * n * 20));
  MLP_OR(m, hipMalloc(&c.Y, sizeof(float) * n * 4));
  MLP_OR(m, hipMemcpy(c.X, x, sizeof(float) * n * 20, hipMemcpyHostToDevice));
  mlp_launch_forward(mlp_view(mlp_carve(m->mem)), c.X, (int)n, c.Y, m->st);
  MLP_OR(m, hipGetLastError());
  MLP_OR(m, hipStreamSynchronize(m->st));
  MLP_OR(m, hipMemcpy(y, c.Y, sizeof(float) * n * 4, hipMemcpyDeviceToHost));
  return UCAC_OK;
}

int ucac_mlp_grad(ucac_mlp* m, const float* x, const float* t, int64_t n, float* grad, double* loss) {
  if (!m || !x || !t || n < 1 || n > (1 << 22)) return m ? (m->err = "bad arguments", UCAC_E_INVAL) : UCAC_E_INVAL;
  MLP_OR(m, hipSetDevice(m->device));
  MlpCall c;
  const int waves = (int)((n + 63) / 64);
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  MLP_OR(m, hipMalloc(&c.X, sizeof(float) * n * 20));
  MLP_OR(m, hipMalloc(&c.Y, sizeof(float) * n * 4));
  MLP_OR(m, hipMalloc(&c.idx, sizeof(int) * n));
  MLP_OR(m, hipMalloc(&c.slots, sizeof(float) * waves * MLP_SLOT));
  MLP_OR(m, hipMalloc(&c.grad, sizeof(float) * MLP_PARAMS));
  MLP_OR(m, hipMalloc(&c.loss, sizeof(double)));
  MLP_OR(m, hipMemcpy(c.X, x, sizeof(float) * n * 20, hipMemcpyHostToDevice));
  MLP_OR(m, hipMemcpy(c.Y, t, sizeof(float) * n * 4, hipMemcpyHostToDevice));
  MLP_OR(m, hipMemcpy(c.idx, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  const MlpBufs b = mlp_carve(m->mem);
  mlp_launch_train(mlp_view(b), c.X, c.Y, c.idx, (int)n, (float)(2.0 / (4.0 * (double)n)), c.slots, m->st);
  mlp_launch_reduce(c.slots, waves, c.grad, c.loss, b.P, m->m1, m->m2, 0, 0.0f, b.W1b, b.W2b, b.W3b, m->st);
  MLP_OR(m, hipGetLastError());
  MLP_OR(m, hipStreamSynchronize(m->st));
  double ls = 0.0;
  MLP_OR(m, hipMemcpy(&ls, c.loss, sizeof(double), hipMemcpyDeviceToHost));
  if (grad) MLP_OR(m, hipMemcpy(grad, c.grad, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost));
  if (loss) *loss = ls / (4.0 * (double)n);
  return UCAC_OK;
}

int ucac_mlp_train(ucac_mlp* m, const float* x, const float* t, int64_t n, int32_t epochs, int32_t batch, double lr,
                   uint64_t seed, double* last_loss) {
  if (!m || !x || !t || n < 1 || n > 0x7fffffff || epochs < 0 || batch < 1 || !(lr > 0.0))
    return m ? (m->err = "bad arguments", UCAC_E_INVAL) : UCAC_E_INVAL;
  MLP_OR(m, hipSetDevice(m->device));
  MlpCall c;
  const int waves = (batch + 63) / 64;
  MLP_OR(m, hipMalloc(&c.X, sizeof(float) * n * 20));
  MLP_OR(m, hipMalloc(&c.Y, sizeof(float) * n * 4));
  MLP_OR(m, hipMalloc(&c.idx, sizeof(int) * n));
  MLP_OR(m, hipMalloc(&c.slots, sizeof(float) * waves * MLP_SLOT));
  MLP_OR(m, hipMalloc(&c.loss, sizeof(double) * 2));
  MLP_OR(m, hipMemcpy(c.X, x, sizeof(float) * n * 20, hipMemcpyHostToDevice));
  MLP_OR(m, hipMemcpy(c.Y, t, sizeof(float) * n * 4, hipMemcpyHostToDevice));
  const MlpBufs b = mlp_carve(m->mem);
  const MlpView v = mlp_view(b);
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  uint64_t rs = seed;
  double epoch_loss = 0.0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(rs) % (uint64_t)(i + 1)]);  // Fisher-Yates
    MLP_OR(m, hipMemcpyAsync(c.idx, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, m->st));
    std::vector<double> bl;
    for (int64_t s0 = 0; s0 < n; s0 += batch) {
      const int nb = (int)std::min<int64_t>(batch, n - s0);
      mlp_launch_train(v, c.X, c.Y, c.idx + s0, nb, (float)(2.0 / (4.0 * nb)), c.slots, m->st);
      ++m->step;
      mlp_launch_reduce(c.slots, (nb + 63) / 64, nullptr, c.loss, b.P, m->m1, m->m2, m->step, (float)lr, b.W1b, b.W2b,
                        b.W3b, m->st);
      MLP_OR(m, hipGetLastError());
      if (e == epochs - 1) {
        double ls = 0.0;
        MLP_OR(m, hipMemcpyAsync(&ls, c.loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
        MLP_OR(m, hipStreamSynchronize(m->st));
        bl.push_back(ls);
      }
    }
    if (e == epochs - 1) {
      epoch_loss = 0.0;
      for (double v2 : bl) epoch_loss += v2;
      epoch_loss /= 4.0 * (double)n;
    }
    MLP_OR(m, hipStreamSynchronize(m->st));  // the next permutation reuses the index buffer
  }
  MLP_OR(m, hipStreamSynchronize(m->st));
  if (last_loss) *last_loss = epoch_loss;
  return UCAC_OK;
}

int ucac_mlp_grad_noalloc(ucac_mlp* m, const float* x, const float* t, int64_t n, float* grad, double* loss,
                          void* stream) {
  if (!m || !x || !t || !grad || !loss) return m ? (m->err = "null argument", UCAC_E_INVAL) : UCAC_E_INVAL;
  if (n < 1 || n > UCAC_MLP_NOALLOC_MAX) {
    char buf[160];
    snprintf(buf, sizeof buf, "n = %lld samples is outside 1..%d, the size of the fixed device scratch",
             (long long)n, UCAC_MLP_NOALLOC_MAX);
    m->err = buf;
    return UCAC_E_INVAL;
  }
  if (m->device < 0 || m->device >= MAX_DEVICES) return m->err = "device ordinal out of range", UCAC_E_INVAL;
  void* base = nullptr;
  hipError_t serr = hipSuccess;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[m->device];
    serr = g_scratch_err[m->device];
  }
  if (!base) return mfail(m, UCAC_E_DEVICE, "device scratch address (hipGetSymbolAddress)", serr);
  MLP_OR(m, hipSetDevice(m->device));
  hipStream_t st = stream ? (hipStream_t)stream : m->st;
  int* idx = (int*)base;
  float* slots = (float*)((unsigned char*)base + NOALLOC_SLOT_OFF);
  const int nb = (int)n, waves = (nb + 63) / 64;
  // identity sample order: every index the training kernel reads is written here first
  hipLaunchKernelGGL(k_iota, dim3((nb + 255) / 256), dim3(256), 0, st, idx, nb);
  MLP_OR(m, hipGetLastError());
  const MlpBufs b = mlp_carve(m->mem);
  // each wavefront overwrites its whole slot (every parameter and its loss sum), so the
  // slots need no clearing; the reduction reads only this call's slots
  mlp_launch_train(mlp_view(b), x, t, idx, nb, (float)(2.0 / (4.0 * (double)n)), slots, st);
  mlp_launch_reduce(slots, waves, grad, loss, b.P, m->m1, m->m2, 0, 0.0f, b.W1b, b.W2b, b.W3b, st);
  MLP_OR(m, hipGetLastError());
  return UCAC_OK;
}

const char* ucac_mlp_last_error(const ucac_mlp* m) { return m ? m->err.c_str() : g_create_error.c_str(); }

void ucac_mlp_destroy(ucac_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->st) (void)hipStreamSynchronize(m->st);
  if (m->mem) (void)hipFree(m->mem);
  if (m->m1) (void)hipFree(m->m1);
  if (m->m2) (void)hipFree(m->m2);
  if (m->st) (void)hipStreamDestroy(m->st);
  delete m;
}

int ucac_dp_batch(int32_t G, int32_t T, const double* tab, const int32_t* min_up, const int32_t* min_dn,
                  const int32_t* u0, const int32_t* hold_on, const int32_t* hold_off, int8_t* u_on, double* cost,
                  int32_t lanes_per_unit, void* stream) {
  if (G < 0 || T < 1 || (lanes_per_unit != 16 && lanes_per_unit != 64))
    return fail(nullptr, UCAC_E_INVAL, "dp_batch: need G >= 0, T >= 1, lanes_per_unit 16 or 64");
  if (G == 0) return UCAC_OK;
  if (!tab || !min_up || !min_dn || !u0 || !hold_on || !hold_off || !u_on || !cost)
    return fail(nullptr, UCAC_E_INVAL, "dp_batch: null pointer");
  if (dp_tables_lds(T, lanes_per_unit) > 65536)
    return fail(nullptr, UCAC_E_INVAL, "dp_batch: horizon %d needs %zu bytes of LDS per block (limit 65536)", T,
                dp_tables_lds(T, lanes_per_unit));
  (void)hipGetLastError();
  launch_dp_tables(tab, G, T, min_up, min_dn, u0, hold_on, hold_off, (signed char*)u_on, cost, lanes_per_unit,
                   (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, UCAC_E_DEVICE, "dp_batch launch failed: %s", hipGetErrorString(e));
  return UCAC_OK;
}

const char* ucac_last_error(const ucac_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void ucac_destroy(ucac_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->par.device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->graphs.clear();
  h->graphs_solve.clear();
  clear_period_graph(h);
  if (h->ev_poll) (void)hipEventDestroy(h->ev_poll);
  if (h->own) (void)hipStreamDestroy(h->own);
  if (h->h_ctl) (void)hipHostFree(h->h_ctl);
  if (h->h_sc) (void)hipHostFree(h->h_sc);
  if (h->arena) (void)hipFree(h->arena);
  if (h->mlp_mem) (void)hipFree(h->mlp_mem);
  if (h->solve_save) (void)hipFree(h->solve_save);
  delete h;
}

}  // extern "C"

// ---- batches: many independent instances, one grouped launch per kernel ----------

struct ucac_batch {
  int device = 0;
  int warm_start = 0;
  std::vector<ucac_handle*> m;
  hipStream_t st = nullptr;
  Member* d_members = nullptr;
  int* d_tables = nullptr;       // per kernel: blk_member [grid], blk_first [n], blk_count [n]
  Group grp[K_COUNT]{};
  int grid[K_COUNT]{};
  int max_T = 1;
  ucac_batch_config cfg{64, 256, 0};
  GraphSet graphs;
  std::vector<int> it0;
  std::string err;
};

namespace {

int bfail(ucac_batch* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf; else g_create_error = buf;
  return code;
}

#define BHIP_OR(b, call)                                                                              \
  do {                                                                                                \
    hipError_t _e = (call);                                                                           \
    if (_e != hipSuccess) return bfail(b, UCAC_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
  } while (0)

int kernel_blocks(int k, const Net& n, const ucac_batch_config& c, int max_T) {
  switch (k) {
    case K_UNITS: return n.G && n.T ? units_blocks(n, units_gpb(max_T, c.dp_lanes, c.branch_block == 64 ? 64 : 256)) : 0;
    case K_BRANCH: return branch_blocks(n, c.branch_block);
    case K_BUS: return bus_blocks(n);
    case K_POST: return post_blocks(n);
    case K_FINALIZE: return 1;
    default: return lambda_blocks(n);
  }
}

// Block tables of every kernel for the configured member order, and the graph.
int batch_build(ucac_batch* b) {
  const int n = (int)b->m.size();
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  if (b->cfg.order == 1)  // largest line work first, so the longest blocks start first
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
      return (long)b->m[a]->T * b->m[a]->L > (long)b->m[c]->T * b->m[c]->L;
    });
  std::vector<int> tab;
  size_t off[K_COUNT];
  for (int k = 0; k < K_COUNT; ++k) {
    std::vector<int> first(n, 0), count(n, 0), member;
    for (int j : order) {
      const int nb = kernel_blocks(k, b->m[j]->net, b->cfg, b->max_T);
      first[j] = (int)member.size();
      count[j] = nb;
      for (int q = 0; q < nb; ++q) member.push_back(j);
    }
    b->grid[k] = (int)member.size();
    off[k] = tab.size();
    tab.insert(tab.end(), member.begin(), member.end());
    tab.insert(tab.end(), first.begin(), first.end());
    tab.insert(tab.end(), count.begin(), count.end());
  }
  if (b->d_tables) { (void)hipFree(b->d_tables); b->d_tables = nullptr; }
  BHIP_OR(b, hipMalloc(&b->d_tables, sizeof(int) * tab.size()));
  BHIP_OR(b, hipMemcpy(b->d_tables, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice));
  for (int k = 0; k < K_COUNT; ++k) {
    Group& g = b->grp[k];
    g.m = b->d_members;
    g.blk_member = b->d_tables + off[k];
    g.blk_first = g.blk_member + b->grid[k];
    g.blk_count = g.blk_first + n;
  }
  b->graphs.clear();
  const char* where = "";
  auto launch = [&](int k, hipStream_t s) {
    if (k == K_FRONT) {
      launch_front_grouped(b->grp[K_UNITS], b->grid[K_UNITS], b->grp[K_BRANCH], b->grid[K_BRANCH], b->warm_start,
                           b->cfg.branch_block, b->cfg.dp_lanes, b->max_T, s);
      return hipGetLastError();
    }
    if (b->grid[k] == 0) return hipSuccess;
    const Group& g = b->grp[k];
    switch (k) {
      case K_BUS: launch_bus_grouped(g, b->grid[k], s); break;
      case K_POST: launch_post_grouped(g, b->grid[k], s); break;
      case K_FINALIZE: launch_finalize_grouped(g, b->grid[k], s); break;
      default: launch_lambda_grouped(g, b->grid[k], s); break;
    }
    return hipGetLastError();
  };
  for (int j = 0; j < N_GRAPHS; ++j) {
    (void)hipGetLastError();
    BHIP_OR(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int r = 0; r < GRAPH_SIZES[j] && le == hipSuccess; ++r) le = enqueue_chain(launch, b->st, &where);
    const hipError_t ce = hipStreamEndCapture(b->st, &b->graphs.g[j]);
    if (le != hipSuccess) return bfail(b, UCAC_E_DEVICE, "grouped launch of %s failed: %s", where, hipGetErrorString(le));
    if (ce != hipSuccess) return bfail(b, UCAC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ce));
    BHIP_OR(b, hipGraphInstantiate(&b->graphs.x[j], b->graphs.g[j], nullptr, nullptr, 0));
  }
  return UCAC_OK;
}

hipError_t batch_launch_iterations(ucac_batch* b, int n) { return b->graphs.launch(n, b->st); }

int batch_set_ctl(ucac_batch* b, int stop_at_tol, double tol) {
  for (ucac_handle* h : b->m) {
    std::memset(h->h_ctl, 0, sizeof(Ctl));
    h->h_ctl->stop_at_tol = stop_at_tol;
    h->h_ctl->tol = tol;
    const double ms[3] = {1e-2, 1e-3, 1e-4};
    for (int q = 0; q < 3; ++q) { h->h_ctl->ms_tol[q] = ms[q]; h->h_ctl->ms_iter[q] = -1; }
    h->h_ctl->conv_iter = -1;
    BHIP_OR(b, hipMemcpyAsync(h->d_ctl, h->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, b->st));
  }
  return UCAC_OK;
}

int batch_read(ucac_batch* b) {
  for (ucac_handle* h : b->m) {
    BHIP_OR(b, hipMemcpyAsync(h->h_sc, h->st.sc, sizeof(double) * NSC, hipMemcpyDeviceToHost, b->st));
    BHIP_OR(b, hipMemcpyAsync(h->h_ctl, h->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, b->st));
  }
  BHIP_OR(b, hipStreamSynchronize(b->st));
  for (size_t k = 0; k < b->m.size(); ++k)
    if (b->m[k]->h_ctl->bad) return bfail(b, UCAC_E_NUMERIC, "member %zu: non-finite residual in the iterate", k);
  return UCAC_OK;
}

// Members whose last iteration left a multiplier update pending get it applied
// (the single-instance flush kernel on the batch stream).  h_ctl must be current.
int batch_flush(ucac_batch* b) {
  bool any = false;
  for (ucac_handle* h : b->m) {
    if (!h->h_ctl->pending) continue;
    any = true;
    launch_lambda(h->net, h->st, h->kp, b->st);
    BHIP_OR(b, hipGetLastError());
    h->h_ctl->pending = 0;
    BHIP_OR(b, hipMemcpyAsync(&h->d_ctl->pending, &h->h_ctl->pending, sizeof(int), hipMemcpyHostToDevice, b->st));
  }
  if (any) BHIP_OR(b, hipStreamSynchronize(b->st));
  return UCAC_OK;
}

}  // namespace

extern "C" {

int ucac_batch_create(const ucac_network* nets, int32_t n, const ucac_params* params, ucac_batch** out) {
  if (!out) return bfail(nullptr, UCAC_E_INVAL, "null output handle");
  *out = nullptr;
  if (!nets || !params || n < 1) return bfail(nullptr, UCAC_E_INVAL, "need at least one network and params");
  if (params->warm_start < 0 || params->warm_start > 1)
    return bfail(nullptr, UCAC_E_INVAL, "batches take the flat (0) or previous-iterate (1) Newton start");
  ucac_batch* b = new ucac_batch();
  b->device = params->device;
  b->warm_start = params->warm_start;
  auto bad = [&](int code) {
    const std::string e = g_create_error;
    ucac_batch_destroy(b);
    g_create_error = e;
    return code;
  };
  for (int k = 0; k < n; ++k) {
    ucac_handle* h = nullptr;
    const int rc = ucac_create(&nets[k], params, &h);
    if (rc != UCAC_OK) {
      g_create_error = "member " + std::to_string(k) + ": " + g_create_error;
      return bad(rc);
    }
    b->m.push_back(h);
    b->max_T = std::max(b->max_T, h->T);
  }
  if (hipSetDevice(b->device) != hipSuccess) return bad(bfail(nullptr, UCAC_E_DEVICE, "hipSetDevice failed"));
  if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess)
    return bad(bfail(nullptr, UCAC_E_DEVICE, "stream create failed"));
  std::vector<Member> hm(n);
  for (int k = 0; k < n; ++k) hm[k] = Member{b->m[k]->net, b->m[k]->st, b->m[k]->kp};
  if (hipMalloc(&b->d_members, sizeof(Member) * n) != hipSuccess ||
      hipMemcpy(b->d_members, hm.data(), sizeof(Member) * n, hipMemcpyHostToDevice) != hipSuccess)
    return bad(bfail(nullptr, UCAC_E_NOMEM, "member table allocation failed"));
  if (batch_build(b) != UCAC_OK) {
    g_create_error = b->err;
    return bad(UCAC_E_DEVICE);
  }
  *out = b;
  return UCAC_OK;
}

int32_t ucac_batch_size(const ucac_batch* b) { return b ? (int32_t)b->m.size() : 0; }

int ucac_batch_member(ucac_batch* b, int32_t k, ucac_handle** member) {
  if (!b || !member) return UCAC_E_INVAL;
  if (k < 0 || k >= (int32_t)b->m.size()) return bfail(b, UCAC_E_INVAL, "member %d out of range", k);
  BHIP_OR(b, hipStreamSynchronize(b->st));
  *member = b->m[k];
  return UCAC_OK;
}

int ucac_batch_step(ucac_batch* b, int32_t n_iters) {
  if (!b) return UCAC_E_INVAL;
  if (n_iters < 0) return bfail(b, UCAC_E_INVAL, "negative iteration count");
  BHIP_OR(b, hipSetDevice(b->device));
  for (ucac_handle* h : b->m) BHIP_OR(b, hipStreamSynchronize(h->stream));
  int rc = batch_set_ctl(b, 0, b->m[0]->par.tol);
  if (rc) return rc;
  BHIP_OR(b, batch_launch_iterations(b, n_iters));
  rc = batch_read(b);
  if (rc) return rc;
  return batch_flush(b);
}

int ucac_batch_solve(ucac_batch* b, double tol, int32_t max_iters, int32_t* iters_done, int32_t* converged) {
  if (!b) return UCAC_E_INVAL;
  if (!(tol > 0.0) || max_iters < 0) return bfail(b, UCAC_E_INVAL, "bad tol or max_iters");
  BHIP_OR(b, hipSetDevice(b->device));
  for (ucac_handle* h : b->m) BHIP_OR(b, hipStreamSynchronize(h->stream));
  int rc = batch_read(b);
  if (rc) return rc;
  const int n = (int)b->m.size();
  std::vector<double> it0(n);
  for (int k = 0; k < n; ++k) {
    ucac_handle* h = b->m[k];
    h->par.tol = tol;
    it0[k] = h->h_sc[SC_ITER];
    h->h_sc[SC_CONV] = 0.0;
    BHIP_OR(b, hipMemcpyAsync(h->st.sc + SC_CONV, h->h_sc + SC_CONV, sizeof(double), hipMemcpyHostToDevice, b->st));
  }
  rc = batch_set_ctl(b, 1, tol);
  if (rc) return rc;
  int launched = 0;
  bool all = false;
  while (!all && launched < max_iters) {
    const int c = std::min(SOLVE_CHUNK, max_iters - launched);
    BHIP_OR(b, batch_launch_iterations(b, c));
    launched += c;
    rc = batch_read(b);
    if (rc) return rc;
    all = true;
    for (ucac_handle* h : b->m) all = all && h->h_sc[SC_CONV] != 0.0;
  }
  rc = batch_flush(b);
  if (rc) return rc;
  int n_conv = 0;
  for (int k = 0; k < n; ++k) {
    const bool cv = b->m[k]->h_sc[SC_CONV] != 0.0;
    n_conv += cv;
    if (iters_done) iters_done[k] = (int32_t)(b->m[k]->h_sc[SC_ITER] - it0[k]);
    if (converged) converged[k] = cv ? 1 : 0;
  }
  return n_conv == n ? UCAC_OK : UCAC_NOT_CONVERGED;
}

int ucac_batch_set_config(ucac_batch* b, const ucac_batch_config* c) {
  if (!b || !c) return UCAC_E_INVAL;
  if ((c->dp_lanes != 16 && c->dp_lanes != 64) || (c->branch_block != 64 && c->branch_block != 256) ||
      (c->order != 0 && c->order != 1))
    return bfail(b, UCAC_E_INVAL, "config: dp_lanes 16|64, branch_block 64|256, order 0|1");
  BHIP_OR(b, hipSetDevice(b->device));
  BHIP_OR(b, hipStreamSynchronize(b->st));
  b->cfg = *c;
  return batch_build(b);
}

int ucac_batch_get_config(const ucac_batch* b, ucac_batch_config* c) {
  if (!b || !c) return UCAC_E_INVAL;
  *c = b->cfg;
  return UCAC_OK;
}

int ucac_batch_autotune(ucac_batch* b, int32_t iters, ucac_batch_config* chosen, double* ms_per_iter, int32_t n_slots) {
  if (!b) return UCAC_E_INVAL;
  if (iters < 1) return bfail(b, UCAC_E_INVAL, "iters must be positive");
  BHIP_OR(b, hipSetDevice(b->device));
  for (ucac_handle* h : b->m) BHIP_OR(b, hipStreamSynchronize(h->stream));
  BHIP_OR(b, hipStreamSynchronize(b->st));
  // every candidate runs from the same saved iterate, which is restored at the end
  size_t total = 0;
  for (ucac_handle* h : b->m) total += h->n_state;
  double* save = nullptr;
  BHIP_OR(b, hipMalloc(&save, sizeof(double) * total));
  auto restore = [&]() -> hipError_t {
    size_t o = 0;
    for (ucac_handle* h : b->m) {
      const hipError_t e = hipMemcpyAsync(h->d_state, save + o, sizeof(double) * h->n_state, hipMemcpyDeviceToDevice, b->st);
      if (e != hipSuccess) return e;
      o += h->n_state;
    }
    return hipStreamSynchronize(b->st);
  };
  {
    size_t o = 0;
    for (ucac_handle* h : b->m) {
      if (hipMemcpyAsync(save + o, h->d_state, sizeof(double) * h->n_state, hipMemcpyDeviceToDevice, b->st) != hipSuccess) {
        (void)hipFree(save);
        return bfail(b, UCAC_E_DEVICE, "state save failed");
      }
      o += h->n_state;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const ucac_batch_config cand[] = {{64, 256, 0}, {16, 256, 0}, {64, 64, 0}, {16, 64, 0},
                                    {64, 256, 1}, {16, 256, 1}, {64, 64, 1}, {16, 64, 1}};
  const int nc = (int)(sizeof cand / sizeof cand[0]);
  double best = 1e300;
  ucac_batch_config bestc = b->cfg;
  int rc = UCAC_OK;
  for (int c = 0; c < nc && rc == UCAC_OK; ++c) {
    b->cfg = cand[c];
    rc = batch_build(b);
    if (rc) break;
    if (restore() != hipSuccess) { rc = bfail(b, UCAC_E_DEVICE, "state restore failed"); break; }
    rc = batch_set_ctl(b, 0, b->m[0]->par.tol);
    if (rc) break;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = batch_launch_iterations(b, 2);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, b->st);
    if (e == hipSuccess) e = batch_launch_iterations(b, iters);
    if (e == hipSuccess) e = hipEventRecord(e1, b->st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { rc = bfail(b, UCAC_E_DEVICE, "tuning run failed: %s", hipGetErrorString(e)); break; }
    const double per = ms / iters;
    if (ms_per_iter && c < n_slots) ms_per_iter[c] = per;
    if (per < best) { best = per; bestc = cand[c]; }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == UCAC_OK) {
    b->cfg = bestc;
    rc = batch_build(b);
  }
  if (rc == UCAC_OK && restore() != hipSuccess) rc = bfail(b, UCAC_E_DEVICE, "state restore failed");
  (void)hipFree(save);
  if (rc == UCAC_OK && chosen) *chosen = bestc;
  if (rc == UCAC_OK) rc = batch_read(b);
  return rc;
}

const char* ucac_batch_last_error(const ucac_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

void ucac_batch_destroy(ucac_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->st) (void)hipStreamSynchronize(b->st);
  b->graphs.clear();
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_members) (void)hipFree(b->d_members);
  if (b->st) (void)hipStreamDestroy(b->st);
  for (ucac_handle* h : b->m) ucac_destroy(h);
  delete b;
}

}  // extern "C"
