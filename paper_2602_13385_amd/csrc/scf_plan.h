// Internal to libscf: the plan object, error reporting, workspace layouts
// and the launch helpers shared by the translation units of the C ABI
// (scf_api.cpp: plans, the step, batched and adjoint paths; scf_cadence.cpp:
// the refresh cadence, the density and the frame).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/scf.h"
#include "host_field.h"
#include "scf_internal.h"


using namespace scf;

namespace scf {
namespace api_detail {
// message of the last failed call on this thread (scf_last_error)
inline thread_local std::string g_last_error;
}  // namespace api_detail
}  // namespace scf

namespace {


scf_status fail(scf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  scf::api_detail::g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(SCF_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                  __FILE__, __LINE__);                                                    \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// basis tables (double precision, host)
// ---------------------------------------------------------------------------
// Monic Gegenbauer recurrence p_n = xi p_{n-1} - beta_n p_{n-2}:
// from n C_n = 2(n+lambda-1) xi C_{n-1} - (n+2 lambda-2) C_{n-2} and the
// leading coefficient k_n = 2^n (lambda)_n / n!.
double gegen_beta(int n, double lam) {
  if (n < 2) return 0.0;
  return (n + 2.0 * lam - 2.0) * (n - 1.0) / (4.0 * (n + lam - 1.0) * (n + lam - 2.0));
}
double gegen_lead(int n, double lam) {
  return std::exp(n * std::log(2.0) + std::lgamma(lam + n) - std::lgamma(lam) - std::lgamma(n + 1.0));
}
// Monic-scaled associated Legendre recurrence Qt_l = c Qt_{l-1} - gamma Qt_{l-2}
double legendre_gamma(int l, int m) {
  if (l < m + 2) return 0.0;
  return (l + m - 1.0) * (l - m - 1.0) / ((2.0 * l - 1.0) * (2.0 * l - 3.0));
}
// rho_lm = d^m P_l / dx^m  /  Qt_l^m
double legendre_rho(int l, int m) {
  double r = 1.0;
  for (int k = 2 * m - 1; k > 1; k -= 2) r *= k;  // (2m-1)!!
  for (int ll = m + 1; ll <= l; ++ll) r *= (2.0 * ll - 1.0) / (ll - m);
  return r;
}
double ylm_norm(int l, int m) {
  double lg = std::lgamma(l - m + 1.0) - std::lgamma(l + m + 1.0);
  return std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * std::exp(lg));
}

// f_nl(s) = -s^l q^(-alpha(2l+1)) C_n^(lambda)(xi) and its s-derivative,
// evaluated with the monic recurrence and its derivative.
void radial_f(double alpha, int l, int n, double s, double& f, double& df) {
  const double lam = (2.0 * l + 1.0) * alpha + 0.5;
  const double t = std::pow(s, 1.0 / alpha);
  const double q = 1.0 + t;
  const double xi = 1.0 - 2.0 / q;
  const double dt = (1.0 / alpha) * std::pow(s, 1.0 / alpha - 1.0);  // dt/ds
  const double dxi = 2.0 * dt / (q * q);
  double p0 = 1.0, p1 = xi, d0 = 0.0, d1 = 1.0, p = 1.0, dp = 0.0;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
  } else if (n == 1) {
    p = xi;
    dp = 1.0;
  } else {
    for (int k = 2; k <= n; ++k) {
      double b = gegen_beta(k, lam);
      double p2 = xi * p1 - b * p0;
      double d2 = p1 + xi * d1 - b * d0;
      p0 = p1;
      p1 = p2;
      d0 = d1;
      d1 = d2;
    }
    p = p1;
    dp = d1;
  }
  const double kn = gegen_lead(n, lam);
  const double pre = std::pow(s, double(l)) * std::pow(q, -alpha * (2.0 * l + 1.0));
  // d pre / ds = pre * (l/s - alpha(2l+1) dt / q)
  const double dpre = (l > 0 ? l * std::pow(s, l - 1.0) * std::pow(q, -alpha * (2.0 * l + 1.0)) : 0.0) -
                      pre * alpha * (2.0 * l + 1.0) * dt / q;
  f = -kn * pre * p;
  df = -kn * (dpre * p + pre * dp * dxi);
}

// Energy-norm normalisation N_nl = (b / 4 pi G) int_0^inf [s^2 f'^2 + l(l+1) f^2] ds.
// alpha = 1: closed form (Hernquist & Ostriker 1992).  Otherwise composite
// 16-point Gauss-Legendre quadrature in v = ln s over [-60, 60].
double norm_nl(double alpha, double b, double G, int n, int l) {
  if (alpha == 1.0) {
    const double K = 0.5 * n * (n + 4.0 * l + 3.0) + (l + 1.0) * (2.0 * l + 1.0);
    const double lg = std::lgamma(n + 4.0 * l + 3.0) - std::lgamma(n + 1.0) - 2.0 * std::lgamma(2.0 * l + 1.5);
    return b / G * K * std::exp(lg - (8.0 * l + 6.0) * std::log(2.0)) / (n + 2.0 * l + 1.5);
  }
  static double xs[16], ws[16];
  static bool init = false;
  if (!init) {
    for (int i = 0; i < 16; ++i) {  // Newton iteration on P_16
      double x = std::cos(M_PI * (i + 0.75) / 16.5);
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= 16; ++k) {
          double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        double dp = 16.0 * (x * p1 - p0) / (x * x - 1.0);
        double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= 16; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = 16.0 * (x * p1 - p0) / (x * x - 1.0);
      xs[i] = x;
      ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    init = true;
  }
  const int panels = 960;
  const double v0 = -60.0, v1 = 60.0, hw = (v1 - v0) / panels;
  double acc = 0.0;
  for (int pnl = 0; pnl < panels; ++pnl) {
    const double c = v0 + (pnl + 0.5) * hw;
    for (int i = 0; i < 16; ++i) {
      const double v = c + 0.5 * hw * xs[i];
      const double s = std::exp(v);
      double f, df;
      radial_f(alpha, l, n, s, f, df);
      double val = (s * s * df * df + l * (l + 1.0) * f * f) * s;
      if (std::isfinite(val)) acc += 0.5 * hw * ws[i] * val;
    }
  }
  return b / (4.0 * M_PI * G) * acc;
}

}  // namespace

struct scf_plan {
  scf_basis basis;
  int dtype;
  int device;
  int nmax, lmax, nmaxc;
  int64_t T;
  int amode;
  Engine* eng;
  int coef_variant = 0;
  int coef_div = 1;  // wave-units of the coefficient pass: one resident round / coef_div
  int field_variant = 0;
  int num_cu = 256;
  int resident[8] = {1, 1, 1, 1, 1, 1, 1, 1};  // resident wave-units per CU per variant
  int gamma_resident = 1;                        // same for the adjoint's gamma pass
  size_t rs;  // sizeof real
  void* d_beta_rad = nullptr;
  void* d_beta_ang = nullptr;
  double* d_cs = nullptr;
  double* d_fw = nullptr;
  double* d_kden = nullptr;  // density constants -K_nl / (4 pi G b^2), [l][n]
  double* d_dtab = nullptr;  // radial derivative table of the matrix-core field pass, [l][2][n]
  std::vector<double> h_cs, h_fw;
  // kernel timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  // batched mode: the captured per-step graph, the stream it is captured on,
  // and pinned host staging for the work list and the centre table
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_g = nullptr;    // kGraphSteps middle steps in one graph
  hipGraphExec_t gexec_g = nullptr;
  std::vector<char> gkey;
  int graph_captures = 0;
  double* h_tab = nullptr;
  size_t h_tab_cap = 0;
  char* h_meta = nullptr;
  size_t h_meta_cap = 0;
  hipEvent_t ev_staging = nullptr;
  bool staging_pending = false;
};

namespace {

enum Kind { K_COEF = 0, K_REDUCE, K_FINALIZE, K_FIELD, K_STEP_FIELD, K_KICK, K_MAKE_W, K_FILL,
            K_BATCH_COEF, K_BATCH_FIELD, K_ADJ, K_SELECT, K_OTHER };
const char* kKindNames[SCF_KERNEL_KINDS] = {"coef", "reduce", "finalize", "field", "field_step",
                                            "kick_drift", "make_w", "fill", "batched_coef",
                                            "batched_step", "adjoint", "select", "other"};

// brackets one launch with events when the plan's timing is on
struct Timed {
  scf_plan* p;
  hipStream_t s;
  int kind;
  hipEvent_t b = nullptr;
  Timed(scf_plan* p_, hipStream_t s_, int k) : p(p_), s(s_), kind(k) {
    if (p && p->prof && p->ev_next + 2 <= p->ev_pool.size() &&
        !(p->cap_stream && s == p->cap_stream)) {
      hipEvent_t a = p->ev_pool[p->ev_next++];
      b = p->ev_pool[p->ev_next++];
      (void)hipEventRecord(a, s);
      p->recs.push_back({kind, a, b});
    }
  }
  ~Timed() {
    if (b) (void)hipEventRecord(b, s);
  }
};

// Coefficient launch geometry: one resident round of wave-units (the
// occupancy of the variant times the CU count), each taking an even share of
// the P-particle stages; returns the unit count and sets *stages.
int coef_units_v(const scf_plan* p, int64_t n, int v, int64_t* stages, int div = 1) {
  if (n <= 0) {
    *stages = 0;
    return 0;
  }
  const int P = p->eng->stage_particles(v);
  *stages = (n + P - 1) / P;
  const int64_t cap = (int64_t)p->resident[v] * p->num_cu / std::max(div, 1);
  return (int)std::min<int64_t>(*stages, std::max<int64_t>(cap, 1));
}

// the plan's variant, and its unit count (fewer, longer units suit small n:
// the per-unit set-up and partial row are amortised over more stages)
int coef_units(const scf_plan* p, int64_t n, int64_t* stages) {
  return coef_units_v(p, n, p->coef_variant, stages, p->coef_div);
}

// rows per unit of variant v when no unit sums more than max_stages stages:
// one when each folds once (its compensation row would stay zero)
int unit_rows(const scf_plan* p, int v, int64_t max_stages) {
  const int f = p->eng->fold_stages(v);
  return (f > 0 && max_stages <= f) ? 1 : p->eng->rows_per_unit(v);
}

// largest partial-row count over the coefficient variants (workspace sizing)
int coef_blocks_max(const scf_plan* p, int64_t n) {
  int nb = 0;
  for (int v = 0; v < p->eng->coef_variants(); ++v) {
    int64_t st;
    nb = std::max(nb, coef_units_v(p, n, v, &st) * p->eng->rows_per_unit(v));
  }
  return nb;
}

constexpr int kReduceChunks = 32;

struct WsLayout {
  size_t partials, red1, coef, W, total;
};

WsLayout ws_layout(const scf_plan* p, int64_t n, int nclusters, int nblocks) {
  nblocks = std::max(nblocks, coef_blocks_max(p, n));  // layout independent of the variant
  WsLayout L;
  size_t off = 0;
  L.partials = off;
  off += align256((size_t)std::max(nblocks, 1) * p->T * p->rs);
  L.red1 = off;
  off += align256((size_t)kReduceChunks * p->T * sizeof(double) * std::max(nclusters, 1));
  L.coef = off;
  off += align256((size_t)p->T * sizeof(double) * std::max(nclusters, 1));
  L.W = off;
  off += align256((size_t)(p->nmaxc + 1) * (p->lmax + 1) * (p->lmax + 1) * p->rs *
                  std::max(nclusters, 1));
  L.total = off;
  (void)n;
  return L;
}

size_t plain_need(const scf_plan* p, int64_t n) { return ws_layout(p, n, 1, 0).total; }

// Batched workspace: the common layout for nclusters, then the centre-table
// chunk, the current centre rows and step counter, and the work lists.
constexpr int kCentreRows = 256;  // centre-table rows uploaded per chunk
constexpr int kGraphSteps = 8;    // middle steps replayed per graph launch

struct BatchLayout {
  WsLayout L;
  size_t tab, cur, ctr, seg_begin, seg_end, seg_slot, rows, blk_cluster, blk_begin, blk_end, total;
  int max_units;
  int64_t max_blocks;
};

BatchLayout batch_layout(const scf_plan* p, int64_t n, int ncl) {
  BatchLayout B;
  int max_units = 0, max_rows = 0;
  for (int v = 0; v < p->eng->coef_variants(); ++v) {
    const int u = p->resident[v] * p->num_cu + ncl;
    max_units = std::max(max_units, u);
    max_rows = std::max(max_rows, u * p->eng->rows_per_unit(v));
  }
  B.max_units = max_units;
  B.max_blocks = (n + 255) / 256 + ncl;
  B.L = ws_layout(p, n, ncl, max_rows);
  size_t off = B.L.total;
  B.tab = off;
  off += align256((size_t)kCentreRows * ncl * 9 * sizeof(double));
  B.cur = off;
  off += align256((size_t)ncl * 9 * sizeof(double));
  B.ctr = off;
  off += 256;
  B.seg_begin = off;
  off += align256((size_t)max_units * 8);
  B.seg_end = off;
  off += align256((size_t)max_units * 8);
  B.seg_slot = off;
  off += align256((size_t)max_units * 4);
  B.rows = off;
  off += align256((size_t)(ncl + 1) * 4);
  B.blk_cluster = off;
  off += align256((size_t)B.max_blocks * 4);
  B.blk_begin = off;
  off += align256((size_t)B.max_blocks * 8);
  B.blk_end = off;
  off += align256((size_t)B.max_blocks * 8);
  B.total = off;
  return B;
}

template <typename R>
void fill_host_params(HostParams<R>& hp, const scf_host* h) {
  std::memset(&hp, 0, sizeof(hp));
  if (!h) return;
  hp.ncomp = h->ncomp;
  hp.G = R(h->G);
  for (int c = 0; c < h->ncomp; ++c) {
    hp.kind[c] = h->comp[c].kind;
    for (int k = 0; k < 3; ++k) hp.p[c][k] = R(h->comp[c].p[k]);
  }
}

scf_status check_host(const scf_host* h) {
  if (!h) return SCF_OK;
  if (h->ncomp < 0 || h->ncomp > SCF_MAX_HOST_COMP)
    return fail(SCF_ERR_INVALID_ARG, "host->ncomp = %d outside [0, %d]", h->ncomp, SCF_MAX_HOST_COMP);
  if (h->ncomp > 0 && !(h->G > 0.0)) return fail(SCF_ERR_INVALID_ARG, "host->G must be > 0");
  for (int c = 0; c < h->ncomp; ++c) {
    const int k = h->comp[c].kind;
    if (k < SCF_HOST_LOG || k > SCF_HOST_PLUMMER)
      return fail(SCF_ERR_INVALID_ARG, "host component %d has unknown kind %d", c, k);
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(h->comp[c].p[q]))
        return fail(SCF_ERR_INVALID_ARG, "host component %d parameter %d is not finite", c, q);
    if (k != SCF_HOST_MN && !(h->comp[c].p[1] > 0.0))
      return fail(SCF_ERR_INVALID_ARG, "host component %d: scale parameter must be > 0", c);
  }
  return SCF_OK;
}

// centre acceleration -grad psi_host(R) in double precision
void centre_accel(const HostParams<double>& H, const double* R, double* g) {
  double gx = 0, gy = 0, gz = 0;
  if (H.ncomp > 0) host_grad<double>(H, R[0], R[1], R[2], gx, gy, gz);
  g[0] = -gx;
  g[1] = -gy;
  g[2] = -gz;
}

template <typename R>
void fill_force_common(ForceArgs<R>& fa, const scf_plan* p) {
  std::memset(&fa, 0, sizeof(fa));
  fa.beta_rad = (const R*)p->d_beta_rad;
  fa.beta_ang = (const R*)p->d_beta_ang;
  fa.binv = R(1.0 / p->basis.b);
  fa.alpha = R(p->basis.alpha);
  fa.inv_alpha = R(1.0 / p->basis.alpha);
  fa.amode = p->amode;
  fa.dtab = p->d_dtab;
}

template <typename R>
void fill_coef_common(CoefArgs<R>& ca, const scf_plan* p) {
  using S = scalar_t<R>;
  std::memset(&ca, 0, sizeof(ca));
  ca.beta_rad = (const S*)p->d_beta_rad;
  ca.beta_ang = (const S*)p->d_beta_ang;
  ca.T = (int)p->T;
  ca.nmax = p->nmax;
  ca.binv = S(1.0 / p->basis.b);
  ca.alpha = S(p->basis.alpha);
  ca.inv_alpha = S(1.0 / p->basis.alpha);
  ca.amode = p->amode;
}

// Sum of `rows` partial rows (FP32 or FP64) in double precision, then the
// coefficients (coef, nullable) and force weights W.  Up to kSmallRows rows:
// one pass (16 coefficients per block of 1024 threads, 64 row groups);
// otherwise chunk sums then their sum (two launches, fixed order either way).
constexpr int kSmallRows = 2048;

scf_status reduce_and_finalize(scf_plan* p, const void* partials, int rows, double* coef, void* W,
                               char* ws, const WsLayout& L, hipStream_t s) {
  if (rows <= kSmallRows) {
    Timed t(p, s, K_REDUCE);
    HIP_TRY(launch_reduce_final_small(p->dtype, partials, rows, (int)p->T, p->nmax, p->lmax,
                                      p->nmaxc, p->d_cs, p->d_fw, coef, W, s));
    return SCF_OK;
  }
  double* red1 = (double*)(ws + L.red1);
  const int nch = std::min(kReduceChunks, rows);
  {
    Timed t(p, s, K_REDUCE);
    HIP_TRY(launch_reduce(p->dtype, partials, rows, (int)p->T, nch, red1, s));
  }
  {
    Timed t(p, s, K_FINALIZE);
    HIP_TRY(launch_finalize(p->dtype, red1, nch, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_cs,
                            p->d_fw, coef, W, s));
  }
  return SCF_OK;
}

// coefficients of n particles into coef (device) and force weights W (device)
template <typename R>
scf_status run_coeffs(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                      const void* m, double* coef, void* W, char* ws, const WsLayout& L, hipStream_t s) {
  int64_t stages;
  const int units = coef_units(p, n, &stages);
  const int rpu = units > 0 ? unit_rows(p, p->coef_variant, (stages + units - 1) / units) : 1;
  const int nb = units * rpu;
  if (n == 0) {
    // empty particle set: all coefficients vanish
    if (coef) {
      Timed t(p, s, K_FILL);
      HIP_TRY(launch_fill(coef, p->T, 0.0, s));
    }
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef ? coef : (double*)(ws + L.coef), (int)p->T, p->nmax,
                          p->lmax, p->nmaxc, p->d_fw, W, s));
    return SCF_OK;
  }
  CoefArgs<R> ca;
  fill_coef_common(ca, p);
  ca.x = (const R*)x;
  ca.y = (const R*)y;
  ca.z = (const R*)z;
  ca.m = (const R*)m;
  ca.begin = 0;
  ca.stages = stages;
  ca.n = n;
  ca.partials = (R*)(ws + L.partials);
  ca.nunits = units;
  ca.one_row = rpu == 1;
  {
    Timed t(p, s, K_COEF);
    HIP_TRY(p->eng->launch_coef(&ca, units, p->coef_variant, s));
  }
  return reduce_and_finalize(p, ca.partials, nb, coef, W, ws, L, s);
}

// Field pass over n particles.  mode 0: a (and psi) into ax, ay, az (pot);
// mode 1: kick by `kick`, drift by `drift` with the drifted positions written
// to xo (default: in place); mode 2: adjoint accumulation (see field_kernel).
template <typename R>
scf_status run_field(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                     void* vz, void* ax, void* ay, void* az, void* pot, const void* W,
                     const HostParams<R>& hp, const double* cen, int mode, double kick,
                     double drift, hipStream_t s, void* xo = nullptr, void* yo = nullptr,
                     void* zo = nullptr, const void* mass = nullptr) {
  if (n == 0) return SCF_OK;
  ForceArgs<R> fa;
  fill_force_common(fa, p);
  fa.x = (R*)x;
  fa.y = (R*)y;
  fa.z = (R*)z;
  fa.xo = (R*)(xo ? xo : x);
  fa.yo = (R*)(yo ? yo : y);
  fa.zo = (R*)(zo ? zo : z);
  fa.mass = (const R*)mass;
  fa.vx = (R*)vx;
  fa.vy = (R*)vy;
  fa.vz = (R*)vz;
  fa.ax = (R*)ax;
  fa.ay = (R*)ay;
  fa.az = (R*)az;
  fa.pot = (R*)pot;
  fa.W = (const R*)W;
  fa.n = n;
  fa.kick = R(kick);
  fa.drift = R(drift);
  fa.host = hp;
  fa.cx = R(cen ? cen[0] : 0.0);
  fa.cy = R(cen ? cen[1] : 0.0);
  fa.cz = R(cen ? cen[2] : 0.0);
  fa.gcx = R(cen ? cen[3] : 0.0);
  fa.gcy = R(cen ? cen[4] : 0.0);
  fa.gcz = R(cen ? cen[5] : 0.0);
  Timed t(p, s, mode == 0 ? K_FIELD : (mode == 1 ? K_STEP_FIELD : K_ADJ));
  HIP_TRY(p->eng->launch_force(&fa, (n + 255) / 256, mode, p->field_variant, s));
  return SCF_OK;
}

// Basis tables of a plan for (alpha, b) (and its nmax, lmax, G): recurrence
// constants, per-coefficient sign and scale, density constants; uploaded to
// the plan's device buffers (allocated on the first call).
hipError_t fill_tables(scf_plan* p, const scf_basis* basis) {
  p->basis = *basis;
  p->amode = basis->alpha == 1.0 ? 0 : (basis->alpha == 0.5 ? 1 : 2);
  const int L1 = p->lmax + 1, NW = p->nmaxc + 1;
  // Legendre table: b_{l,m} at [m L1 + l] (b_{m,m} = -1 starts the order
  // recurrence of the field pass), then the integers 0..lmax at [L1 L1 + k]
  std::vector<double> brad((size_t)L1 * NW, 0.0), bang((size_t)L1 * L1 + L1, 0.0);
  for (int l = 0; l <= p->lmax; ++l) {
    const double lam = (2.0 * l + 1.0) * basis->alpha + 0.5;
    for (int n = 0; n <= p->nmaxc; ++n) brad[(size_t)l * NW + n] = gegen_beta(n, lam);
  }
  for (int m = 0; m <= p->lmax; ++m)
    for (int l = 0; l <= p->lmax; ++l) bang[(size_t)m * L1 + l] = l == m ? -1.0 : legendre_gamma(l, m);
  for (int k = 0; k <= p->lmax; ++k) bang[(size_t)L1 * L1 + k] = k;
  const int L2 = L1 * L1;
  p->h_cs.assign(p->T, 0.0);
  p->h_fw.assign(p->T, 0.0);
  for (int n = 0; n <= p->nmax; ++n) {
    for (int l = 0; l <= p->lmax; ++l) {
      const double lam = (2.0 * l + 1.0) * basis->alpha + 0.5;
      const double Nnl = norm_nl(basis->alpha, basis->b, basis->G, n, l);
      const double kn = gegen_lead(n, lam);
      for (int j = 0; j <= 2 * l; ++j) {
        const int m = (j + 1) / 2;
        const double kappa = -(kn / std::sqrt(Nnl)) * ylm_norm(l, m) * ((m & 1) ? -1.0 : 1.0) *
                             legendre_rho(l, m);
        const bool sin_part = j > 0 && (j % 2 == 0);
        const double sigma = sin_part ? 1.0 : -1.0;
        const double w = j == 0 ? 1.0 : (sin_part ? -2.0 : 2.0);
        const int64_t t = (int64_t)n * L2 + l * l + j;
        p->h_cs[t] = sigma * kappa;
        p->h_fw[t] = w * kappa;
      }
    }
  }
  // device copies: allocated on the first call, overwritten afterwards
  auto upload_real = [&](const std::vector<double>& v, void** dst) -> hipError_t {
    if (!*dst) {
      hipError_t e = hipMalloc(dst, v.size() * p->rs + 16);
      if (e != hipSuccess) return e;
    }
    if (p->rs == 4) {
      std::vector<float> f(v.begin(), v.end());
      return hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    return hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
  };
  hipError_t e = upload_real(brad, &p->d_beta_rad);
  if (e == hipSuccess) e = upload_real(bang, &p->d_beta_ang);
  if (e == hipSuccess && !p->d_cs) e = hipMalloc((void**)&p->d_cs, p->T * 8);
  if (e == hipSuccess) e = hipMemcpy(p->d_cs, p->h_cs.data(), p->T * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && !p->d_fw) e = hipMalloc((void**)&p->d_fw, p->T * 8);
  if (e == hipSuccess) e = hipMemcpy(p->d_fw, p->h_fw.data(), p->T * 8, hipMemcpyHostToDevice);
  {
    // density basis: the radial Laplacian of s^l (1 + s^(1/alpha))^(-p) C_n^lambda(xi)
    // is -K_nl s^(1/alpha - 2) (1 + s^(1/alpha))^(-2) times the same function,
    // K_nl = [n(n + 2 lambda) + p(p + 1)] / alpha^2, p = alpha (2l + 1)
    std::vector<double> kd((size_t)L1 * NW, 0.0);
    const double a = basis->alpha;
    for (int l = 0; l <= p->lmax; ++l)
      for (int n = 0; n <= p->nmax; ++n) {
        const double pp = a * (2.0 * l + 1.0), lam = pp + 0.5;
        const double K = (n * (n + 2.0 * lam) + pp * (pp + 1.0)) / (a * a);
        kd[(size_t)l * NW + n] = -K / (4.0 * M_PI * basis->G * basis->b * basis->b);
      }
    if (e == hipSuccess && !p->d_kden) e = hipMalloc((void**)&p->d_kden, kd.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(p->d_kden, kd.data(), kd.size() * 8, hipMemcpyHostToDevice);
  }
  {
    // the xi-derivative of the monic Gegenbauer basis in the same basis:
    // d C_n^lam / d xi = 2 lam C_{n-1}^(lam+1) = 2 sum_{k = n-1, n-3, ..} (k + lam) C_k^lam,
    // so for p_n = C_n^lam / kappa_n (kappa_n = 2^n (lam)_n / n!, the leading
    // coefficient) d p_n / d xi = sum_k D_nk p_k with D_nk = 2 (k + lam) kappa_k / kappa_n
    // for odd n - k > 0.  The matrix-core field pass needs the coefficients
    // W'_k = sum_n D_nk W_n = 2 (k + lam) kappa_k S_k, S_k = sum_{n = k+1, k+3, ..} W_n / kappa_n,
    // a suffix sum it forms per row; stored per degree: [l][0][n] = 1 / kappa_n,
    // [l][1][k] = 2 (k + lam) kappa_k.
    std::vector<double> dt((size_t)L1 * 2 * NW, 0.0);
    for (int l = 0; l <= p->lmax; ++l) {
      const double lam = (2.0 * l + 1.0) * basis->alpha + 0.5;
      double kap = 1.0;
      for (int n = 0; n <= p->nmaxc; ++n) {
        dt[((size_t)l * 2 + 0) * NW + n] = 1.0 / kap;
        dt[((size_t)l * 2 + 1) * NW + n] = 2.0 * (n + lam) * kap;
        kap *= 2.0 * (lam + n) / (n + 1.0);
      }
    }
    if (e == hipSuccess && !p->d_dtab) e = hipMalloc((void**)&p->d_dtab, dt.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(p->d_dtab, dt.data(), dt.size() * 8, hipMemcpyHostToDevice);
  }
  return e;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// gamma-pass launch geometry (one resident round, like the coefficient pass)
int gamma_units(const scf_plan* p, int64_t n, int64_t* stages) {
  if (n <= 0) {
    *stages = 0;
    return 0;
  }
  const int P = p->eng->gamma_stage_particles();
  *stages = (n + P - 1) / P;
  const int64_t cap = (int64_t)p->gamma_resident * p->num_cu;
  return (int)std::min<int64_t>(*stages, std::max<int64_t>(cap, 1));
}

// Adjoint workspace: the common layout (partials sized for both passes), the
// segment's positions X_k and force weights W_k (k = 0..nsteps), the gamma
// weights W', velocity and acceleration scratch, the Hessian-vector kernel's
// block sums of every kick and the per-kick host sums S_k.
struct AdjLayout {
  WsLayout L;
  size_t X, Wsv, Wp, V, A, hp, S, total;
  int64_t nblk;
  size_t wsz;
};

AdjLayout adj_layout(const scf_plan* p, int64_t n, int nsteps) {
  AdjLayout A;
  int64_t st;
  const int grows = gamma_units(p, n, &st) * p->eng->gamma_rows_per_unit();
  A.L = ws_layout(p, n, 1, grows);
  A.wsz = (size_t)(p->nmaxc + 1) * (p->lmax + 1) * (p->lmax + 1);
  A.nblk = (n + 255) / 256;
  const size_t rs = p->rs;
  size_t off = A.L.total;
  A.X = off;
  off += align256((size_t)(nsteps + 1) * 3 * n * rs);
  A.Wsv = off;
  off += align256((size_t)(nsteps + 1) * A.wsz * rs);
  A.Wp = off;
  off += align256(A.wsz * rs);
  A.V = off;
  off += align256((size_t)3 * n * rs);
  A.A = off;
  off += align256((size_t)3 * n * rs);
  A.hp = off;
  off += align256((size_t)(nsteps + 1) * std::max<int64_t>(A.nblk, 1) * 32 * rs);
  A.S = off;
  off += align256((size_t)(nsteps + 1) * 32 * sizeof(double));
  A.total = off;
  return A;
}

// gamma_t = sum_i mu_i . grad b_t(x_i), mu = c (ex, ey, ez), turned into the
// force weights W' of Eq. (total_potential) (the same scales as the forward
// coefficients)
template <typename R>
scf_status run_gamma(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                     const void* ex, const void* ey, const void* ez, double c, void* Wout, char* ws,
                     const WsLayout& L, hipStream_t s) {
  int64_t stages;
  const int units = gamma_units(p, n, &stages);
  CoefArgs<Dual<R>> ca;
  fill_coef_common(ca, p);
  ca.x = (const R*)x;
  ca.y = (const R*)y;
  ca.z = (const R*)z;
  ca.ex = (const R*)ex;
  ca.ey = (const R*)ey;
  ca.ez = (const R*)ez;
  ca.escale = R(c);
  ca.begin = 0;
  ca.n = n;
  ca.stages = stages;
  ca.nunits = units;
  ca.partials = (acc_t<Dual<R>>*)(ws + L.partials);
  {
    Timed t(p, s, K_ADJ);
    HIP_TRY(p->eng->launch_gamma(&ca, units, s));
  }
  const int rows = units * p->eng->gamma_rows_per_unit();
  return reduce_and_finalize(p, ws + L.partials, rows, nullptr, Wout, ws, L, s);
}

bool ptr_ok(const void* q) { return q != nullptr; }

// workspace regions are laid out at 256-byte offsets from its start
bool ws_aligned(const void* ws) { return ((uintptr_t)ws & 255) == 0; }

}  // namespace
