// libscf C ABI: plan management, basis tables, argument validation, the
// double-precision centre orbit (Sec. 2.1) and the launch sequences of the
// hot path.  Declared in include/scf.h.
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

namespace {

thread_local std::string g_last_error;

scf_status fail(scf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
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

// partial-sum rows of the current variant
int coef_rows(const scf_plan* p, int units) {
  return units * p->eng->rows_per_unit(p->coef_variant);
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
// coefficients (coef, nullable) and force weights W.  Few rows: one pass;
// otherwise chunk sums then their sum (two launches, fixed order either way).
constexpr int kSmallRows = 512;

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
  const int nb = coef_rows(p, units);
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

extern "C" {

int64_t scf_ncoef(int32_t nmax, int32_t lmax) {
  if (nmax < 0 || lmax < 0) return 0;
  return (int64_t)(nmax + 1) * (lmax + 1) * (lmax + 1);
}

const char* scf_status_string(scf_status st) {
  switch (st) {
    case SCF_OK: return "SCF_OK";
    case SCF_ERR_INVALID_ARG: return "SCF_ERR_INVALID_ARG";
    case SCF_ERR_UNSUPPORTED: return "SCF_ERR_UNSUPPORTED";
    case SCF_ERR_WORKSPACE: return "SCF_ERR_WORKSPACE";
    case SCF_ERR_NONFINITE: return "SCF_ERR_NONFINITE";
    case SCF_ERR_HIP: return "SCF_ERR_HIP";
  }
  return "unknown scf_status";
}

const char* scf_last_error(void) { return g_last_error.c_str(); }

const char* scf_kernel_name(int32_t kind) {
  if (kind < 0 || kind >= SCF_KERNEL_KINDS) return "unknown";
  return kKindNames[kind];
}

int32_t scf_plan_num_variants(const scf_plan* p) { return p ? p->eng->coef_variants() : 0; }

int32_t scf_plan_variant(const scf_plan* p) { return p ? p->coef_variant : -1; }

int32_t scf_plan_coef_units_div(const scf_plan* p) { return p ? p->coef_div : -1; }

scf_status scf_plan_set_coef_units_div(scf_plan* p, int32_t div) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (div != 1 && div != 2 && div != 4 && div != 8)
    return fail(SCF_ERR_INVALID_ARG, "div = %d is not 1, 2, 4 or 8", div);
  p->coef_div = div;
  return SCF_OK;
}

scf_status scf_plan_set_variant(scf_plan* p, int32_t v) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (v < 0 || v >= p->eng->coef_variants())
    return fail(SCF_ERR_INVALID_ARG, "variant %d outside [0, %d)", v, p->eng->coef_variants());
  p->coef_variant = v;
  return SCF_OK;
}

const char* scf_plan_describe(const scf_plan* p) { return p ? p->eng->describe() : ""; }

scf_status scf_autotune(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                        const void* m, void* ws, size_t ws_bytes, void* stream, double* best_ms) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n <= 0) return SCF_OK;
  if (!(x && y && z && m)) return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double* coef = (double*)((char*)ws + ws_layout(p, n, 1, 0).coef);
  const int saved = p->coef_variant;
  const bool prof = p->prof;
  p->prof = false;
  const int saved_div = p->coef_div;
  int best = saved, best_div = saved_div;
  float bms = 1e30f;
  for (int cand = 0; cand < 4 * p->eng->coef_variants(); ++cand) {
    const int v = cand / 4, div = 1 << (cand % 4);
    p->coef_variant = v;
    p->coef_div = div;
    float tot = 0.f;
    for (int rep = 0; rep < 4; ++rep) {
      HIP_TRY(hipEventRecord(e0, s));
      scf_status st = scf_coeffs(p, n, x, y, z, m, coef, ws, ws_bytes, stream);
      if (st != SCF_OK) {
        p->coef_variant = saved;
        p->coef_div = saved_div;
        p->prof = prof;
        return st;
      }
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tot += ms;  // the first repetition warms up
    }
    if (tot < bms) {
      bms = tot;
      best = v;
      best_div = div;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->coef_variant = best;
  p->coef_div = best_div;
  p->prof = prof;
  if (best_ms) *best_ms = bms / 3.0;
  return SCF_OK;
}

int32_t scf_plan_num_field_variants(const scf_plan* p) { return p ? p->eng->field_variants() : 0; }

int32_t scf_plan_field_variant(const scf_plan* p) { return p ? p->field_variant : -1; }

scf_status scf_plan_set_field_variant(scf_plan* p, int32_t v) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (v < 0 || v >= p->eng->field_variants())
    return fail(SCF_ERR_INVALID_ARG, "field variant %d outside [0, %d)", v, p->eng->field_variants());
  p->field_variant = v;
  return SCF_OK;
}

scf_status scf_autotune_field(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                              const void* m, void* ax, void* ay, void* az, void* ws,
                              size_t ws_bytes, void* stream, double* best_ms) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n <= 0) return SCF_OK;
  if (!(x && y && z && m && ax && ay && az))
    return fail(SCF_ERR_INVALID_ARG, "particle and output arrays must be non-null");
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L = ws_layout(p, n, 1, 0);
  char* w = (char*)ws;
  const bool prof = p->prof;
  p->prof = false;
  const int saved = p->field_variant;
  scf_status st = p->dtype == SCF_F32
                      ? run_coeffs<float>(p, n, x, y, z, m, (double*)(w + L.coef), w + L.W, w, L, s)
                      : run_coeffs<double>(p, n, x, y, z, m, (double*)(w + L.coef), w + L.W, w, L, s);
  if (st != SCF_OK) {
    p->prof = prof;
    return st;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = saved;
  float bms = 1e30f;
  for (int v = 0; v < p->eng->field_variants(); ++v) {
    p->field_variant = v;
    float tot = 0.f;
    for (int rep = 0; rep < 4; ++rep) {
      HIP_TRY(hipEventRecord(e0, s));
      if (p->dtype == SCF_F32) {
        HostParams<float> hp;
        fill_host_params(hp, nullptr);
        st = run_field<float>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax, ay,
                              az, nullptr, w + L.W, hp, nullptr, 0, 0.0, 0.0, s);
      } else {
        HostParams<double> hp;
        fill_host_params(hp, nullptr);
        st = run_field<double>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax,
                               ay, az, nullptr, w + L.W, hp, nullptr, 0, 0.0, 0.0, s);
      }
      if (st != SCF_OK) {
        p->field_variant = saved;
        p->prof = prof;
        return st;
      }
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tot += ms;
    }
    if (tot < bms) {
      bms = tot;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->field_variant = best;
  p->prof = prof;
  if (best_ms) *best_ms = bms / 3.0;
  return SCF_OK;
}

scf_status scf_power_spectrum(scf_plan* p, int32_t ncoefsets, const double* coef, double* power,
                              void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (ncoefsets < 0) return fail(SCF_ERR_INVALID_ARG, "ncoefsets = %d < 0", ncoefsets);
  if (ncoefsets == 0) return SCF_OK;
  if (!coef || !power) return fail(SCF_ERR_INVALID_ARG, "coef and power must be non-null");
  HIP_TRY(launch_power(coef, p->nmax, p->lmax, ncoefsets, power, (hipStream_t)stream));
  return SCF_OK;
}

scf_status scf_tidal_norm(const scf_host* host, const double* pos, double* norm) {
  if (!host || !pos || !norm) return fail(SCF_ERR_INVALID_ARG, "host, pos and norm must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  HostParams<double> hd;
  fill_host_params(hd, host);
  double s = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double e[3] = {c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0};
    double h[3];
    host_hess_vec<double>(hd, pos[0], pos[1], pos[2], e[0], e[1], e[2], h[0], h[1], h[2]);
    s += h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
  }
  *norm = std::sqrt(s);
  return SCF_OK;
}

scf_status scf_profile_enable(scf_plan* p, int32_t enable) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (enable && p->ev_pool.empty()) {
    p->ev_pool.resize(8192);
    for (auto& e : p->ev_pool) HIP_TRY(hipEventCreate(&e));
  }
  p->prof = enable != 0;
  return SCF_OK;
}

scf_status scf_profile_read(scf_plan* p, scf_kernel_time* out) {
  if (!p || !out) return fail(SCF_ERR_INVALID_ARG, "plan and out must be non-null");
  for (int k = 0; k < SCF_KERNEL_KINDS; ++k) out[k] = scf_kernel_time{k, 0, 0.0};
  for (const auto& r : p->recs) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    out[r.kind].count += 1;
    out[r.kind].total_ms += ms;
  }
  p->recs.clear();
  p->ev_next = 0;
  return SCF_OK;
}

scf_status scf_plan_create(scf_plan** out, const scf_basis* basis, int32_t dtype, uint32_t flags) {
  if (!out || !basis) return fail(SCF_ERR_INVALID_ARG, "plan and basis must be non-null");
  *out = nullptr;
  if (flags != 0) return fail(SCF_ERR_INVALID_ARG, "flags must be 0");
  if (dtype != SCF_F32 && dtype != SCF_F64) return fail(SCF_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (basis->nmax < 0 || basis->lmax < 0)
    return fail(SCF_ERR_INVALID_ARG, "nmax and lmax must be >= 0");
  if (!(basis->alpha > 0.0 && basis->alpha <= 1.0))
    return fail(SCF_ERR_UNSUPPORTED, "alpha = %g outside (0, 1]", basis->alpha);
  if (!(basis->b > 0.0) || !std::isfinite(basis->b)) return fail(SCF_ERR_INVALID_ARG, "b must be > 0");
  if (!(basis->G > 0.0) || !std::isfinite(basis->G)) return fail(SCF_ERR_INVALID_ARG, "G must be > 0");
  Engine* eng = find_engine(dtype, basis->nmax, basis->lmax);
  if (!eng)
    return fail(SCF_ERR_UNSUPPORTED, "no kernel for nmax = %d, lmax = %d", basis->nmax, basis->lmax);
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  scf_plan* p = new scf_plan();
  p->dtype = dtype;
  p->device = device;
  p->nmax = basis->nmax;
  p->lmax = basis->lmax;
  p->nmaxc = eng->nmaxc();
  p->T = scf_ncoef(basis->nmax, basis->lmax);
  p->eng = eng;
  p->rs = eng->real_size();
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess && prop.multiProcessorCount > 0)
      p->num_cu = prop.multiProcessorCount;
    for (int v = 0; v < eng->coef_variants() && v < 8; ++v) p->resident[v] = eng->max_resident_units(v);
    p->gamma_resident = eng->gamma_resident_units();
  }
  hipError_t e = fill_tables(p, basis);
  if (e != hipSuccess) {
    scf_plan_destroy(p);
    return fail(SCF_ERR_HIP, "plan allocation failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return SCF_OK;
}

void scf_plan_destroy(scf_plan* p) {
  if (!p) return;
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->ev_staging) {
    (void)hipEventSynchronize(p->ev_staging);
    (void)hipEventDestroy(p->ev_staging);
  }
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->gexec_g) (void)hipGraphExecDestroy(p->gexec_g);
  if (p->graph_g) (void)hipGraphDestroy(p->graph_g);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->h_tab) (void)hipHostFree(p->h_tab);
  if (p->h_meta) (void)hipHostFree(p->h_meta);
  if (p->d_beta_rad) (void)hipFree(p->d_beta_rad);
  if (p->d_beta_ang) (void)hipFree(p->d_beta_ang);
  if (p->d_kden) (void)hipFree(p->d_kden);
  if (p->d_cs) (void)hipFree(p->d_cs);
  if (p->d_fw) (void)hipFree(p->d_fw);
  delete p;
}

scf_status scf_workspace_size(const scf_plan* p, int64_t n, int32_t nclusters, size_t* bytes) {
  if (!p || !bytes) return fail(SCF_ERR_INVALID_ARG, "plan and bytes must be non-null");
  if (n < 0 || nclusters < 1) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nclusters >= 1");
  if (nclusters > (1 << 20)) return fail(SCF_ERR_INVALID_ARG, "nclusters = %d too large", nclusters);
  *bytes = std::max(plain_need(p, n), batch_layout(p, n, nclusters).total);
  return SCF_OK;
}

scf_status scf_coeffs(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                      const void* m, double* coef, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (!coef) return fail(SCF_ERR_INVALID_ARG, "coef is null");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(m)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(p, n, 1, 0);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (p->dtype == SCF_F32)
    return run_coeffs<float>(p, n, x, y, z, m, coef, w + L.W, w, L, s);
  return run_coeffs<double>(p, n, x, y, z, m, coef, w + L.W, w, L, s);
}

scf_status scf_forces(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                      const double* coef, const scf_host* host, const double* centre, void* ax,
                      void* ay, void* az, void* pot, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (!coef) return fail(SCF_ERR_INVALID_ARG, "coef is null");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(ax) && ptr_ok(ay) && ptr_ok(az)))
    return fail(SCF_ERR_INVALID_ARG, "particle and output arrays must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  const bool with_host = host && host->ncomp > 0;
  if (with_host && !centre) return fail(SCF_ERR_INVALID_ARG, "centre is null with a host potential");
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(p, n, 1, 0);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  {
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw, w + L.W, s));
  }
  double cen[6] = {0, 0, 0, 0, 0, 0};
  if (with_host) {
    HostParams<double> hd;
    fill_host_params(hd, host);
    double g[3];
    host_grad<double>(hd, centre[0], centre[1], centre[2], g[0], g[1], g[2]);
    for (int i = 0; i < 3; ++i) {
      cen[i] = centre[i];
      cen[3 + i] = g[i];
    }
  }
  if (p->dtype == SCF_F32) {
    HostParams<float> hp;
    fill_host_params(hp, with_host ? host : nullptr);
    return run_field<float>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax, ay,
                            az, pot, w + L.W, hp, cen, 0, 0.0, 0.0, s);
  }
  HostParams<double> hp;
  fill_host_params(hp, with_host ? host : nullptr);
  return run_field<double>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax, ay, az,
                           pot, w + L.W, hp, cen, 0, 0.0, 0.0, s);
}

scf_status scf_step(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy, void* vz,
                    const void* m, void* ax, void* ay, void* az, uint32_t step_flags,
                    const scf_host* host, double* centre, double dt, int32_t nsteps,
                    double* coef_last, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0 || nsteps < 0) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nsteps >= 0");
  if (!std::isfinite(dt)) return fail(SCF_ERR_INVALID_ARG, "dt is not finite");
  if (step_flags & ~SCF_STEP_ACC_VALID) return fail(SCF_ERR_INVALID_ARG, "unknown step flags");
  if (!centre) return fail(SCF_ERR_INVALID_ARG, "centre is null");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(ax) && ptr_ok(ay) && ptr_ok(az)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(p, n, 1, 0);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool with_host = host && host->ncomp > 0;
  HostParams<double> hd;
  fill_host_params(hd, with_host ? host : nullptr);
  // centre orbit on the host, double precision, same leapfrog
  double R[3] = {centre[0], centre[1], centre[2]}, V[3] = {centre[3], centre[4], centre[5]};
  auto cen_row = [&](double* row) {
    double g[3] = {0, 0, 0};
    if (with_host) host_grad<double>(hd, R[0], R[1], R[2], g[0], g[1], g[2]);
    for (int i = 0; i < 3; ++i) {
      row[i] = R[i];
      row[3 + i] = g[i];
    }
  };
  double* coef_int = (double*)(w + L.coef);
  void* W = w + L.W;
  const double h = 0.5 * dt;
  auto go = [&](auto tag) -> scf_status {
    using Rt = decltype(tag);
    HostParams<Rt> hp;
    fill_host_params(hp, with_host ? host : nullptr);
    double row[6];
    scf_status st;
    if (!(step_flags & SCF_STEP_ACC_VALID) || nsteps == 0) {
      // a(x0) from the particles themselves
      cen_row(row);
      st = run_coeffs<Rt>(p, n, x, y, z, m, nsteps == 0 && coef_last ? coef_last : coef_int, W, w, L, s);
      if (st != SCF_OK) return st;
      st = run_field<Rt>(p, n, x, y, z, vx, vy, vz, ax, ay, az, nullptr, W, hp, row, 0, 0.0, 0.0, s);
      if (st != SCF_OK) return st;
    }
    if (nsteps == 0) return SCF_OK;
    // opening half kick and drift with the stored accelerations
    {
      Timed t(p, s, K_KICK);
      HIP_TRY(launch_kick_drift(p->dtype, n, x, y, z, vx, vy, vz, ax, ay, az, h, dt, s));
    }
    double gc[3];
    centre_accel(hd, R, gc);
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
    for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    for (int k = 1; k <= nsteps; ++k) {
      const bool last = k == nsteps;
      cen_row(row);
      st = run_coeffs<Rt>(p, n, x, y, z, m, last && coef_last ? coef_last : coef_int, W, w, L, s);
      if (st != SCF_OK) return st;
      // closing half kick of step k merged with the opening half kick of
      // step k+1, then the drift of step k+1
      st = run_field<Rt>(p, n, x, y, z, vx, vy, vz, ax, ay, az, nullptr, W, hp, row, 1,
                         last ? h : dt, last ? 0.0 : dt, s);
      if (st != SCF_OK) return st;
      centre_accel(hd, R, gc);
      for (int i = 0; i < 3; ++i) V[i] += (last ? h : dt) * gc[i];
      if (!last)
        for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    }
    return SCF_OK;
  };
  scf_status st = p->dtype == SCF_F32 ? go(float(0)) : go(double(0));
  if (st != SCF_OK) return st;
  for (int i = 0; i < 3; ++i) {
    centre[i] = R[i];
    centre[3 + i] = V[i];
  }
  return SCF_OK;
}

scf_status scf_step_batched(scf_plan* p, int32_t nclusters, const int64_t* offsets, void* x, void* y,
                            void* z, void* vx, void* vy, void* vz, const void* m, void* ax,
                            void* ay, void* az, uint32_t step_flags, const scf_host* host,
                            double* centres, double dt, int32_t nsteps, double* coef_last, void* ws,
                            size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (nclusters < 1 || nsteps < 0) return fail(SCF_ERR_INVALID_ARG, "need nclusters >= 1 and nsteps >= 0");
  if (!offsets || !centres) return fail(SCF_ERR_INVALID_ARG, "offsets and centres must be non-null");
  if (!std::isfinite(dt)) return fail(SCF_ERR_INVALID_ARG, "dt is not finite");
  if (step_flags & ~(SCF_STEP_ACC_VALID | SCF_STEP_NO_GRAPH | SCF_STEP_GRAPH))
    return fail(SCF_ERR_INVALID_ARG, "unknown step flags");
  if (offsets[0] != 0) return fail(SCF_ERR_INVALID_ARG, "offsets[0] must be 0");
  for (int c = 0; c < nclusters; ++c)
    if (offsets[c + 1] < offsets[c])
      return fail(SCF_ERR_INVALID_ARG, "offsets must be non-decreasing (cluster %d)", c);
  const int64_t n = offsets[nclusters];
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(ax) && ptr_ok(ay) && ptr_ok(az)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  const int ncl = nclusters;
  const BatchLayout B = batch_layout(p, n, ncl);
  if (!ws || ws_bytes < B.total)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", B.total, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool with_host = host && host->ncomp > 0;
  HostParams<double> hd;
  fill_host_params(hd, with_host ? host : nullptr);
  const bool acc_valid = (step_flags & SCF_STEP_ACC_VALID) && nsteps > 0;
  const bool use_graph = (step_flags & SCF_STEP_GRAPH) && !(step_flags & SCF_STEP_NO_GRAPH);

  // ---- work lists (host), staged in pinned memory --------------------------
  const int v = p->coef_variant;
  const int P = p->eng->stage_particles(v);
  const int rpu = p->eng->rows_per_unit(v);
  const int cap = std::max(1, p->resident[v] * p->num_cu);
  std::vector<int64_t> stg(ncl);
  int64_t st_tot = 0;
  for (int c = 0; c < ncl; ++c) {
    stg[c] = (offsets[c + 1] - offsets[c] + P - 1) / P;
    st_tot += stg[c];
  }
  std::vector<int64_t> sb, se;
  std::vector<int32_t> slot, rows(ncl + 1, 0), bcl;
  std::vector<int64_t> bb, be;
  for (int c = 0; c < ncl; ++c) {
    rows[c] = (int32_t)(sb.size() * rpu);
    if (stg[c] == 0) continue;
    int64_t uc = (int64_t)((double)cap * (double)stg[c] / (double)st_tot);
    uc = std::max<int64_t>(1, std::min<int64_t>(uc, stg[c]));
    for (int64_t u = 0; u < uc; ++u) {
      const int64_t s0 = stg[c] * u / uc, s1 = stg[c] * (u + 1) / uc;
      sb.push_back(offsets[c] + s0 * P);
      se.push_back(std::min(offsets[c] + s1 * P, offsets[c + 1]));
      slot.push_back((int32_t)slot.size());
    }
  }
  rows[ncl] = (int32_t)(sb.size() * rpu);
  for (int c = 0; c < ncl; ++c)
    for (int64_t b0 = offsets[c]; b0 < offsets[c + 1]; b0 += 256) {
      bcl.push_back(c);
      bb.push_back(b0);
      be.push_back(std::min(b0 + 256, offsets[c + 1]));
    }
  const int U = (int)sb.size();
  const int64_t nblk = (int64_t)bcl.size();
  if (U > B.max_units || nblk > B.max_blocks)
    return fail(SCF_ERR_INVALID_ARG, "internal: work list larger than its workspace");

  // ---- centre orbit (host, double): rows k = 0..nsteps of R, grad psi_host(R)
  const int64_t nrows = (int64_t)nsteps + 1;
  const size_t tab_elems = (size_t)nrows * ncl * 9;
  const size_t meta_bytes = (size_t)U * 20 + (size_t)(ncl + 1) * 4 + (size_t)nblk * 20;
  if (p->staging_pending) {
    HIP_TRY(hipEventSynchronize(p->ev_staging));
    p->staging_pending = false;
  }
  if (p->h_tab_cap < tab_elems) {
    if (p->h_tab) HIP_TRY(hipHostFree(p->h_tab));
    p->h_tab = nullptr;
    p->h_tab_cap = 0;
    HIP_TRY(hipHostMalloc((void**)&p->h_tab, tab_elems * sizeof(double), hipHostMallocDefault));
    p->h_tab_cap = tab_elems;
  }
  if (p->h_meta_cap < meta_bytes) {
    if (p->h_meta) HIP_TRY(hipHostFree(p->h_meta));
    p->h_meta = nullptr;
    p->h_meta_cap = 0;
    HIP_TRY(hipHostMalloc((void**)&p->h_meta, meta_bytes, hipHostMallocDefault));
    p->h_meta_cap = meta_bytes;
  }
  if (!p->ev_staging) HIP_TRY(hipEventCreateWithFlags(&p->ev_staging, hipEventDisableTiming));
  const double h = 0.5 * dt;
  std::vector<double> cnew(6 * (size_t)ncl);
  for (int c = 0; c < ncl; ++c) {
    double R[3] = {centres[6 * c], centres[6 * c + 1], centres[6 * c + 2]};
    double V[3] = {centres[6 * c + 3], centres[6 * c + 4], centres[6 * c + 5]};
    auto put_row = [&](int64_t k) {
      double g[3] = {0, 0, 0};
      if (with_host) host_grad<double>(hd, R[0], R[1], R[2], g[0], g[1], g[2]);
      double* row = p->h_tab + ((size_t)k * ncl + c) * 9;
      for (int i = 0; i < 3; ++i) {
        row[i] = R[i];
        row[3 + i] = g[i];
        row[6 + i] = 0.0;
      }
    };
    put_row(0);
    if (nsteps > 0) {
      double gc[3];
      centre_accel(hd, R, gc);
      for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
      for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
      for (int k = 1; k <= nsteps; ++k) {
        const bool last = k == nsteps;
        put_row(k);
        centre_accel(hd, R, gc);
        for (int i = 0; i < 3; ++i) V[i] += (last ? h : dt) * gc[i];
        if (!last)
          for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
      }
    }
    for (int i = 0; i < 3; ++i) {
      cnew[6 * c + i] = R[i];
      cnew[6 * c + 3 + i] = V[i];
    }
  }
  {
    char* q = p->h_meta;
    auto put = [&](const void* src, size_t bytes) {
      if (bytes) std::memcpy(q, src, bytes);
      q += bytes;
    };
    put(sb.data(), (size_t)U * 8);
    put(se.data(), (size_t)U * 8);
    put(slot.data(), (size_t)U * 4);
    put(rows.data(), (size_t)(ncl + 1) * 4);
    put(bcl.data(), (size_t)nblk * 4);
    put(bb.data(), (size_t)nblk * 8);
    put(be.data(), (size_t)nblk * 8);
    const char* q0 = p->h_meta;
    size_t o = 0;
    auto up = [&](size_t dst, size_t bytes) -> hipError_t {
      hipError_t e = bytes ? hipMemcpyAsync(w + dst, q0 + o, bytes, hipMemcpyHostToDevice, s)
                           : hipSuccess;
      o += bytes;
      return e;
    };
    HIP_TRY(up(B.seg_begin, (size_t)U * 8));
    HIP_TRY(up(B.seg_end, (size_t)U * 8));
    HIP_TRY(up(B.seg_slot, (size_t)U * 4));
    HIP_TRY(up(B.rows, (size_t)(ncl + 1) * 4));
    HIP_TRY(up(B.blk_cluster, (size_t)nblk * 4));
    HIP_TRY(up(B.blk_begin, (size_t)nblk * 8));
    HIP_TRY(up(B.blk_end, (size_t)nblk * 8));
  }
  // uploads rows [k0, k0 + kCentreRows) of the centre table and restarts the
  // device row counter
  auto upload_rows = [&](int64_t k0) -> scf_status {
    const int64_t k1 = std::min<int64_t>(k0 + kCentreRows, nrows);
    HIP_TRY(hipMemcpyAsync(w + B.tab, p->h_tab + (size_t)k0 * ncl * 9,
                           (size_t)(k1 - k0) * ncl * 9 * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_set_int((int*)(w + B.ctr), 0, s));
    return SCF_OK;
  };

  const int nch = std::max(1, std::min(kReduceChunks, rows[ncl] > 0 ? (rows[ncl] + ncl - 1) / ncl : 1));
  const int64_t W_stride = (int64_t)(p->nmaxc + 1) * (p->lmax + 1) * (p->lmax + 1);
  double* coef_int = (double*)(w + B.L.coef);
  void* Wb = w + B.L.W;

  auto go = [&](auto tag) -> scf_status {
    using Rt = decltype(tag);
    HostParams<Rt> hp;
    fill_host_params(hp, with_host ? host : nullptr);
    CoefArgs<Rt> ca;
    fill_coef_common(ca, p);
    ca.x = (const Rt*)x;
    ca.y = (const Rt*)y;
    ca.z = (const Rt*)z;
    ca.m = (const Rt*)m;
    ca.seg_begin = (const int64_t*)(w + B.seg_begin);
    ca.seg_end = (const int64_t*)(w + B.seg_end);
    ca.seg_slot = (const int32_t*)(w + B.seg_slot);
    ca.n = n;
    ca.nunits = U;
    ca.partials = (Rt*)(w + B.L.partials);
    ForceArgs<Rt> fa;
    fill_force_common(fa, p);
    fa.x = (Rt*)x;
    fa.y = (Rt*)y;
    fa.z = (Rt*)z;
    fa.xo = (Rt*)x;
    fa.yo = (Rt*)y;
    fa.zo = (Rt*)z;
    fa.vx = (Rt*)vx;
    fa.vy = (Rt*)vy;
    fa.vz = (Rt*)vz;
    fa.ax = (Rt*)ax;
    fa.ay = (Rt*)ay;
    fa.az = (Rt*)az;
    fa.W = (const Rt*)Wb;
    fa.n = n;
    fa.host = hp;
    fa.blk_cluster = (const int32_t*)(w + B.blk_cluster);
    fa.blk_begin = (const int64_t*)(w + B.blk_begin);
    fa.blk_end = (const int64_t*)(w + B.blk_end);
    fa.centre_tab = (const double*)(w + B.cur);
    fa.W_stride = W_stride;
    // one step's kernels: coefficients of every cluster, their reduction and
    // finalisation (which also selects this step's centre rows), then the
    // fused field + kick (+ drift) pass
    auto enqueue = [&](hipStream_t q, double kick, double drift, double* coef) -> scf_status {
      {
        Timed t(p, q, K_BATCH_COEF);
        HIP_TRY(p->eng->launch_coef(&ca, U, v, q));
      }
      HIP_TRY(launch_reduce_batched(p->dtype, ca.partials, (const int32_t*)(w + B.rows), ncl,
                                    (int)p->T, nch, (double*)(w + B.L.red1), q));
      HIP_TRY(launch_finalize_batched(p->dtype, (const double*)(w + B.L.red1), nch, (int)p->T,
                                      p->nmax, p->lmax, p->nmaxc, p->d_cs, p->d_fw, coef, Wb,
                                      W_stride, (const double*)(w + B.tab), ncl,
                                      (double*)(w + B.cur), (int*)(w + B.ctr), q));
      ForceArgs<Rt> f2 = fa;
      f2.kick = Rt(kick);
      f2.drift = Rt(drift);
      HIP_TRY(p->eng->launch_force(&f2, nblk, 1, p->field_variant, q));
      return SCF_OK;
    };
    scf_status st = upload_rows(acc_valid ? 1 : 0);
    if (st != SCF_OK) return st;
    int64_t chunk0 = acc_valid ? 1 : 0;
    if (!acc_valid) {
      // a(x0): field pass with no kick and no drift (v is rewritten unchanged)
      st = enqueue(s, 0.0, 0.0, nsteps == 0 && coef_last ? coef_last : coef_int);
      if (st != SCF_OK) return st;
    }
    if (nsteps == 0) return SCF_OK;
    {
      Timed t(p, s, K_KICK);
      HIP_TRY(launch_kick_drift(p->dtype, n, x, y, z, vx, vy, vz, ax, ay, az, h, dt, s));
    }
    // the graph of one middle step (kick dt, drift dt), captured once per
    // distinct argument set on the plan's capture stream
    if (use_graph && nsteps > 1) {
      std::vector<char> key;
      auto add = [&](const void* q, size_t b) {
        key.insert(key.end(), (const char*)q, (const char*)q + b);
      };
      add(&ca, sizeof(ca));
      add(&fa, sizeof(fa));
      add(&dt, sizeof(dt));
      add(&U, sizeof(U));
      add(&nblk, sizeof(nblk));
      add(&nch, sizeof(nch));
      add(&v, sizeof(v));
      add(&p->field_variant, sizeof(p->field_variant));
      add(&coef_int, sizeof(coef_int));
      if (!p->gexec || key != p->gkey) {
        if (p->gexec) HIP_TRY(hipGraphExecDestroy(p->gexec));
        if (p->graph) HIP_TRY(hipGraphDestroy(p->graph));
        if (p->gexec_g) HIP_TRY(hipGraphExecDestroy(p->gexec_g));
        if (p->graph_g) HIP_TRY(hipGraphDestroy(p->graph_g));
        p->gexec = nullptr;
        p->graph = nullptr;
        p->gexec_g = nullptr;
        p->graph_g = nullptr;
        p->gkey.clear();
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        // one middle step, and kGraphSteps of them in a row (the centre rows
        // advance on the device, so consecutive steps are the same nodes)
        for (int rep : {1, kGraphSteps}) {
          HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
          scf_status cs = SCF_OK;
          for (int r = 0; r < rep && cs == SCF_OK; ++r) cs = enqueue(p->cap_stream, dt, dt, coef_int);
          hipGraph_t g = nullptr;
          hipError_t ee = hipStreamEndCapture(p->cap_stream, &g);
          if (cs != SCF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
          }
          HIP_TRY(ee);
          hipGraphExec_t ge = nullptr;
          hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          if (ie != hipSuccess) {
            (void)hipGraphDestroy(g);
            HIP_TRY(ie);
          }
          if (rep == 1) {
            p->graph = g;
            p->gexec = ge;
          } else {
            p->graph_g = g;
            p->gexec_g = ge;
          }
        }
        p->gkey = key;
        p->graph_captures += 1;
      }
    }
    for (int64_t k = 1; k <= nsteps;) {
      if (k - chunk0 >= kCentreRows) {
        chunk0 = k;
        st = upload_rows(k);
        if (st != SCF_OK) return st;
      }
      const bool last = k == nsteps;
      // a run of kGraphSteps middle steps inside the current centre chunk
      const bool group = use_graph && k + kGraphSteps - 1 < nsteps &&
                         k + kGraphSteps - 1 - chunk0 < kCentreRows;
      if (group) {
        Timed t(p, s, K_BATCH_FIELD);
        HIP_TRY(hipGraphLaunch(p->gexec_g, s));
        k += kGraphSteps;
        continue;
      }
      if (!last && use_graph) {
        Timed t(p, s, K_BATCH_FIELD);
        HIP_TRY(hipGraphLaunch(p->gexec, s));
      } else {
        st = enqueue(s, last ? h : dt, last ? 0.0 : dt, last && coef_last ? coef_last : coef_int);
        if (st != SCF_OK) return st;
      }
      ++k;
    }
    return SCF_OK;
  };
  scf_status st = p->dtype == SCF_F32 ? go(float(0)) : go(double(0));
  HIP_TRY(hipEventRecord(p->ev_staging, s));
  p->staging_pending = true;
  if (st == SCF_OK) std::copy(cnew.begin(), cnew.end(), centres);
  return st;
}

int32_t scf_plan_graph_captures(const scf_plan* p) { return p ? p->graph_captures : 0; }

scf_status scf_adjoint_workspace_size(const scf_plan* p, int64_t n, int32_t nsteps, size_t* bytes) {
  if (!p || !bytes) return fail(SCF_ERR_INVALID_ARG, "plan and bytes must be non-null");
  if (n < 0 || nsteps < 0) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nsteps >= 0");
  *bytes = std::max(plain_need(p, n), adj_layout(p, n, nsteps).total);
  return SCF_OK;
}

scf_status scf_step_adjoint(scf_plan* p, int64_t n, const void* x0, const void* y0, const void* z0,
                            const void* vx0, const void* vy0, const void* vz0, const void* m,
                            const scf_host* host, const double* centre0, double dt, int32_t nsteps,
                            void* const* lam, double* lam_centre, double* grad_host, void* ws,
                            size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0 || nsteps < 0) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nsteps >= 0");
  if (!std::isfinite(dt)) return fail(SCF_ERR_INVALID_ARG, "dt is not finite");
  if (!centre0 || !lam_centre || !lam) return fail(SCF_ERR_INVALID_ARG, "centre0, lam and lam_centre must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  const bool with_host = host && host->ncomp > 0;
  if (with_host && !grad_host) return fail(SCF_ERR_INVALID_ARG, "grad_host is null with a host potential");
  if (n > 0) {
    if (!(ptr_ok(x0) && ptr_ok(y0) && ptr_ok(z0) && ptr_ok(vx0) && ptr_ok(vy0) && ptr_ok(vz0) &&
          ptr_ok(m)))
      return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
    for (int q = 0; q < 6; ++q)
      if (!lam[q]) return fail(SCF_ERR_INVALID_ARG, "lam[%d] is null", q);
  }
  const AdjLayout A = adj_layout(p, n, nsteps);
  if (!ws || ws_bytes < A.total)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", A.total, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (nsteps == 0) return SCF_OK;  // the identity map
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const size_t rs = p->rs;
  HostParams<double> hd;
  fill_host_params(hd, with_host ? host : nullptr);
  const double h = 0.5 * dt;
  // centre orbit (host, double): R_k at the kick times k = 0..nsteps
  std::vector<double> Rk(3 * (size_t)(nsteps + 1));
  {
    double R[3] = {centre0[0], centre0[1], centre0[2]}, V[3] = {centre0[3], centre0[4], centre0[5]};
    for (int i = 0; i < 3; ++i) Rk[i] = R[i];
    double gc[3];
    centre_accel(hd, R, gc);
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
    for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    for (int k = 1; k <= nsteps; ++k) {
      for (int i = 0; i < 3; ++i) Rk[3 * k + i] = R[i];
      if (k == nsteps) break;
      centre_accel(hd, R, gc);
      for (int i = 0; i < 3; ++i) V[i] += dt * gc[i];
      for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    }
  }
  auto row_of = [&](int k, double* row) {
    double g[3] = {0, 0, 0};
    if (with_host) host_grad<double>(hd, Rk[3 * k], Rk[3 * k + 1], Rk[3 * k + 2], g[0], g[1], g[2]);
    for (int i = 0; i < 3; ++i) {
      row[i] = Rk[3 * k + i];
      row[3 + i] = g[i];
    }
  };
  std::vector<double> S((size_t)(nsteps + 1) * 32, 0.0);
  auto Xk = [&](int k, int c) -> char* { return w + A.X + ((size_t)k * 3 + c) * n * rs; };
  auto Wk = [&](int k) -> char* { return w + A.Wsv + (size_t)k * A.wsz * rs; };
  char* Vb[3] = {w + A.V, w + A.V + n * rs, w + A.V + 2 * n * rs};
  char* Ab[3] = {w + A.A, w + A.A + n * rs, w + A.A + 2 * n * rs};

  auto go = [&](auto tag) -> scf_status {
    using Rt = decltype(tag);
    HostParams<Rt> hp, none;
    fill_host_params(hp, with_host ? host : nullptr);
    fill_host_params(none, nullptr);
    double row[6];
    scf_status st;
    if (n > 0) {
      // ---- forward recompute of the segment, keeping X_k and W_k --------------
      const void* src[6] = {x0, y0, z0, vx0, vy0, vz0};
      for (int c = 0; c < 3; ++c) {
        HIP_TRY(hipMemcpyAsync(Xk(0, c), src[c], n * rs, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(Vb[c], src[3 + c], n * rs, hipMemcpyDeviceToDevice, s));
      }
      row_of(0, row);
      st = run_coeffs<Rt>(p, n, Xk(0, 0), Xk(0, 1), Xk(0, 2), m, (double*)(w + A.L.coef), Wk(0), w,
                          A.L, s);
      if (st != SCF_OK) return st;
      st = run_field<Rt>(p, n, Xk(0, 0), Xk(0, 1), Xk(0, 2), Vb[0], Vb[1], Vb[2], Ab[0], Ab[1],
                         Ab[2], nullptr, Wk(0), hp, row, 0, 0.0, 0.0, s);
      if (st != SCF_OK) return st;
      for (int c = 0; c < 3; ++c)
        HIP_TRY(hipMemcpyAsync(Xk(1, c), Xk(0, c), n * rs, hipMemcpyDeviceToDevice, s));
      HIP_TRY(launch_kick_drift(p->dtype, n, Xk(1, 0), Xk(1, 1), Xk(1, 2), Vb[0], Vb[1], Vb[2], Ab[0],
                                Ab[1], Ab[2], h, dt, s));
      for (int k = 1; k <= nsteps; ++k) {
        st = run_coeffs<Rt>(p, n, Xk(k, 0), Xk(k, 1), Xk(k, 2), m, (double*)(w + A.L.coef), Wk(k),
                            w, A.L, s);
        if (st != SCF_OK) return st;
        if (k == nsteps) break;
        row_of(k, row);
        st = run_field<Rt>(p, n, Xk(k, 0), Xk(k, 1), Xk(k, 2), Vb[0], Vb[1], Vb[2], Ab[0], Ab[1],
                           Ab[2], nullptr, Wk(k), hp, row, 1, dt, dt, s, Xk(k + 1, 0),
                           Xk(k + 1, 1), Xk(k + 1, 2));
        if (st != SCF_OK) return st;
      }
      // ---- reverse sweep over the kicks k = nsteps..0 ---------------------------
      for (int k = nsteps; k >= 0; --k) {
        const double c = (k == nsteps || k == 0) ? h : dt;
        st = run_gamma<Rt>(p, n, Xk(k, 0), Xk(k, 1), Xk(k, 2), lam[3], lam[4], lam[5], c,
                           w + A.Wp, w, A.L, s);
        if (st != SCF_OK) return st;
        HvpArgs<Rt> ha;
        std::memset(&ha, 0, sizeof(ha));
        ha.x = (const Rt*)Xk(k, 0);
        ha.y = (const Rt*)Xk(k, 1);
        ha.z = (const Rt*)Xk(k, 2);
        ha.lvx = (const Rt*)lam[3];
        ha.lvy = (const Rt*)lam[4];
        ha.lvz = (const Rt*)lam[5];
        ha.c = Rt(c);
        ha.lx = (Rt*)lam[0];
        ha.ly = (Rt*)lam[1];
        ha.lz = (Rt*)lam[2];
        ha.W = (const Rt*)Wk(k);
        ha.beta_rad = (const Rt*)p->d_beta_rad;
        ha.beta_ang = (const Rt*)p->d_beta_ang;
        ha.n = n;
        ha.binv = Rt(1.0 / p->basis.b);
        ha.alpha = Rt(p->basis.alpha);
        ha.inv_alpha = Rt(1.0 / p->basis.alpha);
        ha.amode = p->amode;
        ha.host = hp;
        ha.cx = Rt(Rk[3 * k]);
        ha.cy = Rt(Rk[3 * k + 1]);
        ha.cz = Rt(Rk[3 * k + 2]);
        ha.partials = (Rt*)(w + A.hp) + (size_t)k * A.nblk * 32;
        {
          Timed t(p, s, K_ADJ);
          HIP_TRY(p->eng->launch_hvp(&ha, A.nblk, s));
        }
        // coefficient part: lambda_x += m a' with a' = -grad sum_t W'_t b_t at X_k,
        // then the reverse drift lambda_v += dt lambda_x (for k > 0)
        st = run_field<Rt>(p, n, Xk(k, 0), Xk(k, 1), Xk(k, 2), lam[3], lam[4], lam[5], lam[0],
                           lam[1], lam[2], nullptr, w + A.Wp, none, nullptr, 2, 0.0,
                           k > 0 ? dt : 0.0, s, nullptr, nullptr, nullptr, m);
        if (st != SCF_OK) return st;
      }
      if (with_host) {
        HIP_TRY(launch_adj_reduce(p->dtype, w + A.hp, A.nblk, nsteps + 1, (double*)(w + A.S), s));
        HIP_TRY(hipMemcpyAsync(S.data(), w + A.S, S.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
      }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return SCF_OK;
  };
  scf_status st = p->dtype == SCF_F32 ? go(float(0)) : go(double(0));
  if (st != SCF_OK) return st;
  // ---- centre cotangents and host-parameter gradient (host, double) ----------
  double* lR = lam_centre;
  double* lV = lam_centre + 3;
  const int nc = with_host ? host->ncomp : 0;
  for (int k = nsteps; k >= 0; --k) {
    const double c = (k == nsteps || k == 0) ? h : dt;
    if (with_host) {
      const double* Sk = S.data() + 32 * (size_t)k;
      const double* R = &Rk[3 * k];
      double hs[3], hn[3];
      const double nu[3] = {c * lV[0], c * lV[1], c * lV[2]};
      // particles: sum_i [-Hess(R + x_i) + Hess(R)] mu_i; the centre's own kick
      host_hess_vec<double>(hd, R[0], R[1], R[2], Sk[3], Sk[4], Sk[5], hs[0], hs[1], hs[2]);
      host_hess_vec<double>(hd, R[0], R[1], R[2], nu[0], nu[1], nu[2], hn[0], hn[1], hn[2]);
      for (int i = 0; i < 3; ++i) lR[i] += Sk[i] + hs[i] - hn[i];
      for (int cc = 0; cc < nc; ++cc)
        for (int kk = 0; kk < 3; ++kk)
          grad_host[3 * cc + kk] +=
              Sk[6 + 3 * cc + kk] +
              host_dgrad_dparam_dot<double>(hd, cc, kk, R[0], R[1], R[2], Sk[3], Sk[4], Sk[5]) -
              host_dgrad_dparam_dot<double>(hd, cc, kk, R[0], R[1], R[2], nu[0], nu[1], nu[2]);
    }
    if (k > 0)
      for (int i = 0; i < 3; ++i) lV[i] += dt * lR[i];
  }
  return SCF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// refresh cadence (Sec. 2.2)
// ---------------------------------------------------------------------------
namespace {

// Cadence workspace: the common layout, then the potential, the keys, the
// bound flags, the selection state, block sums and offsets, an acceleration
// scratch, the new weights, the compacted changed particles, the orbit
// samples and two coefficient vectors.
struct CadLayout {
  WsLayout L;
  size_t pot, keys, bound, state, mpart, cnt, off, total, acc, wnew, compact, snaps, ctmp, mom,
      res, all;
};

CadLayout cad_layout(const scf_plan* p, int64_t n, int ns_max) {
  CadLayout C;
  C.L = ws_layout(p, n, 1, 0);
  const size_t rs = p->rs, nn = (size_t)std::max<int64_t>(n, 1);
  const size_t nblk = (nn + 255) / 256;
  size_t off = C.L.total;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  C.pot = take(nn * rs);
  C.keys = take(nn * 8);
  C.bound = take(nn);
  C.state = take(sizeof(SelectState));
  C.mpart = take(nblk * 8);
  C.cnt = take(nblk * 4);
  C.off = take(nblk * 8);
  C.total = take(8);
  C.acc = take(3 * nn * rs);
  C.wnew = take(nn * rs);
  C.compact = take((3 * (size_t)ns_max + 1) * nn * rs);
  C.snaps = take(3 * (size_t)ns_max * nn * rs);
  C.ctmp = take((size_t)p->T * 8);
  C.mom = take(nblk * 4 * 8);
  C.res = take(4 * 8);
  C.all = off;
  return C;
}

double tidal_norm_host(const HostParams<double>& hd, const double* R) {
  double s = 0.0;
  for (int c = 0; c < 3; ++c) {
    double h[3];
    host_hess_vec<double>(hd, R[0], R[1], R[2], c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0,
                          c == 2 ? 1.0 : 0.0, h[0], h[1], h[2]);
    s += h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
  }
  return std::sqrt(s);
}

// Leapfrog in the frozen potential of the force weights W; the centre (R, V)
// follows the host-only leapfrog in double precision.
template <typename R>
scf_status frozen_steps(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                        void* vz, void* ax, void* ay, void* az, bool acc_valid, const void* W,
                        const HostParams<double>& hd, bool with_host, double* Rc, double* Vc,
                        double dt, int nsteps, hipStream_t s) {
  HostParams<R> hp;
  std::memset(&hp, 0, sizeof(hp));
  if (with_host) {
    hp.ncomp = hd.ncomp;
    hp.G = R(hd.G);
    for (int c = 0; c < hd.ncomp; ++c) {
      hp.kind[c] = hd.kind[c];
      for (int k = 0; k < 3; ++k) hp.p[c][k] = R(hd.p[c][k]);
    }
  }
  auto cen_row = [&](double* row) {
    double g[3] = {0, 0, 0};
    if (with_host) host_grad<double>(hd, Rc[0], Rc[1], Rc[2], g[0], g[1], g[2]);
    for (int i = 0; i < 3; ++i) {
      row[i] = Rc[i];
      row[3 + i] = g[i];
    }
  };
  double row[6];
  scf_status st;
  if (!acc_valid || nsteps == 0) {
    cen_row(row);
    st = run_field<R>(p, n, x, y, z, vx, vy, vz, ax, ay, az, nullptr, W, hp, row, 0, 0.0, 0.0, s);
    if (st != SCF_OK) return st;
  }
  if (nsteps == 0) return SCF_OK;
  const double h = 0.5 * dt;
  {
    Timed t(p, s, K_KICK);
    HIP_TRY(launch_kick_drift(p->dtype, n, x, y, z, vx, vy, vz, ax, ay, az, h, dt, s));
  }
  double gc[3];
  centre_accel(hd, Rc, gc);
  for (int i = 0; i < 3; ++i) Vc[i] += h * gc[i];
  for (int i = 0; i < 3; ++i) Rc[i] += dt * Vc[i];
  for (int k = 1; k <= nsteps; ++k) {
    const bool last = k == nsteps;
    cen_row(row);
    // closing half kick of step k merged with the opening half kick of step
    // k+1, then the drift of step k+1; a at the new positions into ax, ay, az
    st = run_field<R>(p, n, x, y, z, vx, vy, vz, ax, ay, az, nullptr, W, hp, row, 1, last ? h : dt,
                      last ? 0.0 : dt, s);
    if (st != SCF_OK) return st;
    centre_accel(hd, Rc, gc);
    for (int i = 0; i < 3; ++i) Vc[i] += (last ? h : dt) * gc[i];
    if (!last)
      for (int i = 0; i < 3; ++i) Rc[i] += dt * Vc[i];
  }
  return SCF_OK;
}

template <typename R>
double key_to_radius(uint64_t key) {
  if constexpr (sizeof(R) == 4) {
    uint32_t b = (uint32_t)key;
    float f;
    std::memcpy(&f, &b, 4);
    return std::sqrt((double)f);
  } else {
    double d;
    std::memcpy(&d, &key, 8);
    return std::sqrt(d);
  }
}

// Selection in the potential of the force weights W (bound test, radix
// selection of r_frac and r_50, weights into w); results to the host.
template <typename R>
scf_status select_impl(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                       const void* vx, const void* vy, const void* vz, const void* m, const void* W,
                       double frac, void* w, uint8_t* bound, void* ax, void* ay, void* az,
                       scf_cadence_state* out, char* ws, const CadLayout& C, hipStream_t s) {
  HostParams<R> none;
  std::memset(&none, 0, sizeof(none));
  void* pot = ws + C.pot;
  scf_status st = run_field<R>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax, ay,
                               az, pot, W, none, nullptr, 0, 0.0, 0.0, s);
  if (st != SCF_OK) return st;
  SelectState* ss = (SelectState*)(ws + C.state);
  {
    Timed t(p, s, K_SELECT);
    HIP_TRY(launch_energy_keys(p->dtype, n, x, y, z, vx, vy, vz, pot, ws + C.keys,
                               bound ? bound : (uint8_t*)(ws + C.bound), s));
    const int hist_blocks = (int)std::min<int64_t>((n + 255) / 256, 4 * (int64_t)p->num_cu);
    HIP_TRY(launch_radix_select(p->dtype, n, ws + C.keys, ss, frac, 0.5, hist_blocks, s));
    HIP_TRY(launch_select_weights(p->dtype, n, ws + C.keys, m, ss, w, (double*)(ws + C.mpart), s));
  }
  SelectState h;
  HIP_TRY(hipMemcpyAsync(&h, ss, offsetof(SelectState, hist), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->nbound = h.nb;
  out->rx = h.nb > 0 ? key_to_radius<R>(h.prefix[0]) : 0.0;
  out->rhm = h.nb > 0 ? key_to_radius<R>(h.prefix[1]) : 0.0;
  out->mbound = h.mbound;
  return SCF_OK;
}

// coef += (1/ns) sum_j a(snapshot j; w1 - w0) over the changed particles;
// the force weights W are overwritten.  Count into *nchanged.
template <typename R>
scf_status delta_impl(scf_plan* p, int64_t n, int ns, const void* const* sx, const void* const* sy,
                      const void* const* sz, const void* w0, const void* w1, double* coef,
                      int64_t* nchanged, char* ws, const CadLayout& C, hipStream_t s) {
  DeltaSnaps ds;
  std::memset(&ds, 0, sizeof(ds));
  ds.ns = ns;
  for (int j = 0; j < ns; ++j) {
    ds.x[j] = sx[j];
    ds.y[j] = sy[j];
    ds.z[j] = sz[j];
  }
  int64_t* total = (int64_t*)(ws + C.total);
  const int64_t cap = std::max<int64_t>(n, 1);
  {
    Timed t(p, s, K_SELECT);
    HIP_TRY(launch_delta_compact(p->dtype, n, w0, w1, ds, (int32_t*)(ws + C.cnt),
                                 (int64_t*)(ws + C.off), total, ws + C.compact, cap, s));
  }
  int64_t nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, total, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (nchanged) *nchanged = nc;
  if (nc == 0) return SCF_OK;
  const R* base = (const R*)(ws + C.compact);
  const R* dw = base + (int64_t)ns * 3 * cap;
  double* ctmp = (double*)(ws + C.ctmp);
  for (int j = 0; j < ns; ++j) {
    const R* sj = base + (int64_t)j * 3 * cap;
    scf_status st = run_coeffs<R>(p, nc, sj, sj + cap, sj + 2 * cap, dw, ctmp, ws + C.L.W, ws, C.L, s);
    if (st != SCF_OK) return st;
    HIP_TRY(launch_axpy(p->T, 1.0 / ns, ctmp, coef, s));
  }
  return SCF_OK;
}

// coef = (1/ns) sum_j a(snapshot j; w); the force weights W are overwritten
template <typename R>
scf_status complete_impl(scf_plan* p, int64_t n, int ns, const void* const* sx,
                         const void* const* sy, const void* const* sz, const void* w, double* coef,
                         char* ws, const CadLayout& C, hipStream_t s) {
  if (ns == 1) return run_coeffs<R>(p, n, sx[0], sy[0], sz[0], w, coef, ws + C.L.W, ws, C.L, s);
  {
    Timed t(p, s, K_FILL);
    HIP_TRY(launch_fill(coef, p->T, 0.0, s));
  }
  double* ctmp = (double*)(ws + C.ctmp);
  for (int j = 0; j < ns; ++j) {
    scf_status st = run_coeffs<R>(p, n, sx[j], sy[j], sz[j], w, ctmp, ws + C.L.W, ws, C.L, s);
    if (st != SCF_OK) return st;
    HIP_TRY(launch_axpy(p->T, 1.0 / ns, ctmp, coef, s));
  }
  return SCF_OK;
}

scf_status check_cadence_ws(const scf_plan* p, int64_t n, int ns_max, const void* ws,
                            size_t ws_bytes) {
  const size_t need = cad_layout(p, n, ns_max).all;
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return SCF_OK;
}

int samples_for(double dti, double mb, double rhm, const scf_cadence* c, double G, int nsub) {
  int ns = 1;
  if (c->n_samples_tdyn > 0 && mb > 0.0 && rhm > 0.0) {
    const double tdyn = c->c_dyn * std::sqrt(rhm * rhm * rhm / (G * mb));
    ns = std::max(1, (int)std::ceil(c->n_samples_tdyn * dti / tdyn));
  }
  return std::min(ns, std::min(nsub, c->ns_max));
}

// rho_SCF (Eq. total_dens) of coef at n points into rho: the field pass's psi
// with density-scaled weights, times the radial factor
template <typename R>
scf_status density_impl(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                        const double* coef, void* rho, char* ws, const CadLayout& C, hipStream_t s) {
  void* W = ws + C.L.W;
  {
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw, W, s));
    HIP_TRY(launch_scale_w(p->dtype, W, p->d_kden, p->lmax, p->nmaxc, s));
  }
  HostParams<R> none;
  std::memset(&none, 0, sizeof(none));
  const size_t nr = (size_t)n * p->rs;
  char* acc = ws + C.acc;
  scf_status st = run_field<R>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, acc,
                               acc + nr, acc + 2 * nr, rho, W, none, nullptr, 0, 0.0, 0.0, s);
  if (st != SCF_OK) return st;
  Timed t(p, s, K_SELECT);
  HIP_TRY(launch_density_factor(p->dtype, n, x, y, z, 1.0 / p->basis.b, 1.0 / p->basis.alpha,
                                p->amode, rho, s));
  return SCF_OK;
}

// core radius and velocity (Sec. 2.1) over w > 0: out = r_core, v[3], mass
template <typename R>
scf_status core_impl(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                     const void* vx, const void* vy, const void* vz, const void* m, const void* w,
                     const double* coef, double* out, char* ws, const CadLayout& C, hipStream_t s) {
  void* rho = ws + C.pot;
  scf_status st = density_impl<R>(p, n, x, y, z, coef, rho, ws, C, s);
  if (st != SCF_OK) return st;
  double r[4];
  {
    Timed t(p, s, K_SELECT);
    HIP_TRY(launch_core_moments(p->dtype, n, x, y, z, vx, vy, vz, m, w, rho, 0, 0.0,
                                (double*)(ws + C.mom), (double*)(ws + C.res), s));
  }
  HIP_TRY(hipMemcpyAsync(r, ws + C.res, sizeof(r), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double rc2 = r[1] > 0.0 ? r[0] / r[1] : 0.0;
  {
    Timed t(p, s, K_SELECT);
    HIP_TRY(launch_core_moments(p->dtype, n, x, y, z, vx, vy, vz, m, w, rho, 1, rc2,
                                (double*)(ws + C.mom), (double*)(ws + C.res), s));
  }
  HIP_TRY(hipMemcpyAsync(r, ws + C.res, sizeof(r), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out[0] = std::sqrt(rc2);
  for (int k = 0; k < 3; ++k) out[1 + k] = r[3] > 0.0 ? r[k] / r[3] : 0.0;
  out[4] = r[3];
  return SCF_OK;
}

// fixed-point search for the a_000 maximum from c (in/out)
scf_status recentre_impl(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                         const void* w, double* c, double tol, int maxit, int32_t* steps, char* ws,
                         const CadLayout& C, hipStream_t s) {
  const double b = p->basis.b;
  int it = 0;
  while (it < maxit) {
    ++it;
    double r[4];
    {
      Timed t(p, s, K_SELECT);
      HIP_TRY(launch_recentre_sums(p->dtype, n, x, y, z, w, c, 1.0 / b, p->basis.alpha, p->amode,
                                   1e-9 * b, (double*)(ws + C.mom), (double*)(ws + C.res), s));
    }
    HIP_TRY(hipMemcpyAsync(r, ws + C.res, sizeof(r), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!(r[0] > 0.0)) break;
    double step2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double cn = r[1 + k] / r[0];
      step2 += (cn - c[k]) * (cn - c[k]);
      c[k] = cn;
    }
    if (std::sqrt(step2) <= tol * b) break;
  }
  if (steps) *steps = it;
  return SCF_OK;
}

// energy norm of the zeroth mode, b alpha B(alpha + 2, alpha) / (4 pi G)
double n00_closed(double alpha, double b, double G) {
  const double beta = std::exp(std::lgamma(alpha + 2.0) + std::lgamma(alpha) - std::lgamma(2.0 * alpha + 2.0));
  return b * alpha * beta / (4.0 * M_PI * G);
}

// (alpha, b) maximising a_000 of the particles with w > 0 about the origin,
// alpha in [amin, 1]: the best point of a coarse grid, then Nelder-Mead in
// (u, ln b) with alpha = amin + (1 - amin) sin^2 u (no bound to handle).  Each
// objective value is one device reduction.  ab: in, the start; out, the result.
scf_status tune_impl(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                     const void* w, double amin, double* ab, double* best_val, char* ws,
                     const CadLayout& C, hipStream_t s) {
  const double G = p->basis.G;
  auto eval = [&](double alpha, double b, double* out) -> scf_status {
    double r[4];
    {
      Timed t(p, s, K_SELECT);
      HIP_TRY(launch_a000_sum(p->dtype, n, x, y, z, w, alpha, 1.0 / b, (double*)(ws + C.mom),
                              (double*)(ws + C.res), s));
    }
    HIP_TRY(hipMemcpyAsync(r, ws + C.res, sizeof(r), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = r[0] / std::sqrt(4.0 * M_PI * n00_closed(alpha, b, G));
    return SCF_OK;
  };
  auto alpha_of = [&](double u) { const double q = std::sin(u); return amin + (1.0 - amin) * q * q; };
  const double lb0 = std::log(ab[1]);
  double fbest = -1.0, ubest = 0.0, lbbest = lb0;
  for (int ia = 0; ia < 7; ++ia) {
    const double alpha = amin + (1.0 - amin) * ia / 6.0;
    for (int ib = 0; ib < 17; ++ib) {
      const double lb = lb0 - 4.0 + 0.5 * ib;
      double f;
      scf_status st = eval(alpha, std::exp(lb), &f);
      if (st != SCF_OK) return st;
      if (f > fbest) {
        fbest = f;
        ubest = std::asin(std::sqrt(std::min(1.0, (alpha - amin) / (1.0 - amin))));
        lbbest = lb;
      }
    }
  }
  // Nelder-Mead (maximisation) on (u, ln b)
  double P[3][2] = {{ubest, lbbest}, {ubest + 0.15, lbbest}, {ubest, lbbest + 0.15}};
  double F[3];
  for (int k = 0; k < 3; ++k) {
    scf_status st = eval(alpha_of(P[k][0]), std::exp(P[k][1]), &F[k]);
    if (st != SCF_OK) return st;
  }
  for (int it = 0; it < 600; ++it) {
    // order: 0 best, 2 worst
    for (int a = 0; a < 2; ++a)
      for (int b2 = 0; b2 < 2 - a; ++b2)
        if (F[b2] < F[b2 + 1]) {
          std::swap(F[b2], F[b2 + 1]);
          std::swap(P[b2][0], P[b2 + 1][0]);
          std::swap(P[b2][1], P[b2 + 1][1]);
        }
    double size = 0.0;
    for (int k = 1; k < 3; ++k)
      size = std::max(size, std::max(std::fabs(P[k][0] - P[0][0]), std::fabs(P[k][1] - P[0][1])));
    if (size < 1e-10) break;
    const double c0 = 0.5 * (P[0][0] + P[1][0]), c1 = 0.5 * (P[0][1] + P[1][1]);
    auto at = [&](double t, double* q) { q[0] = c0 + t * (P[2][0] - c0); q[1] = c1 + t * (P[2][1] - c1); };
    double xr[2], fr;
    at(-1.0, xr);
    scf_status st = eval(alpha_of(xr[0]), std::exp(xr[1]), &fr);
    if (st != SCF_OK) return st;
    if (fr > F[0]) {
      double xe[2], fe;
      at(-2.0, xe);
      st = eval(alpha_of(xe[0]), std::exp(xe[1]), &fe);
      if (st != SCF_OK) return st;
      if (fe > fr) {
        P[2][0] = xe[0]; P[2][1] = xe[1]; F[2] = fe;
      } else {
        P[2][0] = xr[0]; P[2][1] = xr[1]; F[2] = fr;
      }
    } else if (fr > F[1]) {
      P[2][0] = xr[0]; P[2][1] = xr[1]; F[2] = fr;
    } else {
      double xc[2], fc;
      at(fr > F[2] ? -0.5 : 0.5, xc);
      st = eval(alpha_of(xc[0]), std::exp(xc[1]), &fc);
      if (st != SCF_OK) return st;
      if (fc > std::max(fr, F[2])) {
        P[2][0] = xc[0]; P[2][1] = xc[1]; F[2] = fc;
      } else {
        for (int k = 1; k < 3; ++k) {
          P[k][0] = P[0][0] + 0.5 * (P[k][0] - P[0][0]);
          P[k][1] = P[0][1] + 0.5 * (P[k][1] - P[0][1]);
          st = eval(alpha_of(P[k][0]), std::exp(P[k][1]), &F[k]);
          if (st != SCF_OK) return st;
        }
      }
    }
  }
  int kb = 0;
  for (int k = 1; k < 3; ++k)
    if (F[k] > F[kb]) kb = k;
  ab[0] = alpha_of(P[kb][0]);
  ab[1] = std::exp(P[kb][1]);
  if (best_val) *best_val = F[kb];
  return SCF_OK;
}

// new (alpha, b) for a plan, after the device has finished queued work
scf_status set_basis_impl(scf_plan* p, double alpha, double b) {
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SCF_ERR_UNSUPPORTED, "alpha = %g outside (0, 1]", alpha);
  if (!(b > 0.0) || !std::isfinite(b)) return fail(SCF_ERR_INVALID_ARG, "b must be > 0");
  HIP_TRY(hipDeviceSynchronize());
  scf_basis nb = p->basis;
  nb.alpha = alpha;
  nb.b = b;
  HIP_TRY(fill_tables(p, &nb));
  return SCF_OK;
}

}  // namespace

extern "C" {

scf_status scf_cadence_workspace_size(const scf_plan* p, int64_t n, int32_t ns_max, size_t* bytes) {
  if (!p || !bytes) return fail(SCF_ERR_INVALID_ARG, "plan and bytes must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (ns_max < 1 || ns_max > SCF_MAX_SAMPLES)
    return fail(SCF_ERR_INVALID_ARG, "ns_max = %d outside [1, %d]", ns_max, SCF_MAX_SAMPLES);
  *bytes = cad_layout(p, n, ns_max).all;
  return SCF_OK;
}

scf_status scf_step_frozen(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                           void* vz, void* ax, void* ay, void* az, uint32_t step_flags,
                           const double* coef, const scf_host* host, double* centre, double dt,
                           int32_t nsteps, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0 || nsteps < 0) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nsteps >= 0");
  if (!std::isfinite(dt)) return fail(SCF_ERR_INVALID_ARG, "dt is not finite");
  if (step_flags & ~SCF_STEP_ACC_VALID) return fail(SCF_ERR_INVALID_ARG, "unknown step flags");
  if (!centre || !coef) return fail(SCF_ERR_INVALID_ARG, "centre and coef must be non-null");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(ax) && ptr_ok(ay) && ptr_ok(az)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  const size_t need = plain_need(p, n);
  if (!ws || ws_bytes < need)
    return fail(SCF_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (!ws_aligned(ws)) return fail(SCF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(p, n, 1, 0);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool with_host = host && host->ncomp > 0;
  HostParams<double> hd;
  fill_host_params(hd, with_host ? host : nullptr);
  {
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw, w + L.W, s));
  }
  double R[3] = {centre[0], centre[1], centre[2]}, V[3] = {centre[3], centre[4], centre[5]};
  const bool av = (step_flags & SCF_STEP_ACC_VALID) != 0;
  scf_status st = p->dtype == SCF_F32
                      ? frozen_steps<float>(p, n, x, y, z, vx, vy, vz, ax, ay, az, av, w + L.W, hd,
                                            with_host, R, V, dt, nsteps, s)
                      : frozen_steps<double>(p, n, x, y, z, vx, vy, vz, ax, ay, az, av, w + L.W, hd,
                                             with_host, R, V, dt, nsteps, s);
  if (st != SCF_OK) return st;
  for (int i = 0; i < 3; ++i) {
    centre[i] = R[i];
    centre[3 + i] = V[i];
  }
  return SCF_OK;
}

scf_status scf_select(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                      const void* vx, const void* vy, const void* vz, const void* m,
                      const double* coef, double frac, void* w, uint8_t* bound,
                      scf_cadence_state* out, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !coef || !out) return fail(SCF_ERR_INVALID_ARG, "plan, coef and out must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (!(frac > 0.0 && frac <= 1.0)) return fail(SCF_ERR_INVALID_ARG, "frac must lie in (0, 1]");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(w)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  hipStream_t s = (hipStream_t)stream;
  char* wsp = (char*)ws;
  {
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw,
                          wsp + C.L.W, s));
  }
  const size_t nr = (size_t)n * p->rs;
  char* acc = wsp + C.acc;
  return p->dtype == SCF_F32
             ? select_impl<float>(p, n, x, y, z, vx, vy, vz, m, wsp + C.L.W, frac, w, bound, acc,
                                  acc + nr, acc + 2 * nr, out, wsp, C, s)
             : select_impl<double>(p, n, x, y, z, vx, vy, vz, m, wsp + C.L.W, frac, w, bound, acc,
                                   acc + nr, acc + 2 * nr, out, wsp, C, s);
}

scf_status scf_coeffs_delta(scf_plan* p, int64_t n, int32_t nsnap, const void* const* snaps,
                            const void* w_old, const void* w_new, double* coef, int64_t* nchanged,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!p || !coef || !snaps) return fail(SCF_ERR_INVALID_ARG, "plan, coef and snaps must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (nsnap < 1 || nsnap > SCF_MAX_SAMPLES)
    return fail(SCF_ERR_INVALID_ARG, "nsnap = %d outside [1, %d]", nsnap, SCF_MAX_SAMPLES);
  if (n > 0) {
    if (!ptr_ok(w_old) || !ptr_ok(w_new)) return fail(SCF_ERR_INVALID_ARG, "weights must be non-null");
    for (int j = 0; j < 3 * nsnap; ++j)
      if (!snaps[j]) return fail(SCF_ERR_INVALID_ARG, "snapshot pointer %d is null", j);
  }
  scf_status cs = check_cadence_ws(p, n, nsnap, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, nsnap);
  hipStream_t s = (hipStream_t)stream;
  const void* sx[SCF_MAX_SAMPLES];
  const void* sy[SCF_MAX_SAMPLES];
  const void* sz[SCF_MAX_SAMPLES];
  for (int j = 0; j < nsnap; ++j) {
    sx[j] = snaps[3 * j];
    sy[j] = snaps[3 * j + 1];
    sz[j] = snaps[3 * j + 2];
  }
  if (n == 0) {
    if (nchanged) *nchanged = 0;
    return SCF_OK;
  }
  return p->dtype == SCF_F32
             ? delta_impl<float>(p, n, nsnap, sx, sy, sz, w_old, w_new, coef, nchanged, (char*)ws, C, s)
             : delta_impl<double>(p, n, nsnap, sx, sy, sz, w_old, w_new, coef, nchanged, (char*)ws, C, s);
}

scf_status scf_cadence_init(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                            const void* vx, const void* vy, const void* vz, const void* m,
                            double frac, double* coef, void* w, scf_cadence_state* state,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!p || !coef || !state) return fail(SCF_ERR_INVALID_ARG, "plan, coef and state must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (!(frac > 0.0 && frac <= 1.0)) return fail(SCF_ERR_INVALID_ARG, "frac must lie in (0, 1]");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(w)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  hipStream_t s = (hipStream_t)stream;
  char* wsp = (char*)ws;
  const size_t nr = (size_t)n * p->rs;
  char* acc = wsp + C.acc;
  auto go = [&](auto tag) -> scf_status {
    using Rt = decltype(tag);
    // coefficients (and force weights) of all particles, then the selection
    scf_status st = run_coeffs<Rt>(p, n, x, y, z, m, coef, wsp + C.L.W, wsp, C.L, s);
    if (st != SCF_OK) return st;
    st = select_impl<Rt>(p, n, x, y, z, vx, vy, vz, m, wsp + C.L.W, frac, w, nullptr, acc, acc + nr,
                         acc + 2 * nr, state, wsp, C, s);
    if (st != SCF_OK) return st;
    const void* sx[1] = {x};
    const void* sy[1] = {y};
    const void* sz[1] = {z};
    return complete_impl<Rt>(p, n, 1, sx, sy, sz, w, coef, wsp, C, s);
  };
  scf_status st = p->dtype == SCF_F32 ? go(float(0)) : go(double(0));
  if (st != SCF_OK) return st;
  state->since = 0;
  HIP_TRY(hipStreamSynchronize(s));
  return SCF_OK;
}

scf_status scf_evolve(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy, void* vz,
                      const void* m, void* ax, void* ay, void* az, const scf_host* host,
                      double* centre, const scf_cadence* cfg, int32_t nint, double* coef, void* w,
                      scf_cadence_state* state, scf_interval_log* log, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!p || !cfg || !centre || !coef || !state)
    return fail(SCF_ERR_INVALID_ARG, "plan, cadence, centre, coef and state must be non-null");
  if (n < 0 || nint < 0) return fail(SCF_ERR_INVALID_ARG, "need n >= 0 and nint >= 0");
  if (!(cfg->eta > 0.0) || !(cfg->dt_max > 0.0) || !(cfg->frac > 0.0 && cfg->frac <= 1.0) ||
      cfg->refresh_every < 1 || cfg->n_samples_tdyn < 0 || cfg->ns_max < 1 ||
      cfg->ns_max > SCF_MAX_SAMPLES || (cfg->n_samples_tdyn > 0 && !(cfg->c_dyn > 0.0)) ||
      (cfg->recentre != 0 && cfg->recentre != 1) || (cfg->retune != 0 && cfg->retune != 1) ||
      (cfg->retune && !(cfg->alpha_min > 0.0 && cfg->alpha_min < 1.0)))
    return fail(SCF_ERR_INVALID_ARG, "invalid cadence parameters");
  if (!host || host->ncomp < 1)
    return fail(SCF_ERR_INVALID_ARG, "the cadence needs a host potential (its tidal tensor sets the interval)");
  scf_status hs = check_host(host);
  if (hs != SCF_OK) return hs;
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(w) && ptr_ok(ax) && ptr_ok(ay) && ptr_ok(az)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, cfg->ns_max, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, cfg->ns_max);
  hipStream_t s = (hipStream_t)stream;
  char* wsp = (char*)ws;
  HostParams<double> hd;
  fill_host_params(hd, host);
  double R[3] = {centre[0], centre[1], centre[2]}, V[3] = {centre[3], centre[4], centre[5]};
  const size_t nr = (size_t)n * p->rs;
  void* W = wsp + C.L.W;
  void* wnew = wsp + C.wnew;
  {
    Timed t(p, s, K_MAKE_W);
    HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw, W, s));
  }
  auto go = [&](auto tag) -> scf_status {
    using Rt = decltype(tag);
    for (int it = 0; it < nint; ++it) {
      const double tn = tidal_norm_host(hd, R);
      const double dti = std::sqrt(cfg->eta) * std::pow(tn * tn / 6.0, -0.25);
      if (!std::isfinite(dti) || !(dti > 0.0))
        return fail(SCF_ERR_INVALID_ARG, "tidal timestep is not finite at the centre (|T| = %g)", tn);
      const int nsub = std::max(1, (int)std::ceil(dti / cfg->dt_max));
      const double h = dti / nsub;
      const int ns = samples_for(dti, state->mbound, state->rhm, cfg, p->basis.G, nsub);
      const void* sx[SCF_MAX_SAMPLES];
      const void* sy[SCF_MAX_SAMPLES];
      const void* sz[SCF_MAX_SAMPLES];
      int done = 0;
      for (int j = 0; j < ns; ++j) {
        const int end = (int)(((int64_t)(j + 1) * nsub + ns - 1) / ns);
        scf_status st = frozen_steps<Rt>(p, n, x, y, z, vx, vy, vz, ax, ay, az, done > 0, W, hd,
                                         true, R, V, h, end - done, s);
        if (st != SCF_OK) return st;
        done = end;
        if (j + 1 < ns) {
          char* dst = wsp + C.snaps + (size_t)j * 3 * nr;
          HIP_TRY(hipMemcpyAsync(dst, x, nr, hipMemcpyDeviceToDevice, s));
          HIP_TRY(hipMemcpyAsync(dst + nr, y, nr, hipMemcpyDeviceToDevice, s));
          HIP_TRY(hipMemcpyAsync(dst + 2 * nr, z, nr, hipMemcpyDeviceToDevice, s));
          sx[j] = dst;
          sy[j] = dst + nr;
          sz[j] = dst + 2 * nr;
        } else {
          sx[j] = x;
          sy[j] = y;
          sz[j] = z;
        }
      }
      // selection at the interval end, in the potential the particles moved in
      scf_cadence_state sel = *state;
      scf_status st = select_impl<Rt>(p, n, x, y, z, vx, vy, vz, m, W, cfg->frac, wnew, nullptr, ax,
                                      ay, az, &sel, wsp, C, s);
      if (st != SCF_OK) return st;
      int64_t nchanged = 0;
      const bool complete = state->since + 1 >= cfg->refresh_every;
      double dx[3] = {0.0, 0.0, 0.0}, dv[3] = {0.0, 0.0, 0.0};
      if (complete) {
        // count of changed weights (no compaction), then the full sums
        DeltaSnaps none;
        std::memset(&none, 0, sizeof(none));
        HIP_TRY(launch_delta_compact(p->dtype, n, w, wnew, none, (int32_t*)(wsp + C.cnt),
                                     (int64_t*)(wsp + C.off), (int64_t*)(wsp + C.total), nullptr, 0, s));
        HIP_TRY(hipMemcpyAsync(&nchanged, wsp + C.total, 8, hipMemcpyDeviceToHost, s));
        if (cfg->recentre) {
          // frame origin to the a_000 maximum of the selected particles:
          // positions, earlier samples and the centre orbit shift with it
          st = recentre_impl(p, n, x, y, z, wnew, dx, 1e-6, 100, nullptr, wsp, C, s);
          if (st != SCF_OK) return st;
          HIP_TRY(launch_shift3(p->dtype, n, x, y, z, dx, s));
          for (int j = 0; j + 1 < ns; ++j)
            HIP_TRY(launch_shift3(p->dtype, n, (void*)sx[j], (void*)sy[j], (void*)sz[j], dx, s));
          for (int k = 0; k < 3; ++k) R[k] += dx[k];
        }
        if (cfg->retune) {
          // basis parameters of the zeroth mode closest to the selected particles
          double ab[2] = {p->basis.alpha, p->basis.b};
          st = tune_impl(p, n, x, y, z, wnew, cfg->alpha_min, ab, nullptr, wsp, C, s);
          if (st != SCF_OK) return st;
          st = set_basis_impl(p, ab[0], ab[1]);
          if (st != SCF_OK) return st;
        }
        st = complete_impl<Rt>(p, n, ns, sx, sy, sz, wnew, coef, wsp, C, s);
        if (st != SCF_OK) return st;
        if (cfg->recentre) {
          // frame velocity to the core velocity of the new potential
          double core[5];
          st = core_impl<Rt>(p, n, x, y, z, vx, vy, vz, m, wnew, coef, core, wsp, C, s);
          if (st != SCF_OK) return st;
          for (int k = 0; k < 3; ++k) dv[k] = core[1 + k];
          HIP_TRY(launch_shift3(p->dtype, n, vx, vy, vz, dv, s));
          for (int k = 0; k < 3; ++k) V[k] += dv[k];
        }
        state->since = 0;
      } else {
        st = delta_impl<Rt>(p, n, ns, sx, sy, sz, w, wnew, coef, &nchanged, wsp, C, s);
        if (st != SCF_OK) return st;
        state->since += 1;
      }
      if (n > 0) HIP_TRY(hipMemcpyAsync(w, wnew, nr, hipMemcpyDeviceToDevice, s));
      {
        Timed t(p, s, K_MAKE_W);
        HIP_TRY(launch_make_w(p->dtype, coef, (int)p->T, p->nmax, p->lmax, p->nmaxc, p->d_fw, W, s));
      }
      HIP_TRY(hipStreamSynchronize(s));
      state->nbound = sel.nbound;
      state->rx = sel.rx;
      state->rhm = sel.rhm;
      state->mbound = sel.mbound;
      if (log) {
        scf_interval_log& e = log[it];
        std::memset(&e, 0, sizeof(e));
        e.dt_int = dti;
        e.nsub = nsub;
        e.nsamples = ns;
        e.complete = complete ? 1 : 0;
        e.nbound = sel.nbound;
        e.nchanged = nchanged;
        e.rx = sel.rx;
        e.rhm = sel.rhm;
        e.mbound = sel.mbound;
        for (int k = 0; k < 3; ++k) {
          e.dx[k] = dx[k];
          e.dv[k] = dv[k];
        }
        e.alpha = p->basis.alpha;
        e.b = p->basis.b;
      }
    }
    return SCF_OK;
  };
  scf_status st = p->dtype == SCF_F32 ? go(float(0)) : go(double(0));
  for (int i = 0; i < 3; ++i) {
    centre[i] = R[i];
    centre[3 + i] = V[i];
  }
  return st;
}



scf_status scf_density(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                       const double* coef, void* rho, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !coef) return fail(SCF_ERR_INVALID_ARG, "plan and coef must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(rho)))
    return fail(SCF_ERR_INVALID_ARG, "point and output arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  hipStream_t s = (hipStream_t)stream;
  return p->dtype == SCF_F32 ? density_impl<float>(p, n, x, y, z, coef, rho, (char*)ws, C, s)
                             : density_impl<double>(p, n, x, y, z, coef, rho, (char*)ws, C, s);
}

scf_status scf_core(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                    const void* vx, const void* vy, const void* vz, const void* m, const void* w,
                    const double* coef, double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !coef || !out) return fail(SCF_ERR_INVALID_ARG, "plan, coef and out must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(vx) && ptr_ok(vy) && ptr_ok(vz) &&
                 ptr_ok(m) && ptr_ok(w)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  hipStream_t s = (hipStream_t)stream;
  return p->dtype == SCF_F32
             ? core_impl<float>(p, n, x, y, z, vx, vy, vz, m, w, coef, out, (char*)ws, C, s)
             : core_impl<double>(p, n, x, y, z, vx, vy, vz, m, w, coef, out, (char*)ws, C, s);
}

scf_status scf_recentre(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                        const void* w, double* centre, double tol, int32_t maxit, int32_t* steps,
                        void* ws, size_t ws_bytes, void* stream) {
  if (!p || !centre) return fail(SCF_ERR_INVALID_ARG, "plan and centre must be non-null");
  if (n < 0 || maxit < 0 || !(tol >= 0.0))
    return fail(SCF_ERR_INVALID_ARG, "need n >= 0, maxit >= 0 and tol >= 0");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(w)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  return recentre_impl(p, n, x, y, z, w, centre, tol, maxit, steps, (char*)ws, C,
                       (hipStream_t)stream);
}


scf_status scf_plan_set_basis(scf_plan* p, double alpha, double b) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  return set_basis_impl(p, alpha, b);
}

scf_status scf_plan_get_basis(const scf_plan* p, scf_basis* out) {
  if (!p || !out) return fail(SCF_ERR_INVALID_ARG, "plan and out must be non-null");
  *out = p->basis;
  return SCF_OK;
}

scf_status scf_tune_basis(scf_plan* p, int64_t n, const void* x, const void* y, const void* z,
                          const void* w, double alpha_min, double* alpha_b, double* a000,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!p || !alpha_b) return fail(SCF_ERR_INVALID_ARG, "plan and alpha_b must be non-null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  if (!(alpha_min > 0.0 && alpha_min < 1.0))
    return fail(SCF_ERR_INVALID_ARG, "alpha_min must lie in (0, 1)");
  if (!(alpha_b[1] > 0.0) || !std::isfinite(alpha_b[1]))
    return fail(SCF_ERR_INVALID_ARG, "the starting b must be > 0");
  if (n > 0 && !(ptr_ok(x) && ptr_ok(y) && ptr_ok(z) && ptr_ok(w)))
    return fail(SCF_ERR_INVALID_ARG, "particle arrays must be non-null");
  scf_status cs = check_cadence_ws(p, n, 1, ws, ws_bytes);
  if (cs != SCF_OK) return cs;
  const CadLayout C = cad_layout(p, n, 1);
  return tune_impl(p, n, x, y, z, w, alpha_min, alpha_b, a000, (char*)ws, C, (hipStream_t)stream);
}

}  // extern "C"
