// libscf C ABI, continued: the refresh cadence of Sec. 2.2 (frozen-potential
// steps, the bound selection, complete and intermediate refreshes, the
// driver), the SCF density (Eq. total_dens), the frame centre and velocity
// (Sec. 2.1) and the basis retuning.  Declared in include/scf.h.
#include "scf_plan.h"

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

void scf_cadence_defaults(scf_cadence* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->eta = 1.0 / 400.0;  // Eq. (tidal_timestep)
  c->dt_max = 0.005;
  c->frac = 0.999;       // r_99.9
  // t_dyn = 4.3451 Myr at M = 1e5 Msun and r = 10 pc, written as
  // c_dyn sqrt(r^3 / (G M)): with G = 4.30091727e-3 pc (km/s)^2 / Msun the
  // square root is sqrt(1000 / 430.091727) pc/(km/s), and 1 pc/(km/s) is
  // 3.0856775814913673e13 km / 3.15576e13 s-per-Myr = 0.977792 Myr
  c->c_dyn = 4.3451 / (std::sqrt(1000.0 / (4.30091727e-3 * 1e5)) *
                       (3.0856775814913673e13 / 3.15576e13));
  c->refresh_every = 5;
  c->n_samples_tdyn = 1;
  c->ns_max = 8;
  c->recentre = 0;
  c->retune = 0;
  c->alpha_min = 0.25;
}

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
