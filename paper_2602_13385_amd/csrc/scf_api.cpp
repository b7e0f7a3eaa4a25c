// libscf C ABI: plan management, basis tables, argument validation, the
// double-precision centre orbit (Sec. 2.1) and the launch sequences of the
// hot path (coefficients, field, step, batched step, adjoint, diagnostics).
// Declared in include/scf.h.
#include <vector>

#include "scf_plan.h"

// Times ncand launch configurations (set(c) selects candidate c, launch()
// runs it on stream s): one untimed launch of each first (code loading, clock
// ramp), then three rounds over all candidates, each timing eight
// back-to-back launches between a pair of events.  A candidate's time is its
// best round; interleaving the rounds spreads clock drift over all
// candidates alike.  best gets the fastest (the first of equals), best_ms its
// time per launch.
template <typename Set, typename Launch>
static scf_status time_candidates(const int ncand, Set set, Launch launch, hipStream_t s,
                                  int& best, float& best_ms) {
  constexpr int kRounds = 3, kLaunches = 8;
  std::vector<float> t(ncand, 1e30f);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  scf_status st = SCF_OK;
  for (int c = 0; c < ncand && st == SCF_OK; ++c) {
    set(c);
    st = launch();
  }
  hipError_t he = hipSuccess;
  for (int r = 0; r < kRounds && st == SCF_OK && he == hipSuccess; ++r)
    for (int c = 0; c < ncand && st == SCF_OK && he == hipSuccess; ++c) {
      set(c);
      he = hipEventRecord(e0, s);
      for (int k = 0; k < kLaunches && st == SCF_OK && he == hipSuccess; ++k) st = launch();
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (ms / kLaunches < t[c]) t[c] = ms / kLaunches;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SCF_OK) return st;
  HIP_TRY(he);
  best = 0;
  for (int c = 1; c < ncand; ++c)
    if (t[c] < t[best]) best = c;
  best_ms = t[best];
  return SCF_OK;
}

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

const char* scf_last_error(void) { return scf::api_detail::g_last_error.c_str(); }

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
  double* coef = (double*)((char*)ws + ws_layout(p, n, 1, 0).coef);
  const int saved = p->coef_variant, saved_div = p->coef_div;
  const bool prof = p->prof;
  p->prof = false;
  // candidates: every kernel variant at a block-count divisor of 1, 2, 4 or 8
  int best = 0;
  float bms = 0.f;
  const scf_status st = time_candidates(
      4 * p->eng->coef_variants(),
      [&](int c) {
        p->coef_variant = c / 4;
        p->coef_div = 1 << (c % 4);
      },
      [&]() { return scf_coeffs(p, n, x, y, z, m, coef, ws, ws_bytes, stream); },
      (hipStream_t)stream, best, bms);
  p->prof = prof;
  if (st != SCF_OK) {
    p->coef_variant = saved;
    p->coef_div = saved_div;
    return st;
  }
  p->coef_variant = best / 4;
  p->coef_div = 1 << (best % 4);
  if (best_ms) *best_ms = bms;
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
  auto launch = [&]() -> scf_status {
    if (p->dtype == SCF_F32) {
      HostParams<float> hp;
      fill_host_params(hp, nullptr);
      return run_field<float>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax,
                              ay, az, nullptr, w + L.W, hp, nullptr, 0, 0.0, 0.0, s);
    }
    HostParams<double> hp;
    fill_host_params(hp, nullptr);
    return run_field<double>(p, n, (void*)x, (void*)y, (void*)z, nullptr, nullptr, nullptr, ax,
                             ay, az, nullptr, w + L.W, hp, nullptr, 0, 0.0, 0.0, s);
  };
  int best = 0;
  float bms = 0.f;
  st = time_candidates(
      p->eng->field_variants(), [&](int c) { p->field_variant = c; }, launch, s, best, bms);
  p->prof = prof;
  if (st != SCF_OK) {
    p->field_variant = saved;
    return st;
  }
  p->field_variant = best;
  if (best_ms) *best_ms = bms;
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
  if (p->d_dtab) (void)hipFree(p->d_dtab);
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

}  // extern "C"

namespace {

// scf_step, and with w_hist non-null scf_step_keep_weights: the force
// weights of the kick at x_k go to row k of w_hist instead of the workspace
scf_status step_impl(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                     void* vz, const void* m, void* ax, void* ay, void* az, uint32_t step_flags,
                     const scf_host* host, double* centre, double dt, int32_t nsteps,
                     double* coef_last, void* w_hist, void* ws, size_t ws_bytes, void* stream) {
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
  const size_t wrow = (size_t)(p->nmaxc + 1) * (p->lmax + 1) * (p->lmax + 1) * p->rs;
  // force weights of the kick at x_k
  auto Wk = [&](int k) -> void* { return w_hist ? (char*)w_hist + (size_t)k * wrow : w + L.W; };
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
      st = run_coeffs<Rt>(p, n, x, y, z, m, nsteps == 0 && coef_last ? coef_last : coef_int, Wk(0),
                          w, L, s);
      if (st != SCF_OK) return st;
      st = run_field<Rt>(p, n, x, y, z, vx, vy, vz, ax, ay, az, nullptr, Wk(0), hp, row, 0, 0.0,
                         0.0, s);
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
      st = run_coeffs<Rt>(p, n, x, y, z, m, last && coef_last ? coef_last : coef_int, Wk(k), w, L,
                          s);
      if (st != SCF_OK) return st;
      // closing half kick of step k merged with the opening half kick of
      // step k+1, then the drift of step k+1
      // (the accelerations are stored on the last step only: the merged
      // kicks of the other steps do not read them back)
      st = run_field<Rt>(p, n, x, y, z, vx, vy, vz, last ? ax : nullptr, last ? ay : nullptr,
                         last ? az : nullptr, nullptr, Wk(k), hp, row, 1, last ? h : dt,
                         last ? 0.0 : dt, s);
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

}  // namespace

extern "C" {

scf_status scf_step(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx, void* vy, void* vz,
                    const void* m, void* ax, void* ay, void* az, uint32_t step_flags,
                    const scf_host* host, double* centre, double dt, int32_t nsteps,
                    double* coef_last, void* ws, size_t ws_bytes, void* stream) {
  return step_impl(p, n, x, y, z, vx, vy, vz, m, ax, ay, az, step_flags, host, centre, dt, nsteps,
                   coef_last, nullptr, ws, ws_bytes, stream);
}

int64_t scf_plan_weights_size(const scf_plan* p) {
  return p ? (int64_t)(p->nmaxc + 1) * (p->lmax + 1) * (p->lmax + 1) : 0;
}

scf_status scf_step_keep_weights(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx,
                                 void* vy, void* vz, const void* m, void* ax, void* ay, void* az,
                                 uint32_t step_flags, const scf_host* host, double* centre,
                                 double dt, int32_t nsteps, double* coef_last, void* w_hist,
                                 void* ws, size_t ws_bytes, void* stream) {
  if (n > 0 && !w_hist) return fail(SCF_ERR_INVALID_ARG, "w_hist is null");
  return step_impl(p, n, x, y, z, vx, vy, vz, m, ax, ay, az, step_flags, host, centre, dt, nsteps,
                   coef_last, n > 0 ? w_hist : nullptr, ws, ws_bytes, stream);
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
  const int cap = std::max(1, p->resident[v] * p->num_cu);
  std::vector<int64_t> stg(ncl);
  int64_t st_tot = 0;
  for (int c = 0; c < ncl; ++c) {
    stg[c] = (offsets[c + 1] - offsets[c] + P - 1) / P;
    st_tot += stg[c];
  }
  std::vector<int64_t> sb, se;
  std::vector<int32_t> slot, unit_start(ncl + 1, 0), rows(ncl + 1, 0), bcl;
  std::vector<int64_t> bb, be;
  int64_t max_stages = 0;
  for (int c = 0; c < ncl; ++c) {
    unit_start[c] = (int32_t)sb.size();
    if (stg[c] == 0) continue;
    int64_t uc = (int64_t)((double)cap * (double)stg[c] / (double)st_tot);
    uc = std::max<int64_t>(1, std::min<int64_t>(uc, stg[c]));
    for (int64_t u = 0; u < uc; ++u) {
      const int64_t s0 = stg[c] * u / uc, s1 = stg[c] * (u + 1) / uc;
      sb.push_back(offsets[c] + s0 * P);
      se.push_back(std::min(offsets[c] + s1 * P, offsets[c + 1]));
      slot.push_back((int32_t)slot.size());
      max_stages = std::max(max_stages, s1 - s0);
    }
  }
  unit_start[ncl] = (int32_t)sb.size();
  // partial rows of cluster c: [rows[c], rows[c+1])
  const int rpu = unit_rows(p, v, max_stages);
  for (int c = 0; c <= ncl; ++c) rows[c] = unit_start[c] * rpu;
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
  // one reduction launch when no cluster has more partial rows than the
  // single-pass kernel takes
  int max_cluster_rows = 0;
  for (int c = 0; c < ncl; ++c) max_cluster_rows = std::max(max_cluster_rows, rows[c + 1] - rows[c]);
  const bool one_pass = max_cluster_rows <= kSmallRows;
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
    ca.one_row = rpu == 1;
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
    auto enqueue = [&](hipStream_t q, double kick, double drift, double* coef,
                       bool store_acc) -> scf_status {
      {
        Timed t(p, q, K_BATCH_COEF);
        HIP_TRY(p->eng->launch_coef(&ca, U, v, q));
      }
      {
        Timed tr(p, q, K_REDUCE);
        if (one_pass) {
          HIP_TRY(launch_reduce_final_batched(
              p->dtype, ca.partials, (const int32_t*)(w + B.rows), ncl, (int)p->T, p->nmax,
              p->lmax, p->nmaxc, p->d_cs, p->d_fw, coef, Wb, W_stride,
              (const double*)(w + B.tab), (double*)(w + B.cur), (int*)(w + B.ctr), q));
        } else {
          HIP_TRY(launch_reduce_batched(p->dtype, ca.partials, (const int32_t*)(w + B.rows), ncl,
                                        (int)p->T, nch, (double*)(w + B.L.red1), q));
          HIP_TRY(launch_finalize_batched(p->dtype, (const double*)(w + B.L.red1), nch, (int)p->T,
                                          p->nmax, p->lmax, p->nmaxc, p->d_cs, p->d_fw, coef, Wb,
                                          W_stride, (const double*)(w + B.tab), ncl,
                                          (double*)(w + B.cur), (int*)(w + B.ctr), q));
        }
      }
      ForceArgs<Rt> f2 = fa;
      f2.kick = Rt(kick);
      f2.drift = Rt(drift);
      if (!store_acc) f2.ax = f2.ay = f2.az = nullptr;
      {
        Timed t(p, q, K_BATCH_FIELD);
        HIP_TRY(p->eng->launch_force(&f2, nblk, 1, p->field_variant, q));
      }
      return SCF_OK;
    };
    scf_status st = upload_rows(acc_valid ? 1 : 0);
    if (st != SCF_OK) return st;
    int64_t chunk0 = acc_valid ? 1 : 0;
    if (!acc_valid) {
      // a(x0): field pass with no kick and no drift (v is rewritten unchanged)
      st = enqueue(s, 0.0, 0.0, nsteps == 0 && coef_last ? coef_last : coef_int, true);
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
      add(&one_pass, sizeof(one_pass));
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
          for (int r = 0; r < rep && cs == SCF_OK; ++r) cs = enqueue(p->cap_stream, dt, dt, coef_int, false);
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
        st = enqueue(s, last ? h : dt, last ? 0.0 : dt, last && coef_last ? coef_last : coef_int,
                     last);
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
                            void* const* lam, double* lam_centre, double* grad_host,
                            const void* w_hist, void* ws, size_t ws_bytes, void* stream) {
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
  // force weights of the kick at X_k: recorded by the forward pass, or
  // recomputed here into the workspace
  auto Wk = [&](int k) -> char* {
    return w_hist ? (char*)w_hist + (size_t)k * A.wsz * rs : w + A.Wsv + (size_t)k * A.wsz * rs;
  };
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
      if (!w_hist) {
        st = run_coeffs<Rt>(p, n, Xk(0, 0), Xk(0, 1), Xk(0, 2), m, (double*)(w + A.L.coef), Wk(0),
                            w, A.L, s);
        if (st != SCF_OK) return st;
      }
      st = run_field<Rt>(p, n, Xk(0, 0), Xk(0, 1), Xk(0, 2), Vb[0], Vb[1], Vb[2], Ab[0], Ab[1],
                         Ab[2], nullptr, Wk(0), hp, row, 0, 0.0, 0.0, s);
      if (st != SCF_OK) return st;
      for (int c = 0; c < 3; ++c)
        HIP_TRY(hipMemcpyAsync(Xk(1, c), Xk(0, c), n * rs, hipMemcpyDeviceToDevice, s));
      HIP_TRY(launch_kick_drift(p->dtype, n, Xk(1, 0), Xk(1, 1), Xk(1, 2), Vb[0], Vb[1], Vb[2], Ab[0],
                                Ab[1], Ab[2], h, dt, s));
      for (int k = 1; k <= nsteps; ++k) {
        if (!w_hist) {
          st = run_coeffs<Rt>(p, n, Xk(k, 0), Xk(k, 1), Xk(k, 2), m, (double*)(w + A.L.coef),
                              Wk(k), w, A.L, s);
          if (st != SCF_OK) return st;
        }
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
