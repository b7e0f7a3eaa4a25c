// Device-side building blocks of the SCF hot path (gfx950).
//
// Notation (Sec. 2, Eq. psi_nlm / Eq. u00 and the Zhao family it belongs to):
//   s = r/b, t = s^(1/alpha), q = 1 + t, xi = (t-1)/(t+1) = 1 - 2/q
//   G_l(r) = s^l q^(-alpha(2l+1)) = g0 * w^l,  g0 = q^(-alpha), w = s q^(-2 alpha)
//   U_nl(r) = -(k_n / sqrt(N_nl)) * G_l(r) * p_n^(l)(xi)
// where p_n^(l) is the monic Gegenbauer polynomial C_n^(lambda_l) / k_n,
// lambda_l = (2l+1) alpha + 1/2, obeying p_n = xi p_{n-1} - beta_n^(l) p_{n-2}.
//   Y_lm(theta, phi) = N_lm (-1)^m rho_lm Qt_l^m(cos theta) (sin theta e^{i phi})^m
// where Qt_l^m is the monic-scaled associated Legendre factor obeying
// Qt_l = c Qt_{l-1} - gamma_lm Qt_{l-2}, Qt_m = 1, Qt_{m+1} = c.
// All normalisations (k_n, N_nl, N_lm, rho_lm, the sign of Eq. a_nlm) are
// folded into per-coefficient double-precision scale tables on the host, so
// the kernels only run the two short recurrences.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "scf_dual.h"

namespace scf {

// Single precision: the hardware reciprocal refined by one Newton step,
// x1 = x0 + x0 (1 - v x0).  The bare v_rcp_f32 result is off by up to an ulp
// with a consistent sign over wide ranges of v, which biases cos(theta) = z/r
// and leaves an isotropic sample with a systematic even-l, m = 0 coefficient
// of about 1e-8 of a_000; the refined value removes that bias.
template <typename R>
__device__ __forceinline__ R d_rcp(R v) {
  if constexpr (std::is_same<R, float>::value) {
    const float x0 = __builtin_amdgcn_rcpf(v);
    return fmaf(x0, fmaf(-v, x0, 1.0f), x0);
  } else {
    return R(1) / v;
  }
}
template <typename R>
__device__ __forceinline__ R d_sqrt(R v) { return std::sqrt(v); }
template <typename R>
__device__ __forceinline__ R d_log2(R v) { return std::log2(v); }
template <typename R>
__device__ __forceinline__ R d_exp2(R v) { return std::exp2(v); }

// the same functions on dual numbers: value and first derivative
template <typename T>
__device__ __forceinline__ Dual<T> d_rcp(Dual<T> a) {
  const T r = d_rcp(a.v);
  return {r, -a.d * r * r};
}
template <typename T>
__device__ __forceinline__ Dual<T> d_sqrt(Dual<T> a) {
  const T s = d_sqrt(a.v);
  return {s, s > T(0) ? a.d * T(0.5) / s : T(0)};
}
template <typename T>
__device__ __forceinline__ Dual<T> d_log2(Dual<T> a) {
  return {d_log2(a.v), a.d / (a.v * T(0.69314718055994530942))};
}
template <typename T>
__device__ __forceinline__ Dual<T> d_exp2(Dual<T> a) {
  const T e = d_exp2(a.v);
  return {e, a.d * e * T(0.69314718055994530942)};
}

// alpha modes: 0 -> alpha = 1, 1 -> alpha = 1/2, 2 -> general 0 < alpha <= 1
struct BasisConsts {
  double binv, alpha, inv_alpha;
  int amode;
};

// Radial / angular geometry of one particle.
template <typename R>
struct Geom {
  R r, ir;         // |x| and 1/|x| (0 at the origin)
  R xi, dxi;       // xi and d xi / dr
  R g0, w, om, kap;  // G_0, G_l/G_{l-1}, and the factors of dG_l/dr
  R c, ux, uy;     // cos(theta), sin(theta) cos(phi), sin(theta) sin(phi)
};

template <typename R>
__device__ __forceinline__ Geom<R> make_geom(R x, R y, R z, R binv, R alpha, R inv_alpha,
                                             int amode) {
  Geom<R> g;
  R r2 = x * x + y * y + z * z;
  g.r = d_sqrt(r2);
  g.ir = g.r > R(0) ? d_rcp(g.r) : R(0);
  R s = g.r * binv;
  R iq;
  if (amode == 0) {
    R q = R(1) + s;
    iq = d_rcp(q);
    g.g0 = iq;
    R iq2 = iq * iq;
    g.w = s * iq2;
    g.om = iq2 * binv;
    g.kap = iq * binv;
    g.dxi = R(2) * iq2 * binv;
  } else if (amode == 1) {
    R q = R(1) + s * s;
    iq = d_rcp(q);
    g.g0 = d_sqrt(iq);
    g.w = s * iq;
    g.om = iq * binv;
    g.kap = s * iq * binv;
    g.dxi = R(4) * s * iq * iq * binv;
  } else {
    R ls = s > R(0) ? d_log2(s) : R(0);
    R t = s > R(0) ? d_exp2(ls * inv_alpha) : R(0);
    R tos = s > R(0) ? d_exp2(ls * (inv_alpha - R(1))) : (alpha == R(1) ? R(1) : R(0));
    R q = R(1) + t;
    iq = d_rcp(q);
    g.g0 = d_exp2(-alpha * d_log2(q));
    R g02 = g.g0 * g.g0;
    g.w = s * g02;
    g.om = g02 * binv;
    g.kap = tos * iq * binv;
    g.dxi = R(2) * iq * iq * tos * binv * inv_alpha;
  }
  g.xi = R(1) - R(2) * iq;
  g.c = z * g.ir;
  g.ux = x * g.ir;
  g.uy = y * g.ir;
  return g;
}

}  // namespace scf
