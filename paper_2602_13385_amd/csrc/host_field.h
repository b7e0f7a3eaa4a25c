// Analytic host-galaxy potentials (Appendix A; the logarithmic halo and the
// Plummer sphere are the textbook forms): gradient of psi_host and, for the
// adjoint, its Hessian-vector product and parameter derivatives.  Used by the
// device kernels (float or double) and by the host-side double-precision
// centre-orbit integrator of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace scf {

enum { HOST_LOG = 1, HOST_HERNQUIST = 2, HOST_NFW = 3, HOST_MN = 4, HOST_PLUMMER = 5 };
constexpr int kMaxHostComp = 8;

template <typename R>
struct HostParams {
  int ncomp;
  int kind[kMaxHostComp];
  R G;
  R p[kMaxHostComp][3];
};

template <typename R>
__host__ __device__ inline R h_sqrt(R v) { return std::sqrt(v); }
template <typename R>
__host__ __device__ inline R h_log1p(R v) { return std::log1p(v); }

// radial profile of a spherical component: psi'(r) and psi''(r)
template <typename R>
__host__ __device__ inline void sph_derivs(int kind, R G, const R* p, R r, R& d1, R& d2) {
  switch (kind) {
    case HOST_LOG: {
      R v2 = p[0] * p[0], D = r * r + p[1] * p[1];
      d1 = v2 * r / D;
      d2 = v2 * (p[1] * p[1] - r * r) / (D * D);
    } break;
    case HOST_HERNQUIST: {
      R ra = r + p[1];
      d1 = G * p[0] / (ra * ra);
      d2 = R(-2) * G * p[0] / (ra * ra * ra);
    } break;
    case HOST_NFW: {
      R x = r / p[1];
      R g = h_log1p(x) - x / (R(1) + x);
      R GM = G * p[0];
      d1 = GM * g / (r * r);
      R q = x / (R(1) + x);
      d2 = -(R(2) * GM * g / (r * r * r)) + GM * q * q / (r * r * r);
    } break;
    case HOST_PLUMMER: {
      R D = r * r + p[1] * p[1], sD = h_sqrt(D);
      d1 = G * p[0] * r / (D * sD);
      d2 = G * p[0] * (p[1] * p[1] - R(2) * r * r) / (D * D * sD);
    } break;
    default:
      d1 = R(0);
      d2 = R(0);
  }
}

// gradient of psi_host at position (px, py, pz)
template <typename R>
__host__ __device__ inline void host_grad(const HostParams<R>& H, R px, R py, R pz, R& gx, R& gy,
                                          R& gz) {
  gx = gy = gz = R(0);
  for (int c = 0; c < H.ncomp; ++c) {
    const R* p = H.p[c];
    if (H.kind[c] == HOST_MN) {
      R zeta = h_sqrt(pz * pz + p[2] * p[2]);
      R zab = p[1] + zeta;
      R D2 = px * px + py * py + zab * zab;
      R D = h_sqrt(D2);
      R f = H.G * p[0] / (D2 * D);
      gx += f * px;
      gy += f * py;
      gz += f * pz * zab / zeta;
    } else {
      R r = h_sqrt(px * px + py * py + pz * pz);
      if (r > R(0)) {
        R d1, d2;
        sph_derivs(H.kind[c], H.G, p, r, d1, d2);
        R s = d1 / r;
        gx += s * px;
        gy += s * py;
        gz += s * pz;
      }
    }
  }
}

// Hessian of psi_host at P applied to (ux, uy, uz)
template <typename R>
__host__ __device__ inline void host_hess_vec(const HostParams<R>& H, R px, R py, R pz, R ux, R uy,
                                              R uz, R& hx, R& hy, R& hz) {
  hx = hy = hz = R(0);
  for (int c = 0; c < H.ncomp; ++c) {
    const R* p = H.p[c];
    if (H.kind[c] == HOST_MN) {
      R GM = H.G * p[0];
      R zeta = h_sqrt(pz * pz + p[2] * p[2]);
      R zab = p[1] + zeta;
      R D2 = px * px + py * py + zab * zab;
      R D = h_sqrt(D2);
      R D3 = D2 * D, D5 = D3 * D2;
      R w = zab * pz / zeta;  // d D^2/2 / dz
      R hxx = GM / D3 - R(3) * GM * px * px / D5;
      R hxy = R(-3) * GM * px * py / D5;
      R hxz = R(-3) * GM * px * w / D5;
      R hyy = GM / D3 - R(3) * GM * py * py / D5;
      R hyz = R(-3) * GM * py * w / D5;
      R hzz = GM * ((pz / zeta) * (pz / zeta) + zab * p[2] * p[2] / (zeta * zeta * zeta)) / D3 -
              R(3) * GM * w * w / D5;
      hx += hxx * ux + hxy * uy + hxz * uz;
      hy += hxy * ux + hyy * uy + hyz * uz;
      hz += hxz * ux + hyz * uy + hzz * uz;
    } else {
      R r = h_sqrt(px * px + py * py + pz * pz);
      if (r > R(0)) {
        R d1, d2;
        sph_derivs(H.kind[c], H.G, p, r, d1, d2);
        R ir = R(1) / r;
        R ex = px * ir, ey = py * ir, ez = pz * ir;
        R eu = ex * ux + ey * uy + ez * uz;
        R t = d1 * ir;
        R a = (d2 - t) * eu;
        hx += a * ex + t * ux;
        hy += a * ey + t * uy;
        hz += a * ez + t * uz;
      }
    }
  }
}

// derivative of grad psi_host with respect to parameter k of component c,
// dotted with (ux, uy, uz)
template <typename R>
__host__ __device__ inline R host_dgrad_dparam_dot(const HostParams<R>& H, int c, int k, R px, R py,
                                                   R pz, R ux, R uy, R uz) {
  const R* p = H.p[c];
  const R G = H.G;
  if (H.kind[c] == HOST_MN) {
    R GM = G * p[0];
    R zeta = h_sqrt(pz * pz + p[2] * p[2]);
    R zab = p[1] + zeta;
    R D2 = px * px + py * py + zab * zab;
    R D = h_sqrt(D2);
    R D3 = D2 * D, D5 = D3 * D2;
    if (k == 0) return G * (px * ux + py * uy + pz * zab / zeta * uz) / D3;
    if (k == 1)
      return R(-3) * GM * zab * (px * ux + py * uy) / D5 +
             GM * pz / zeta * (R(1) / D3 - R(3) * zab * zab / D5) * uz;
    R b = p[2];
    return R(-3) * GM * zab * b / (zeta * D5) * (px * ux + py * uy) +
           GM * pz * b *
               (R(1) / (zeta * zeta * D3) - zab / (zeta * zeta * zeta * D3) -
                R(3) * zab * zab / (zeta * zeta * D5)) *
               uz;
  }
  R r = h_sqrt(px * px + py * py + pz * pz);
  if (!(r > R(0))) return R(0);
  R e = (px * ux + py * uy + pz * uz) / r;
  R dp = R(0);
  switch (H.kind[c]) {
    case HOST_LOG: {
      R D = r * r + p[1] * p[1];
      dp = (k == 0) ? R(2) * p[0] * r / D : (k == 1) ? R(-2) * p[0] * p[0] * r * p[1] / (D * D) : R(0);
    } break;
    case HOST_HERNQUIST: {
      R ra = r + p[1];
      dp = (k == 0) ? G / (ra * ra) : (k == 1) ? R(-2) * G * p[0] / (ra * ra * ra) : R(0);
    } break;
    case HOST_NFW: {
      R x = r / p[1];
      R g = h_log1p(x) - x / (R(1) + x);
      dp = (k == 0) ? G * g / (r * r)
                    : (k == 1) ? -G * p[0] * x * x / (p[1] * r * r * (R(1) + x) * (R(1) + x)) : R(0);
    } break;
    case HOST_PLUMMER: {
      R D = r * r + p[1] * p[1], sD = h_sqrt(D);
      dp = (k == 0) ? G * r / (D * sD) : (k == 1) ? R(-3) * G * p[0] * r * p[1] / (D * D * sD) : R(0);
    } break;
    default:
      break;
  }
  return dp * e;
}

}  // namespace scf
