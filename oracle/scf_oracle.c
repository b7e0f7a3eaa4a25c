/*
 * FP64 CPU oracle for the basis-expansion (SCF) N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the GPU library.  Everything is double precision and follows the
 * paper's definitions in the paper's order:
 *
 *  * Sec. 2, Eq. (total_potential) and Eq. (psi_nlm): the cluster potential is
 *    psi(r) = sum_{nlm} a_nlm U_n^l(r) Y_l^m(theta, phi), and each basis pair
 *    solves Poisson's equation, so the density pair is fixed by the potential.
 *  * Sec. 2, Eqs. (a_nlm)/(sumanlm): bi-orthogonality isolates each
 *    coefficient, a_nlm = -int rho psi*_nlm, estimated from particles as
 *    a_nlm = -sum_k m_k psi*_nlm(r_k).
 *  * Sec. 2, Eq. (u00): the zeroth radial mode of the tunable Zhao (1996) basis
 *    is proportional to (1 + (r/b)^(1/alpha))^(-alpha).  The paper defers the
 *    higher modes to its companion paper; the oracle uses the Zhao family that
 *    this zeroth mode belongs to,
 *        f_nl(s) = -s^l (1 + s^(1/alpha))^(-alpha(2l+1)) C_n^(lambda_l)(xi),
 *        lambda_l = (2l+1) alpha + 1/2,  xi = (s^(1/alpha)-1)/(s^(1/alpha)+1),
 *    s = r/b (alpha = 1: Hernquist & Ostriker 1992; alpha = 1/2: Clutton-Brock
 *    1973).  Its normalisation is fixed by the minus sign of Eq. (a_nlm):
 *    -int rho_nlm psi*_n'l'm' = delta, i.e. after integrating Poisson's
 *    equation by parts, orthonormality in the energy inner product
 *        N_nl = (b / 4 pi G) int_0^inf [s^2 f'(s)^2 + l(l+1) f(s)^2] ds,
 *        U_nl(r) = f_nl(r/b) / sqrt(N_nl).
 *    N_nl is computed here by quadrature of that definition.
 *  * Y_l^m: complex orthonormal spherical harmonics with the Condon-Shortley
 *    phase, a_{nl,-m} = (-1)^m conj(a_nlm) being implied for a real density.
 *  * Sec. 2.1: the cluster frame is accelerating and non-rotating, centred on a
 *    test particle that follows the host potential; a star at x in that frame
 *    feels -grad psi_SCF(x) - grad psi_host(R + x) + grad psi_host(R).
 *  * Appendix A: host potential components (Hernquist, NFW, Miyamoto-Nagai),
 *    their forces and tidal tensors.  The logarithmic halo and the Plummer
 *    sphere are textbook forms (the paper does not write them out).
 *
 * Derivatives of the basis functions are exact: the radial factor is carried
 * as a one-dimensional second-order jet and the angular factor as a solid
 * harmonic r^l Y_l^m (a polynomial in x, y, z) carried with its exact
 * gradient and Hessian, so poles need no special treatment.  At r = 0 exactly
 * the alpha = 1 basis has a direction-dependent cusp; the oracle returns a
 * zero SCF acceleration there (and the generators never place a particle
 * within 1e-6 of the centre).
 *
 * Parity status: pinned (see the oracle tests) by closed forms, library
 * routines, finite differences and the paper's printed orbit table.
 */
#include "scf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t orc_ncoef(int32_t nmax, int32_t lmax) {
  if (nmax < 0 || lmax < 0) return 0;
  return (int64_t)(nmax + 1) * (lmax + 1) * (lmax + 1);
}

/* ------------------------------------------------------------------------ */
/* Gegenbauer polynomials (textbook three-term recurrence)                  */
/* ------------------------------------------------------------------------ */
double orc_gegenbauer(int32_t n, double lambda, double x) {
  if (n == 0) return 1.0;
  double c0 = 1.0, c1 = 2.0 * lambda * x;
  for (int32_t k = 2; k <= n; ++k) {
    double c2 = (2.0 * (k + lambda - 1.0) * x * c1 - (k + 2.0 * lambda - 2.0) * c0) / k;
    c0 = c1;
    c1 = c2;
  }
  return c1;
}

/* ------------------------------------------------------------------------ */
/* one-dimensional second-order jets: value, first and second derivative    */
/* ------------------------------------------------------------------------ */
typedef struct { double v, d, dd; } jet;

static jet j_const(double c) { jet r = {c, 0.0, 0.0}; return r; }
static jet j_add(jet a, jet b) { jet r = {a.v + b.v, a.d + b.d, a.dd + b.dd}; return r; }
static jet j_scale(jet a, double c) { jet r = {c * a.v, c * a.d, c * a.dd}; return r; }
static jet j_mul(jet a, jet b) {
  jet r = {a.v * b.v, a.d * b.v + a.v * b.d, a.dd * b.v + 2.0 * a.d * b.d + a.v * b.dd};
  return r;
}
static jet j_recip(jet a) {
  double iv = 1.0 / a.v;
  jet r = {iv, -a.d * iv * iv, 2.0 * a.d * a.d * iv * iv * iv - a.dd * iv * iv};
  return r;
}
/* a^p for a.v > 0 (or p a non-negative integer when a.v == 0) */
static jet j_pow(jet a, double p) {
  if (p == 1.0) return a;
  if (p == 0.0) return j_const(1.0);
  jet r;
  r.v = pow(a.v, p);
  double d1 = p * pow(a.v, p - 1.0);
  double d2 = (p == 2.0) ? 2.0 : p * (p - 1.0) * pow(a.v, p - 2.0);
  r.d = d1 * a.d;
  r.dd = d2 * a.d * a.d + d1 * a.dd;
  return r;
}

/* reduced radial function  h_nl(s) = -(1 + s^(1/alpha))^(-alpha(2l+1)) C_n(xi)
 * (so that f_nl(s) = s^l h_nl(s)) as jets in s, n = 0..nmax */
static void reduced_radial_jets(double alpha, int32_t l, int32_t nmax, double s, jet* out) {
  jet js = {s, 1.0, 0.0};
  jet t = j_pow(js, 1.0 / alpha);
  jet q = j_add(j_const(1.0), t);
  jet iq = j_recip(q);
  jet xi = j_add(j_const(1.0), j_scale(iq, -2.0)); /* (t-1)/(t+1) = 1 - 2/q */
  jet pre = j_pow(q, -alpha * (2.0 * l + 1.0));
  double lam = (2.0 * l + 1.0) * alpha + 0.5;
  jet c0 = j_const(1.0);
  jet c1 = j_scale(xi, 2.0 * lam);
  for (int32_t n = 0; n <= nmax; ++n) {
    jet cn;
    if (n == 0) cn = c0;
    else if (n == 1) cn = c1;
    else {
      jet c2 = j_scale(j_add(j_scale(j_mul(xi, c1), 2.0 * (n + lam - 1.0)),
                             j_scale(c0, -(n + 2.0 * lam - 2.0))),
                       1.0 / n);
      c0 = c1;
      c1 = c2;
      cn = c2;
    }
    out[n] = j_scale(j_mul(pre, cn), -1.0);
  }
}

void orc_radial_raw(double alpha, int32_t l, int32_t nmax, double s, double* f, double* dfds) {
  jet* h = (jet*)malloc(sizeof(jet) * (nmax + 1));
  reduced_radial_jets(alpha, l, nmax, s, h);
  jet js = {s, 1.0, 0.0};
  jet sl = j_pow(js, (double)l);
  for (int32_t n = 0; n <= nmax; ++n) {
    jet fn = j_mul(sl, h[n]);
    if (f) f[n] = fn.v;
    if (dfds) dfds[n] = fn.d;
  }
  free(h);
}

/* Energy inner product by quadrature.  With s = e^v the integral becomes
 * int [s^2 f1' f2' + l(l+1) f1 f2] s dv over the whole real line; the
 * substitution v = 2 sinh(t) makes the integrand decay double-exponentially
 * and the trapezoidal rule in t converges geometrically. */
double orc_energy_inner(const orc_basis* B, int32_t l, int32_t n1, int32_t n2) {
  const double h = 1.0 / 64.0, tmax = 4.6;
  int32_t nmx = n1 > n2 ? n1 : n2;
  double* f = (double*)malloc(sizeof(double) * (nmx + 1));
  double* df = (double*)malloc(sizeof(double) * (nmx + 1));
  double acc = 0.0;
  int32_t K = (int32_t)(tmax / h);
  for (int32_t k = -K; k <= K; ++k) {
    double t = k * h;
    double v = 2.0 * sinh(t), dv = 2.0 * cosh(t);
    double s = exp(v);
    orc_radial_raw(B->alpha, l, nmx, s, f, df);
    double integrand = s * s * df[n1] * df[n2] + (double)l * (l + 1.0) * f[n1] * f[n2];
    if (isfinite(integrand)) acc += integrand * s * dv;
  }
  free(f);
  free(df);
  return B->b / (4.0 * M_PI * B->G) * acc * h;
}

void orc_norms(const orc_basis* B, double* N) {
  for (int32_t n = 0; n <= B->nmax; ++n)
    for (int32_t l = 0; l <= B->lmax; ++l) N[n * (B->lmax + 1) + l] = orc_energy_inner(B, l, n, n);
}

void orc_radial(const orc_basis* B, int32_t l, double r, double* U, double* dU) {
  int32_t nmax = B->nmax;
  double* f = (double*)malloc(sizeof(double) * (nmax + 1));
  double* df = (double*)malloc(sizeof(double) * (nmax + 1));
  orc_radial_raw(B->alpha, l, nmax, r / B->b, f, df);
  for (int32_t n = 0; n <= nmax; ++n) {
    double Nn = orc_energy_inner(B, l, n, n);
    double inv = 1.0 / sqrt(Nn);
    if (U) U[n] = f[n] * inv;
    if (dU) dU[n] = df[n] * inv / B->b;
  }
  free(f);
  free(df);
}

/* ------------------------------------------------------------------------ */
/* spherical harmonics                                                       */
/* ------------------------------------------------------------------------ */
/* N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) */
static double ylm_norm(int32_t l, int32_t m) {
  double r = (2.0 * l + 1.0) / (4.0 * M_PI);
  for (int32_t k = l - m + 1; k <= l + m; ++k) r /= k;
  return sqrt(r);
}

/* Y_lm(theta, phi) = N_lm P_l^m(cos theta) e^{i m phi} with
 * P_l^m(x) = (-1)^m (1-x^2)^{m/2} d^m P_l / dx^m; the derivative factor obeys
 * the associated-Legendre recurrence in l. */
void orc_ylm(int32_t lmax, double theta, double phi, double* re, double* im) {
  double c = cos(theta), sn = sin(theta);
  for (int32_t m = 0; m <= lmax; ++m) {
    double dfact = 1.0; /* (2m-1)!! */
    for (int32_t k = 2 * m - 1; k > 1; k -= 2) dfact *= k;
    double qm2 = 0.0, qm1 = 0.0;
    for (int32_t l = m; l <= lmax; ++l) {
      double q;
      if (l == m) q = dfact;
      else if (l == m + 1) q = (2.0 * m + 1.0) * c * qm1;
      else q = ((2.0 * l - 1.0) * c * qm1 - (l + m - 1.0) * qm2) / (l - m);
      qm2 = qm1;
      qm1 = q;
      double P = ((m & 1) ? -1.0 : 1.0) * pow(sn, m) * q;
      double Nlm = ylm_norm(l, m);
      int32_t idx = l * (l + 1) / 2 + m;
      re[idx] = Nlm * P * cos(m * phi);
      im[idx] = Nlm * P * sin(m * phi);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* three-dimensional second-order numbers: value, gradient, Hessian         */
/* Hessian order xx, xy, xz, yy, yz, zz                                      */
/* ------------------------------------------------------------------------ */
typedef struct { double v, g[3], h[6]; } hd;

static const int HI[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static void hd_zero(hd* a) { memset(a, 0, sizeof(hd)); }
static hd hd_c(double c) { hd r; hd_zero(&r); r.v = c; return r; }
static hd hd_var(double x, int i) { hd r; hd_zero(&r); r.v = x; r.g[i] = 1.0; return r; }
static hd hd_add(hd a, hd b, int ord) {
  hd r;
  r.v = a.v + b.v;
  if (ord >= 1) for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] + b.g[i];
  if (ord >= 2) for (int i = 0; i < 6; ++i) r.h[i] = a.h[i] + b.h[i];
  return r;
}
static hd hd_scale(hd a, double c, int ord) {
  hd r;
  r.v = c * a.v;
  if (ord >= 1) for (int i = 0; i < 3; ++i) r.g[i] = c * a.g[i];
  if (ord >= 2) for (int i = 0; i < 6; ++i) r.h[i] = c * a.h[i];
  return r;
}
static hd hd_mul(hd a, hd b, int ord) {
  hd r;
  r.v = a.v * b.v;
  if (ord >= 1)
    for (int i = 0; i < 3; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  if (ord >= 2)
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        int k = HI[i][j];
        r.h[k] = a.v * b.h[k] + b.v * a.h[k] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
      }
  return r;
}
/* lift a radial jet F(r) to a function of (x, y, z) */
static hd hd_from_radial(jet F, const double* p, double r, int ord) {
  hd out;
  hd_zero(&out);
  out.v = F.v;
  if (ord >= 1 && r > 0.0) {
    double u[3] = {p[0] / r, p[1] / r, p[2] / r};
    for (int i = 0; i < 3; ++i) out.g[i] = F.d * u[i];
    if (ord >= 2)
      for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
          out.h[HI[i][j]] = F.dd * u[i] * u[j] + (F.d / r) * ((i == j ? 1.0 : 0.0) - u[i] * u[j]);
  }
  return out;
}

/* All real basis functions b_t(x) of the stored layout, with derivatives up to
 * order ord.  b_{nl,0} = U_nl Y_l0, b_{nl,2m-1} = Re(U_nl Y_lm),
 * b_{nl,2m} = Im(U_nl Y_lm).  Built as U_nl(r)/r^l (a radial jet) times the
 * solid harmonic r^l Y_lm = N_lm (-1)^m (x+iy)^m Pi_l^m(z, r^2), where
 * Pi_l^m = r^(l-m) d^m P_l/dx^m (cos theta) obeys the same recurrence as the
 * associated Legendre functions.  invsqrtN[n*(lmax+1)+l] = N_nl^(-1/2). */
static void basis_eval(const orc_basis* B, const double* invsqrtN, const double* p, int ord,
                       hd* out /* ncoef */, hd* Zre, hd* Zim /* (lmax+1)^2 scratch */,
                       jet* rad /* nmax+1 */) {
  const int32_t nmax = B->nmax, lmax = B->lmax, L1 = lmax + 1;
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  hd X = hd_var(p[0], 0), Y = hd_var(p[1], 1), Z = hd_var(p[2], 2);
  hd R2 = hd_add(hd_add(hd_mul(X, X, ord), hd_mul(Y, Y, ord), ord), hd_mul(Z, Z, ord), ord);
  /* solid harmonics, index l*l + m for 0 <= m <= l */
  hd Ere = hd_c(1.0), Eim = hd_c(0.0); /* (x+iy)^m */
  for (int32_t m = 0; m <= lmax; ++m) {
    if (m > 0) {
      hd nre = hd_add(hd_mul(Ere, X, ord), hd_scale(hd_mul(Eim, Y, ord), -1.0, ord), ord);
      hd nim = hd_add(hd_mul(Ere, Y, ord), hd_mul(Eim, X, ord), ord);
      Ere = nre;
      Eim = nim;
    }
    double dfact = 1.0;
    for (int32_t k = 2 * m - 1; k > 1; k -= 2) dfact *= k;
    hd pim2 = hd_c(0.0), pim1 = hd_c(0.0);
    for (int32_t l = m; l <= lmax; ++l) {
      hd pi;
      if (l == m) pi = hd_c(dfact);
      else if (l == m + 1) pi = hd_scale(hd_mul(Z, pim1, ord), 2.0 * m + 1.0, ord);
      else
        pi = hd_scale(hd_add(hd_scale(hd_mul(Z, pim1, ord), 2.0 * l - 1.0, ord),
                             hd_scale(hd_mul(R2, pim2, ord), -(l + m - 1.0), ord), ord),
                      1.0 / (l - m), ord);
      pim2 = pim1;
      pim1 = pi;
      double c = ylm_norm(l, m) * ((m & 1) ? -1.0 : 1.0);
      Zre[l * l + m] = hd_scale(hd_mul(Ere, pi, ord), c, ord);
      Zim[l * l + m] = hd_scale(hd_mul(Eim, pi, ord), c, ord);
    }
  }
  for (int32_t l = 0; l <= lmax; ++l) {
    reduced_radial_jets(B->alpha, l, nmax, r / B->b, rad);
    /* U_nl / r^l = h_nl(r/b) b^-l / sqrt(N); d/dr = (1/b) d/ds */
    double scl = pow(B->b, -(double)l);
    for (int32_t n = 0; n <= nmax; ++n) {
      double c = scl * invsqrtN[n * L1 + l];
      jet F = {c * rad[n].v, c * rad[n].d / B->b, c * rad[n].dd / (B->b * B->b)};
      hd Fh = hd_from_radial(F, p, r, ord);
      int64_t base = (int64_t)n * L1 * L1 + (int64_t)l * l;
      out[base] = hd_mul(Fh, Zre[l * l], ord);
      for (int32_t m = 1; m <= l; ++m) {
        out[base + 2 * m - 1] = hd_mul(Fh, Zre[l * l + m], ord);
        out[base + 2 * m] = hd_mul(Fh, Zim[l * l + m], ord);
      }
    }
  }
}

typedef struct {
  orc_basis B;
  int64_t T;
  double* invsqrtN;
} basis_ctx;

static void ctx_init(basis_ctx* c, const orc_basis* B) {
  c->B = *B;
  c->T = orc_ncoef(B->nmax, B->lmax);
  int32_t L1 = B->lmax + 1;
  c->invsqrtN = (double*)malloc(sizeof(double) * (B->nmax + 1) * L1);
  orc_norms(B, c->invsqrtN);
  for (int32_t i = 0; i < (B->nmax + 1) * L1; ++i) c->invsqrtN[i] = 1.0 / sqrt(c->invsqrtN[i]);
}
static void ctx_free(basis_ctx* c) { free(c->invsqrtN); }

/* per-thread scratch for basis_eval */
typedef struct { hd* b; hd* zre; hd* zim; jet* rad; } scratch;
static void scratch_init(scratch* s, const orc_basis* B, int64_t T) {
  int32_t L2 = (B->lmax + 1) * (B->lmax + 1);
  s->b = (hd*)malloc(sizeof(hd) * T);
  s->zre = (hd*)malloc(sizeof(hd) * L2);
  s->zim = (hd*)malloc(sizeof(hd) * L2);
  s->rad = (jet*)malloc(sizeof(jet) * (B->nmax + 1));
}
static void scratch_free(scratch* s) { free(s->b); free(s->zre); free(s->zim); free(s->rad); }

/* stored-coefficient sign: Re a = -sum m Re b, Im a = +sum m Im b */
static double coef_sign(int64_t t, int32_t lmax) {
  int32_t L2 = (lmax + 1) * (lmax + 1);
  int32_t lj = (int32_t)(t % L2);
  int32_t l = (int32_t)floor(sqrt((double)lj));
  while (l * l > lj) --l;
  while ((l + 1) * (l + 1) <= lj) ++l;
  int32_t j = lj - l * l;
  return (j > 0 && (j % 2) == 0) ? 1.0 : -1.0;
}
/* weight of a stored coefficient in psi: 1 for m = 0, 2 Re(.) for m > 0 */
static double psi_weight(int64_t t, int32_t lmax) {
  int32_t L2 = (lmax + 1) * (lmax + 1);
  int32_t lj = (int32_t)(t % L2);
  int32_t l = (int32_t)floor(sqrt((double)lj));
  while (l * l > lj) --l;
  while ((l + 1) * (l + 1) <= lj) ++l;
  int32_t j = lj - l * l;
  if (j == 0) return 1.0;
  return (j % 2 == 1) ? 2.0 : -2.0;
}

/* Neumaier compensated accumulation */
static void neu_add(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
  else *c += (x - t) + *s;
  *s = t;
}

/* Deterministic reduction sum_k w_k(t) over particles: fixed chunks, each
 * chunk summed in order, chunks combined in order.  kernel(k, scratch, acc)
 * adds particle k's contribution into acc[T] (sum) via neu_add on (s, c). */
#define ORC_CHUNK 1024

/* ------------------------------------------------------------------------ */
/* coefficients                                                             */
/* ------------------------------------------------------------------------ */
int orc_coeffs(const orc_basis* B, int64_t n, const double* x, const double* y, const double* z,
               const double* m, double* coef) {
  if (!B || B->nmax < 0 || B->lmax < 0 || n < 0 || !coef) return 1;
  basis_ctx C;
  ctx_init(&C, B);
  const int64_t T = C.T;
  int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
  double* part = (double*)calloc((size_t)(nch > 0 ? nch : 1) * T * 2, sizeof(double));
#pragma omp parallel
  {
    scratch S;
    scratch_init(&S, B, T);
#pragma omp for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
      double* ps = part + c * T * 2;
      int64_t k1 = (c + 1) * ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
      for (int64_t k = c * ORC_CHUNK; k < k1; ++k) {
        double p[3] = {x[k], y[k], z[k]};
        basis_eval(B, C.invsqrtN, p, 0, S.b, S.zre, S.zim, S.rad);
        for (int64_t t = 0; t < T; ++t) neu_add(&ps[2 * t], &ps[2 * t + 1], m[k] * S.b[t].v);
      }
    }
    scratch_free(&S);
  }
  for (int64_t t = 0; t < T; ++t) {
    double s = 0.0, cc = 0.0;
    for (int64_t c = 0; c < nch; ++c) {
      neu_add(&s, &cc, part[(c * T + t) * 2]);
      neu_add(&s, &cc, part[(c * T + t) * 2 + 1]);
    }
    coef[t] = coef_sign(t, B->lmax) * (s + cc);
  }
  free(part);
  ctx_free(&C);
  return 0;
}

/* psi and its derivatives at one point from stored coefficients */
static hd field_point(const basis_ctx* C, const double* coef, const double* p, int ord,
                      scratch* S) {
  basis_eval(&C->B, C->invsqrtN, p, ord, S->b, S->zre, S->zim, S->rad);
  hd psi = hd_c(0.0);
  for (int64_t t = 0; t < C->T; ++t)
    psi = hd_add(psi, hd_scale(S->b[t], psi_weight(t, C->B.lmax) * coef[t], ord), ord);
  return psi;
}

int orc_field(const orc_basis* B, const double* coef, int64_t n, const double* x, const double* y,
              const double* z, double* pot, double* gx, double* gy, double* gz) {
  if (!B || !coef || n < 0) return 1;
  basis_ctx C;
  ctx_init(&C, B);
  int ord = (gx || gy || gz) ? 1 : 0;
#pragma omp parallel
  {
    scratch S;
    scratch_init(&S, B, C.T);
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      double p[3] = {x[k], y[k], z[k]};
      hd psi = field_point(&C, coef, p, ord, &S);
      double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      if (pot) pot[k] = psi.v;
      double g[3] = {0.0, 0.0, 0.0};
      if (r > 0.0) { g[0] = -psi.g[0]; g[1] = -psi.g[1]; g[2] = -psi.g[2]; }
      if (gx) gx[k] = g[0];
      if (gy) gy[k] = g[1];
      if (gz) gz[k] = g[2];
    }
    scratch_free(&S);
  }
  ctx_free(&C);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* host potentials (Appendix A; logarithmic and Plummer are textbook)       */
/* ------------------------------------------------------------------------ */
/* spherical components: psi(r), psi'(r), psi''(r) and d psi'/d p_k */
static void sph_profile(const orc_comp* c, double G, double r, double* psi, double* d1,
                        double* d2, double* dp /* 3 */) {
  dp[0] = dp[1] = dp[2] = 0.0;
  switch (c->kind) {
    case ORC_HOST_LOG: {
      double v0 = c->p[0], rc = c->p[1], D = r * r + rc * rc;
      *psi = 0.5 * v0 * v0 * log(D);
      *d1 = v0 * v0 * r / D;
      *d2 = v0 * v0 * (rc * rc - r * r) / (D * D);
      dp[0] = 2.0 * v0 * r / D;
      dp[1] = -2.0 * v0 * v0 * r * rc / (D * D);
    } break;
    case ORC_HOST_HERNQUIST: {
      double M = c->p[0], a = c->p[1], ra = r + a;
      *psi = -G * M / ra;
      *d1 = G * M / (ra * ra);
      *d2 = -2.0 * G * M / (ra * ra * ra);
      dp[0] = G / (ra * ra);
      dp[1] = -2.0 * G * M / (ra * ra * ra);
    } break;
    case ORC_HOST_NFW: {
      double M = c->p[0], rs = c->p[1], xx = r / rs;
      double g = log1p(xx) - xx / (1.0 + xx);
      *psi = (r > 0.0) ? -G * M * log1p(xx) / r : -G * M / rs;
      *d1 = (r > 0.0) ? G * M * g / (r * r) : 0.0;
      /* psi'' = -d f_r / dr with the paper's expression for d f_r / dr */
      *d2 = (r > 0.0) ? -(2.0 * G * M * g / (r * r * r)) *
                            (1.0 - (1.0 / (2.0 * g)) * (xx / (1.0 + xx)) * (xx / (1.0 + xx)))
                      : G * M / (2.0 * rs * rs * rs) * 0.0;
      dp[0] = (r > 0.0) ? G * g / (r * r) : 0.0;
      dp[1] = (r > 0.0) ? -G * M * xx * xx / (rs * r * r * (1.0 + xx) * (1.0 + xx)) : 0.0;
    } break;
    case ORC_HOST_PLUMMER: {
      double M = c->p[0], a = c->p[1], D = r * r + a * a, sD = sqrt(D);
      *psi = -G * M / sD;
      *d1 = G * M * r / (D * sD);
      *d2 = G * M * (a * a - 2.0 * r * r) / (D * D * sD);
      dp[0] = G * r / (D * sD);
      dp[1] = -3.0 * G * M * r * a / (D * D * sD);
    } break;
    default:
      *psi = *d1 = *d2 = 0.0;
  }
}

static void comp_eval(const orc_comp* c, double G, const double* pos, double* pot, double* grad,
                      double* hess, double* dgrad /* [3][3] or NULL */) {
  double x = pos[0], y = pos[1], z = pos[2];
  if (c->kind == ORC_HOST_MN) {
    double M = c->p[0], a = c->p[1], b = c->p[2];
    double zeta = sqrt(z * z + b * b), zab = a + zeta;
    double D2 = x * x + y * y + zab * zab, D = sqrt(D2), D3 = D2 * D, D5 = D3 * D2;
    double GM = G * M;
    *pot += -GM / D;
    grad[0] += GM * x / D3;
    grad[1] += GM * y / D3;
    grad[2] += GM * zab * z / (zeta * D3);
    double h[3][3];
    h[0][0] = GM / D3 - 3.0 * GM * x * x / D5;
    h[0][1] = -3.0 * GM * x * y / D5;
    h[0][2] = -3.0 * GM * x * zab * z / (zeta * D5);
    h[1][1] = GM / D3 - 3.0 * GM * y * y / D5;
    h[1][2] = -3.0 * GM * y * zab * z / (zeta * D5);
    h[2][2] = GM * ((z / zeta) * (z / zeta) + zab * b * b / (zeta * zeta * zeta)) / D3 -
              3.0 * GM * (zab * z / zeta) * (zab * z / zeta) / D5;
    h[1][0] = h[0][1];
    h[2][0] = h[0][2];
    h[2][1] = h[1][2];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) hess[i * 3 + j] += h[i][j];
    if (dgrad) {
      /* d/dM */
      dgrad[0] = G * x / D3;
      dgrad[1] = G * y / D3;
      dgrad[2] = G * zab * z / (zeta * D3);
      /* d/da : dD/da = zab/D */
      dgrad[3] = -3.0 * GM * x * zab / D5;
      dgrad[4] = -3.0 * GM * y * zab / D5;
      dgrad[5] = GM * z / zeta * (1.0 / D3 - 3.0 * zab * zab / D5);
      /* d/db : dzeta/db = b/zeta, dD/db = zab b/(zeta D) */
      dgrad[6] = -3.0 * GM * x * zab * b / (zeta * D5);
      dgrad[7] = -3.0 * GM * y * zab * b / (zeta * D5);
      dgrad[8] = GM * z * b *
                 (1.0 / (zeta * zeta * D3) - zab / (zeta * zeta * zeta * D3) -
                  3.0 * zab * zab / (zeta * zeta * D5));
    }
    return;
  }
  double r = sqrt(x * x + y * y + z * z);
  double psi, d1, d2, dp[3];
  sph_profile(c, G, r, &psi, &d1, &d2, dp);
  *pot += psi;
  if (r > 0.0) {
    double u[3] = {x / r, y / r, z / r};
    for (int i = 0; i < 3; ++i) grad[i] += d1 * u[i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        hess[i * 3 + j] += d2 * u[i] * u[j] + (d1 / r) * ((i == j ? 1.0 : 0.0) - u[i] * u[j]);
    if (dgrad)
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) dgrad[k * 3 + i] = dp[k] * u[i];
  } else {
    for (int i = 0; i < 3; ++i) hess[i * 3 + i] += d2;
    if (dgrad)
      for (int k = 0; k < 9; ++k) dgrad[k] = 0.0;
  }
}

void orc_host_eval(const orc_host* H, const double* pos, double* pot, double* grad, double* hess) {
  double p = 0.0, g[3] = {0, 0, 0}, h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (H)
    for (int32_t c = 0; c < H->ncomp; ++c) comp_eval(&H->comp[c], H->G, pos, &p, g, h, NULL);
  if (pot) *pot = p;
  if (grad) memcpy(grad, g, sizeof(g));
  if (hess) memcpy(hess, h, sizeof(h));
}

void orc_host_dgrad_dparam(const orc_host* H, const double* pos, double* out) {
  if (!H) return;
  for (int32_t c = 0; c < H->ncomp; ++c) {
    double p = 0.0, g[3] = {0, 0, 0}, h[9];
    memset(h, 0, sizeof(h));
    comp_eval(&H->comp[c], H->G, pos, &p, g, h, out + c * 9);
  }
}

/* ------------------------------------------------------------------------ */
/* leapfrog in the accelerating cluster frame                               */
/* ------------------------------------------------------------------------ */
/* acceleration of every particle: -grad psi_SCF(x) - grad psi_host(R + x)
 * + grad psi_host(R) (Sec. 2.1) */
static void accel_all(const orc_basis* B, const orc_host* H, int64_t n, const double* x,
                      const double* y, const double* z, const double* m, const double* R,
                      double* coef, double* ax, double* ay, double* az) {
  if (n == 0) return;
  orc_coeffs(B, n, x, y, z, m, coef);
  orc_field(B, coef, n, x, y, z, NULL, ax, ay, az);
  if (H && H->ncomp > 0) {
    double g0[3];
    orc_host_eval(H, R, NULL, g0, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
      double p[3] = {R[0] + x[k], R[1] + y[k], R[2] + z[k]}, g[3];
      orc_host_eval(H, p, NULL, g, NULL);
      ax[k] += -g[0] + g0[0];
      ay[k] += -g[1] + g0[1];
      az[k] += -g[2] + g0[2];
    }
  }
}

static void centre_accel(const orc_host* H, const double* R, double* g) {
  double gr[3] = {0, 0, 0};
  if (H && H->ncomp > 0) orc_host_eval(H, R, NULL, gr, NULL);
  g[0] = -gr[0];
  g[1] = -gr[1];
  g[2] = -gr[2];
}

int orc_step(const orc_basis* B, const orc_host* H, int64_t n, double* x, double* y, double* z,
             double* vx, double* vy, double* vz, const double* m, double* centre, double dt,
             int32_t nsteps, double* coef_last, double* acc) {
  if (!B || n < 0 || nsteps < 0 || !centre) return 1;
  int64_t T = orc_ncoef(B->nmax, B->lmax);
  double* coef = (double*)malloc(sizeof(double) * T);
  double* ax = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* ay = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* az = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* R = centre;
  double* V = centre + 3;
  double gc[3];
  accel_all(B, H, n, x, y, z, m, R, coef, ax, ay, az);
  centre_accel(H, R, gc);
  const double h = 0.5 * dt;
  for (int32_t s = 0; s < nsteps; ++s) {
    for (int64_t k = 0; k < n; ++k) {
      vx[k] += h * ax[k];
      vy[k] += h * ay[k];
      vz[k] += h * az[k];
    }
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
    for (int64_t k = 0; k < n; ++k) {
      x[k] += dt * vx[k];
      y[k] += dt * vy[k];
      z[k] += dt * vz[k];
    }
    for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    accel_all(B, H, n, x, y, z, m, R, coef, ax, ay, az);
    centre_accel(H, R, gc);
    for (int64_t k = 0; k < n; ++k) {
      vx[k] += h * ax[k];
      vy[k] += h * ay[k];
      vz[k] += h * az[k];
    }
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
  }
  if (coef_last) memcpy(coef_last, coef, sizeof(double) * T);
  if (acc)
    for (int64_t k = 0; k < n; ++k) {
      acc[k] = ax[k];
      acc[n + k] = ay[k];
      acc[2 * n + k] = az[k];
    }
  free(coef);
  free(ax);
  free(ay);
  free(az);
  return 0;
}

/* Kick-drift-kick leapfrog in a frozen SCF potential (Sec. 2.2: between
 * refreshes the particles move in the potential of fixed coefficients coef,
 * plus the host's differential field about the centre, which follows the
 * same leapfrog in the host alone). */
static void accel_frozen(const orc_basis* B, const orc_host* H, int64_t n, const double* x,
                         const double* y, const double* z, const double* coef, const double* R,
                         double* ax, double* ay, double* az) {
  if (n == 0) return;
  orc_field(B, coef, n, x, y, z, NULL, ax, ay, az);
  if (H && H->ncomp > 0) {
    double g0[3];
    orc_host_eval(H, R, NULL, g0, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
      double p[3] = {R[0] + x[k], R[1] + y[k], R[2] + z[k]}, g[3];
      orc_host_eval(H, p, NULL, g, NULL);
      ax[k] += -g[0] + g0[0];
      ay[k] += -g[1] + g0[1];
      az[k] += -g[2] + g0[2];
    }
  }
}

int orc_step_frozen(const orc_basis* B, const orc_host* H, int64_t n, double* x, double* y,
                    double* z, double* vx, double* vy, double* vz, const double* coef,
                    double* centre, double dt, int32_t nsteps) {
  if (!B || n < 0 || nsteps < 0 || !centre || !coef) return 1;
  double* ax = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* ay = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* az = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  double* R = centre;
  double* V = centre + 3;
  double gc[3];
  const double h = 0.5 * dt;
  accel_frozen(B, H, n, x, y, z, coef, R, ax, ay, az);
  centre_accel(H, R, gc);
  for (int32_t s = 0; s < nsteps; ++s) {
    for (int64_t k = 0; k < n; ++k) {
      vx[k] += h * ax[k];
      vy[k] += h * ay[k];
      vz[k] += h * az[k];
    }
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
    for (int64_t k = 0; k < n; ++k) {
      x[k] += dt * vx[k];
      y[k] += dt * vy[k];
      z[k] += dt * vz[k];
    }
    for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    accel_frozen(B, H, n, x, y, z, coef, R, ax, ay, az);
    centre_accel(H, R, gc);
    for (int64_t k = 0; k < n; ++k) {
      vx[k] += h * ax[k];
      vy[k] += h * ay[k];
      vz[k] += h * az[k];
    }
    for (int i = 0; i < 3; ++i) V[i] += h * gc[i];
  }
  free(ax);
  free(ay);
  free(az);
  return 0;
}

/* Power per degree (Sec. 3.5, Fig. power_spectrum_time_series):
 * E_l = sum_n sum_{m=-l}^{l} |a_nlm|^2; with a_{nl,-m} = (-1)^m conj(a_nlm)
 * this is sum_n [a_nl0^2 + 2 sum_{m>=1} (Re^2 + Im^2)]. */
void orc_power(int32_t nmax, int32_t lmax, const double* coef, double* El) {
  const int64_t L2 = (int64_t)(lmax + 1) * (lmax + 1);
  for (int32_t l = 0; l <= lmax; ++l) {
    double s = 0.0;
    for (int32_t n = 0; n <= nmax; ++n)
      for (int32_t j = 0; j <= 2 * l; ++j) {
        const double a = coef[n * L2 + l * l + j];
        s += (j == 0 ? 1.0 : 2.0) * a * a;
      }
    El[l] = s;
  }
}

/* Frobenius norm of the host's tidal tensor T_ij = -d^2 psi_host / dx_i dx_j
 * at pos (Sec. 2.2, Eq. tidal_tensor). */
double orc_tidal_norm(const orc_host* H, const double* pos) {
  double h[9];
  orc_host_eval(H, pos, NULL, NULL, h);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += h[i] * h[i];
  return sqrt(s);
}

int orc_orbit(const orc_host* H, double* centre, double dt, int32_t nsteps, double* traj) {
  if (!centre || nsteps < 0) return 1;
  double* R = centre;
  double* V = centre + 3;
  double g[3];
  const double h = 0.5 * dt;
  if (traj) memcpy(traj, centre, sizeof(double) * 6);
  centre_accel(H, R, g);
  for (int32_t s = 0; s < nsteps; ++s) {
    for (int i = 0; i < 3; ++i) V[i] += h * g[i];
    for (int i = 0; i < 3; ++i) R[i] += dt * V[i];
    centre_accel(H, R, g);
    for (int i = 0; i < 3; ++i) V[i] += h * g[i];
    if (traj) memcpy(traj + 6 * (int64_t)(s + 1), centre, sizeof(double) * 6);
  }
  return 0;
}

int orc_step_batched(const orc_basis* B, const orc_host* H, int32_t nclust, const int64_t* off,
                     double* x, double* y, double* z, double* vx, double* vy, double* vz,
                     const double* m, double* centres, double dt, int32_t nsteps,
                     double* coef_last) {
  if (!B || nclust < 0 || !off) return 1;
  int64_t T = orc_ncoef(B->nmax, B->lmax);
  for (int32_t c = 0; c < nclust; ++c) {
    int64_t a = off[c], n = off[c + 1] - off[c];
    if (n < 0) return 1;
    int rc = orc_step(B, H, n, x + a, y + a, z + a, vx + a, vy + a, vz + a, m + a,
                      centres + 6 * c, dt, nsteps, coef_last ? coef_last + c * T : NULL, NULL);
    if (rc) return rc;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* discrete adjoint of orc_step                                             */
/* ------------------------------------------------------------------------ */
/* With beta_t = sum_k m_k b_t(x_k) the SCF acceleration is
 *   a_i = sum_t w_t beta_t grad b_t(x_i),  w_t = 1 (m = 0) or 2 (m > 0),
 * (psi = -sum_t w_t beta_t b_t).  For cotangents mu_i of a_i the vector-
 * Jacobian product with respect to x_j is
 *   sum_t w_t beta_t Hess b_t(x_j) mu_j + m_j grad(sum_t w_t gamma_t b_t)(x_j),
 *   gamma_t = sum_i mu_i . grad b_t(x_i).
 * The tidal part a_i += h(R + x_i) - h(R), h = -grad psi_host, contributes
 * -Hess psi_host(R + x_j) mu_j to x_j, sum_i [-Hess(R + x_i) + Hess(R)] mu_i
 * to R and sum_i mu_i . [-dgrad/dp(R + x_i) + dgrad/dp(R)] to each host
 * parameter. */
static double psi_w(int64_t t, int32_t lmax) { return fabs(psi_weight(t, lmax)); }

static void accel_vjp(const basis_ctx* C, const orc_host* H, int64_t n, const double* x,
                      const double* y, const double* z, const double* m, const double* R,
                      const double* mu /* 3n: x,y,z blocks */, double* lam /* 3n, += */,
                      double* lamR /* 3, += */, double* gp /* ncomp*3, += */) {
  const int64_t T = C->T;
  const int32_t lmax = C->B.lmax;
  /* beta_t */
  double* beta = (double*)malloc(sizeof(double) * T);
  orc_coeffs(&C->B, n, x, y, z, m, beta);
  for (int64_t t = 0; t < T; ++t) beta[t] *= coef_sign(t, lmax); /* stored -> beta */
  /* gamma_t = sum_i mu_i . grad b_t(x_i), deterministic chunked reduction */
  int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
  double* part = (double*)calloc((size_t)(nch > 0 ? nch : 1) * T * 2, sizeof(double));
#pragma omp parallel
  {
    scratch S;
    scratch_init(&S, &C->B, T);
#pragma omp for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
      double* ps = part + c * T * 2;
      int64_t k1 = (c + 1) * ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
      for (int64_t k = c * ORC_CHUNK; k < k1; ++k) {
        double p[3] = {x[k], y[k], z[k]};
        basis_eval(&C->B, C->invsqrtN, p, 1, S.b, S.zre, S.zim, S.rad);
        double mk[3] = {mu[k], mu[n + k], mu[2 * n + k]};
        for (int64_t t = 0; t < T; ++t)
          neu_add(&ps[2 * t], &ps[2 * t + 1],
                  mk[0] * S.b[t].g[0] + mk[1] * S.b[t].g[1] + mk[2] * S.b[t].g[2]);
      }
    }
    scratch_free(&S);
  }
  double* gam = (double*)malloc(sizeof(double) * T);
  for (int64_t t = 0; t < T; ++t) {
    double s = 0.0, cc = 0.0;
    for (int64_t c = 0; c < nch; ++c) {
      neu_add(&s, &cc, part[(c * T + t) * 2]);
      neu_add(&s, &cc, part[(c * T + t) * 2 + 1]);
    }
    gam[t] = s + cc;
  }
  free(part);
  int nc = H ? H->ncomp : 0;
  double g0dp[8 * 9];
  double hR[9];
  if (nc > 0) {
    orc_host_eval(H, R, NULL, NULL, hR);
    orc_host_dgrad_dparam(H, R, g0dp);
  }
  /* per-particle terms; host reductions per chunk in fixed order */
  double* hpart = (double*)calloc((size_t)(nch > 0 ? nch : 1) * (3 + 24), sizeof(double));
#pragma omp parallel
  {
    scratch S;
    scratch_init(&S, &C->B, T);
#pragma omp for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
      int64_t k1 = (c + 1) * ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
      double* hp = hpart + c * 27;
      for (int64_t k = c * ORC_CHUNK; k < k1; ++k) {
        double p[3] = {x[k], y[k], z[k]};
        double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        double mk[3] = {mu[k], mu[n + k], mu[2 * n + k]};
        basis_eval(&C->B, C->invsqrtN, p, 2, S.b, S.zre, S.zim, S.rad);
        double Hs[6] = {0, 0, 0, 0, 0, 0}, G1[3] = {0, 0, 0};
        for (int64_t t = 0; t < T; ++t) {
          double w = psi_w(t, lmax);
          for (int q = 0; q < 6; ++q) Hs[q] += w * beta[t] * S.b[t].h[q];
          for (int q = 0; q < 3; ++q) G1[q] += w * gam[t] * S.b[t].g[q];
        }
        double out[3];
        for (int i = 0; i < 3; ++i) {
          out[i] = 0.0;
          if (r > 0.0) {
            for (int j = 0; j < 3; ++j) out[i] += Hs[HI[i][j]] * mk[j];
            out[i] += m[k] * G1[i];
          }
        }
        if (nc > 0) {
          double P[3] = {R[0] + p[0], R[1] + p[1], R[2] + p[2]}, hP[9], dP[8 * 9];
          orc_host_eval(H, P, NULL, NULL, hP);
          orc_host_dgrad_dparam(H, P, dP);
          for (int i = 0; i < 3; ++i) {
            double s = 0.0, sR = 0.0;
            for (int j = 0; j < 3; ++j) {
              s += -hP[i * 3 + j] * mk[j];
              sR += (-hP[i * 3 + j] + hR[i * 3 + j]) * mk[j];
            }
            out[i] += s;
            hp[i] += sR;
          }
          for (int cc = 0; cc < nc; ++cc)
            for (int kk = 0; kk < 3; ++kk) {
              double s = 0.0;
              for (int i = 0; i < 3; ++i)
                s += mk[i] * (-dP[(cc * 3 + kk) * 3 + i] + g0dp[(cc * 3 + kk) * 3 + i]);
              hp[3 + cc * 3 + kk] += s;
            }
        }
        lam[k] += out[0];
        lam[n + k] += out[1];
        lam[2 * n + k] += out[2];
      }
    }
    scratch_free(&S);
  }
  for (int64_t c = 0; c < nch; ++c) {
    for (int i = 0; i < 3; ++i) lamR[i] += hpart[c * 27 + i];
    for (int q = 0; q < nc * 3; ++q) gp[q] += hpart[c * 27 + 3 + q];
  }
  free(hpart);
  free(gam);
  free(beta);
}

/* centre kick cotangent: V += h g(R), g = -grad psi_host; nu = h lam_V */
static void centre_vjp(const orc_host* H, const double* R, const double* nu, double* lamR,
                       double* gp) {
  if (!H || H->ncomp == 0) return;
  double hR[9], dR[8 * 9];
  orc_host_eval(H, R, NULL, NULL, hR);
  orc_host_dgrad_dparam(H, R, dR);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) lamR[i] += -hR[i * 3 + j] * nu[j];
  for (int c = 0; c < H->ncomp; ++c)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += -dR[(c * 3 + k) * 3 + i] * nu[i];
      gp[c * 3 + k] += s;
    }
}

int orc_step_adjoint(const orc_basis* B, const orc_host* H, int64_t n, const double* x0,
                     const double* y0, const double* z0, const double* vx0, const double* vy0,
                     const double* vz0, const double* m, const double* centre0, double dt,
                     int32_t nsteps, double* lam, double* lam_centre, double* grad_host) {
  if (!B || n < 0 || nsteps < 0 || !lam || !lam_centre || !grad_host) return 1;
  /* forward trajectory: positions and centre at every step time */
  double* X = (double*)malloc(sizeof(double) * 3 * n * (nsteps + 1) + 8);
  double* RC = (double*)malloc(sizeof(double) * 3 * (nsteps + 1));
  double* x = (double*)malloc(sizeof(double) * 6 * n + 8);
  memcpy(x, x0, sizeof(double) * n);
  memcpy(x + n, y0, sizeof(double) * n);
  memcpy(x + 2 * n, z0, sizeof(double) * n);
  memcpy(x + 3 * n, vx0, sizeof(double) * n);
  memcpy(x + 4 * n, vy0, sizeof(double) * n);
  memcpy(x + 5 * n, vz0, sizeof(double) * n);
  double cen[6];
  memcpy(cen, centre0, sizeof(cen));
  memcpy(X, x, sizeof(double) * 3 * n);
  memcpy(RC, cen, sizeof(double) * 3);
  for (int32_t s = 0; s < nsteps; ++s) {
    orc_step(B, H, n, x, x + n, x + 2 * n, x + 3 * n, x + 4 * n, x + 5 * n, m, cen, dt, 1, NULL,
             NULL);
    memcpy(X + (int64_t)(s + 1) * 3 * n, x, sizeof(double) * 3 * n);
    memcpy(RC + 3 * (s + 1), cen, sizeof(double) * 3);
  }
  basis_ctx C;
  ctx_init(&C, B);
  const double h = 0.5 * dt;
  double* lx = lam;          /* 3n */
  double* lv = lam + 3 * n;  /* 3n */
  double* lR = lam_centre;   /* 3 */
  double* lV = lam_centre + 3;
  double* mu = (double*)malloc(sizeof(double) * 3 * n + 8);
  for (int32_t s = nsteps - 1; s >= 0; --s) {
    const double* xa = X + (int64_t)(s + 1) * 3 * n;
    const double* Ra = RC + 3 * (s + 1);
    /* closing half kicks at step s+1 */
    for (int64_t q = 0; q < 3 * n; ++q) mu[q] = h * lv[q];
    double nu[3] = {h * lV[0], h * lV[1], h * lV[2]};
    accel_vjp(&C, H, n, xa, xa + n, xa + 2 * n, m, Ra, mu, lx, lR, grad_host);
    centre_vjp(H, Ra, nu, lR, grad_host);
    /* drift */
    for (int64_t q = 0; q < 3 * n; ++q) lv[q] += dt * lx[q];
    for (int i = 0; i < 3; ++i) lV[i] += dt * lR[i];
    /* opening half kicks at step s */
    const double* xb = X + (int64_t)s * 3 * n;
    const double* Rb = RC + 3 * s;
    for (int64_t q = 0; q < 3 * n; ++q) mu[q] = h * lv[q];
    double nu2[3] = {h * lV[0], h * lV[1], h * lV[2]};
    accel_vjp(&C, H, n, xb, xb + n, xb + 2 * n, m, Rb, mu, lx, lR, grad_host);
    centre_vjp(H, Rb, nu2, lR, grad_host);
  }
  free(mu);
  ctx_free(&C);
  free(x);
  free(X);
  free(RC);
  return 0;
}
