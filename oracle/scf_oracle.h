/*
 * FP64 CPU oracle for the basis-expansion (SCF) N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this library: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * Every routine here is the plain definition written out in double precision,
 * in the order the paper states it, with no tiling, fusion or reordering:
 *   - potential expansion            (Sec. 2, Eqs. total_potential / psi_nlm)
 *   - coefficient estimator          (Sec. 2, Eqs. a_nlm / sumanlm)
 *   - zeroth radial mode             (Sec. 2, Eq. u00; higher modes of the same
 *                                     Zhao (1996) family, see scf_oracle.c)
 *   - host potentials                (Appendix A)
 *   - cluster frame / centre orbit   (Sec. 2.1)
 * plus a kick-drift-kick leapfrog and its exact discrete adjoint.
 *
 * Coefficient storage (shared convention of the ABI, documented, not code):
 *   index(n, l, j) = n*(lmax+1)^2 + l*l + j,  j = 0 -> Re a_{nl0},
 *   j = 2m-1 -> Re a_{nlm}, j = 2m -> Im a_{nlm} for 1 <= m <= l.
 */
#ifndef SCF_ORACLE_H
#define SCF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nmax, lmax;
  double alpha, b, G;
} orc_basis;

enum { ORC_HOST_LOG = 1, ORC_HOST_HERNQUIST = 2, ORC_HOST_NFW = 3,
       ORC_HOST_MN = 4, ORC_HOST_PLUMMER = 5 };

typedef struct {
  int32_t kind, pad;
  double p[3];
} orc_comp;

typedef struct {
  int32_t ncomp, pad;
  double G;
  orc_comp comp[8];
} orc_host;

int64_t orc_ncoef(int32_t nmax, int32_t lmax);

/* OpenMP threads the oracle's parallel loops use, and a setter (n > 0). */
int32_t orc_num_threads(void);
void orc_set_threads(int32_t n);

/* Gegenbauer polynomial C_n^lambda(x) by the three-term recurrence. */
double orc_gegenbauer(int32_t n, double lambda, double x);

/* Unnormalised radial function f_nl(s) and df/ds, n = 0..nmax. */
void orc_radial_raw(double alpha, int32_t l, int32_t nmax, double s, double* f, double* dfds);

/* Energy inner product (b/(4 pi G)) * int [s^2 f1' f2' + l(l+1) f1 f2] ds. */
double orc_energy_inner(const orc_basis* B, int32_t l, int32_t n1, int32_t n2);

/* Normalisation N[n*(lmax+1)+l] = energy inner product of (n,l) with itself. */
void orc_norms(const orc_basis* B, double* N);

/* Normalised U_nl(r) and dU/dr for n = 0..nmax. */
void orc_radial(const orc_basis* B, int32_t l, double r, double* U, double* dU);

/* Complex orthonormal Y_lm, 0 <= m <= l <= lmax, index l(l+1)/2 + m. */
void orc_ylm(int32_t lmax, double theta, double phi, double* re, double* im);

/* a_{nlm} = -sum_k m_k U_nl(r_k) conj(Y_lm(theta_k, phi_k)). */
int orc_coeffs(const orc_basis* B, int64_t n, const double* x, const double* y,
               const double* z, const double* m, double* coef);

/* psi_SCF and g = -grad psi_SCF at n points (any output pointer may be NULL). */
int orc_field(const orc_basis* B, const double* coef, int64_t n, const double* x,
              const double* y, const double* z, double* pot, double* gx, double* gy,
              double* gz);

/* Host potential, gradient, Hessian (row-major 3x3) at one point. */
void orc_host_eval(const orc_host* H, const double* pos, double* pot, double* grad,
                   double* hess);

/* d(grad psi_host)/d(param) for every (component, parameter) pair:
 * out[(c*3 + k)*3 + i] = d (d psi / d x_i) / d p_{c,k}. */
void orc_host_dgrad_dparam(const orc_host* H, const double* pos, double* out);

/* Kick-drift-kick leapfrog in the accelerating cluster frame.  state is
 * x,y,z,vx,vy,vz (each n doubles) updated in place; centre is R[3],V[3]
 * updated in place.  coef_last (may be NULL) receives the coefficients of the
 * final positions; acc (may be NULL, 3n) receives the final accelerations. */
int orc_step(const orc_basis* B, const orc_host* H, int64_t n, double* x, double* y,
             double* z, double* vx, double* vy, double* vz, const double* m,
             double* centre, double dt, int32_t nsteps, double* coef_last, double* acc);

/* nsteps kick-drift-kick steps in the frozen SCF potential of coef plus the
 * host's differential field (Sec. 2.2, between refreshes); the centre
 * (R, V, in/out) follows the same leapfrog in the host alone. */
int orc_step_frozen(const orc_basis* B, const orc_host* H, int64_t n, double* x, double* y,
                    double* z, double* vx, double* vy, double* vz, const double* coef,
                    double* centre, double dt, int32_t nsteps);

/* Power per degree E_l = sum_{n,m} |a_nlm|^2 (m = -l..l), l = 0..lmax. */
void orc_power(int32_t nmax, int32_t lmax, const double* coef, double* El);

/* Frobenius norm of the tidal tensor -Hess psi_host at pos. */
double orc_tidal_norm(const orc_host* H, const double* pos);

/* Test-particle (cluster-centre) orbit in the host alone, same leapfrog.
 * centre R,V updated in place; traj (may be NULL) receives (nsteps+1)*6. */
int orc_orbit(const orc_host* H, double* centre, double dt, int32_t nsteps, double* traj);

/* The same for several clusters concatenated, offsets[nclust+1]; centres is
 * nclust*6, coef_last is nclust*ncoef. */
int orc_step_batched(const orc_basis* B, const orc_host* H, int32_t nclust,
                     const int64_t* offsets, double* x, double* y, double* z, double* vx,
                     double* vy, double* vz, const double* m, double* centres, double dt,
                     int32_t nsteps, double* coef_last);

/* Discrete adjoint of orc_step over nsteps from the given initial state.
 * lam (6n, in: dL/d final state ordered x,y,z,vx,vy,vz; out: dL/d initial
 * state), lam_centre (6, in: dL/d final R,V; out: dL/d initial R,V) and
 * grad_host (ncomp*3, accumulated: dL/d host parameters). */
int orc_step_adjoint(const orc_basis* B, const orc_host* H, int64_t n, const double* x0,
                     const double* y0, const double* z0, const double* vx0,
                     const double* vy0, const double* vz0, const double* m,
                     const double* centre0, double dt, int32_t nsteps, double* lam,
                     double* lam_centre, double* grad_host);

#ifdef __cplusplus
}
#endif
#endif
