/*
 * scf.h -- C ABI of libscf, the MI355X (gfx950) implementation of the
 * basis-expansion ("self-consistent field", SCF) N-body hot path.
 *
 * The method (Sec. 2, Eqs. total_potential, psi_nlm, a_nlm, sumanlm): the
 * cluster potential is expanded in bi-orthogonal basis pairs
 *     psi(x) = sum_{n,l,m} a_nlm U_n^l(r) Y_l^m(theta, phi)
 * whose coefficients are estimated from the N particles as
 *     a_nlm = -sum_k m_k U_n^l(r_k) conj(Y_l^m(theta_k, phi_k)).
 * The radial functions are the Zhao (1996) family whose zeroth mode is
 * Eq. (u00), U_0^0 ~ (1 + (r/b)^(1/alpha))^(-alpha):
 *     U_n^l(r) = -s^l (1 + s^(1/alpha))^(-alpha(2l+1)) C_n^(lambda_l)(xi) / sqrt(N_nl),
 *     s = r/b, xi = (s^(1/alpha)-1)/(s^(1/alpha)+1), lambda_l = (2l+1)alpha + 1/2,
 * normalised so that -int rho_nlm psi*_n'l'm' = delta (energy inner product
 * N_nl = (b/4 pi G) int [s^2 f'^2 + l(l+1) f^2] ds).  alpha = 1 is the
 * Hernquist-Ostriker basis, alpha = 1/2 the Clutton-Brock basis; any
 * 0 < alpha <= 1 is accepted.  Y_l^m are complex orthonormal harmonics with the
 * Condon-Shortley phase.  Stars are integrated in the accelerating,
 * non-rotating cluster frame of Sec. 2.1, centred on a test particle that
 * orbits the analytic host potential of Appendix A:
 *     a_i = -grad psi_SCF(x_i) - grad psi_host(R + x_i) + grad psi_host(R).
 *
 * CONVENTIONS
 *  - Particle arrays are structure-of-arrays, one contiguous device array per
 *    component (x, y, z, vx, vy, vz, m, ax, ay, az), element type float for a
 *    plan of dtype SCF_F32 and double for SCF_F64.
 *  - Coefficients are always double, n-major:
 *        index(n, l, j) = n*(lmax+1)^2 + l*l + j,
 *        j = 0 -> Re a_nl0;  j = 2m-1 -> Re a_nlm;  j = 2m -> Im a_nlm  (1<=m<=l),
 *    a_{nl,-m} = (-1)^m conj(a_nlm) being implied.
 *  - Device pointers are caller-owned (e.g. torch tensors).  The workspace is a
 *    caller-allocated, 256-byte-aligned device buffer of at least the size
 *    returned by the matching *_workspace_size query; the library allocates no
 *    device memory on these calls (plans allocate their small tables at
 *    creation).  Output arrays must not alias input arrays unless stated.  Host structs and host arrays are read (and, where stated,
 *    written) during the call only.
 *  - stream is a hipStream_t (NULL = the null stream).  Calls enqueue work and
 *    return; device outputs are valid once the stream reaches that point.
 *    Host outputs (centre states, host gradients) are valid on return.
 *  - Errors: arguments are validated before any launch; on error nothing is
 *    enqueued and outputs are untouched.  HIP failures return SCF_ERR_HIP.
 *    scf_last_error() gives a thread-local message for the last failure.
 *    n == 0 is a valid, successful call.  No C++ exception crosses the ABI.
 */
#ifndef SCF_H
#define SCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCF_OK = 0,
  SCF_ERR_INVALID_ARG = 1, /* null pointer, negative size, bad enum, bad offsets */
  SCF_ERR_UNSUPPORTED = 2, /* (nmax, lmax) or alpha outside the compiled range */
  SCF_ERR_WORKSPACE = 3,   /* workspace pointer null or smaller than required */
  SCF_ERR_NONFINITE = 4,   /* reserved: non-finite input detected */
  SCF_ERR_HIP = 5          /* a HIP runtime call failed (message in scf_last_error) */
} scf_status;

typedef enum { SCF_F32 = 0, SCF_F64 = 1 } scf_dtype;

/* Basis (Sec. 2): n = 0..nmax, l = 0..lmax inclusive; scale radius b > 0,
 * exponent 0 < alpha <= 1, gravitational constant G > 0. */
typedef struct {
  int32_t nmax, lmax;
  double alpha, b, G;
} scf_basis;

/* Host-potential components (Appendix A; LOG and PLUMMER are the textbook
 * forms).  Parameters p[]:
 *   SCF_HOST_LOG        psi = (v0^2/2) ln(r^2 + rc^2)            p = {v0, rc}
 *   SCF_HOST_HERNQUIST  psi = -G M / (r + a)                       p = {M, a}
 *   SCF_HOST_NFW        psi = -G M ln(1 + r/rs) / r                p = {M, rs}
 *   SCF_HOST_MN         psi = -G M / sqrt(R^2 + (a + sqrt(z^2+b^2))^2)  p = {M, a, b}
 *   SCF_HOST_PLUMMER    psi = -G M / sqrt(r^2 + a^2)               p = {M, a}   */
enum {
  SCF_HOST_LOG = 1,
  SCF_HOST_HERNQUIST = 2,
  SCF_HOST_NFW = 3,
  SCF_HOST_MN = 4,
  SCF_HOST_PLUMMER = 5
};
#define SCF_MAX_HOST_COMP 8

typedef struct {
  int32_t kind, pad;
  double p[3];
} scf_host_comp;

typedef struct {
  int32_t ncomp, pad; /* 0 <= ncomp <= SCF_MAX_HOST_COMP; 0 = isolated cluster */
  double G;
  scf_host_comp comp[SCF_MAX_HOST_COMP];
} scf_host;

typedef struct scf_plan scf_plan;

/* scf_step flags */
#define SCF_STEP_ACC_VALID 1u /* ax, ay, az already hold a(x) at entry */
#define SCF_STEP_NO_GRAPH 2u  /* scf_step_batched: launch the kernels directly (the default) */
#define SCF_STEP_GRAPH 4u     /* scf_step_batched: replay the middle steps from HIP graphs */

/* (nmax+1)(lmax+1)^2, or 0 for negative arguments. */
int64_t scf_ncoef(int32_t nmax, int32_t lmax);

/* Create a plan for one basis and dtype on the current HIP device: basis
 * tables (normalisations of Sec. 2, recurrence constants) are computed in
 * double precision on the host and copied to the device.  flags must be 0. */
scf_status scf_plan_create(scf_plan** plan, const scf_basis* basis, int32_t dtype, uint32_t flags);
void scf_plan_destroy(scf_plan* plan);

/* Workspace bytes for scf_coeffs / scf_forces / scf_step on n particles
 * (nclusters = 1) or for scf_step_batched with nclusters clusters totalling n. */
scf_status scf_workspace_size(const scf_plan* plan, int64_t n, int32_t nclusters, size_t* bytes);

/* Coefficients of Eq. (sumanlm): coef (device, ncoef doubles) receives
 * a_nlm = -sum_k m_k U_nl(r_k) conj(Y_lm), about the origin of x, y, z.
 * Single-precision plans accumulate each lane's terms in single precision
 * over at most 16 stages of its thread block (about 150 particles at nmax 16,
 * lmax 10, whatever n is), then add the block's sums into a (hi, lo) pair of
 * single-precision partials with an error-free two-sum; double-precision
 * plans accumulate in double precision.  The partials of all blocks are
 * summed in double precision in a fixed order. */
scf_status scf_coeffs(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                      const void* m, double* coef, void* ws, size_t ws_bytes, void* stream);

/* Accelerations at n points from coefficients coef (device, ncoef doubles):
 * a = -grad psi_SCF (Eq. total_potential) plus, if host != NULL and
 * host->ncomp > 0, the tidal term -grad psi_host(centre + x) + grad psi_host(centre)
 * with centre[3] a host array.  pot (nullable) receives psi_SCF. */
scf_status scf_forces(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                      const double* coef, const scf_host* host, const double* centre, void* ax,
                      void* ay, void* az, void* pot, void* ws, size_t ws_bytes, void* stream);

/* nsteps kick-drift-kick leapfrog steps of size dt in the cluster frame:
 * every step recomputes the coefficients from all particles (Eq. sumanlm),
 * the SCF + tidal accelerations, and kicks/drifts the particles.  The frame
 * centre (centre[6] = R, V, host array, in/out) follows the same leapfrog in
 * the host potential alone, in double precision on the host.  The state
 * (x, y, z, vx, vy, vz, and ax, ay, az = a at the final positions) is
 * synchronised on return.  With SCF_STEP_ACC_VALID ax, ay, az must hold a(x)
 * at entry; otherwise the call first evaluates it.  coef_last (device,
 * nullable) receives the coefficients of the final positions. */
scf_status scf_step(scf_plan* plan, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                    void* vz, const void* m, void* ax, void* ay, void* az, uint32_t step_flags,
                    const scf_host* host, double* centre, double dt, int32_t nsteps,
                    double* coef_last, void* ws, size_t ws_bytes, void* stream);

/* Elements of one force-weight row of the plan, (nmax bound + 1)(lmax + 1)^2:
 * the coefficients of Eq. (total_potential) times their normalisations, in
 * the plan's real type, as the field kernels read them. */
int64_t scf_plan_weights_size(const scf_plan* plan);

/* scf_step that also keeps the force weights of every kick: row k of w_hist
 * (device, (nsteps + 1) * scf_plan_weights_size(plan) elements of the plan's
 * real type, caller-owned) receives the weights from the coefficients at x_k,
 * k = 1..nsteps, and row 0 those at the starting positions when the call
 * evaluates a(x0) (without SCF_STEP_ACC_VALID; otherwise row 0 is left as it
 * is).  The rows let scf_step_adjoint replay the segment without its
 * coefficient passes.  Everything else is as for scf_step. */
scf_status scf_step_keep_weights(scf_plan* plan, int64_t n, void* x, void* y, void* z, void* vx,
                                 void* vy, void* vz, const void* m, void* ax, void* ay, void* az,
                                 uint32_t step_flags, const scf_host* host, double* centre,
                                 double dt, int32_t nsteps, double* coef_last, void* w_hist,
                                 void* ws, size_t ws_bytes, void* stream);

/* scf_step for nclusters independent clusters concatenated in the particle
 * arrays: cluster c owns particles [offsets[c], offsets[c+1]) (host array of
 * nclusters+1 entries, offsets[0] = 0, non-decreasing; n = offsets[nclusters]).
 * Each cluster has its own coefficients (Eq. sumanlm over its own particles)
 * and frame centre (centres: host, nclusters*6 = R, V per cluster, in/out,
 * advanced in double precision on the host); all share the host potential.
 * One step is one launch each of the coefficient, reduction, finalisation and
 * field kernels for all clusters together, driven by static work lists (a
 * cluster's particle ranges per wave-unit, its partial rows, its 256-particle
 * field blocks) built on the host per call.  The kernels are launched
 * directly on stream by default.  With SCF_STEP_GRAPH (and without
 * SCF_STEP_NO_GRAPH) the middle steps (all but the last) are instead
 * replayed from HIP graphs of one and of eight steps, captured once on a
 * plan-owned stream and recaptured when pointers, sizes, dt or the host
 * change; the results are bitwise identical.  On the MI355X the direct
 * launches are the faster of the two.  The per-step centre rows are uploaded in chunks of 256
 * steps and selected on the device.  The workspace must come from
 * scf_workspace_size(plan, n, nclusters).  step_flags and the returned state
 * are as for scf_step; coef_last (device, nullable) receives nclusters*ncoef
 * doubles, cluster-major.  A plan must not run two batched calls
 * concurrently (the graph and the pinned staging buffers are per plan). */
scf_status scf_step_batched(scf_plan* plan, int32_t nclusters, const int64_t* offsets, void* x,
                            void* y, void* z, void* vx, void* vy, void* vz, const void* m,
                            void* ax, void* ay, void* az, uint32_t step_flags, const scf_host* host,
                            double* centres, double dt, int32_t nsteps, double* coef_last,
                            void* ws, size_t ws_bytes, void* stream);

/* Reverse mode of scf_step over one segment of nsteps steps starting from
 * the synchronised state (x0..vz0, centre0[6], host array).  The forward
 * segment is recomputed on the device from that state.  lam[6] are device
 * arrays (x, y, z, vx, vy, vz components) holding dL/d(final state) on entry
 * and dL/d(initial state) on return; lam_centre[6] (host, in/out) likewise
 * for the centre R, V; grad_host (host, host->ncomp*3 doubles) accumulates
 * dL/d(host parameters p[]).  w_hist (device, nullable) holds the force
 * weights of the segment's kicks 0..nsteps as scf_step_keep_weights wrote them
 * for the same starting state (without SCF_STEP_ACC_VALID); with them the
 * recompute runs only the field passes, without w_hist it also recomputes the
 * coefficients.  Blocks until the results are on the host. */
scf_status scf_step_adjoint(scf_plan* plan, int64_t n, const void* x0, const void* y0,
                            const void* z0, const void* vx0, const void* vy0, const void* vz0,
                            const void* m, const scf_host* host, const double* centre0, double dt,
                            int32_t nsteps, void* const* lam, double* lam_centre,
                            double* grad_host, const void* w_hist, void* ws, size_t ws_bytes,
                            void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): scf_step
 * with no workspace argument.  The workspace is a file-scope device array of
 * scf_noalloc_scratch_bytes() bytes (64 MiB) that every GPU the library runs
 * on holds until the process ends; its device address is looked up once per
 * device on the first call there.  The call allocates nothing.  Arguments,
 * state, results and errors are those of scf_step; in addition the call
 * returns SCF_ERR_WORKSPACE, with nothing enqueued, when the plan's step
 * needs more than the array holds (scf_workspace_size's single-cluster figure
 * for this n, which stops growing once n covers one resident round of the
 * coefficient pass), and SCF_ERR_INVALID_ARG when the current device is not
 * the plan's.  All calls on one GPU share the array: calls that overlap on
 * one GPU (other host threads, or streams without ordering between them) race
 * on it. */
size_t scf_noalloc_scratch_bytes(void);
scf_status scf_step_noalloc(scf_plan* plan, int64_t n, void* x, void* y, void* z, void* vx,
                            void* vy, void* vz, const void* m, void* ax, void* ay, void* az,
                            uint32_t step_flags, const scf_host* host, double* centre, double dt,
                            int32_t nsteps, double* coef_last, void* stream);

/* Workspace bytes for scf_step_adjoint (grows with n * nsteps: the segment's
 * positions are kept on the device). */
scf_status scf_adjoint_workspace_size(const scf_plan* plan, int64_t n, int32_t nsteps,
                                      size_t* bytes);

/* Diagnostics (Sec. 3.5, Fig. power_spectrum_time_series).
 * scf_power_spectrum: for each of ncoefsets coefficient vectors (device,
 * ncoefsets*ncoef doubles, as written by the calls above) the power per
 * degree E_l = sum_n sum_{m=-l..l} |a_nlm|^2 = sum_n [a_nl0^2 + 2 sum_{m>=1}
 * (Re^2 + Im^2)] into power (device, ncoefsets*(lmax+1) doubles), on stream.
 * sum_l E_l = -2 W with W = 1/2 sum_k m_k psi_SCF(x_k).
 * scf_tidal_norm: the Frobenius norm of the host's tidal tensor
 * T_ij = -d^2 psi_host / dx_i dx_j (Sec. 2.2, Eq. tidal_tensor) at pos[3]
 * (host arrays, double precision, no device work). */
scf_status scf_power_spectrum(scf_plan* plan, int32_t ncoefsets, const double* coef,
                              double* power, void* stream);
scf_status scf_tidal_norm(const scf_host* host, const double* pos, double* norm);

/* ---- Refresh cadence (Sec. 2.2) ----------------------------------------
 * Between refreshes the particles move in a frozen SCF potential.  The
 * integration interval is Delta t_int = sqrt(eta) (|T|_F^2 / 6)^(-1/4)
 * (Eq. tidal_timestep) with T the host tidal tensor (Eq. tidal_tensor) at the
 * centre at the start of the interval; it is covered by ceil(Delta t_int /
 * dt_max) equal kick-drift-kick substeps.  At its end the particles are
 * selected in the potential they moved in: a particle is bound when
 * |v|^2/2 + psi_SCF(x) < 0 (cluster frame; the paper's direct pair sum is
 * replaced by psi_SCF, with the kinetic factor 1/2), r_x is the k-th smallest
 * radius of the bound particles with k = ceil(x N_b) (an energy Lagrange
 * radius), and only bound particles with r <= r_x enter the coefficient sum,
 * with weight m (x = 0.999 in the paper).  Every refresh_every-th interval is
 * a complete refresh: the coefficients of Eq. (sumanlm) over the selected
 * particles.  The others are intermediate refreshes: the particles whose
 * weight changed are added with weight w_new - w_old (recaptured: +m, lost:
 * -m).  Orbit samples: N_s = max(1, ceil(n_s Delta t_int / t_dyn)) (capped by
 * the substep count and ns_max), t_dyn = c_dyn sqrt(r_hm^3 / (G M_b)) with the
 * bound mass M_b and r_hm = r_50 of the previous selection; sample j is the
 * positions after substep ceil((j+1) nsub / N_s), and a refresh averages its
 * sums over the samples.  Radii are compared through |x|^2 = (x x + y y) + z z
 * with every operation rounded in the plan's precision.  With recentre set, a
 * complete refresh first moves the frame origin to the maximum of a_000 over
 * the selected particles (scf_recentre from the current origin, tol 1e-6 b,
 * at most 100 steps; positions, samples and the centre orbit's R shift), then
 * computes the coefficients, then moves the frame velocity to the core
 * velocity of the new potential (scf_core; velocities and V shift).  With
 * retune, a complete refresh (after any recentring) also sets the plan's
 * alpha and b to scf_tune_basis's result over the selected particles before
 * the coefficients are computed, so the coefficients and the plan's basis
 * change together. */
#define SCF_MAX_SAMPLES 16
typedef struct {
  double eta;             /* Eq. tidal_timestep parameter (1/400 in the paper), > 0 */
  double dt_max;          /* largest substep, > 0 */
  double frac;            /* x of the selection radius r_x, in (0, 1] (0.999) */
  double c_dyn;           /* t_dyn = c_dyn sqrt(r_hm^3 / (G M_b)); 2.91430 restates the
                             paper's formula (4.3451 Myr at 1e5 Msun, 10 pc) for any units */
  int32_t refresh_every;  /* complete refresh every this many intervals (5), >= 1 */
  int32_t n_samples_tdyn; /* orbit samples per t_dyn (the paper: 1); 0: one sample at the end */
  int32_t ns_max;         /* most samples per interval, 1..SCF_MAX_SAMPLES */
  int32_t recentre;       /* 1: at complete refreshes move the frame to the a_000 maximum
                             and the core velocity (scf_recentre, scf_core) */
  int32_t retune;         /* 1: at complete refreshes retune alpha and b (scf_tune_basis;
                             the plan's basis changes) */
  int32_t pad;
  double alpha_min;       /* lower bound of alpha for retune, in (0, 1) */
} scf_cadence;

/* The paper's cadence parameters (Sec. 2.2): eta = 1/400, dt_max = 0.005,
 * frac = 0.999, a complete refresh every fifth interval, one orbit sample per
 * t_dyn with c_dyn restating t_dyn = 4.3451 Myr at 1e5 Msun and 10 pc
 * (2.91430...), at most 8 samples per interval, no recentring or retuning,
 * alpha_min = 0.25. */
void scf_cadence_defaults(scf_cadence* cadence);

/* Cadence state carried between calls (host, in/out). */
typedef struct {
  int32_t since;  /* intervals since the last complete refresh */
  int32_t pad;
  int64_t nbound; /* of the last selection: bound count N_b, */
  double rx;      /* r_x, */
  double rhm;     /* r_50, */
  double mbound;  /* and bound mass M_b */
} scf_cadence_state;

/* One record per integration interval (host). */
typedef struct {
  double dt_int;          /* Delta t_int */
  int32_t nsub, nsamples; /* substeps and orbit samples */
  int32_t complete, pad;  /* 1: complete refresh, 0: intermediate */
  int64_t nbound, nchanged; /* bound particles; particles whose weight changed */
  double rx, rhm, mbound;
  double dx[3], dv[3];    /* frame shift applied at this interval's end (recentre) */
  double alpha, b;        /* the plan's basis after this interval (retune) */
} scf_interval_log;

/* Workspace bytes for scf_select, scf_coeffs_delta, scf_cadence_init and
 * scf_evolve on n particles keeping up to ns_max orbit samples. */
scf_status scf_cadence_workspace_size(const scf_plan* plan, int64_t n, int32_t ns_max,
                                      size_t* bytes);

/* nsteps kick-drift-kick steps of size dt in the frozen potential of coef
 * (device, ncoef doubles) plus the host's differential field; the centre
 * (centre[6], host, in/out) follows the same leapfrog in the host alone, in
 * double precision.  State and flags as for scf_step (ax, ay, az hold a(x)
 * at the final positions on return). */
scf_status scf_step_frozen(scf_plan* plan, int64_t n, void* x, void* y, void* z, void* vx,
                           void* vy, void* vz, void* ax, void* ay, void* az, uint32_t step_flags,
                           const double* coef, const scf_host* host, double* centre, double dt,
                           int32_t nsteps, void* ws, size_t ws_bytes, void* stream);

/* Selection in the potential of coef: w (device, n, plan dtype) receives
 * m [bound and r <= r_frac], bound (device bytes, nullable) the bound flags,
 * out (host) N_b, r_frac, r_50 and M_b (its since field is left as is).
 * Blocks until out is written. */
scf_status scf_select(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                      const void* vx, const void* vy, const void* vz, const void* m,
                      const double* coef, double frac, void* w, uint8_t* bound,
                      scf_cadence_state* out, void* ws, size_t ws_bytes, void* stream);

/* Intermediate refresh: coef (device, in/out) += (1/nsnap) sum_j
 * a(snapshot j; w_new - w_old), the coefficients of Eq. (sumanlm) of the
 * particles whose weight changed, at nsnap position snapshots (snaps: host
 * array of 3*nsnap device pointers x_0, y_0, z_0, x_1, ...), 1 <= nsnap <=
 * SCF_MAX_SAMPLES.  The changed particles are compacted first, so the cost
 * follows their number, written to *nchanged (host).  Blocks until done. */
scf_status scf_coeffs_delta(scf_plan* plan, int64_t n, int32_t nsnap, const void* const* snaps,
                            const void* w_old, const void* w_new, double* coef, int64_t* nchanged,
                            void* ws, size_t ws_bytes, void* stream);

/* Start of a cadence: the coefficients of all particles, the selection in
 * their potential (fraction frac), and a complete refresh over the selected
 * particles into coef (device); w (device) receives the weights and state
 * (host) the selection, with since = 0.  Blocks. */
scf_status scf_cadence_init(scf_plan* plan, int64_t n, const void* x, const void* y,
                            const void* z, const void* vx, const void* vy, const void* vz,
                            const void* m, double frac, double* coef, void* w,
                            scf_cadence_state* state, void* ws, size_t ws_bytes, void* stream);

/* nint integration intervals of the cadence from the state (x..vz, centre),
 * the current coefficients coef (device, in/out), the current weights w
 * (device, in/out) and the cadence state (host, in/out).  ax, ay, az are
 * scratch (device, n each; a(x) in the last potential on return).  log
 * (host, nullable) receives nint records.  Blocks once per interval (the
 * selection's results come to the host). */
scf_status scf_evolve(scf_plan* plan, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                      void* vz, const void* m, void* ax, void* ay, void* az,
                      const scf_host* host, double* centre, const scf_cadence* cadence,
                      int32_t nint, double* coef, void* w, scf_cadence_state* state,
                      scf_interval_log* log, void* ws, size_t ws_bytes, void* stream);

/* Density and frame core (Sec. 2, Eq. total_dens; Sec. 2.1).
 * scf_density: rho_SCF = sum a_nlm D_n^l Y_l^m at n points (rho: device, n,
 * plan dtype) from coef (device).  The density basis follows from Poisson's
 * equation, nabla^2 psi^(nlm) = 4 pi G rho^(nlm), in closed form through the
 * Gegenbauer differential equation:
 *     D_n^l(r) = -K_nl s^(1/alpha - 2) (1 + s^(1/alpha))^(-2) U_n^l(r) / (4 pi G b^2),
 *     K_nl = [n(n + 2 lambda_l) + p_l(p_l + 1)] / alpha^2,  p_l = alpha(2l+1).
 * At r = 0 the value is not finite for alpha > 1/2 (the basis' central cusp).
 * scf_core: over the particles with w > 0 (device, plan dtype), the core
 * radius r_core = sqrt(sum rho^2 r^2 / sum rho^2) with rho = rho_SCF of coef at
 * each particle, and the mass-weighted mean velocity of those with r <= r_core
 * (the frame velocity of Sec. 2.1); r^2 is formed in double precision.
 * out (host, 5 doubles) = r_core, v_core[3], core mass; all zero when no
 * particle has w > 0.  Blocks.  Both use the workspace of
 * scf_cadence_workspace_size(plan, n, 1). */
scf_status scf_density(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                       const double* coef, void* rho, void* ws, size_t ws_bytes, void* stream);
scf_status scf_core(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                    const void* vx, const void* vy, const void* vz, const void* m, const void* w,
                    const double* coef, double* out, void* ws, size_t ws_bytes, void* stream);

/* Frame centre (Sec. 2.1): the origin that maximises the monopole
 * coefficient a_000 of the particles with w > 0.  About c, a_000(c) is
 * proportional to sum_k w_k g(|x_k - c|), g(r) = (1 + (r/b)^(1/alpha))^(-alpha)
 * (Eq. u00); its stationary points satisfy c = sum w omega x / sum w omega
 * with omega = -g'(r)/r, and this fixed-point iteration (which never lowers
 * a_000) runs from centre (host in/out, 3 doubles) until a step is at most
 * tol * b or maxit steps are taken (*steps, nullable, receives the count).
 * Particles within 1e-9 b of the current point are left out of a step.  The
 * per-particle terms and sums are in double precision.  Blocks; workspace of
 * scf_cadence_workspace_size(plan, n, 1). */
scf_status scf_recentre(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                        const void* w, double* centre, double tol, int32_t maxit, int32_t* steps,
                        void* ws, size_t ws_bytes, void* stream);

/* Basis parameters (Sec. 2, Eq. u00 and the text after it): alpha and b are
 * tuned so that the zeroth mode matches the cluster potential.  About the
 * origin, a_000 = Y_00 sum_k w_k f(r_k) / sqrt(N_00) with
 * f = (1 + (r/b)^(1/alpha))^(-alpha) and the energy norm
 * N_00 = b alpha B(alpha + 2, alpha) / (4 pi G) (B the Beta function); the
 * basis is orthonormal in that norm, so a_000 is the projection of the
 * cluster potential on the unit zeroth mode and its maximum picks the zeroth
 * mode closest to it.  scf_tune_basis maximises it over alpha in
 * [alpha_min, 1] and b > 0 for the particles with w > 0: the best point of a
 * 7 x 17 grid in (alpha, ln b) about the start, then a Nelder-Mead search
 * with alpha = alpha_min + (1 - alpha_min) sin^2 u; each value is a
 * double-precision device reduction.  alpha_b (host, 2 doubles): in, the
 * start (alpha, b); out, the maximum; a000 (host, nullable) its value.
 * Blocks; workspace of scf_cadence_workspace_size(plan, n, 1).
 * scf_plan_set_basis replaces a plan's alpha and b (nmax, lmax, G and dtype
 * stay): the basis tables are recomputed and copied to the device after the
 * device has finished all queued work.  Coefficients computed before the
 * change belong to the old basis.  scf_plan_get_basis reads the current one. */
scf_status scf_tune_basis(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                          const void* w, double alpha_min, double* alpha_b, double* a000,
                          void* ws, size_t ws_bytes, void* stream);
scf_status scf_plan_set_basis(scf_plan* plan, double alpha, double b);
scf_status scf_plan_get_basis(const scf_plan* plan, scf_basis* out);

/* Launch configuration.  Single-precision plans have one coefficient
 * kernel (blocks of four waves sharing each stage of particles, compensated
 * folds); double-precision plans have three compiled variants (lanes per
 * particle in the basis phase).  The grid is one resident round of units
 * divided by 1, 2, 4 or 8 (fewer, longer units amortise their set-up and
 * partial rows when n is small).
 * scf_autotune times each (variant, divisor) on the given particles
 * (synchronising the stream) and keeps the fastest for the plan; best_ms
 * (nullable) receives its time per call in milliseconds.  Timing: one
 * untimed call of each candidate, then three interleaved rounds of eight
 * back-to-back calls per candidate; a candidate's time is its best round.
 * scf_autotune_field times the field variants the same way.
 * Variants give results that agree to rounding (the particle sums are grouped
 * differently); a fixed variant is bitwise reproducible. */
int32_t scf_plan_num_variants(const scf_plan* plan);
/* Number of HIP graphs the plan has captured for scf_step_batched so far. */
int32_t scf_plan_graph_captures(const scf_plan* plan);
int32_t scf_plan_variant(const scf_plan* plan);
scf_status scf_plan_set_variant(scf_plan* plan, int32_t variant);
int32_t scf_plan_coef_units_div(const scf_plan* plan);
scf_status scf_plan_set_coef_units_div(scf_plan* plan, int32_t div);
const char* scf_plan_describe(const scf_plan* plan);
scf_status scf_autotune(scf_plan* plan, int64_t n, const void* x, const void* y, const void* z,
                        const void* m, void* ws, size_t ws_bytes, void* stream, double* best_ms);

/* The field kernel has compiled variants too.  Variants 0 and 1 evaluate the
 * radial sums of Eq. total_potential on the vector ALUs, under two register
 * budgets per thread (the compiler's own, or one that allows at least 4 waves
 * per SIMD); their results are bitwise identical.  Single-precision plans add
 * variants 2 and 3: the same sums as 4x4x1 matrix-core (MFMA) products in
 * persistent blocks, again under two register budgets (the compiler's own, or
 * 5 waves per SIMD); these two agree bitwise with each other and, since they
 * sum in another order, with variants 0 and 1 to the single-precision force
 * tolerance.  The last two variants (4 and 5 in single, 2 and 3 in double
 * precision) run the vector-ALU sums with each particle's degrees split over
 * 2 or 4 waves of one block, which add their partial sums through LDS: more
 * waves for few particles; they agree with variants 0 and 1 to the force
 * tolerance of the plan's precision.  The batched step runs variant 1's
 * kernel for every variant above 0 (its per-cluster blocks measured faster
 * on the vector ALUs), and the adjoint's accumulation pass runs variant 0's
 * for variants 0 to 3 and the split kernels for theirs.  scf_autotune_field
 * computes the coefficients of the given particles, times each variant on
 * the forces at those particles (written to ax, ay, az, device, caller-owned;
 * synchronising the stream) and keeps the fastest for the plan; best_ms
 * (nullable) receives its time. */
int32_t scf_plan_num_field_variants(const scf_plan* plan);
int32_t scf_plan_field_variant(const scf_plan* plan);
scf_status scf_plan_set_field_variant(scf_plan* plan, int32_t variant);
scf_status scf_autotune_field(scf_plan* plan, int64_t n, const void* x, const void* y,
                              const void* z, const void* m, void* ax, void* ay, void* az, void* ws,
                              size_t ws_bytes, void* stream, double* best_ms);

/* Kernel timing (tracing): when enabled, every kernel the plan launches is
 * bracketed by HIP events on its stream; scf_profile_read synchronises on
 * those events and returns, per kernel kind, the launch count and the summed
 * event-to-event duration in milliseconds since the last read, then resets.
 * out must hold SCF_KERNEL_KINDS entries. */
#define SCF_KERNEL_KINDS 13
typedef struct {
  int32_t kind, count;
  double total_ms;
} scf_kernel_time;
scf_status scf_profile_enable(scf_plan* plan, int32_t enable);
scf_status scf_profile_read(scf_plan* plan, scf_kernel_time* out);
const char* scf_kernel_name(int32_t kind);

/* Issue-rate microbenchmark (measurement only; the ceilings the kernels'
 * roofline fractions are read against).  kind 0: single-precision FMA chains
 * (16 independent chains per lane), 1: the same with 32 chains, 2: 4x4x1
 * (16-block) FP32 MFMA chains, 3: 16x16x4 FP32 MFMA, 4: 32x32x2 FP32 MFMA,
 * 5: the work of kinds 0 and 2 (at the same iters) in every wave, as
 * independent chains (its time against the sum of theirs shows whether the
 * vector ALU and the matrix core overlap).  waves_per_simd (1..8) waves share each SIMD (blocks of four waves,
 * waves_per_simd blocks per compute unit); iters sets the length.  scratch is
 * a device buffer of at least 4 * waves_per_simd * (compute units) bytes that
 * the kernel may write.  Returns the achieved TFLOP/s and the kernel time of
 * the second of two launches on the null stream (blocks). */
scf_status scf_bench_ceiling(int32_t kind, int32_t waves_per_simd, int32_t iters, void* scratch,
                             double* tflops, double* ms);

const char* scf_status_string(scf_status status);
const char* scf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SCF_H */
