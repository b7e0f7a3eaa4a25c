// Internal interfaces of libscf: the per-(dtype, nmax, lmax) kernel engines
// and the argument blocks their launchers take.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "host_field.h"
#include "scf_dual.h"

namespace scf {

// Kernel arguments of the coefficient (particle-sum) kernel.  R is the
// arithmetic type (float, double, or Dual<T> for the adjoint's gamma pass,
// whose positions are x + eps escale (ex, ey, ez) with unit weights and whose
// sums keep only the eps part).
template <typename R>
struct CoefArgs {
  using S = scalar_t<R>;
  const S* x;
  const S* y;
  const S* z;
  const S* m;
  const S* ex;  // dual mode: direction of the eps parts
  const S* ey;
  const S* ez;
  S escale;
  const int64_t* seg_begin;  // per-block particle range [seg_begin[b], seg_end[b])
  const int64_t* seg_end;
  const int32_t* seg_slot;   // per-block output slot (partials row)
  int64_t begin, n;          // used when seg_begin == nullptr: the particles
  int64_t stages;            // [begin, n) form `stages` stages, split evenly: unit u
                             // takes stages [u*stages/nunits, (u+1)*stages/nunits)
  int nunits;                // number of wave-units (particle ranges)
  const S* beta_rad;         // [(lmax+1)][(NMAXC+1)]  monic Gegenbauer recurrence
  const S* beta_ang;         // [(lmax+1)][(lmax+1)] monic Legendre recurrence [m][l], then 0..lmax
  acc_t<R>* partials;        // [nblocks][T]
  int one_row;               // single-precision block kernel: every unit folds its
                             // sums once, so it writes its hi row only (no lo row)
  int T, nmax;
  S binv, alpha, inv_alpha;
  int amode;
};

// Kernel arguments of the field (force / kick-drift) kernel.
template <typename R>
struct ForceArgs {
  R* x;
  R* y;
  R* z;
  R* xo;  // step mode: drifted positions are written here (may equal x, y, z)
  R* yo;
  R* zo;
  R* vx;  // adjoint mode: lambda_v
  R* vy;
  R* vz;
  R* ax;  // adjoint mode: lambda_x
  R* ay;
  R* az;
  R* pot;
  const R* mass;  // adjoint mode
  const R* W;         // [(lmax+1)^2][(NMAXC+1)] force weights, n fastest
  const R* beta_rad;  // as in CoefArgs
  const R* beta_ang;
  int64_t n;
  R binv, alpha, inv_alpha;
  int amode;
  R kick, drift;      // step mode: v += kick * a; x += drift * v
  HostParams<R> host;
  R cx, cy, cz;       // frame centre R
  R gcx, gcy, gcz;    // grad psi_host(R) (host, double precision, rounded)
  // batched mode: per-block cluster id table and per-cluster tables
  const int32_t* blk_cluster;  // nullable
  const int64_t* blk_begin;    // particle range of each block (batched mode)
  const int64_t* blk_end;
  const double* centre_tab;    // [nclusters][9]: R, grad psi_host(R), unused
  int64_t W_stride;            // elements between clusters' W tables
  // matrix-core field pass: per degree, 1 / kappa_n and 2 (n + lam) kappa_n
  // (kappa_n the leading coefficient of C_n^lam), [l][2][NMAXC + 1]
  const double* dtab;
};

// Kernel arguments of the adjoint's Hessian-vector kernel (T = float or double).
template <typename T>
struct HvpArgs {
  const T* x;
  const T* y;
  const T* z;
  const T* lvx;  // lambda_v: the cotangent direction is mu = c lambda_v
  const T* lvy;
  const T* lvz;
  T c;
  T* lx;  // lambda_x (accumulated)
  T* ly;
  T* lz;
  const T* W;  // force weights of the coefficients at x
  const T* beta_rad;
  const T* beta_ang;
  int64_t n;
  T binv, alpha, inv_alpha;
  int amode;
  HostParams<T> host;
  T cx, cy, cz;  // frame centre R
  T* partials;   // [nblocks][32] block sums of the host terms (host present)
};

// Job descriptions handed to an engine.
struct Engine {
  virtual ~Engine() {}
  virtual int nmaxc() const = 0;
  virtual int lmax() const = 0;
  virtual int dtype() const = 0;
  virtual size_t real_size() const = 0;
  // coefficient-kernel variants (basis-phase lanes per particle, waves per block)
  virtual int coef_variants() const = 0;
  // particles per wave-stage of variant v
  virtual int stage_particles(int v) const = 0;
  // partial-sum rows written per wave-unit (at most), and resident wave-units per CU
  virtual int rows_per_unit(int v) const = 0;
  // stages a unit of variant v sums before it folds them into its rows; a
  // unit of at most that many stages writes one row (0: rows_per_unit always)
  virtual int fold_stages(int v) const = 0;
  virtual int max_resident_units(int v) const = 0;
  // launches variant v of the coefficient kernel over nunits wave-units
  virtual hipError_t launch_coef(const void* args, int nunits, int v, hipStream_t s) const = 0;
  // launches the field kernel; mode 0 = forces, 1 = kick/drift step,
  // 2 = adjoint accumulation (lambda_x += m a, lambda_v += drift lambda_x)
  // field-kernel launch variants (register budget); fv < field_variants()
  virtual int field_variants() const = 0;
  virtual hipError_t launch_force(const void* args, int64_t nblocks, int mode, int fv,
                                  hipStream_t s) const = 0;
  // adjoint: the gamma pass (coefficient kernel on dual positions, one
  // variant) and the Hessian-vector kernel
  virtual int gamma_stage_particles() const = 0;
  virtual int gamma_rows_per_unit() const = 0;
  virtual int gamma_resident_units() const = 0;
  virtual hipError_t launch_gamma(const void* args, int nunits, hipStream_t s) const = 0;
  virtual hipError_t launch_hvp(const void* args, int64_t nblocks, hipStream_t s) const = 0;
  virtual const char* describe() const = 0;
};

Engine* find_engine(int dtype, int nmax, int lmax);
Engine* find_engine_f32_exact(int nmax, int lmax);
Engine* find_engine_f32_generic(int nmax, int lmax);
Engine* find_engine_f64_exact(int nmax, int lmax);
Engine* find_engine_f64_generic(int nmax, int lmax);

// Small kernels independent of (nmax, lmax).
hipError_t launch_reduce(int dtype, const void* partials, int nblocks, int T, int nchunks,
                         double* red1, hipStream_t s);
hipError_t launch_finalize(int dtype, const double* red1, int nchunks, int T, int nmax, int lmax,
                           int nmaxc, const double* cs, const double* fw, double* coef, void* W,
                           hipStream_t s);
// launch_reduce + launch_finalize in one pass, for few partial rows
hipError_t launch_reduce_final_small(int dtype, const void* partials, int nblocks, int T, int nmax,
                                    int lmax, int nmaxc, const double* cs, const double* fw,
                                    double* coef, void* W, hipStream_t s);
hipError_t launch_make_w(int dtype, const double* coef, int T, int nmax, int lmax, int nmaxc,
                         const double* fw, void* W, hipStream_t s);
hipError_t launch_kick_drift(int dtype, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                             void* vz, const void* ax, const void* ay, const void* az, double kick,
                             double drift, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// batched mode (cluster-segmented) reduction and finalisation
hipError_t launch_reduce_batched(int dtype, const void* partials, const int32_t* rows, int ncl,
                                 int T, int nchunks, double* red1, hipStream_t s);
hipError_t launch_finalize_batched(int dtype, const double* red1, int nchunks, int T, int nmax,
                                   int lmax, int nmaxc, const double* cs, const double* fw,
                                   double* coef, void* W, int64_t W_stride,
                                   const double* centre_tab, int ncl, double* cur, int* step,
                                   hipStream_t s);
// launch_reduce_batched + launch_finalize_batched in one pass, for few rows per cluster
hipError_t launch_reduce_final_batched(int dtype, const void* partials, const int32_t* rows, int ncl,
                                      int T, int nmax, int lmax, int nmaxc, const double* cs,
                                      const double* fw, double* coef, void* W, int64_t W_stride,
                                      const double* centre_tab, double* cur, int* step,
                                      hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
// power per degree of ncl coefficient vectors (ncl x T in, ncl x (lmax+1) out)
hipError_t launch_power(const double* coef, int nmax, int lmax, int ncl, double* El,
                        hipStream_t s);
// adjoint: the double-precision sums of the Hessian-vector kernel's 32 block
// sums, for nkicks kicks ([nkicks][nblocks][32] -> [nkicks][32])
hipError_t launch_adj_reduce(int dtype, const void* partials, int64_t nblocks, int nkicks,
                             double* out, hipStream_t s);

// ---- refresh cadence (selection and intermediate refresh) -----------------
// State of the two-target radix selection (device): the selected key bits and
// remaining ranks per target, the bound count, the ranks k_t and bound mass.
struct SelectState {
  uint64_t prefix[2];
  int64_t rank[2];
  int64_t k[2];
  int64_t nb;
  double mbound;
  uint32_t hist[2][256];
};
constexpr int kMaxSamples = 16;  // orbit samples per interval (positions kept)
struct DeltaSnaps {
  int ns;
  const void* x[kMaxSamples];
  const void* y[kMaxSamples];
  const void* z[kMaxSamples];
};
// bound flags (nullable) and squared-radius keys (u32 for FP32, u64 for FP64)
hipError_t launch_energy_keys(int dtype, int64_t n, const void* x, const void* y, const void* z,
                              const void* vx, const void* vy, const void* vz, const void* pot,
                              void* keys, uint8_t* bound, hipStream_t s);
// the keys of ranks ceil(frac_t N_b), t = 0, 1, among the bound keys
hipError_t launch_radix_select(int dtype, int64_t n, const void* keys, SelectState* st,
                               double frac0, double frac1, int hist_blocks, hipStream_t s);
// weights m [key <= selected key of target 0] and the bound mass
hipError_t launch_select_weights(int dtype, int64_t n, const void* keys, const void* m,
                                 SelectState* st, void* w, double* mass_part, hipStream_t s);
// stable compaction of the particles with w0 != w1: positions of every
// snapshot ([snapshot][x, y, z][cap]) and w1 - w0 ([cap]) into out (nullable:
// count only); the count into *total
hipError_t launch_delta_compact(int dtype, int64_t n, const void* w0, const void* w1,
                                const DeltaSnaps& snaps, int32_t* cnt, int64_t* off,
                                int64_t* total, void* out, int64_t cap, hipStream_t s);
// y += a x on n doubles
hipError_t launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s);
// density (Eq. total_dens): force weights scaled by kd[l][n], then the radial
// factor s^(1/alpha-2) (1 + s^(1/alpha))^-2 applied to the field pass's psi
hipError_t launch_scale_w(int dtype, void* W, const double* kd, int lmax, int nmaxc,
                          hipStream_t s);
hipError_t launch_density_factor(int dtype, int64_t n, const void* x, const void* y, const void* z,
                                 double binv, double inv_alpha, int amode, void* rho,
                                 hipStream_t s);
// core moments over w > 0 (mode 0: rho^2 r^2, rho^2; mode 1, r^2 <= r2max:
// m v, m): block sums into part[nblk][4], their fixed-order sum into res[4]
hipError_t launch_core_moments(int dtype, int64_t n, const void* x, const void* y, const void* z,
                               const void* vx, const void* vy, const void* vz, const void* m,
                               const void* w, const void* rho, int mode, double r2max,
                               double* part, double* res, hipStream_t s);
// frame centre: fixed-order double sums of (w omega, w omega x, y, z) about c
// into part[nblk][4] and res[4]
hipError_t launch_recentre_sums(int dtype, int64_t n, const void* x, const void* y, const void* z,
                                const void* w, const double* c, double binv, double alpha,
                                int amode, double rmin, double* part, double* res, hipStream_t s);
// sum over w > 0 of w (1 + (|x|/b)^(1/alpha))^(-alpha) into res[0] (double)
hipError_t launch_a000_sum(int dtype, int64_t n, const void* x, const void* y, const void* z,
                           const void* w, double alpha, double binv, double* part, double* res,
                           hipStream_t s);
// a_k -= d[k] on three arrays of n
hipError_t launch_shift3(int dtype, int64_t n, void* a0, void* a1, void* a2, const double* d,
                         hipStream_t s);

}  // namespace scf
