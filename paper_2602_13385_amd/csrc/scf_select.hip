// Selection and refresh kernels of the refresh cadence (Sec. 2.2): the bound
// test and squared-radius keys, an exact radix selection of the energy
// Lagrange radii, the selection weights with the bound mass, the compaction
// of the particles whose weight changed (intermediate refresh), and an FP64
// axpy on coefficient vectors.  All HBM-bound, one pass each.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "scf_internal.h"

namespace scf {
namespace {

template <typename R>
struct KeyOf;
template <>
struct KeyOf<float> {
  using K = uint32_t;
  static __device__ __forceinline__ K bits(float v) { return __float_as_uint(v); }
};
template <>
struct KeyOf<double> {
  using K = uint64_t;
  static __device__ __forceinline__ K bits(double v) { return (K)__double_as_longlong(v); }
};

// |v|^2/2 + psi < 0 marks a bound particle; its key is the bit pattern of
// |x|^2 = ((x x + y y) + z z) with every operation rounded (a non-negative
// float orders like its bits), unbound particles get the all-ones key.
template <typename R>
__global__ void __launch_bounds__(256) energy_keys_kernel(int64_t n, const R* __restrict__ x,
                                                          const R* __restrict__ y,
                                                          const R* __restrict__ z,
                                                          const R* __restrict__ vx,
                                                          const R* __restrict__ vy,
                                                          const R* __restrict__ vz,
                                                          const R* __restrict__ pot,
                                                          typename KeyOf<R>::K* __restrict__ keys,
                                                          uint8_t* __restrict__ bound) {
#pragma clang fp contract(off)
  using K = typename KeyOf<R>::K;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const R xi = x[i], yi = y[i], zi = z[i];
  const R ux = vx[i], uy = vy[i], uz = vz[i];
  const R e = R(0.5) * ((ux * ux + uy * uy) + uz * uz) + pot[i];
  const bool b = e < R(0);
  const R r2 = (xi * xi + yi * yi) + zi * zi;
  keys[i] = b ? KeyOf<R>::bits(r2) : ~K(0);
  if (bound) bound[i] = b ? 1 : 0;
}

// Histogram of one 8-bit digit (bits [shift, shift+8)) of the keys whose
// higher bits equal each target's prefix, for two targets at once.
template <typename K>
__global__ void __launch_bounds__(256) radix_hist_kernel(int64_t n, const K* __restrict__ keys,
                                                         SelectState* st, int shift, int first) {
  __shared__ uint32_t h[2][256];
  h[0][threadIdx.x] = 0;
  h[1][threadIdx.x] = 0;
  __syncthreads();
  const int hs = shift + 8;
  const K p0 = first ? K(0) : (K)st->prefix[0] >> hs;
  const K p1 = first ? K(0) : (K)st->prefix[1] >> hs;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const K k = keys[i];
    const unsigned d = (unsigned)(k >> shift) & 255u;
    const K hi = hs >= (int)(8 * sizeof(K)) ? K(0) : k >> hs;
    if (first || hi == p0) atomicAdd(&h[0][d], 1u);
    if (first || hi == p1) atomicAdd(&h[1][d], 1u);
  }
  __syncthreads();
  for (int t = 0; t < 2; ++t) {
    const uint32_t c = h[t][threadIdx.x];
    if (c) atomicAdd(&st->hist[t][threadIdx.x], c);
  }
}

__global__ void __launch_bounds__(256) select_clear_kernel(SelectState* st) {
  st->hist[0][threadIdx.x] = 0;
  st->hist[1][threadIdx.x] = 0;
  if (threadIdx.x < 2) {
    st->prefix[threadIdx.x] = 0;
    st->rank[threadIdx.x] = 0;
    st->k[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) {
    st->nb = 0;
    st->mbound = 0.0;
  }
}

// One block: picks each target's digit (the bucket that holds its remaining
// rank), extends the prefix and clears the histograms for the next digit.
// On the first digit it also derives the bound count (keys below all-ones)
// and the ranks k_t = ceil(frac_t N_b), clamped to [1, N_b].
__global__ void __launch_bounds__(256) radix_pick_kernel(SelectState* st, int shift, int first,
                                                         int64_t n, double frac0, double frac1) {
  __shared__ uint32_t cnt[256];
  __shared__ int64_t scan[256];
  const int tid = threadIdx.x;
  if (first) {
    if (tid == 0) {
      const int64_t nb = n - (int64_t)st->hist[0][255];
      st->nb = nb;
      const double fr[2] = {frac0, frac1};
      for (int t = 0; t < 2; ++t) {
        int64_t k = nb > 0 ? (int64_t)ceil(fr[t] * (double)nb) : 0;
        if (nb > 0) k = k < 1 ? 1 : (k > nb ? nb : k);
        st->k[t] = k;
        st->rank[t] = k > 0 ? k - 1 : 0;
        st->prefix[t] = 0;
      }
    }
    __syncthreads();
  }
  for (int t = 0; t < 2; ++t) {
    const uint32_t c = st->hist[t][tid];
    cnt[tid] = c;
    scan[tid] = c;
    __syncthreads();
    // inclusive prefix sum over the 256 bins (Hillis-Steele)
    for (int off = 1; off < 256; off <<= 1) {
      const int64_t v = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    const int64_t r = st->rank[t];
    const int64_t lo = scan[tid] - (int64_t)cnt[tid], hi = scan[tid];
    __syncthreads();
    if (st->nb > 0 && cnt[tid] > 0 && r >= lo && r < hi) {
      st->prefix[t] |= (uint64_t)tid << shift;
      st->rank[t] = r - lo;
    }
    __syncthreads();
    st->hist[t][tid] = 0;
    __syncthreads();
  }
}

// w = m on bound particles with key <= the selected key, else 0; per-block
// double sums of the bound mass (fixed order).
template <typename R>
__global__ void __launch_bounds__(256) select_weights_kernel(int64_t n,
                                                             const typename KeyOf<R>::K* __restrict__ keys,
                                                             const R* __restrict__ m,
                                                             const SelectState* st,
                                                             R* __restrict__ w,
                                                             double* __restrict__ mass_part) {
  using K = typename KeyOf<R>::K;
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double mb = 0.0;
  if (i < n) {
    const K k = keys[i];
    const K kx = (K)st->prefix[0];
    const R mi = m[i];
    const bool b = k != ~K(0);
    w[i] = (st->nb > 0 && b && k <= kx) ? mi : R(0);
    if (b) mb = (double)mi;
  }
  red[threadIdx.x] = mb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) mass_part[blockIdx.x] = red[0];
}

// bound mass: the block sums added in a fixed order
__global__ void __launch_bounds__(256) mass_sum_kernel(const double* __restrict__ part, int64_t nblk,
                                                       SelectState* st) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) st->mbound = red[0];
}

// ---- compaction of the particles whose weight changed ----------------------
template <typename R>
__global__ void __launch_bounds__(256) delta_count_kernel(int64_t n, const R* __restrict__ w0,
                                                          const R* __restrict__ w1,
                                                          int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool f = i < n && w0[i] != w1[i];
  const unsigned long long bal = __ballot(f);
  __shared__ int32_t wc[4];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// exclusive scan of the block counts (one block of 1024 threads, each over a
// contiguous chunk); total into *total
__global__ void __launch_bounds__(1024) delta_scan_kernel(const int32_t* __restrict__ cnt,
                                                          int64_t nblk, int64_t* __restrict__ off,
                                                          int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  const int64_t chunk = (nblk + 1023) / 1024;
  const int64_t b0 = threadIdx.x * chunk;
  const int64_t b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += cnt[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t c = 0;
    for (int t = 0; t < 1024; ++t) {
      const int64_t v = part[t];
      part[t] = c;
      c += v;
    }
    *total = c;
  }
  __syncthreads();
  int64_t c = part[threadIdx.x];
  for (int64_t b = b0; b < b1; ++b) {
    off[b] = c;
    c += cnt[b];
  }
}

// stable scatter of the changed particles: positions of every snapshot and
// the weight change dw = w1 - w0
template <typename R>
__global__ void __launch_bounds__(256) delta_scatter_kernel(int64_t n, const R* __restrict__ w0,
                                                            const R* __restrict__ w1,
                                                            const int64_t* __restrict__ off,
                                                            DeltaSnaps snaps, R* __restrict__ out,
                                                            int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool f = i < n && w0[i] != w1[i];
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ int32_t wc[4];
  if (lane == 0) wc[wv] = __popcll(bal);
  __syncthreads();
  if (!f) return;
  int32_t base = 0;
  for (int q = 0; q < wv; ++q) base += wc[q];
  const int32_t below = __popcll(bal & ((1ull << lane) - 1ull));
  const int64_t o = off[blockIdx.x] + base + below;
  // layout: [snapshot][x, y, z][cap], then dw[cap]
  for (int j = 0; j < snaps.ns; ++j) {
    R* dst = out + (int64_t)j * 3 * cap;
    dst[o] = ((const R*)snaps.x[j])[i];
    dst[cap + o] = ((const R*)snaps.y[j])[i];
    dst[2 * cap + o] = ((const R*)snaps.z[j])[i];
  }
  out[(int64_t)snaps.ns * 3 * cap + o] = w1[i] - w0[i];
}

__global__ void __launch_bounds__(256) axpy_kernel(int64_t n, double a, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// ---- density (Eq. total_dens) and the core of Sec. 2.1 ---------------------
// W rows of degree l scaled by kd[l][n] (the density constants times
// -1/(4 pi G b^2)); layout W[(l^2 + j) NW + n]
template <typename R>
__global__ void __launch_bounds__(256) scale_w_kernel(R* __restrict__ W, const double* __restrict__ kd,
                                                      int lmax, int nw) {
  const int L2 = (lmax + 1) * (lmax + 1);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= L2 * nw) return;
  const int n = i % nw, lj = i / nw;
  int l = 0;
  while ((l + 1) * (l + 1) <= lj) ++l;
  W[i] = R((double)W[i] * kd[l * nw + n]);
}

// rho = s^(1/alpha - 2) (1 + s^(1/alpha))^(-2) psi_K, s = r/b (in place)
template <typename R>
__global__ void __launch_bounds__(256) density_factor_kernel(int64_t n, const R* __restrict__ x,
                                                             const R* __restrict__ y,
                                                             const R* __restrict__ z, R binv,
                                                             R inv_alpha, int amode,
                                                             R* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const R s = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]) * binv;
  R f;
  if (amode == 0) {
    f = R(1) / (s * (R(1) + s) * (R(1) + s));
  } else if (amode == 1) {
    const R t = s * s;
    f = R(1) / ((R(1) + t) * (R(1) + t));
  } else {
    const R t = pow(s, inv_alpha);
    f = pow(s, inv_alpha - R(2)) / ((R(1) + t) * (R(1) + t));
  }
  rho[i] *= f;
}

// Block sums (fixed order) over the particles with w > 0 of
//   mode 0: rho^2 r^2, rho^2
//   mode 1 (r^2 <= r2max only): m vx, m vy, m vz, m
// with r^2 = (x x + y y) + z z in double precision; out[blk][4].
template <typename R>
__global__ void __launch_bounds__(256) core_moments_kernel(int64_t n, const R* __restrict__ x,
                                                           const R* __restrict__ y,
                                                           const R* __restrict__ z,
                                                           const R* __restrict__ vx,
                                                           const R* __restrict__ vy,
                                                           const R* __restrict__ vz,
                                                           const R* __restrict__ m,
                                                           const R* __restrict__ w,
                                                           const R* __restrict__ rho, int mode,
                                                           double r2max, double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double red[4][256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n && w[i] > R(0)) {
    const double xi = x[i], yi = y[i], zi = z[i];
    const double r2 = (xi * xi + yi * yi) + zi * zi;
    if (mode == 0) {
      const double d = rho[i];
      q[1] = d * d;
      q[0] = q[1] * r2;
    } else if (r2 <= r2max) {
      const double mi = m[i];
      q[0] = mi * (double)vx[i];
      q[1] = mi * (double)vy[i];
      q[2] = mi * (double)vz[i];
      q[3] = mi;
    }
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = q[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[(int64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// the block sums of core_moments_kernel added in a fixed order: res[4]
__global__ void __launch_bounds__(256) moments_sum_kernel(const double* __restrict__ part,
                                                          int64_t nblk, double* __restrict__ res) {
  __shared__ double red[4][256];
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblk; b += 256)
    for (int k = 0; k < 4; ++k) q[k] += part[b * 4 + k];
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = q[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) res[threadIdx.x] = red[threadIdx.x][0];
}

// ---- frame centre (Sec. 2.1) ------------------------------------------------
// Block sums (fixed order) of w omega, w omega x, w omega y, w omega z with
// omega = t (1 + t)^(-alpha-1) / r^2, t = (r/b)^(1/alpha), r = |x - c|, over
// the particles with w > 0 and r > rmin; all in double precision.
template <typename R>
__global__ void __launch_bounds__(256) recentre_sums_kernel(int64_t n, const R* __restrict__ x,
                                                            const R* __restrict__ y,
                                                            const R* __restrict__ z,
                                                            const R* __restrict__ w, double cx,
                                                            double cy, double cz, double binv,
                                                            double alpha, int amode, double rmin,
                                                            double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double red[4][256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n && w[i] > R(0)) {
    const double xi = x[i], yi = y[i], zi = z[i];
    const double dx = xi - cx, dy = yi - cy, dz = zi - cz;
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (r > rmin) {
      const double s = r * binv;
      double om;
      if (amode == 0) {
        om = s / ((1.0 + s) * (1.0 + s) * (r * r));
      } else if (amode == 1) {
        const double t = s * s;
        om = t / ((1.0 + t) * sqrt(1.0 + t) * (r * r));
      } else {
        const double t = pow(s, 1.0 / alpha);
        om = t * pow(1.0 + t, -alpha - 1.0) / (r * r);
      }
      om *= (double)w[i];
      q[0] = om;
      q[1] = om * xi;
      q[2] = om * yi;
      q[3] = om * zi;
    }
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = q[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[(int64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Block sums (fixed order) of w (1 + (r/b)^(1/alpha))^(-alpha), r = |x|, over
// the particles with w > 0, in double precision: the zeroth mode's projection
// for the basis (alpha, b) up to its norm (out[blk][4], slot 0).
template <typename R>
__global__ void __launch_bounds__(256) a000_sum_kernel(int64_t n, const R* __restrict__ x,
                                                       const R* __restrict__ y,
                                                       const R* __restrict__ z,
                                                       const R* __restrict__ w, double alpha,
                                                       double binv, double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q = 0.0;
  if (i < n && w[i] > R(0)) {
    const double xi = x[i], yi = y[i], zi = z[i];
    const double s = sqrt((xi * xi + yi * yi) + zi * zi) * binv;
    double f;
    if (alpha == 1.0)
      f = 1.0 / (1.0 + s);
    else if (alpha == 0.5)
      f = 1.0 / sqrt(1.0 + s * s);
    else
      f = pow(1.0 + pow(s, 1.0 / alpha), -alpha);
    q = (double)w[i] * f;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[(int64_t)blockIdx.x * 4 + threadIdx.x] = threadIdx.x == 0 ? red[0] : 0.0;
}

// a -= d for three arrays (a frame shift of positions or velocities)
template <typename R>
__global__ void __launch_bounds__(256) shift3_kernel(int64_t n, R* __restrict__ a0, R* __restrict__ a1,
                                                     R* __restrict__ a2, double d0, double d1,
                                                     double d2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  a0[i] = R((double)a0[i] - d0);
  a1[i] = R((double)a1[i] - d1);
  a2[i] = R((double)a2[i] - d2);
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_energy_keys(int dtype, int64_t n, const void* x, const void* y, const void* z,
                              const void* vx, const void* vy, const void* vz, const void* pot,
                              void* keys, uint8_t* bound, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dtype == 0)
    energy_keys_kernel<float><<<blocks_of(n), 256, 0, s>>>(
        n, (const float*)x, (const float*)y, (const float*)z, (const float*)vx, (const float*)vy,
        (const float*)vz, (const float*)pot, (uint32_t*)keys, bound);
  else
    energy_keys_kernel<double><<<blocks_of(n), 256, 0, s>>>(
        n, (const double*)x, (const double*)y, (const double*)z, (const double*)vx,
        (const double*)vy, (const double*)vz, (const double*)pot, (uint64_t*)keys, bound);
  return hipGetLastError();
}

hipError_t launch_radix_select(int dtype, int64_t n, const void* keys, SelectState* st,
                               double frac0, double frac1, int hist_blocks, hipStream_t s) {
  const int kbits = dtype == 0 ? 32 : 64;
  const unsigned g = (unsigned)(hist_blocks > 0 ? hist_blocks : 1);
  select_clear_kernel<<<1, 256, 0, s>>>(st);
  for (int shift = kbits - 8; shift >= 0; shift -= 8) {
    const int first = shift == kbits - 8;
    if (dtype == 0)
      radix_hist_kernel<uint32_t><<<g, 256, 0, s>>>(n, (const uint32_t*)keys, st, shift, first);
    else
      radix_hist_kernel<uint64_t><<<g, 256, 0, s>>>(n, (const uint64_t*)keys, st, shift, first);
    radix_pick_kernel<<<1, 256, 0, s>>>(st, shift, first, n, frac0, frac1);
  }
  return hipGetLastError();
}

hipError_t launch_select_weights(int dtype, int64_t n, const void* keys, const void* m,
                                 SelectState* st, void* w, double* mass_part, hipStream_t s) {
  const int64_t nblk = n > 0 ? (int64_t)blocks_of(n) : 0;
  if (n > 0) {
    if (dtype == 0)
      select_weights_kernel<float><<<blocks_of(n), 256, 0, s>>>(
          n, (const uint32_t*)keys, (const float*)m, st, (float*)w, mass_part);
    else
      select_weights_kernel<double><<<blocks_of(n), 256, 0, s>>>(
          n, (const uint64_t*)keys, (const double*)m, st, (double*)w, mass_part);
  }
  mass_sum_kernel<<<1, 256, 0, s>>>(mass_part, nblk, st);
  return hipGetLastError();
}

hipError_t launch_delta_compact(int dtype, int64_t n, const void* w0, const void* w1,
                                const DeltaSnaps& snaps, int32_t* cnt, int64_t* off,
                                int64_t* total, void* out, int64_t cap, hipStream_t s) {
  const int64_t nblk = n > 0 ? (int64_t)blocks_of(n) : 0;
  if (n > 0) {
    if (dtype == 0)
      delta_count_kernel<float><<<blocks_of(n), 256, 0, s>>>(n, (const float*)w0,
                                                              (const float*)w1, cnt);
    else
      delta_count_kernel<double><<<blocks_of(n), 256, 0, s>>>(n, (const double*)w0,
                                                               (const double*)w1, cnt);
  }
  delta_scan_kernel<<<1, 1024, 0, s>>>(cnt, nblk, off, total);
  if (n > 0 && out) {
    if (dtype == 0)
      delta_scatter_kernel<float><<<blocks_of(n), 256, 0, s>>>(
          n, (const float*)w0, (const float*)w1, off, snaps, (float*)out, cap);
    else
      delta_scatter_kernel<double><<<blocks_of(n), 256, 0, s>>>(
          n, (const double*)w0, (const double*)w1, off, snaps, (double*)out, cap);
  }
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  axpy_kernel<<<blocks_of(n), 256, 0, s>>>(n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_scale_w(int dtype, void* W, const double* kd, int lmax, int nmaxc,
                          hipStream_t s) {
  const int nw = nmaxc + 1, cnt = (lmax + 1) * (lmax + 1) * nw;
  if (dtype == 0)
    scale_w_kernel<float><<<blocks_of(cnt), 256, 0, s>>>((float*)W, kd, lmax, nw);
  else
    scale_w_kernel<double><<<blocks_of(cnt), 256, 0, s>>>((double*)W, kd, lmax, nw);
  return hipGetLastError();
}

hipError_t launch_density_factor(int dtype, int64_t n, const void* x, const void* y, const void* z,
                                 double binv, double inv_alpha, int amode, void* rho,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dtype == 0)
    density_factor_kernel<float><<<blocks_of(n), 256, 0, s>>>(
        n, (const float*)x, (const float*)y, (const float*)z, (float)binv, (float)inv_alpha, amode,
        (float*)rho);
  else
    density_factor_kernel<double><<<blocks_of(n), 256, 0, s>>>(
        n, (const double*)x, (const double*)y, (const double*)z, binv, inv_alpha, amode,
        (double*)rho);
  return hipGetLastError();
}

hipError_t launch_core_moments(int dtype, int64_t n, const void* x, const void* y, const void* z,
                               const void* vx, const void* vy, const void* vz, const void* m,
                               const void* w, const void* rho, int mode, double r2max,
                               double* part, double* res, hipStream_t s) {
  const int64_t nblk = n > 0 ? (int64_t)blocks_of(n) : 0;
  if (n > 0) {
    if (dtype == 0)
      core_moments_kernel<float><<<blocks_of(n), 256, 0, s>>>(
          n, (const float*)x, (const float*)y, (const float*)z, (const float*)vx,
          (const float*)vy, (const float*)vz, (const float*)m, (const float*)w,
          (const float*)rho, mode, r2max, part);
    else
      core_moments_kernel<double><<<blocks_of(n), 256, 0, s>>>(
          n, (const double*)x, (const double*)y, (const double*)z, (const double*)vx,
          (const double*)vy, (const double*)vz, (const double*)m, (const double*)w,
          (const double*)rho, mode, r2max, part);
  }
  moments_sum_kernel<<<1, 256, 0, s>>>(part, nblk, res);
  return hipGetLastError();
}

hipError_t launch_recentre_sums(int dtype, int64_t n, const void* x, const void* y, const void* z,
                                const void* w, const double* c, double binv, double alpha,
                                int amode, double rmin, double* part, double* res, hipStream_t s) {
  const int64_t nblk = n > 0 ? (int64_t)blocks_of(n) : 0;
  if (n > 0) {
    if (dtype == 0)
      recentre_sums_kernel<float><<<blocks_of(n), 256, 0, s>>>(
          n, (const float*)x, (const float*)y, (const float*)z, (const float*)w, c[0], c[1], c[2],
          binv, alpha, amode, rmin, part);
    else
      recentre_sums_kernel<double><<<blocks_of(n), 256, 0, s>>>(
          n, (const double*)x, (const double*)y, (const double*)z, (const double*)w, c[0], c[1],
          c[2], binv, alpha, amode, rmin, part);
  }
  moments_sum_kernel<<<1, 256, 0, s>>>(part, nblk, res);
  return hipGetLastError();
}

hipError_t launch_shift3(int dtype, int64_t n, void* a0, void* a1, void* a2, const double* d,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dtype == 0)
    shift3_kernel<float><<<blocks_of(n), 256, 0, s>>>(n, (float*)a0, (float*)a1, (float*)a2, d[0],
                                                      d[1], d[2]);
  else
    shift3_kernel<double><<<blocks_of(n), 256, 0, s>>>(n, (double*)a0, (double*)a1, (double*)a2,
                                                       d[0], d[1], d[2]);
  return hipGetLastError();
}

hipError_t launch_a000_sum(int dtype, int64_t n, const void* x, const void* y, const void* z,
                           const void* w, double alpha, double binv, double* part, double* res,
                           hipStream_t s) {
  const int64_t nblk = n > 0 ? (int64_t)blocks_of(n) : 0;
  if (n > 0) {
    if (dtype == 0)
      a000_sum_kernel<float><<<blocks_of(n), 256, 0, s>>>(n, (const float*)x, (const float*)y,
                                                          (const float*)z, (const float*)w, alpha,
                                                          binv, part);
    else
      a000_sum_kernel<double><<<blocks_of(n), 256, 0, s>>>(n, (const double*)x, (const double*)y,
                                                           (const double*)z, (const double*)w,
                                                           alpha, binv, part);
  }
  moments_sum_kernel<<<1, 256, 0, s>>>(part, nblk, res);
  return hipGetLastError();
}

}  // namespace scf
