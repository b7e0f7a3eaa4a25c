// Small kernels of the SCF hot path that do not depend on (nmax, lmax): the
// double-precision cross-block reductions of the coefficient sums, the force
// weights, the standalone kick-drift, fills, the batched-mode reductions and
// the adjoint's reduction of its host sums; and the engine lookup.
#include <hip/hip_runtime.h>

#include "scf_internal.h"

namespace scf {

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// partial sums over blocks: red1[chunk][t] = sum_{b in chunk} partials[b][t] (double)
template <typename R>
__global__ void __launch_bounds__(256) reduce_kernel(const R* __restrict__ partials, int nblocks,
                                                     int T, int per_chunk, double* red1) {
  __shared__ double sh[4][64];
  const int ti = threadIdx.x & 63, kc = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + ti;
  const int b0 = blockIdx.y * per_chunk;
  int b1 = b0 + per_chunk;
  if (b1 > nblocks) b1 = nblocks;
  double s = 0.0;
  if (t < T) {
#pragma unroll 8
    for (int b = b0 + kc; b < b1; b += 4) s += double(partials[(int64_t)b * T + t]);
  }
  sh[kc][ti] = s;
  __syncthreads();
  if (kc == 0 && t < T)
    red1[(int64_t)blockIdx.y * T + t] = ((sh[0][ti] + sh[1][ti]) + sh[2][ti]) + sh[3][ti];
}

// a_t = cs_t * (sum of the chunk sums of t), in a fixed order (4 strided
// chunk subsets, then their sum), and the force weights W[(l,j)][n] =
// fw_t a_t; rows n in (nmax, nmaxc] of W are zero.
template <typename R>
__device__ __forceinline__ void finalize_block(const double* __restrict__ red1, int nchunks, int T,
                                               int nmax, int lmax, int nmaxc,
                                               const double* __restrict__ cs,
                                               const double* __restrict__ fw, double* coef, R* W,
                                               int cb, int ncb) {
  __shared__ double sh[4][64];
  const int L2 = (lmax + 1) * (lmax + 1);
  const int ti = threadIdx.x & 63, kc = threadIdx.x >> 6;
  const int t = cb * 64 + ti;
  double s = 0.0;
  if (t < T) {
#pragma unroll 8
    for (int c = kc; c < nchunks; c += 4) s += red1[(int64_t)c * T + t];
  }
  sh[kc][ti] = s;
  __syncthreads();
  if (kc == 0 && t < T) {
    const double tot = ((sh[0][ti] + sh[1][ti]) + sh[2][ti]) + sh[3][ti];
    const int n = t / L2, lj = t % L2;
    const double cv = cs[t] * tot;
    if (coef) coef[t] = cv;
    W[lj * (nmaxc + 1) + n] = R(fw[t] * cv);
  }
  const int npad = (nmaxc - nmax) * L2;
  for (int q = cb * blockDim.x + threadIdx.x; q < npad; q += ncb * blockDim.x) {
    const int n = nmax + 1 + q / L2, lj = q % L2;
    W[lj * (nmaxc + 1) + n] = R(0);
  }
}

// Single-pass reduction and finalisation of up to a few thousand partial
// rows [r0, r1), for a block of 1024 threads and the 16 coefficients
// t = 16 cb .. 16 cb + 15: thread (g, c) sums rows r0 + g, r0 + g + 64, ..
// of coefficient 16 cb + c in double precision (each wave reads four 64-byte
// row pieces per load), the 64 row-group sums of a coefficient are then added
// pairwise in a fixed order, and a_t = cs_t * sum and W[(l,j)][n] = fw_t a_t
// are written; rows n in (nmax, nmaxc] of W are zero.
template <typename R>
__device__ __forceinline__ void reduce_final_cols(const R* __restrict__ partials, int r0, int r1,
                                                  int T, int nmax, int lmax, int nmaxc,
                                                  const double* __restrict__ cs,
                                                  const double* __restrict__ fw, double* coef,
                                                  R* W, int cb, int ncb) {
  __shared__ double sh[64][16];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int t = cb * 16 + c;
  double s = 0.0;
  if (t < T) {
#pragma unroll 8
    for (int b = r0 + g; b < r1; b += 64) s += double(partials[(int64_t)b * T + t]);
  }
  sh[g][c] = s;
  __syncthreads();
  for (int h = 32; h >= 1; h >>= 1) {
    if (g < h) sh[g][c] += sh[g + h][c];
    __syncthreads();
  }
  const int L2 = (lmax + 1) * (lmax + 1);
  if (g == 0 && t < T) {
    const int n = t / L2, lj = t % L2;
    const double cv = cs[t] * sh[0][c];
    if (coef) coef[t] = cv;
    W[lj * (nmaxc + 1) + n] = R(fw[t] * cv);
  }
  const int npad = (nmaxc - nmax) * L2;
  for (int q = cb * blockDim.x + threadIdx.x; q < npad; q += ncb * blockDim.x) {
    const int n = nmax + 1 + q / L2, lj = q % L2;
    W[lj * (nmaxc + 1) + n] = R(0);
  }
}

// Coefficient chunk of a block: blocks are dealt to the 8 XCDs in turn
// (block b runs on XCD b mod 8), so chunk (b mod 8) per + b / 8 gives each
// XCD a contiguous range of chunks, and the two 64-byte halves of a row's
// 128-byte line are read through one L2 (the grid is a multiple of 8 blocks).
__device__ __forceinline__ int xcd_chunk() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}
constexpr int grid_chunks(int T) { return ((T + 15) / 16 + 7) / 8 * 8; }

template <typename R>
__global__ void __launch_bounds__(1024) reduce_final_small_kernel(
    const R* __restrict__ partials, int nblocks, int T, int nmax, int lmax, int nmaxc,
    const double* __restrict__ cs, const double* __restrict__ fw, double* coef, R* W) {
  reduce_final_cols<R>(partials, 0, nblocks, T, nmax, lmax, nmaxc, cs, fw, coef, W, xcd_chunk(),
                       gridDim.x);
}

template <typename R>
__global__ void __launch_bounds__(256) finalize_kernel(const double* __restrict__ red1, int nchunks,
                                                       int T, int nmax, int lmax, int nmaxc,
                                                       const double* __restrict__ cs,
                                                       const double* __restrict__ fw, double* coef,
                                                       R* W) {
  finalize_block<R>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw, coef, W, blockIdx.x, gridDim.x);
}

template <typename R>
__global__ void __launch_bounds__(256) make_w_kernel(const double* __restrict__ coef, int T, int nmax,
                                                     int lmax, int nmaxc,
                                                     const double* __restrict__ fw, R* W) {
  const int L2 = (lmax + 1) * (lmax + 1);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (nmaxc + 1) * L2) return;
  const int lj = e / (nmaxc + 1), n = e % (nmaxc + 1);
  if (n > nmax) {
    W[e] = R(0);
    return;
  }
  const int t = n * L2 + lj;
  W[e] = R(fw[t] * coef[t]);
}

template <typename R>
__global__ void __launch_bounds__(256) kick_drift_kernel(int64_t n, R* x, R* y, R* z, R* vx, R* vy,
                                                         R* vz, const R* ax, const R* ay,
                                                         const R* az, R kick, R drift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  R u = fma(kick, ax[i], vx[i]), v = fma(kick, ay[i], vy[i]), w = fma(kick, az[i], vz[i]);
  vx[i] = u;
  vy[i] = v;
  vz[i] = w;
  x[i] = fma(drift, u, x[i]);
  y[i] = fma(drift, v, y[i]);
  z[i] = fma(drift, w, z[i]);
}

// Batched reduction: cluster c owns partial rows [rows[c], rows[c+1]);
// red1[c][chunk][t] sums its rows of one chunk (double).
template <typename R>
__global__ void __launch_bounds__(256) reduce_batched_kernel(const R* __restrict__ partials,
                                                             const int32_t* __restrict__ rows,
                                                             int T, int nchunks, double* red1) {
  __shared__ double sh[4][64];
  const int ti = threadIdx.x & 63, kc = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + ti;
  const int c = blockIdx.z;
  const int r0 = rows[c], r1 = rows[c + 1];
  const int per_chunk = (r1 - r0 + nchunks - 1) / nchunks;
  const int b0 = r0 + blockIdx.y * per_chunk;
  int b1 = b0 + per_chunk;
  if (b1 > r1) b1 = r1;
  double s = 0.0;
  if (t < T)
    for (int b = b0 + kc; b < b1; b += 4) s += double(partials[(int64_t)b * T + t]);
  sh[kc][ti] = s;
  __syncthreads();
  if (kc == 0 && t < T)
    red1[((int64_t)c * nchunks + blockIdx.y) * T + t] =
        ((sh[0][ti] + sh[1][ti]) + sh[2][ti]) + sh[3][ti];
}

// Batched finalisation: coef[c][t] and W[c][.] of every cluster.  Block
// (0, 0) also copies row *step of the centre table into cur (the rows the
// field pass of this step reads) and then advances *step.
template <typename R>
__global__ void __launch_bounds__(256) finalize_batched_kernel(
    const double* __restrict__ red1, int nchunks, int T, int nmax, int lmax, int nmaxc,
    const double* __restrict__ cs, const double* __restrict__ fw, double* coef, R* W,
    int64_t W_stride, const double* __restrict__ centre_tab, int ncl, double* cur, int* step) {
  const int c = blockIdx.y;
  if (blockIdx.x == 0 && c == 0 && step) {
    const int k = *step;
    for (int i = threadIdx.x; i < ncl * 9; i += blockDim.x)
      cur[i] = centre_tab[(int64_t)k * ncl * 9 + i];
    __syncthreads();
    if (threadIdx.x == 0) *step = k + 1;
  }
  finalize_block<R>(red1 + (int64_t)c * nchunks * T, nchunks, T, nmax, lmax, nmaxc, cs, fw,
                    coef ? coef + (int64_t)c * T : nullptr, W + (int64_t)c * W_stride, blockIdx.x,
                    gridDim.x);
}

// Batched single-pass reduction and finalisation: block (cb, c) reduces
// cluster c's rows [rows[c], rows[c+1]) for coefficients 16 cb .. 16 cb + 15
// (as reduce_final_cols); block (0, 0) also copies row *step of the centre
// table into cur and then advances *step (as finalize_batched_kernel).
template <typename R>
__global__ void __launch_bounds__(1024) reduce_final_batched_kernel(
    const R* __restrict__ partials, const int32_t* __restrict__ rows, int T, int nmax, int lmax,
    int nmaxc, const double* __restrict__ cs, const double* __restrict__ fw, double* coef, R* W,
    int64_t W_stride, const double* __restrict__ centre_tab, int ncl, double* cur, int* step) {
  const int c = blockIdx.y;
  if (blockIdx.x == 0 && c == 0 && step) {
    const int k = *step;
    for (int i = threadIdx.x; i < ncl * 9; i += blockDim.x)
      cur[i] = centre_tab[(int64_t)k * ncl * 9 + i];
    __syncthreads();
    if (threadIdx.x == 0) *step = k + 1;
  }
  reduce_final_cols<R>(partials, rows[c], rows[c + 1], T, nmax, lmax, nmaxc, cs, fw,
                       coef ? coef + (int64_t)c * T : nullptr, W + (int64_t)c * W_stride,
                       xcd_chunk(), gridDim.x);
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_reduce(int dtype, const void* partials, int nblocks, int T, int nchunks,
                         double* red1, hipStream_t s) {
  if (nblocks <= 0 || T <= 0) return hipSuccess;
  const int per_chunk = (nblocks + nchunks - 1) / nchunks;
  dim3 grid((T + 63) / 64, nchunks);
  if (dtype == 0)
    reduce_kernel<float><<<grid, 256, 0, s>>>((const float*)partials, nblocks, T, per_chunk, red1);
  else
    reduce_kernel<double><<<grid, 256, 0, s>>>((const double*)partials, nblocks, T, per_chunk, red1);
  return hipGetLastError();
}

hipError_t launch_reduce_final_small(int dtype, const void* partials, int nblocks, int T, int nmax,
                                    int lmax, int nmaxc, const double* cs, const double* fw,
                                    double* coef, void* W, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  const int grid = grid_chunks(T);
  if (dtype == 0)
    reduce_final_small_kernel<float><<<grid, 1024, 0, s>>>((const float*)partials, nblocks, T, nmax,
                                                           lmax, nmaxc, cs, fw, coef, (float*)W);
  else
    reduce_final_small_kernel<double><<<grid, 1024, 0, s>>>((const double*)partials, nblocks, T,
                                                            nmax, lmax, nmaxc, cs, fw, coef,
                                                            (double*)W);
  return hipGetLastError();
}

hipError_t launch_finalize(int dtype, const double* red1, int nchunks, int T, int nmax, int lmax,
                           int nmaxc, const double* cs, const double* fw, double* coef, void* W,
                           hipStream_t s) {
  const int grid = (T + 63) / 64;
  if (dtype == 0)
    finalize_kernel<float><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw, coef,
                                                (float*)W);
  else
    finalize_kernel<double><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw, coef,
                                                 (double*)W);
  return hipGetLastError();
}

hipError_t launch_make_w(int dtype, const double* coef, int T, int nmax, int lmax, int nmaxc,
                         const double* fw, void* W, hipStream_t s) {
  const int ne = (nmaxc + 1) * (lmax + 1) * (lmax + 1);
  const int grid = (ne + 255) / 256;
  if (dtype == 0)
    make_w_kernel<float><<<grid, 256, 0, s>>>(coef, T, nmax, lmax, nmaxc, fw, (float*)W);
  else
    make_w_kernel<double><<<grid, 256, 0, s>>>(coef, T, nmax, lmax, nmaxc, fw, (double*)W);
  return hipGetLastError();
}

hipError_t launch_kick_drift(int dtype, int64_t n, void* x, void* y, void* z, void* vx, void* vy,
                             void* vz, const void* ax, const void* ay, const void* az, double kick,
                             double drift, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = (n + 255) / 256;
  if (dtype == 0)
    kick_drift_kernel<float><<<dim3((unsigned)grid), 256, 0, s>>>(
        n, (float*)x, (float*)y, (float*)z, (float*)vx, (float*)vy, (float*)vz, (const float*)ax,
        (const float*)ay, (const float*)az, (float)kick, (float)drift);
  else
    kick_drift_kernel<double><<<dim3((unsigned)grid), 256, 0, s>>>(
        n, (double*)x, (double*)y, (double*)z, (double*)vx, (double*)vy, (double*)vz,
        (const double*)ax, (const double*)ay, (const double*)az, kick, drift);
  return hipGetLastError();
}

hipError_t launch_reduce_batched(int dtype, const void* partials, const int32_t* rows, int ncl,
                                 int T, int nchunks, double* red1, hipStream_t s) {
  if (ncl <= 0 || T <= 0) return hipSuccess;
  dim3 grid((T + 63) / 64, nchunks, ncl);
  if (dtype == 0)
    reduce_batched_kernel<float><<<grid, 256, 0, s>>>((const float*)partials, rows, T, nchunks, red1);
  else
    reduce_batched_kernel<double><<<grid, 256, 0, s>>>((const double*)partials, rows, T, nchunks,
                                                       red1);
  return hipGetLastError();
}

hipError_t launch_finalize_batched(int dtype, const double* red1, int nchunks, int T, int nmax,
                                   int lmax, int nmaxc, const double* cs, const double* fw,
                                   double* coef, void* W, int64_t W_stride,
                                   const double* centre_tab, int ncl, double* cur, int* step,
                                   hipStream_t s) {
  if (ncl <= 0) return hipSuccess;
  dim3 grid((T + 63) / 64, ncl);
  if (dtype == 0)
    finalize_batched_kernel<float><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs, fw,
                                                        coef, (float*)W, W_stride, centre_tab, ncl,
                                                        cur, step);
  else
    finalize_batched_kernel<double><<<grid, 256, 0, s>>>(red1, nchunks, T, nmax, lmax, nmaxc, cs,
                                                         fw, coef, (double*)W, W_stride,
                                                         centre_tab, ncl, cur, step);
  return hipGetLastError();
}

hipError_t launch_reduce_final_batched(int dtype, const void* partials, const int32_t* rows, int ncl,
                                      int T, int nmax, int lmax, int nmaxc, const double* cs,
                                      const double* fw, double* coef, void* W, int64_t W_stride,
                                      const double* centre_tab, double* cur, int* step,
                                      hipStream_t s) {
  if (ncl <= 0 || T <= 0) return hipSuccess;
  dim3 grid(grid_chunks(T), ncl);
  if (dtype == 0)
    reduce_final_batched_kernel<float><<<grid, 1024, 0, s>>>(
        (const float*)partials, rows, T, nmax, lmax, nmaxc, cs, fw, coef, (float*)W, W_stride,
        centre_tab, ncl, cur, step);
  else
    reduce_final_batched_kernel<double><<<grid, 1024, 0, s>>>(
        (const double*)partials, rows, T, nmax, lmax, nmaxc, cs, fw, coef, (double*)W, W_stride,
        centre_tab, ncl, cur, step);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  set_int_kernel<<<1, 64, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint helpers
// ---------------------------------------------------------------------------
// out[k][q] = sum over blocks b of partials[k][b][q], q < 32, for every kick
// k (one block each), in double and in a fixed order (8 strided block
// subsets, then their sum)
template <typename R>
__global__ void __launch_bounds__(256) adj_reduce_kernel(const R* __restrict__ partials,
                                                         int64_t nblocks, double* out) {
  __shared__ double sh[8][32];
  const int q = threadIdx.x & 31, part = threadIdx.x >> 5;
  const R* pk = partials + (int64_t)blockIdx.x * nblocks * 32;
  double s = 0.0;
  for (int64_t b = part; b < nblocks; b += 8) s += double(pk[b * 32 + q]);
  sh[part][q] = s;
  __syncthreads();
  if (part == 0) {
    double t = 0.0;
    for (int k = 0; k < 8; ++k) t += sh[k][q];
    out[(int64_t)blockIdx.x * 32 + q] = t;
  }
}

hipError_t launch_adj_reduce(int dtype, const void* partials, int64_t nblocks, int nkicks,
                             double* out, hipStream_t s) {
  if (nkicks <= 0) return hipSuccess;
  if (dtype == 0)
    adj_reduce_kernel<float><<<nkicks, 256, 0, s>>>((const float*)partials, nblocks, out);
  else
    adj_reduce_kernel<double><<<nkicks, 256, 0, s>>>((const double*)partials, nblocks, out);
  return hipGetLastError();
}

// Power per degree: E_l = sum_n [a_nl0^2 + 2 sum_{m>=1} (Re^2 + Im^2)], one
// block per degree, a fixed-order tree over the block.
__global__ void __launch_bounds__(256) power_kernel(const double* __restrict__ coef, int nmax,
                                                    int lmax, double* El) {
  __shared__ double sh[256];
  const int l = blockIdx.x;
  const int L2 = (lmax + 1) * (lmax + 1);
  const int per = 2 * l + 1;
  double s = 0.0;
  for (int q = threadIdx.x; q < (nmax + 1) * per; q += blockDim.x) {
    const int n = q / per, j = q % per;
    const double a = coef[(int64_t)n * L2 + l * l + j];
    s += (j == 0 ? 1.0 : 2.0) * a * a;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) El[l] = sh[0];
}

hipError_t launch_power(const double* coef, int nmax, int lmax, int ncl, double* El,
                        hipStream_t s) {
  const int64_t T = (int64_t)(nmax + 1) * (lmax + 1) * (lmax + 1);
  for (int c = 0; c < ncl; ++c) {
    power_kernel<<<lmax + 1, 256, 0, s>>>(coef + c * T, nmax, lmax, El + (int64_t)c * (lmax + 1));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

Engine* find_engine(int dtype, int nmax, int lmax) {
  if (nmax < 0 || lmax < 0) return nullptr;
  Engine* e = dtype == 0 ? find_engine_f32_exact(nmax, lmax) : find_engine_f64_exact(nmax, lmax);
  if (e) return e;
  return dtype == 0 ? find_engine_f32_generic(nmax, lmax) : find_engine_f64_generic(nmax, lmax);
}

}  // namespace scf
