// Vector-ALU and matrix-core throughput microbenchmarks (measurement only):
// the issue-rate ceilings that the kernels' roofline fractions are read
// against.  Each lane runs NCH independent single-precision FMA chains (or
// MFMA chains) so that no dependency stalls the issue; waves_per_simd waves
// share each SIMD.
#include <hip/hip_runtime.h>

#include "../../include/scf.h"
#include "scf_plan.h"

namespace {

template <int NCH>
__global__ void __launch_bounds__(256) fma_chains_kernel(float* out, int iters, float b, float c) {
  float acc[NCH];
#pragma unroll
  for (int i = 0; i < NCH; ++i) acc[i] = float(threadIdx.x + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int i = 0; i < NCH; ++i) acc[i] = fmaf(acc[i], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NCH; ++i) s += acc[i];
  if (s == 1234.5f) out[blockIdx.x] = s;  // keeps the chains live
}

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef float mf16 __attribute__((ext_vector_type(16)));

// MFMA chains: kind 0 = 4x4x1 (16 blocks), 1 = 16x16x4, 2 = 32x32x2 (FP32)
template <int KIND>
__global__ void __launch_bounds__(256) mfma_chains_kernel(float* out, int iters, float a, float b) {
  if constexpr (KIND == 0) {
    mf4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c3, 0, 0, 0);
      }
    }
    const float s = c0[0] + c1[1] + c2[2] + c3[3];
    if (s == 1234.5f) out[blockIdx.x] = s;
  } else if constexpr (KIND == 1) {
    mf4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
      }
    }
    const float s = c0[0] + c1[1] + c2[2] + c3[3];
    if (s == 1234.5f) out[blockIdx.x] = s;
  } else {
    mf16 c0 = {}, c1 = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
      }
    }
    const float s = c0[0] + c1[1];
    if (s == 1234.5f) out[blockIdx.x] = s;
  }
}

// Both in one wave: per step four 4x4x1 MFMA chains and 16 FMA chains,
// independent of each other (the same per-wave counts as kinds 0 and 2 at the
// same iters), so that a pipe able to overlap them would finish in the time
// of the longer of the two.
__global__ void __launch_bounds__(256) mixed_chains_kernel(float* out, int iters, float a, float b) {
  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = float(threadIdx.x + i);
  mf4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c3, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = fmaf(acc[i], a, b);
    }
  }
  float s = c0[0] + c1[1] + c2[2] + c3[3];
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i];
  if (s == 1234.5f) out[blockIdx.x] = s;
}

}  // namespace

extern "C" {

scf_status scf_bench_ceiling(int32_t kind, int32_t waves_per_simd, int32_t iters, void* scratch,
                             double* tflops, double* ms) {
  if (!tflops || !ms || !scratch) return fail(SCF_ERR_INVALID_ARG, "null argument");
  if (kind < 0 || kind > 5 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1)
    return fail(SCF_ERR_INVALID_ARG, "bad kind, waves_per_simd or iters");
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // blocks of four waves (one per SIMD), waves_per_simd blocks per CU
  const int nblk = ncu * waves_per_simd;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float* out = (float*)scratch;
  double flop_per_thread = 0.0;
  auto launch = [&]() {
    switch (kind) {
      case 0:
        fma_chains_kernel<16><<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 16 * 8 * (double)iters;
        break;
      case 1:
        fma_chains_kernel<32><<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 32 * 8 * (double)iters;
        break;
      case 2:  // 16 blocks x 4x4x1 = 256 MACs per instruction per wave
        mfma_chains_kernel<0><<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 256 * 32 * (double)iters / 64.0;
        break;
      case 3:  // 16x16x4 = 1024 MACs
        mfma_chains_kernel<1><<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 1024 * 32 * (double)iters / 64.0;
        break;
      case 4:  // 32x32x2 = 2048 MACs
        mfma_chains_kernel<2><<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 2048 * 16 * (double)iters / 64.0;
        break;
      default:  // kinds 0 and 2 in one wave
        mixed_chains_kernel<<<nblk, 256>>>(out, iters, 0.999f, 1e-3f);
        flop_per_thread = 2.0 * 16 * 8 * (double)iters + 2.0 * 256 * 32 * (double)iters / 64.0;
        break;
    }
  };
  launch();  // warm-up
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e0, nullptr));
  launch();
  HIP_TRY(hipEventRecord(e1, nullptr));
  HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t;
  *tflops = flop_per_thread * 256.0 * nblk / (t * 1e-3) / 1e12;
  return SCF_OK;
}

}  // extern "C"
