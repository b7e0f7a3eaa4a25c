// Allocation-free variant of scf_step for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The workspace of the step (partial rows of the
// coefficient pass, the double-precision chunk sums, the coefficients and the
// force weights) comes from one file-scope device array instead of the caller.
//
// Every GPU the library runs on holds its own copy of the array (kScratchBytes)
// until the process ends; all calls on one GPU share it and it keeps the last
// call's contents.  The step writes every byte it later reads (each partial
// row in full, every chunk sum, every coefficient and weight), so nothing is
// cleared between calls.  Calls that overlap on one GPU (two host threads, or
// two streams without ordering between them) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scf_plan.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// Device address of this device's copy of the array.  In host code `scratch`
// names a host-side stand-in, not device memory, so the address is looked up
// once per device (with that device current) and only it is used afterwards.
scf_status scratch_for_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SCF_ERR_UNSUPPORTED, "device %d beyond the %d devices with static scratch", dev,
                kMaxDevices);
  std::call_once(g_scratch_once[dev], [dev]() {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? ptr : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return fail(SCF_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch_ptr[dev];
  return SCF_OK;
}

}  // namespace

extern "C" {

size_t scf_noalloc_scratch_bytes(void) { return kScratchBytes; }

scf_status scf_step_noalloc(scf_plan* p, int64_t n, void* x, void* y, void* z, void* vx,
                            void* vy, void* vz, const void* m, void* ax, void* ay, void* az,
                            uint32_t step_flags, const scf_host* host, double* centre, double dt,
                            int32_t nsteps, double* coef_last, void* stream) {
  if (!p) return fail(SCF_ERR_INVALID_ARG, "plan is null");
  if (n < 0) return fail(SCF_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
  const size_t need = plain_need(p, n);
  if (need > kScratchBytes)
    return fail(SCF_ERR_WORKSPACE,
                "this plan's step needs %zu bytes of workspace; the static scratch holds %zu",
                need, kScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device)
    return fail(SCF_ERR_INVALID_ARG, "plan belongs to device %d, current device is %d", p->device,
                dev);
  void* ws = nullptr;
  scf_status st = scratch_for_device(dev, &ws);
  if (st != SCF_OK) return st;
  return scf_step(p, n, x, y, z, vx, vy, vz, m, ax, ay, az, step_flags, host, centre, dt, nsteps,
                  coef_last, ws, kScratchBytes, stream);
}

}  // extern "C"
