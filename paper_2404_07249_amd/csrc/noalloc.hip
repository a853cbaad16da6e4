// Power spectrum without any allocation (pb3_power_noalloc): the forward
// transform and the binned sums of pb3_power, with their workspace (the
// z-pass and y-pass outputs, the compact spectrum and the per-chunk sums)
// carved from a file-scope device array instead of the plan's workspace.
//
// The array is one per GPU: its device address is looked up once per
// device (hipGetSymbolAddress with that device current) and kept; host code
// passes that address, never the array's name, to kernels.  Every call on a
// GPU uses the same memory, so calls that overlap on one GPU race; nothing
// in it needs to start at zero (every pass writes its whole output before
// the next pass reads it).

#include <hip/hip_runtime.h>

#include <mutex>

#include "pb3_internal.h"

namespace pb3 {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// bytes of the power path's workspace at the plan's geometry
static size_t power_scratch_bytes(const pb3_plan& p) {
  return up256(sizeof(float2) * (size_t)p.Nx * p.Ny * p.Kz) + up256(sizeof(float2) * (size_t)p.Nx * p.Lcy * p.Kz) +
         up256(sizeof(float2) * ncompact(p)) + up256(sizeof(double) * (size_t)(p.n_chunks > 0 ? p.n_chunks : 1));
}

// device address of this device's array (looked up on the first call here)
static pb3_status scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    set_error("device index beyond the supported range");
    return PB3_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PB3_OK;
}

}  // namespace pb3

using namespace pb3;

extern "C" {

pb3_status pb3_power_noalloc(pb3_plan* plan, const float* delta_dev, double* pk_dev, void* stream) {
  if (!plan || !delta_dev || !pk_dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (!plan->device) {
    set_error("plan has no device state (created with PB3_FLAG_HOST_ONLY)");
    return PB3_EINVAL;
  }
  pb3_status st = check_field_ptr(delta_dev, "delta");
  if (st != PB3_OK) return st;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device_id) {
    set_error("plan was created on another device");
    return PB3_EINVAL;
  }
  const size_t need = power_scratch_bytes(*plan);
  if (need > kNoAllocBytes) {
    set_error("the plan's power spectrum needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string(kNoAllocBytes) + " bytes of the static array");
    return PB3_EUNSUPPORTED;
  }
  void* base = nullptr;
  if ((st = scratch_for(dev, &base)) != PB3_OK) return st;
  char* c = (char*)base;
  auto take = [&](size_t n) {
    char* r = c;
    c += up256(n);
    return (void*)r;
  };
  Exec x;
  x.ws.base = base;
  x.ws.bytes = need;
  x.ws.f1 = (float2*)take(sizeof(float2) * (size_t)plan->Nx * plan->Ny * plan->Kz);
  x.ws.f2 = (float2*)take(sizeof(float2) * (size_t)plan->Nx * plan->Lcy * plan->Kz);
  x.ws.dc = (float2*)take(sizeof(float2) * ncompact(*plan));
  x.ws.ppart = (double*)take(sizeof(double) * (size_t)(plan->n_chunks > 0 ? plan->n_chunks : 1));
  x.io.delta[0] = delta_dev;
  x.io.pk[0] = pk_dev;
  const hipStream_t s = (hipStream_t)stream;
  if ((e = launch_fwd_z(*plan, x, s)) != hipSuccess) return hip_fail(e, "fwd_z");
  if ((e = launch_fwd_y(*plan, x, s)) != hipSuccess) return hip_fail(e, "fwd_y");
  if ((e = launch_fwd_x(*plan, x, s)) != hipSuccess) return hip_fail(e, "fwd_x");
  if ((e = launch_power(*plan, x, s, true)) != hipSuccess) return hip_fail(e, "power");
  return PB3_OK;
}

}  // extern "C"
