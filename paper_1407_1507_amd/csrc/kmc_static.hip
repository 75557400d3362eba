// Allocation-free form of the count (kmc_count_static): every scratch buffer
// of the job is carved from one static device array, so the call makes no
// device or pinned-host allocation.  For callers that cannot allocate: code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc.
//
// The array is a file-scope __device__ object: each device the library runs
// on holds its own copy, at its own address, until the process ends.  In host
// code the array's name is only a host-side stand-in, so its device address is
// taken once per device with hipGetSymbolAddress (with that device current)
// and only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/kmc.h"
#include "kmc_internal.h"

static __device__ __align__(256) uint8_t scratch[KMC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceScratch {
  std::mutex mu;          // one call at a time on a device (they share the array)
  void* ptr = nullptr;    // device address of `scratch` on that device
};

DeviceScratch& device_scratch(int dev) {
  static DeviceScratch* table = new DeviceScratch[kMaxDevices];  // lives until exit
  return table[dev];
}

}  // namespace

extern "C" kmc_status kmc_count_static(kmc_ctx* ctx, const kmc_reads* reads,
                                       const kmc_params* params, void* stream,
                                       uint64_t* keys_out, uint32_t* counts_out,
                                       uint64_t out_cap, uint64_t* n_out,
                                       uint64_t* bin_offsets, kmc_stats* stats) {
  if (!ctx || !n_out) return KMC_ERR_INVALID_ARG;
  *n_out = 0;
  const int dev = kmc::ctx_device(ctx);
  if (dev < 0 || dev >= kMaxDevices) return KMC_ERR_DEVICE;
  DeviceScratch& ds = device_scratch(dev);
  std::lock_guard<std::mutex> lk(ds.mu);
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  if (!ds.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      kmc::ctx_set_error(ctx, "hipGetSymbolAddress of the static scratch failed");
      return KMC_ERR_DEVICE;
    }
    ds.ptr = p;
  }
  return kmc::count_static_impl(ctx, reads, params, stream, ds.ptr, KMC_STATIC_SCRATCH_BYTES,
                                keys_out, counts_out, out_cap, n_out, bin_offsets, stats);
}
