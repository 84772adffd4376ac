// noalloc.hip -- links_simulate_noalloc: links_simulate with its workspace in a
// fixed device array instead of allocated device memory, for callers that cannot
// allocate (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The array below is one per GPU: each device that loads the library holds its
// own copy, at its own address, until the process ends.  Host code never passes
// the array's name to a kernel or a copy (in host code it names a host-side
// stand-in, not device memory): links_create looks up this device's address of
// the array once per device (hipGetSymbolAddress, with the device current) and
// every call uses that address.
//
// Every call on a device shares its array and leaves its contents behind; the
// passes clear what must start at zero (work counters, bucket histograms) with
// fill kernels.  Calls that overlap in time on one device race: they must be
// issued on one stream or synchronised with each other.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/links.h"
#include "kernels.h"

namespace {

static __device__ __align__(256) unsigned char scratch[LINKS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device
int g_table_T[kMaxDevices];              // steps of the crank table each array holds

}  // namespace

namespace links {

// Called by links_create with `device` current.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return report_error(LINKS_ERR_ARG, "device index above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return LINKS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return report_error(LINKS_ERR_DEVICE, "hipGetSymbolAddress of the allocation-free scratch area failed");
  }
  g_table_T[device] = -1;
  g_ptr[device] = static_cast<unsigned char*>(p);
  return LINKS_OK;
}

}  // namespace links

extern "C" int links_simulate_noalloc(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts,
                                      links_sim_out* out, void* stream) {
  if (!ctx) return links::report_error(LINKS_ERR_ARG, "ctx is NULL");
  const int dev = links::ctx_device(ctx);
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev >= 0 && dev < kMaxDevices) base = g_ptr[dev];
  }
  if (!base) return links::report_error(LINKS_ERR_DEVICE, "the allocation-free scratch area of this device is not set up");
  return links::simulate_in_arena(ctx, batch, opts, out, stream, base, LINKS_NOALLOC_SCRATCH_BYTES, &g_table_T[dev]);
}
