// static_run.cpp -- mhs_run_static: the one-instance reduction with its
// workspace in a static device array, for callers that cannot allocate.
//
// `scratch` is a file-scope device array; every device the library runs on
// holds its own copy until the process ends.  In host code its name is only
// a host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// ever passed to kernels or copies.
#include "host.h"

#include <mutex>

namespace mhsk {
int run_without_allocation(const mhs_instance* inst, uint32_t flags, char* ws, size_t ws_bytes,
                           hipStream_t stream, mhs_summary* sum, int32_t* death_e, int32_t* death_v);
}  // namespace mhsk

using namespace mhsk;

static __device__ __align__(256) char scratch[MHS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];          // one call at a time per device
char* g_scratch[kMaxDevices] = {};     // device address of `scratch`, per device
}  // namespace

extern "C" int mhs_run_static(const mhs_instance* inst, uint32_t flags, void* hip_stream, mhs_summary* summary,
                              int32_t* death_e, int32_t* death_v) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(MHS_EDEVICE, "no current device");
  if (dev < 0 || dev >= kMaxDevices) return set_error(MHS_EINVAL, "device ordinal beyond 63");
  std::lock_guard<std::mutex> g(g_mu[dev]);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return set_error(MHS_EDEVICE, "cannot find the static scratch on this device");
    g_scratch[dev] = (char*)p;
  }
  return run_without_allocation(inst, flags, g_scratch[dev], MHS_STATIC_SCRATCH_BYTES, (hipStream_t)hip_stream,
                                summary, death_e, death_v);
}
