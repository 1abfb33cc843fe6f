// rbc_matmul_noalloc (include/rbc.h): rbc_matmul with its workspace in a fixed
// device array instead of a caller's buffer, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).  The call
// runs exactly the kernels of rbc_matmul, so C is the same to the bit.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "handles.hpp"
#include "launches.hpp"

namespace {

// Each device that runs this library holds one copy until the process ends.
__device__ __align__(256) char scratch[RBC_NOALLOC_MAX_WORKSPACE];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of this device's copy, looked up once per device with that
// device current.  In host code `scratch` names a host-side stand-in, never
// usable as a device pointer.
rbc_status scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return rbc::fail(RBC_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return RBC_OK;
}

}  // namespace

extern "C" rbc_status rbc_matmul_noalloc(rbc_plan h, const void* A, int64_t lda, const void* B, int64_t ldb,
                                         void* C, int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale,
                                         void* stream) {
  try {
    if (!h) return rbc::fail(RBC_EINVAL, "null plan");
    if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return rbc::fail(RBC_EINVAL, "bad mode %d", (int)mode);
    rbc::Plan& p = h->p;
    if (p.ws_bytes > (size_t)RBC_NOALLOC_MAX_WORKSPACE)
      return rbc::fail(RBC_EINVAL, "plan needs %zu bytes of workspace; the fixed device array holds %zu",
                       p.ws_bytes, (size_t)RBC_NOALLOC_MAX_WORKSPACE);
    if (!p.dev_tables)
      return rbc::fail(RBC_EINVAL, "the plan's coefficient tables are not on the device yet (they are "
                                   "uploaded by the plan's first rbc_matmul on this device)");
    if (p.timing) return rbc::fail(RBC_EINVAL, "stage timing creates events: turn it off for this call");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rbc::fail(RBC_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return rbc::fail(RBC_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    if (dev != p.device)
      return rbc::fail(RBC_EINVAL, "plan was first used on device %d, now %d", p.device, dev);
    void* ws = nullptr;
    rbc_status st = scratch_address(dev, &ws);
    if (st != RBC_OK) return st;
    std::vector<int32_t> s, pm;
    rbc::seeded_draws(p, seed, mode, s, pm);
    return rbc::matmul_impl(p, A, lda, B, ldb, C, ldc, s.data(), pm.data(), kappa_scale, ws,
                            (size_t)RBC_NOALLOC_MAX_WORKSPACE, stream);
  } catch (...) {
    return rbc::fail(RBC_ENOMEM, "host allocation failed");
  }
}
