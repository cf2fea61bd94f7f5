// dp_compute_noalloc: one force evaluation whose workspace is a file-scope device array,
// for callers that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid allocation).  The array is 64 MiB on every device the
// library initialises a handle on, held until the process ends.  Its device address is
// looked up once per device, at the first dp_init on that device, with the device
// current; host code uses only that address, never the array's host-side name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/dp.h"
#include "kernels.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

namespace dp {

// called by dp_init with `device` current
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return DP_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return DP_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return DP_ERR_HIP;
  g_scratch_ptr[device] = p;
  return DP_OK;
}

}  // namespace dp

extern "C" int dp_compute_noalloc(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                                  const double* box, double* energy, double* forces, double* virial,
                                  double* atom_energy, void* stream) {
  if (!h) return DP_ERR_ARG;
  const int dev = dp::handle_device(h);
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) p = g_scratch_ptr[dev];
  }
  if (!p) return dp::set_error(h, DP_ERR_HIP, "dp_compute_noalloc: scratch array address unknown on this device");
  if (!box) return dp::set_error(h, DP_ERR_ARG, "null box");
  size_t need = 0;
  const int rc = dp::compute_ws_bytes(h, natoms, box, &need);
  if (rc != DP_OK) return rc;
  if (need > kScratchBytes)
    return dp::set_error(h, DP_ERR_WORKSPACE,
                         "dp_compute_noalloc: this frame needs " + std::to_string(need) +
                             " bytes of workspace; the built-in scratch array holds " +
                             std::to_string(kScratchBytes) + " (use dp_compute with a caller workspace)");
  return dp_compute(h, natoms, coords, types, box, energy, forces, virial, atom_energy, p, kScratchBytes, stream);
}
