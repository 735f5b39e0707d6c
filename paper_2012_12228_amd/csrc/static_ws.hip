// Allocation-free initialisation: ftafqmc_init_ueg with the workspace taken from a file-scope
// device array instead of the caller, for callers that cannot allocate device memory.
//
// The array `scratch` exists once per device (each device that loads the library holds its
// FTAFQMC_STATIC_WORKSPACE_BYTES until the process ends).  In host code its name is only a
// stand-in: its device address is obtained once per device with hipGetSymbolAddress, and that
// address is what the library hands to its kernels.  One handle per device may hold the array
// at a time (a second init on the device returns FTAFQMC_E_STATE until the first handle is
// destroyed); work enqueued through handles of different processes or threads that overlap on
// one device would race on it.  Every buffer the kernels read is written by the library before
// it is read (ftafqmc_init_ueg sets the tables and the walker state), so stale contents from a
// previous handle do not matter.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ftafqmc.h"
#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[FTAFQMC_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
void* scratch_addr[MAX_DEVICES];     // device address of `scratch` on each device, once known
ftafqmc_t holder[MAX_DEVICES];       // the live handle that uses the device's array, if any
std::mutex lock;

}  // namespace

void static_ws_release(ftafqmc_t h) {
  if (!h) return;
  std::lock_guard<std::mutex> g(lock);
  for (int d = 0; d < MAX_DEVICES; ++d)
    if (holder[d] == h) holder[d] = nullptr;
}

extern "C" int ftafqmc_init_ueg_static(const ftafqmc_params* p, int n_sys, void* stream, ftafqmc_t* out) {
  if (!p || n_sys < 1 || !out) return lib_init_error(FTAFQMC_E_ARG, "null parameters or output");
  for (int i = 0; i < n_sys; ++i)
    if (p[i].flags & (FTAFQMC_OVERLAP | FTAFQMC_GRAPH))
      return lib_init_error(FTAFQMC_E_ARG, "the static workspace takes no FTAFQMC_OVERLAP or FTAFQMC_GRAPH "
                                           "(they create streams and graphs)");
  size_t need = 0;
  if (ftafqmc_workspace_bytes(p, n_sys, &need) != FTAFQMC_OK)
    return lib_init_error(FTAFQMC_E_ARG, "invalid system parameters");
  if (need > (size_t)FTAFQMC_STATIC_WORKSPACE_BYTES)
    return lib_init_error(FTAFQMC_E_ARG, "systems need more workspace than the static maximum "
                                         "FTAFQMC_STATIC_WORKSPACE_BYTES (use ftafqmc_init_ueg)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return lib_init_error(FTAFQMC_E_HIP, "no current device");
  std::lock_guard<std::mutex> g(lock);
  if (holder[dev]) return lib_init_error(FTAFQMC_E_STATE, "the device's static workspace is held by a live handle");
  if (!scratch_addr[dev]) {
    void* addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !addr) return lib_init_error(FTAFQMC_E_HIP, "hipGetSymbolAddress of the static workspace failed");
    scratch_addr[dev] = addr;
  }
  const int rc = init_ueg_impl(p, n_sys, scratch_addr[dev], (size_t)FTAFQMC_STATIC_WORKSPACE_BYTES, stream, out, true);
  if (rc == FTAFQMC_OK) holder[dev] = *out;
  return rc;
}
