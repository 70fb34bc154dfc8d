// hlb_noalloc.hip -- hlb_create_noalloc: a context whose workspace is a
// static device array of the library instead of caller-allocated memory,
// for callers that cannot allocate device memory.
//
// The array lives in the library's code object, so every GPU the library
// runs on holds its own copy from the first use until the process ends.  In
// host code the array's name is only a host-side stand-in: its device
// address is obtained once per device with hipGetSymbolAddress, with that
// device current, and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hlb.h"

constexpr size_t kScratchBytes = size_t(HLB_NOALLOC_MAX_BYTES);

// The workspace of a no-allocation context.  Never passed to a kernel by its
// name: host code uses only the address hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices];      // device address of `scratch` per device, once obtained
const hlb_ctx *g_owner[kMaxDevices];  // the live context over a device's array, if any

}  // namespace

// Internal functions of hlb_api.hip (not part of the ABI): context creation
// over a given workspace, and the message that hlb_last_error(NULL) reports.
hlb_status hlb_internal_create(hlb_ctx **out, int lattice, int storage, int nx, int ny, int nz, const hlb_params *p,
                               void *workspace, size_t bytes, void *stream, bool static_ws);
void hlb_internal_set_create_error(const std::string &msg);

// Called by hlb_destroy for a context over the static array: the array of
// its device is free again.
void hlb_internal_release_noalloc(const hlb_ctx *c) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto &o : g_owner)
    if (o == c) o = nullptr;
}

extern "C" hlb_status hlb_create_noalloc(hlb_ctx **out, int lattice, int storage, int nx, int ny, int nz,
                                          const hlb_params *p, void *stream) {
  if (!out) {
    hlb_internal_set_create_error("out is NULL");
    return HLB_EINVAL;
  }
  *out = nullptr;
  size_t bytes = 0;
  hlb_status s = hlb_workspace_size_params(lattice, storage, nx, ny, nz, p, &bytes);
  if (s != HLB_OK) return s;  // hlb_workspace_size set the message
  if (bytes > kScratchBytes) {
    hlb_internal_set_create_error("hlb_create_noalloc: this lattice needs " + std::to_string(bytes) +
                                  " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                  " bytes of the static array; use hlb_create with a caller workspace");
    return HLB_ESHAPE;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    hlb_internal_set_create_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return HLB_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    hlb_internal_set_create_error("hlb_create_noalloc: device index out of range");
    return HLB_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_owner[dev]) {
    hlb_internal_set_create_error(
        "hlb_create_noalloc: the static array of this device already holds a live context; destroy it first");
    return HLB_ESTATE;
  }
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      hlb_internal_set_create_error(std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
      return HLB_EHIP;
    }
    g_ptr[dev] = ptr;
  }
  // Every array of the context is written before it is read (hlb_init_fields
  // or hlb_set_state writes the state, a step writes u*, a reduction its
  // partial sums), so the previous context's contents need no clearing.
  s = hlb_internal_create(out, lattice, storage, nx, ny, nz, p, g_ptr[dev], kScratchBytes, stream, true);
  if (s != HLB_OK) return s;
  g_owner[dev] = *out;
  return HLB_OK;
}
