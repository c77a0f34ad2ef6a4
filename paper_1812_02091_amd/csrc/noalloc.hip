// The scratch region of lcemd_topl_noalloc: a file-scope device array, so
// that calls which cannot allocate (graph capture, tight serving loops)
// still have room for tables, distance rows and candidate lists.  Each GPU
// holds its own copy of the array at its own address from module load to
// process end; its address is looked up once per device, with that device
// current, and only that address is ever handed to kernels or copies.
#include <mutex>

#include "context.h"

namespace {
constexpr size_t kNoAllocBytes = size_t(256) << 20;  // 256 MiB per device
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_mu;
void* g_ptr[64] = {};
}  // namespace

namespace lcemd_host {

size_t noalloc_capacity() { return kNoAllocBytes; }

int noalloc_setup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= 64) return LCEMD_E_NO_DEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return LCEMD_E_HIP;
    }
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return LCEMD_OK;
}

}  // namespace lcemd_host
