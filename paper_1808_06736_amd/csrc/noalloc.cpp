// esn_setpts_noalloc: esn_setpts for callers that cannot allocate device
// memory.  The bin sort's scratch (digit counts, the published tile counts of
// the radix passes, the records between passes, the sorted keys) lives in one
// static device array per GPU instead of plan memory.
#include <mutex>

#include "esn_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;   // 128 MiB per GPU
constexpr int kMaxDevices = 64;

// The shared scratch.  In host code this name is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (looked up once
// per device, with that device current).
void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return nullptr;
    g_ptr[device] = ptr;
  }
  return g_ptr[device];
}

}  // namespace

extern "C" int esn_setpts_noalloc(esn_plan p, int64_t M, int coord_prec, const void* x,
                                  const void* y, const void* z) {
  if (!p || p->type == 3) return ESN_ERR_BAD_ARG;
  void* ptr = scratch_ptr(p->device);
  if (!ptr) return ESN_ERR_HIP;
  const void* xs[3] = {x, y, z};
  return esn::setpts_impl(p, M, coord_prec, xs, ptr, kScratchBytes);
}
