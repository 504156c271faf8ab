// Allocation-free surrogate prediction: sur_predict with every workspace of
// its forward pass (hidden activations, split-K partial sums) cut from a
// fixed device array of the library instead of its allocator, for callers
// that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/ctm_opt.h"
#include "engine.h"
#include "surrogate.h"

using namespace ctm;

// 16 MiB: enough for batches of about 3000 inputs of the 5000 -> 256 -> 256 -> 1 network.
constexpr size_t kScratchBytes = (size_t)16 << 20;

// One copy per GPU, present from the loading of the code object to the end
// of the process.  Host code must not pass this name to a kernel or a copy:
// on the host it only stands for the symbol; its device address comes from
// hipGetSymbolAddress (per device, in sur_scratch_setup).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* current_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch_ptr[dev];
}

}  // namespace

namespace ctm {

int sur_scratch_setup() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[dev]) return (int)hipSuccess;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  g_scratch_ptr[dev] = p;
  return (int)hipSuccess;
}

}  // namespace ctm

extern "C" int sur_predict_noalloc(sur_net* s, const float* X, int batch, float* y) {
  if (!s || !X || !y || batch < 1) return CTM_EINVAL;
  try {
    const int64_t need = sur_predict_workspace_bytes(s->n_in, s->width, batch);
    if (need > (int64_t)kScratchBytes)
      throw Error(CTM_EINVAL, "sur_predict_noalloc: batch " + std::to_string(batch) + " needs " +
                                  std::to_string(need) + " bytes of scratch, the maximum is " +
                                  std::to_string(kScratchBytes));
    void* p = current_scratch();
    if (!p) {
      // first call on a device the network was not created on
      HIP_CHECK((hipError_t)sur_scratch_setup());
      p = current_scratch();
      if (!p) throw Error(CTM_EHIP, "sur_predict_noalloc: no scratch on the current device");
    }
    ArenaScope arena(&s->dev, p, kScratchBytes);
    sur_predict_impl(s, X, batch, y);
    return CTM_OK;
  } catch (const Error& e) {
    s->err = e.what();
    return e.code;
  }
}
