// Forward render that allocates nothing: for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Every intermediate of
// the preprocess -> bin/sort -> raster sequence lives in one fixed device array per GPU, held by the
// library until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "drk_internal.hpp"

namespace drk {

constexpr size_t kNoAllocBytes = size_t(128) << 20;   // the fixed array: 128 MiB per device
constexpr int kNoAllocDevices = 64;

// The array itself.  Host code never uses this name as an address: it takes the device address of
// each GPU's copy from hipGetSymbolAddress once and passes that to the kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};
}  // namespace

}  // namespace drk

using namespace drk;

extern "C" drk_status drk_render_fwd_noalloc(const drk_scene* scene, const drk_camera* cam, const drk_opts* opts,
                                              float* rgb, float* T_final, void* stream) {
  if (!scene || !cam || !opts || !rgb) { set_error("null argument"); return DRK_EINVAL; }
  if (opts->counters != 0) { set_error("drk_render_fwd_noalloc writes no per-pixel counters (opts.counters must be 0)"); return DRK_EINVAL; }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) {
    set_error("drk_render_fwd_noalloc: no usable current device");
    return DRK_EDEVICE;
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      // once per device, with that device current: the device address of its copy of the array
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        return DRK_EDEVICE;
      }
      g_scratch_ptr[dev] = p;
    }
    base = g_scratch_ptr[dev];
  }
  return render_placed(base, kNoAllocBytes, scene, cam, opts, rgb, T_final, reinterpret_cast<hipStream_t>(stream));
}
