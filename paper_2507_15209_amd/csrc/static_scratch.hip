// static_scratch.hip -- the value-and-gradient entry point for callers that
// cannot allocate (code under HIP graph capture, tight serving loops): the
// scratch memory every call needs lives in one file-scope device array of
// fixed size instead of a caller-provided workspace.
//
// Each GPU that runs this library holds its own copy of the array for the
// life of the process.  Host code never uses the array's name as a device
// address: the address of each device's copy is taken once per device with
// hipGetSymbolAddress (that device current) and kept; kernels receive it as
// they receive a workspace.  Calls on one GPU share that GPU's copy.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "mp3.h"

namespace mp3 {
void set_last_error(const std::string& msg);
}

namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// the address of the current device's copy of scratch (taken on first use)
int device_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    mp3::set_last_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return MP3_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    mp3::set_last_error("device index beyond the static scratch table");
    return MP3_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      mp3::set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return MP3_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MP3_OK;
}

}  // namespace

extern "C" {

size_t mp3_static_scratch_bytes(void) { return kStaticScratchBytes; }

int mp3_zeta_value_and_grad_static(mp3_plan_t plan, const void* delta, const double* dzeta, double* zeta,
                                   void* ddelta, const float* pos, const float* w, const int64_t* np_off, void* dw,
                                   void* stream) {
  if (!plan) {
    mp3::set_last_error("plan is NULL");
    return MP3_EINVAL;
  }
  int32_t batch = 0;
  if (int s = mp3_plan_info(plan, nullptr, nullptr, nullptr, nullptr, &batch)) return s;
  const int64_t np_total = np_off ? np_off[batch] : 0;
  if (np_total < 0) {
    mp3::set_last_error("np_off[batch] must be >= 0");
    return MP3_EINVAL;
  }
  size_t need = 0;
  if (int s = mp3_workspace_size(plan, np_total, &need)) return s;
  if (need > kStaticScratchBytes) {
    mp3::set_last_error("this call needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                        std::to_string(kStaticScratchBytes) + " (use mp3_zeta_value_and_grad with a workspace)");
    return MP3_EWORKSPACE;
  }
  void* ws = nullptr;
  if (int s = device_scratch(&ws)) return s;
  return mp3_zeta_value_and_grad(plan, delta, dzeta, zeta, ddelta, pos, w, np_off, dw, ws, kStaticScratchBytes,
                                 stream);
}

}  // extern "C"
