// sgwls_filter for callers that cannot allocate device memory (code under
// graph capture, serving loops, harnesses that forbid allocation): the
// filter's workspace is a file-scope device array instead of a caller buffer.
#include "sgwls.h"
#include "sgwls_internal.hpp"

#include <mutex>

namespace {

// Scratch of sgwls_filter_noalloc on every device the library runs on (held
// until the process ends).  Its host-side name is only a symbol: kernels get
// the device address that hipGetSymbolAddress returns for it.
constexpr size_t kScratchBytes = SGWLS_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device
// with that device current; nullptr if the lookup fails.
void* device_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mutex);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[dev] = ptr;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" sgwls_status sgwls_filter_noalloc(const float* f, const float* g, float* u, int C,
                                             int M, int N, const sgwls_params* p,
                                             const float* lambda_dev, float* saved,
                                             void* stream) {
  const sgwls_status st = sgwls_validate(C, M, N, p);
  if (st != SGWLS_OK) return st;
  const size_t need = sgwls_workspace_bytes(C, M, N, p, saved ? 1 : 0);
  if (need == 0 || need > kScratchBytes) return SGWLS_E_WORKSPACE;
  void* ws = device_scratch();
  if (!ws) return SGWLS_E_HIP;
  // Everything the filter reads from its workspace it writes first in the
  // same call, so the array needs no clearing between calls.  Three
  // launches per pass: the caller could not read a fused pass's wait error
  // back from the library's array.
  const sgwls::NoFusedScope three_launches;
  return sgwls_filter(f, g, u, C, M, N, p, lambda_dev, saved, ws, kScratchBytes, stream);
}
