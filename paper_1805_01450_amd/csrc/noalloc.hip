// The allocation-free form of qgm_amplitudes_device: its device workspace
// (constant-step results, packed bitstrings, per-item results, the work-queue
// counter, slice-sum partials and item memory) is a fixed array in the
// library's own device image instead of caller memory, so a caller that
// cannot allocate (code under graph capture, tight serving loops) needs none.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qgm.h"

namespace qgm {
qgm_status run_on_fixed_workspace(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                                  uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream,
                                  double* d_partial);
qgm_status fail_status(qgm_status s, const char* msg);
}  // namespace qgm

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // QGM_NOALLOC_SCRATCH_BYTES in qgm.h
static_assert(kScratchBytes == QGM_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

// One copy per device, allocated by the runtime when the library's code
// object is loaded there and kept until the process ends.  Host code never
// uses this name as an address: it is a host-side stand-in; the device
// address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
qgm_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return qgm::fail_status(QGM_E_HIP, "hipGetDevice failed or device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return qgm::fail_status(QGM_E_HIP, "hipGetSymbolAddress(scratch) failed");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return QGM_OK;
}

}  // namespace

extern "C" qgm_status qgm_amplitudes_device_noalloc(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs,
                                                   const double* d_params, uint64_t s_begin, uint64_t s_end,
                                                   void* hip_stream, double* d_partial) {
  if (!p) return qgm::fail_status(QGM_E_ARG, "null plan");
  void* ws = nullptr;
  qgm_status s = scratch_for_current_device(&ws);
  if (s) return s;
  return qgm::run_on_fixed_workspace(p, d_bits, n_bs, d_params, s_begin, s_end, ws, kScratchBytes, hip_stream,
                                     d_partial);
}
