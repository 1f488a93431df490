// Allocation-free variant of bgk_fine_propagate_moments (include/bgk.h).
//
// The batched lift -> fine propagation -> projection of Algorithm 2's jump
// loop needs a device workspace: two phase-space ping-pong buffers, the
// per-wave moment partials, Maxwellian factor rows and per-cell sums.  Here
// that workspace is a file-scope device array of fixed size, so the call
// itself allocates nothing (no hipMalloc, no library allocation, no timing
// events, no host-side bookkeeping) and can run inside HIP graph capture or
// a loop that must not allocate.  Every call on a device shares that
// device's array.
#include <mutex>

#include "bgk_internal.h"

namespace bgk {
namespace {

// Each device that loads the library holds its own copy of this array until
// the process ends.  In host code the name stands for a host-side symbol,
// not a device address: host code uses only the address returned for it by
// hipGetSymbolAddress on each device.
static __device__ __align__(256) unsigned char scratch[BGK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_of_current_device(void** out) {
  int dev = -1;
  BGK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal out of range for the no-allocation scratch table");
    return BGK_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BGK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) {
      set_error("no-allocation scratch has no 256-byte aligned device address");
      return BGK_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BGK_OK;
}

// Clears the sticky status word at the head of the scratch (a kernel, not a
// memset node, so that a captured call replays correctly).
__global__ void k_clear_status(int* st) {
  if (threadIdx.x == 0) *st = 0;
}

// The call's status for the caller's device int: BGK_OK, or
// BGK_E_NONPHYSICAL when a lift or reduction raised the sticky word.
__global__ void k_copy_status(const int* st, int32_t* out) {
  if (threadIdx.x == 0) *out = *st == 0 ? BGK_OK : BGK_E_NONPHYSICAL;
}

}  // namespace
}  // namespace bgk

using namespace bgk;

extern "C" int bgk_fine_propagate_moments_noalloc(const bgk_problem* prob, int32_t batch,
                                                  const double* V_in, double* V_out,
                                                  double t_span, int32_t* status,
                                                  void* stream) {
  // host-side checks first: nothing touches the device before the size test
  int rc = check_problem(prob);
  if (rc) return rc;
  if (batch < 1) {
    set_error("batch must be >= 1");
    return BGK_E_INVALID;
  }
  const size_t need = propagate_ws_bytes(*prob, batch);
  if (need > (size_t)BGK_NOALLOC_SCRATCH_BYTES) {
    set_error("bgk_fine_propagate_moments_noalloc: this batch needs " + std::to_string(need) +
              " bytes of scratch; the static scratch holds " +
              std::to_string((size_t)BGK_NOALLOC_SCRATCH_BYTES) + " bytes");
    return BGK_E_WORKSPACE;
  }
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* st = &reinterpret_cast<WsHeader*>(ws)->status;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
  BGK_HIP(hipGetLastError());
  noalloc_mode(true);
  rc = propagate_plain(prob, batch, V_in, V_out, t_span, ws, (size_t)BGK_NOALLOC_SCRATCH_BYTES,
                       stream);
  noalloc_mode(false);
  if (rc) return rc;
  if (status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, st, status);
    BGK_HIP(hipGetLastError());
  }
  return BGK_OK;
}
