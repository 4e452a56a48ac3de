// fock_diag_fwd_static: fock_diag_fwd with library-owned scratch memory, for
// callers that cannot allocate device memory.  The scratch is one file-scope
// device array; in host code its name is only a host-side stand-in, so every
// host use goes through the device address that hipGetSymbolAddress returns
// for the current device (resolved once per device, on the entry point's
// first call there).
#include <mutex>

#include "fd_internal.h"

namespace fd {
namespace {

// Largest forward workspace the entry point accepts: the prep block, F0 in
// node order and the two-level family rings of one sweep.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;

// Each device holds its own copy from module load until the process ends.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (the device is current
// when hipGetSymbolAddress runs).
fd_status scratch_address(void** ptr, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return FD_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *err = "device ordinal beyond the static scratch table";
    return FD_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e);
      return FD_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return FD_OK;
}

bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace
}  // namespace fd

extern "C" fd_status fock_diag_fwd_static(fd_plan p, const void* A, const void* b, const void* c, void* rho,
                                          hipStream_t stream) {
  if (!p) return fd::api_fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  const size_t al = P.dt == FD_C64 ? 8 : 16;
  for (const void* q : {A, b, c, static_cast<const void*>(rho)}) {
    if (!q) return fd::api_fail(FD_ERR_INVALID_ARG, "a required device pointer is NULL");
    if (!fd::aligned_to(q, al)) return fd::api_fail(FD_ERR_INVALID_ARG, "complex buffers must be aligned to their element size");
  }
  // the b = 0 schedule only on the caller's promise: no synchronising read of b
  const bool odd = P.odd_for(P.flags == FD_B_ZERO);
  const size_t need = fd::fwd_layout(P, odd, false, 0).total;
  if (need > fd::kStaticScratchBytes)
    return fd::api_fail(FD_ERR_WORKSPACE, "the sweep needs " + std::to_string(need) +
                                              " bytes of scratch, more than the static array's " +
                                              std::to_string(fd::kStaticScratchBytes));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fd::api_fail(FD_ERR_HIP, "hipGetDevice failed");
  if (!P.d_pn || P.device != dev)
    return fd::api_fail(FD_ERR_INVALID_ARG,
                        "the plan has no device tables on the current device: make one fock_diag_fwd (or "
                        "detection_probs, fock_diag_vjp, fock_diag_jvp) call with it on this device first");
  void* ws = nullptr;
  std::string err;
  const fd_status s = fd::scratch_address(&ws, &err);
  if (s != FD_OK) return fd::api_fail(s, err);
  // no per-kernel timing events for this call (they would be created on demand)
  const uint32_t tmask = P.timing.mask;
  P.timing.mask = 0;
  const hipError_t e = fd::run_forward(P, odd, A, b, c, rho, ws, nullptr, stream);
  P.timing.mask = tmask;
  if (e != hipSuccess) return fd::api_fail(FD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return fd::api_ok();
}
