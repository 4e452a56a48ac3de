// Device-side entry points of the library replaced by failing stubs, so the
// host code (planner and C ABI) links without the GPU objects: the sanitizer
// driver only takes host paths, and a stub reached by mistake fails loudly.
#include <cstdio>
#include <cstdlib>

#include "fd_internal.h"

namespace fd {
namespace {
[[noreturn]] void reached(const char* what) {
  std::fprintf(stderr, "host sanitizer driver reached a device path: %s\n", what);
  std::abort();
}
}  // namespace

hipError_t run_forward(const Plan&, bool, const void*, const void*, const void*, void*, void*, void*, hipStream_t,
                       StopRule*) { reached("run_forward"); }
hipError_t run_vjp(const Plan&, bool, const void*, const void*, const void*, const void*, const void*, void*, void*,
                   void*, void*, hipStream_t) { reached("run_vjp"); }
hipError_t run_jvp(const Plan&, const void*, const void*, const void*, const void*, const void*, const void*, void*,
                   void*, void*, hipStream_t) { reached("run_jvp"); }
hipError_t run_state_fwd(const Plan&, bool, const void*, const void*, const void*, void*, void*, hipStream_t) {
  reached("run_state_fwd");
}
hipError_t run_state_jvp(const Plan&, const void*, const void*, const void*, const void*, const void*, void*,
                         hipStream_t) { reached("run_state_jvp"); }
hipError_t run_state_vjp(const Plan&, const void*, const void*, const void*, void*, void*, void*, void*, hipStream_t) {
  reached("run_state_vjp");
}
fd_status run_forward_batch(int, Plan* const*, const bool*, const void* const*, const void* const*,
                            const void* const*, void* const*, void* const*, hipStream_t, std::string*) {
  reached("run_forward_batch");
}
void batch_forget(uint64_t) {}
fd_status batch_set_tuning(const fd_batch_tuning&) { return FD_OK; }
fd_batch_tuning batch_get_tuning() { return fd_batch_tuning{2, 64, 4}; }
}  // namespace fd
