// Batched persistent sweep kernel for any batch (up to 8 detected modes and
// 2 undetected modes).
#include "batch_sweep.h"

namespace fd {

hipError_t batch_sweep_md8(bool c64, const BatchSweepArgs* a, int* per_cu, hipStream_t st) {
  return batch_sweep_impl<8, 8, 4>(c64, a, per_cu, st);
}

}  // namespace fd
