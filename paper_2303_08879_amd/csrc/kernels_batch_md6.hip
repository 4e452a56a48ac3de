// Batched persistent sweep kernel for batches of circuits with at most 6 modes
// and at most one undetected mode (Algorithm 1: <= 6 detected modes;
// Algorithm 2: <= 5 detected modes).
#include "batch_sweep.h"

namespace fd {

hipError_t batch_sweep_md6(bool c64, const BatchSweepArgs* a, int* per_cu, hipStream_t st) {
  return batch_sweep_impl<6, 5, 2>(c64, a, per_cu, st);
}

}  // namespace fd
