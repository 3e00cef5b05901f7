// Step kernels of the BF16 population store (see lbm_step.h).
#include "lbm_step.h"

namespace lbmwf {

template hipError_t launch_step_store<StoreBF16>(bool odd, int bc, const StepArgs& a, hipStream_t s);
template hipError_t launch_batch_store<StoreBF16>(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst,
                                              int ntiles, hipStream_t s);

}  // namespace lbmwf
