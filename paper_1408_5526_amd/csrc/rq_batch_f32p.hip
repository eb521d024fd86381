// rq_batch_f32p.hip -- batch kernel instance (float, no Greeks); one
// translation unit per instance so that they compile in parallel.
#include "rq_batch_kernel.h"

namespace rq {

hipError_t launch_batch_f32p(const BatchArgs &b, int grid, hipStream_t st) { return launch_batch_t<float, false, 0>(b, grid, st); }
int batch_occ_f32p() { return batch_blocks_per_cu_t<float, false, 0>(); }

}  // namespace rq
