// rq_batch_f32g.hip -- batch kernel instance (float, Greeks: true); one
// translation unit per instance so that they compile in parallel.
#include "rq_batch_kernel.h"

namespace rq {

hipError_t launch_batch_f32g(const BatchArgs &b, int grid, hipStream_t st) { return launch_batch_t<float, true>(b, grid, st); }
int batch_occ_f32g() { return batch_blocks_per_cu_t<float, true>(); }

}  // namespace rq
