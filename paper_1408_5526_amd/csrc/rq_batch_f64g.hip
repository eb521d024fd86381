// rq_batch_f64g.hip -- batch kernel instance (double, Greeks: true); one
// translation unit per instance so that they compile in parallel.
#include "rq_batch_kernel.h"

namespace rq {

hipError_t launch_batch_f64g(const BatchArgs &b, int grid, hipStream_t st) { return launch_batch_t<double, true>(b, grid, st); }
int batch_occ_f64g() { return batch_blocks_per_cu_t<double, true>(); }

}  // namespace rq
