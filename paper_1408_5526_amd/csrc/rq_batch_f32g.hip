// rq_batch_f32g.hip -- batch kernel instances (float, Greeks: the forward
// phase and the reverse phase); one translation unit per precision so that
// they compile in parallel.
#include "rq_batch_kernel.h"

namespace rq {

hipError_t launch_batch_f32g(const BatchArgs &b, int grid, int phase, hipStream_t st)
{
    return phase == 1 ? launch_batch_t<float, true, 1>(b, grid, st) : launch_batch_t<float, true, 2>(b, grid, st);
}
int batch_occ_f32g(int phase)
{
    return phase == 1 ? batch_blocks_per_cu_t<float, true, 1>() : batch_blocks_per_cu_t<float, true, 2>();
}

}  // namespace rq
