// rq_lmm_adj32.hip -- FP32 instantiations of the LIBOR adjoint kernels (forward and reverse halves).
#include "rq_lmm_adj.h"

namespace rq {

hipError_t launch_lmm_adjoint_f32(const LmmArgs &a, int n_factors, int part, hipStream_t st)
{
    return launch_adj_prec<float, false>(a, n_factors, part, st);
}

}  // namespace rq
