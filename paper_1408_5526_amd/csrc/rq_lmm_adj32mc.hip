// rq_lmm_adj32mc.hip -- FP32 instantiations of the LIBOR adjoint kernels for pseudo-random (Philox) points.
#include "rq_lmm_adj.h"

namespace rq {

hipError_t launch_lmm_adjoint_f32mc(const LmmArgs &a, int n_factors, int part, hipStream_t st)
{
    return launch_adj_prec<float, true>(a, n_factors, part, st);
}

}  // namespace rq
