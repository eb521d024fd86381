// rq_lmm_adj64mc.hip -- FP64 instantiations of the LIBOR adjoint kernels for pseudo-random (Philox) points.
#include "rq_lmm_adj.h"

namespace rq {

hipError_t launch_lmm_adjoint_f64mc(const LmmArgs &a, int n_factors, int part, hipStream_t st)
{
    return launch_adj_prec<double, true>(a, n_factors, part, st);
}

}  // namespace rq
