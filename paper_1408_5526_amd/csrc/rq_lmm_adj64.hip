// rq_lmm_adj64.hip -- FP64 instantiations of the LIBOR adjoint kernels and the dispatch.
#include "rq_lmm_adj.h"

namespace rq {

hipError_t launch_lmm_adjoint_f64(const LmmArgs &a, int n_factors, int part, hipStream_t st)
{
    return launch_adj_prec<double, false>(a, n_factors, part, st);
}

hipError_t launch_lmm_adjoint(const LmmArgs &a, int n_factors, int fp32, int part, hipStream_t st)
{
    if (a.g.mc)
        return fp32 ? launch_lmm_adjoint_f32mc(a, n_factors, part, st)
                    : launch_lmm_adjoint_f64mc(a, n_factors, part, st);
    return fp32 ? launch_lmm_adjoint_f32(a, n_factors, part, st) : launch_lmm_adjoint_f64(a, n_factors, part, st);
}

}  // namespace rq
