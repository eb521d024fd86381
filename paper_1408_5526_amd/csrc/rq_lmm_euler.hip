// rq_lmm_euler.hip -- the LIBOR pricing kernel (rq_lmm.h) with the plain
// Euler step, for Halton and for pseudo-random (Philox) points.
#include "rq_lmm.h"

namespace rq {

hipError_t launch_lmm_euler(const LmmArgs &a, int n_factors, int fp32, hipStream_t st)
{
    return a.g.mc ? launch_lmm_gen_t<2, true>(a, n_factors, fp32, st) : launch_lmm_gen_t<0, true>(a, n_factors, fp32, st);
}

}  // namespace rq
