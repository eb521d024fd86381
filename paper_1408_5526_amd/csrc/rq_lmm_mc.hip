// rq_lmm_mc.hip -- the LIBOR pricing kernel (rq_lmm.h) for pseudo-random
// (Philox) points.
#include "rq_lmm.h"

namespace rq {

hipError_t launch_lmm_mc(const LmmArgs &a, int n_factors, int fp32, hipStream_t st)
{
    return launch_lmm_gen_t<2>(a, n_factors, fp32, st);
}

}  // namespace rq
