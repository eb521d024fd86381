// rq_lmm.hip -- the LIBOR pricing kernel (rq_lmm.h) for Halton points, and
// the launch dispatch over point generators.
#include "rq_lmm.h"

namespace rq {

hipError_t launch_lmm(const LmmArgs &a, int n_factors, int fp32, hipStream_t st)
{
    if (a.euler) return launch_lmm_euler(a, n_factors, fp32, st);
    if (a.g.mc) return launch_lmm_mc(a, n_factors, fp32, st);
    return a.g.perm_on ? launch_lmm_gen_t<1>(a, n_factors, fp32, st) : launch_lmm_gen_t<0>(a, n_factors, fp32, st);
}

}  // namespace rq
