// rq_reduce.h -- reductions over path blocks (theta) and over replications
// (RQ, sd, SE), each a fixed-order Neumaier sum, so results are
// bit-reproducible run to run.
#pragma once

#include "rq_device.h"

namespace rq {

// theta[m][o] for outputs o = first, first + step, ... of replication m.
__device__ __forceinline__ void reduce_one(const ReduceArgs &a, int m, int first, int step)
{
    for (int o = first; o < a.n_out; o += step) {
        Acc acc{0.0, 0.0};
        const double *p = a.partial + (size_t)m * a.n_blk * a.stride + a.off + o;
        for (int b = 0; b < a.n_blk; ++b) acc_add(acc, p[(size_t)b * a.stride]);
        a.theta[(size_t)m * a.n_out + o] = (acc.s + acc.c) / a.Nd;
    }
}

// mean, sd (M-1) and SE of output o over the replications.
__device__ __forceinline__ void finalize_one(const FinalizeArgs &a, int o)
{
    Acc s{0.0, 0.0};
    for (int m = 0; m < a.M; ++m) acc_add(s, a.theta[(size_t)m * a.n_out + o]);
    const double mu = (s.s + s.c) / (double)a.M;
    Acc q{0.0, 0.0};
    for (int m = 0; m < a.M; ++m) {
        const double d = a.theta[(size_t)m * a.n_out + o] - mu;
        acc_add(q, __dmul_rn(d, d));
    }
    const double sd = a.M > 1 ? sqrt((q.s + q.c) / (double)(a.M - 1)) : __builtin_nan("");
    if (a.mean) a.mean[o] = mu;
    if (a.sd) a.sd[o] = sd;
    if (a.se) a.se[o] = a.M > 1 ? sd / sqrt((double)a.M) : __builtin_nan("");
}

}  // namespace rq
