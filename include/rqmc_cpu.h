/* rqmc_cpu.h -- the recursive Halton generator on the host CPU: the paper's
 * fastest CPU method (Algorithm 2, the recursive form of the radical
 * inverse; Table 1), built as a multi-core, SIMD baseline beside the GPU's
 * counter-based generator (rq_sequence in rqmc.h).  A separate library
 * (librqmc_cpu.so): no GPU entry point calls it and it calls none.
 *
 * Points, starts and permutations follow the conventions of rqmc.h: point i
 * of replication m in dimension j is phi_{p_j}((n_j^m + i) mod P_j) with
 * D_j digits, the correctly rounded FP64 value of R / P_j, the start n_j^m
 * drawn from SplitMix64 keyed by (seed, m_offset + m, j), the optional
 * permutation per base drawn by Fisher-Yates (RQ_PERM_RANDOM), leading
 * zeros unpermuted.  The results are bit-identical to rq_sequence's.
 *
 * Method.  Algorithm 2 advances the radical inverse of consecutive indices
 * by carrying in the digit expansion (only the digits that change are
 * touched).  Here it runs on exact integer partial sums, and the low k
 * digits (p^k >= 64) are split off: within a block of p^k consecutive
 * indices, R = R_high + T[a] with T[a] the (permuted) contribution of the
 * low digits a, so a block is one vector add and one vector divide per
 * point; Algorithm 2's carry runs once per block, on the high digits.
 * Threads take (replication, index tile) pairs; each tile starts from the
 * digit expansion of its first index (the counter-based start of
 * Algorithm 3) and continues recursively.
 *
 * Errors: the rq_status codes of rqmc.h (RQ_EINVAL for bad arguments,
 * RQ_ERANGE beyond the prime table or for N > P_j, RQ_EUNSUPPORTED for
 * flags other than RQ_START_ZERO and RQ_PERM_RANDOM).  Never aborts. */
#ifndef RQMC_CPU_H
#define RQMC_CPU_H

#include <stddef.h>
#include <stdint.h>

#include "rqmc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* cpu_sequence(s, N, M, seed): out host [M][N][s] FP64, as rq_sequence.
 *   threads   worker threads (0: all the process may use)
 * rq_cpu_last_error() says why a call failed. */
rq_status rq_cpu_sequence(int s, int64_t N, int M, uint64_t seed, int flags, int64_t m_offset,
                    double *out, int threads);

/* cpu_alg2_run: the exact integers R of `count` consecutive indices
 * n, n+1, ... (mod p^D) of one base by the blocked recursion above;
 * sigma: host [p] digit permutation or NULL (identity).  out host [count]
 * uint64.  A verification entry for wraps at P and small starts. */
rq_status rq_cpu_alg2_run(uint32_t p, const int32_t *sigma, uint64_t n, int64_t count, uint64_t *out);

/* Threads the library uses when threads = 0. */
int rq_cpu_max_threads(void);

const char *rq_cpu_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RQMC_CPU_H */
