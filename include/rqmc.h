/*
 * rqmc.h -- C ABI of the MI355X (gfx950) randomized quasi-Monte Carlo
 * pricing library.
 *
 * Method (Xu & Okten, "High Performance Financial Simulation Using
 * Randomized Quasi-Monte Carlo Methods"):
 *   - M independent randomisations of an s-dimensional Halton sequence
 *     (random-start, optionally randomly permuted: "Rasrap", section
 *     "Randomized-quasi Monte Carlo sequences", eqs. (1)-(3), Algorithm 3);
 *   - each point mapped through the inverse normal CDF;
 *   - LIBOR market model caplets (SDE of the caplet section, log-Euler,
 *     spot measure) or Caflisch mortgage-backed securities (MBS section);
 *   - estimates theta_N^m = (1/N) sum_i f(q_i^m), the grand average
 *     RQ_{M,N} = (1/M) sum_m theta_N^m, its sample standard deviation and
 *     standard error (Introduction).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Points.  Replication m (global index m_offset + m) in dimension j uses
 *   the j-th prime p_j (p_0 = 2), D_j = max{D : p_j^D <= 2^53} digits,
 *   P_j = p_j^{D_j}, and a start n_j^m uniform on [0, P_j) drawn from
 *   SplitMix64 (Steele, Lea & Flood 2014) keyed by (seed, m_global, j).
 *   Point i (0-based) is x_{i,j}^m = phi_{p_j}((n_j^m + i) mod P_j), the
 *   radical inverse with D_j digits, returned as the correctly rounded FP64
 *   value of the exact rational R/P_j.  Point 0 of a replication is
 *   phi(n), as in Algorithm 3, step 2.
 * Flags (bitwise or):
 *   RQ_START_ZERO   every start is 0: plain Halton (one replication
 *                   suffices; the others repeat it).
 *   RQ_PERM_RANDOM  one random digit permutation per base (eq. (3)),
 *                   shared by all replications; digits above the top
 *                   nonzero digit stay unpermuted.  Fisher-Yates from the
 *                   identity with SplitMix64 draws at counters
 *                   2^60 + (j 65536 + t) 64 + attempt.
 *   RQ_OUT_DIGITS   rq_sequence only: emit the exact integers R (uint64)
 *                   instead of the FP64 points.
 *   RQ_PERM_PER_REP the other reading of the random permutations: every
 *                   replication draws its own permutation of every base
 *                   (same Fisher-Yates, on the SplitMix64 stream seeded with
 *                   output 2^62 + m_global of the seed's stream); generated
 *                   on the device, M * (sum of the s primes) uint16 of
 *                   workspace.  Alternative to RQ_PERM_RANDOM; not in
 *                   batches.
 *   RQ_MC_PHILOX    pseudo-random points instead of Halton (the paper's
 *                   Philox comparison): coordinate j of point i of
 *                   replication m_global is word (j mod 4) of Philox4x64-10
 *                   (Salmon, Moraes, Dror & Shaw, SC'11) at counter
 *                   (j/4, i, 0, 0) under key (seed, m_global), mapped to
 *                   ((x >> 11) + 1/2) 2^-53.  Excludes the three flags above;
 *                   N is not limited by P_j.
 *   RQ_LMM_EULER    rq_price_caplets only: the plain Euler step of the
 *                   paper's discretised LIBOR SDE, L_n <- L_n + mu_n L_n delta
 *                   + L_n sqrt(delta) a_n . Z, instead of the log-Euler step.
 *                   Not with Greeks or RQ_PERM_RANDOM (RQ_EUNSUPPORTED), not
 *                   in batches.  The FP32 form steps log2 L by log2 of the
 *                   Euler factor, kept >= 2^-100 (an Euler step that would
 *                   make a rate negative is outside the FP32 form).
 * Normals.  Dimension j of a path maps to z = Phi^{-1}(x) (Wichura's
 *   AS241 in FP64; the FP32 form folds r = min(x, 1-x) in FP64 first).
 * Memory.  Every pointer named "device" is a device (HBM) address on the
 *   current HIP device; every pointer named "host" is host memory read
 *   during the call only.  The caller owns all buffers, including the
 *   workspace `ws` (device, 256-byte aligned, at least the size returned
 *   by the matching *_workspace function).  The library keeps no device
 *   state between calls: concurrent calls need distinct workspaces.
 * Streams.  `stream` is a hipStream_t (NULL = the legacy default stream).
 *   Work is enqueued asynchronously; results are valid once the stream
 *   has been synchronised.  The small per-call parameter tables are copied
 *   from host memory with hipMemcpyAsync, which HIP may perform
 *   synchronously for pageable memory.
 * Errors.  Arguments are validated before anything is enqueued; a non-OK
 *   status means nothing was launched unless it is RQ_EHIP.  The message of
 *   the last non-OK status of the calling thread is rq_last_error().  The
 *   library never aborts or exits.
 */
#ifndef RQMC_H
#define RQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RQ_OK = 0,
    RQ_EINVAL = 1,        /* null pointer, non-positive size, bad model value */
    RQ_ERANGE = 2,        /* size beyond what the method or library supports */
    RQ_ENOMEM = 3,        /* host allocation failed */
    RQ_EHIP = 4,          /* a HIP call failed; see rq_last_error() */
    RQ_EWORKSPACE = 5,    /* ws_bytes smaller than required, or ws misaligned */
    RQ_EUNSUPPORTED = 6   /* valid request outside this build's capabilities */
} rq_status;

typedef enum { RQ_FP64 = 0, RQ_FP32 = 1 } rq_precision;

enum {
    RQ_START_RANDOM = 0,
    RQ_START_ZERO = 1,
    RQ_PERM_RANDOM = 2,
    RQ_OUT_DIGITS = 4,
    RQ_MC_PHILOX = 8,
    RQ_LMM_EULER = 16,
    RQ_PERM_PER_REP = 32
};

/* Limits of this build. */
#define RQ_MAX_DIM 4096          /* s <= 4096 (primes up to 38873)          */
#define RQ_MAX_FWD 80            /* LIBOR forwards per model                */
#define RQ_MAX_FACTORS 3         /* factors d of the LIBOR model            */
#define RQ_MAX_MONTHS 4096       /* MBS term in months                      */
#define RQ_MAX_REPLICATION (1LL << 40)  /* m_offset + M                    */

/* LIBOR market model (caplet section).  Forwards L_1..L_n over
 * [T_n, T_n + delta] with T_n = n*delta; the simulation steps from one
 * tenor date to the next (step delta) under the spot measure with the
 * log-Euler form of the discretised SDE.  Constant vol vectors
 * a_n = sigma[n] * loadings[n-1][:].  Path dimension k*n_factors + f drives
 * factor f of step k (s = n_fwd * n_factors).
 *   L0        host [n_fwd+1]  L_0(0)..L_n(0) > 0; L_0(0) only enters the
 *                             numeraire (1 + delta L_0(0)).
 *   sigma     host [n_fwd+1]  sigma[n] >= 0 for n >= 1; sigma[0] unused.
 *   loadings  host [n_fwd][n_factors], row-major, each row of unit length
 *                             (|row| - 1| <= 1e-9).
 *   strike    host [n_fwd]    K_1..K_n; NaN = no caplet on that forward.
 * Outputs per path (n_out = n_fwd + 1): o = n-1 is the caplet on L_n,
 * delta (L_n(T_n) - K_n)^+ paid at T_{n+1}, divided by the spot numeraire
 * prod_{j=0..n} (1 + delta L_j(T_j)); o = n_fwd is the book (sum). */
typedef struct {
    int n_fwd;
    int n_factors;
    double delta;
    const double *L0;
    const double *sigma;
    const double *loadings;
    const double *strike;
} rq_lmm_model;

/* Caflisch MBS model (MBS section), unit principal, level payment
 * c = i0/(1-(1+i0)^{-months}); monthly rate i_k = K0 e^{sigma z_k} i_{k-1}
 * with K0 = exp(-sigma^2/2); prepayment w_k = K1 + K2 atan(K3 i_k + K4);
 * PV = sum_k u_k c r_k ((1-w_k) + w_k c_k).  One output per path (n_out =
 * 1); dimension k-1 drives month k (s = months). */
typedef struct {
    int months;
    double i0, sigma, K1, K2, K3, K4;
} rq_mbs_params;

/* Results, all device pointers owned by the caller, FP64:
 *   theta  [M][n_out]  per-replication estimates theta_N^m
 *   mean   [n_out]     RQ_{M,N}
 *   sd     [n_out]     sample standard deviation of theta (denominator
 *                      M-1; NaN when M == 1)
 *   se     [n_out]     sd / sqrt(M)
 * Any of mean/sd/se may be NULL to skip it; theta is required. */
typedef struct {
    double *theta;
    double *mean;
    double *sd;
    double *se;
} rq_result;

/* Workspace sizes in bytes for the call with the same arguments.
 * Return 0 when the arguments would be rejected (rq_last_error says why). */
size_t rq_sequence_workspace(int s, int64_t N, int M, int flags);
size_t rq_caplets_workspace(const rq_lmm_model *model, int64_t N, int M, int flags,
                            rq_precision prec, int with_greeks);
size_t rq_mbs_workspace(const rq_mbs_params *params, int64_t N, int M, int flags,
                        rq_precision prec, int with_greeks);

/* sequence(s, N, M, seed): the points themselves (Algorithm 3 for every
 * base, all replications in one launch).
 *   out  device [M][N][s] FP64 points, or uint64 integers R when
 *        RQ_OUT_DIGITS is set (x = R / P_j).
 * Limits: s <= RQ_MAX_DIM, N <= P_j for every j, m_offset + M <=
 * RQ_MAX_REPLICATION, M*N*s*8 bytes addressable. */
rq_status rq_sequence(int s, int64_t N, int M, uint64_t seed, int flags, int64_t m_offset,
                      void *out, void *ws, size_t ws_bytes, void *stream);

/* price_caplets(model, N, M): caplets and book of the LIBOR market model.
 *   out       results with n_out = n_fwd + 1
 *   grad      NULL, or pathwise Greeks of the book from the adjoint kernels,
 *             n_g = 2 n_fwd + 1 outputs per replication: [0, n_fwd)
 *             dbook/dL_n(0) for n = 1..n_fwd (strikes held fixed); [n_fwd]
 *             dbook/dL_0(0) (the spot rate, through the numeraire);
 *             [n_fwd + 1, 2 n_fwd + 1) dbook/dsigma_n for n = 1..n_fwd
 *             (the adjoint carries a sigma_n below 2^-60, zero included,
 *             as 2^-60: its state and prices are unchanged to rounding and
 *             its vega is the derivative there).
 *             theta holds the per-replication estimates, mean/sd/se their
 *             grand average and spread (as for prices).
 *   per_path  optional device [M][N][n_out] FP64: every path's discounted
 *             payoffs (a verification hook; NULL in production)
 *   prec      RQ_FP64: all path arithmetic in FP64.  RQ_FP32: forwards,
 *             drifts and normals in FP32 (the fixing value's 2^X too);
 *             digits, points, numeraire, payoffs and all reductions stay
 *             FP64.
 * With grad != NULL the prices come from the adjoint's forward pass (same
 * scheme; it keeps its state in log2 units, so FP64 prices agree with the
 * pricing kernel's to rounding).  The adjoint runs as two kernels over
 * chunks of 64-path blocks: the forward passes store every step's w and the
 * final states in the workspace (at most 64 GiB, sized by
 * rq_caplets_workspace), then the payoffs and reverse sweeps read them. */
rq_status rq_price_caplets(const rq_lmm_model *model, int64_t N, int M, uint64_t seed,
                           int64_t m_offset, int flags, rq_precision prec,
                           const rq_result *out, const rq_result *grad, double *per_path,
                           void *ws, size_t ws_bytes, void *stream);

/* The adjoint's store region (see rq_price_caplets): at most `bytes` per
 * chunk, counted in FP64 (at least one 64-path task per chunk); 0 restores
 * the default, 64 GiB.  Process-wide; it changes the workspace size that
 * rq_caplets_workspace reports for calls with Greeks and the number of
 * kernel launches, never the results (each task's arithmetic and partial
 * row are the same in any chunk).  Set it before sizing the workspace. */
rq_status rq_set_adjoint_store_limit(size_t bytes);

/* price_caplets_noalloc: rq_price_caplets without a caller workspace, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, hosts that forbid allocation during a run).  It
 * allocates nothing: the workspace is a fixed device array of
 * RQ_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library, one per GPU, held
 * until the process ends; its address on the current device is looked up
 * on the first call there.  Arguments, outputs and results are those of
 * rq_price_caplets with the same arguments (same kernels); with grad the
 * adjoint's store region takes whatever the tables and partial sums leave
 * of the array, in as many chunks as that needs.
 * Errors: as rq_price_caplets, plus RQ_ERANGE when the tables and partial
 * sums (M * ceil(N / 256) * (n_fwd + 1) doubles without Greeks,
 * M * ceil(N / 64) * (3 n_fwd + 2) with them), plus one stored 64-path
 * task with Greeks, do not fit the array; nothing is launched then.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other host threads) race and must be serialised by
 * the caller.  The array keeps the last call's contents; each call writes
 * every byte it later reads. */
#define RQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rq_status rq_price_caplets_noalloc(const rq_lmm_model *model, int64_t N, int M, uint64_t seed,
                                   int64_t m_offset, int flags, rq_precision prec,
                                   const rq_result *out, const rq_result *grad, double *per_path,
                                   void *stream);

/* price_mbs(params, N, M): present value of the mortgage pool.
 *   grad  NULL, or the pathwise total derivative dPV/di0 (one output per
 *         replication; rates scale with i0 and the payment c and the
 *         annuity factors c_k move with it), carried forward along each
 *         path as a tangent.
 *   prec  RQ_FP32 keeps the rate, prepayment and pool fraction in FP32 and
 *         the discount factor, cash-flow products and reductions in FP64. */
rq_status rq_price_mbs(const rq_mbs_params *params, int64_t N, int M, uint64_t seed,
                       int64_t m_offset, int flags, rq_precision prec, const rq_result *out,
                       const rq_result *grad, double *per_path, void *ws, size_t ws_bytes,
                       void *stream);

/* inv_normal: the inverse standard normal CDF used on every path
 * dimension, applied elementwise (a verification and utility entry).
 *   u     device [n] FP64 points in [0, 1)
 *   z     device [n], FP64 (RQ_FP64: Wichura's AS241) or FP32 (RQ_FP32: the
 *         FP32 form of the pricing kernels, relative error ~2e-7)
 * Values below 2^-64 in the fold min(u, 1-u) are clamped to it. */
rq_status rq_inv_normal(int64_t n, const double *u, void *z, rq_precision prec, void *stream);

/* ---- Batches of instruments ------------------------------------------------
 * price_batch: many instruments (LIBOR books and MBS pools of any supported
 * shape, each with its own N, M, seed, m_offset and flags) priced in ONE
 * persistent launch.  Work items are (instrument, replication, block of 64
 * paths); waves take them from an atomic queue, so small and large
 * instruments share the GPU without a launch per instrument.  Each item
 * writes its own partial sums, so the results do not depend on the tuning:
 * for every instrument they are bit-identical to those of any other chunk,
 * grid or order, and equal (to the rounding of the block sums) to what the
 * single-instrument entry points return for it.  (Not in the paper: a
 * serving form of the same method.) */
enum { RQ_INST_LMM = 0, RQ_INST_MBS = 1 };

typedef struct {
    int kind;                     /* RQ_INST_LMM or RQ_INST_MBS */
    const rq_lmm_model *lmm;      /* host, kind RQ_INST_LMM (NULL otherwise) */
    const rq_mbs_params *mbs;     /* host, kind RQ_INST_MBS (NULL otherwise) */
    int64_t N;                    /* points per replication */
    int M;                        /* replications */
    uint64_t seed;
    int64_t m_offset;
    int flags;                    /* RQ_START_ZERO / RQ_PERM_RANDOM */
} rq_instrument;

/* Launch shape of the batch (all fields 0 = automatic):
 *   chunk         work items taken per queue grab (0: from the item count)
 *   waves_per_cu  persistent blocks (one wave each) per compute unit (0: as
 *                 many as are resident, from the occupancy calculator)
 *   order         RQ_ORDER_COST: instruments in decreasing estimated cost
 *                 (longest first); RQ_ORDER_GIVEN: the caller's order */
enum { RQ_ORDER_COST = 0, RQ_ORDER_GIVEN = 1 };
typedef struct {
    int chunk;
    int waves_per_cu;
    int order;
} rq_tuning;

/* Workspace bytes for price_batch / autotune_batch with these arguments
 * (0 if they would be rejected). */
size_t rq_batch_workspace(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks);

/* price_batch(inst[n_inst]): per instrument k, the results of
 * rq_price_caplets / rq_price_mbs with the same arguments.
 *   inst      host [n_inst], 1 <= n_inst <= 65536
 *   tuning    NULL or a launch shape (see rq_tuning)
 *   outs      host [n_inst] rq_result (device buffers as for the single
 *             entry points: theta [M_k][n_out_k] required)
 *   grads     host [n_inst] or NULL; with with_greeks, the Greeks of each
 *             instrument (LIBOR: the 2 n_fwd + 1 of rq_price_caplets; MBS:
 *             dPV/di0)
 *   t_first, t_last  device [n_inst] uint64 or both NULL: the earliest start
 *             and latest end of instrument k's work items, in ticks of the
 *             device real-time counter (rq_realtime_hz)
 * No per-path output.  Errors name the offending instrument. */
rq_status rq_price_batch(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                         const rq_tuning *tuning, const rq_result *outs, const rq_result *grads,
                         uint64_t *t_first, uint64_t *t_last, void *ws, size_t ws_bytes, void *stream);

/* autotune_batch: the project's launch-shape autotuner for price_batch.
 * Candidates: the automatic shape (all zero) in both orders, and chunk
 * (work items per queue grab) in {1, 2, 4, 8, 16} x waves_per_cu in {the
 * resident count, half of it} x both orders (22 shapes).  After one untimed
 * run it times every candidate once; a batch of more than 2^28 paths is
 * screened on a probe of itself (each instrument's M divided by the power
 * of two that brings the probe near 2^28 paths, at least 1) and the three
 * fastest shapes there, with the automatic one in cost order, are timed on
 * the full batch (after one untimed full run), so the choice is not slower
 * than price_batch without a tuning beyond timing noise.  The fastest shape is returned in *best
 * (its full-batch time in ms in *best_ms unless NULL) and kept for this
 * batch's signature (precision, Greeks, and per instrument its kind,
 * shape, N, M and flags): rq_price_batch with tuning == NULL then uses it.
 * With the environment variable RQ_TUNING_CACHE naming a file, the choice
 * is also appended there and read back by later processes.  The outputs
 * hold the last run's results.  Synchronises the stream. */
rq_status rq_autotune_batch(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                            const rq_result *outs, const rq_result *grads, rq_tuning *best, double *best_ms,
                            void *ws, size_t ws_bytes, void *stream);

/* batch_tuning: the launch shape rq_price_batch uses for this batch when
 * called with tuning == NULL: the autotuner's choice for its signature
 * (*from_autotuner = 1), else all zero, i.e. automatic (*from_autotuner =
 * 0).  Host only; validates the list like rq_batch_workspace. */
rq_status rq_batch_tuning(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                          rq_tuning *out, int *from_autotuner);

/* Frequency (Hz) of the device real-time counter of the batch timestamps. */
rq_status rq_realtime_hz(double *hz);

/* lmm_pca_loadings: unit-row factor loadings for the LIBOR model, from the
 * n_factors principal components of the forward correlation
 * rho_ij = exp(-beta |T_i - T_j|), T_i = i delta (i = 1..n_fwd): with
 * eigenpairs (lambda_f, e_f) in descending order, row i is
 * (sqrt(lambda_f) e_f[i])_f rescaled to unit length, each e_f signed so
 * that e_f[0] > 0.  (A model input, not part of the paper's method: the
 * paper's caplet is one-factor; the multi-factor workloads use this
 * reduction.)  Host computation (Jacobi rotations), no device work.
 *   out   host [n_fwd][n_factors], row-major, written on RQ_OK
 * Errors: RQ_ERANGE for n_fwd outside [1, RQ_MAX_FWD] or n_factors outside
 * [1, min(RQ_MAX_FACTORS, n_fwd)]; RQ_EINVAL for delta <= 0, beta <= 0 or
 * out == NULL. */
rq_status rq_lmm_pca_loadings(int n_fwd, int n_factors, double delta, double beta, double *out);

/* Kernel timing instrumentation.  Between rq_timer_begin and rq_timer_end
 * every entry point records a pair of HIP events on its stream around its
 * main path kernels (the LIBOR or MBS pricing kernel, the two adjoint
 * kernels over all their chunks, or the sequence kernel), for the first
 * max_launches calls of the process; setup, copies
 * and reductions are outside the pair.  rq_timer_end waits for the recorded
 * events and returns the summed kernel time (ms) and the number of timed
 * launches.  Process-wide; not meant for concurrent use from several
 * threads. */
rq_status rq_timer_begin(int max_launches);
rq_status rq_timer_end(double *total_ms, int *n_launches);

/* After rq_timer_end: the summed time (ms) and launch count of one half of
 * the two-kernel adjoint behind rq_price_caplets with Greeks, part 1 the
 * forward kernel (forward passes, storing w and the final states), part 2
 * the reverse kernel (payoffs, reverse sweeps), over the same calls.  Both
 * are 0 when no such call was timed.
 * Errors: RQ_EINVAL for part outside {1, 2} or while the timer runs. */
rq_status rq_timer_part(int part, double *total_ms, int *n_launches);

/* Thread-local message describing the last non-OK status ("" if none). */
const char *rq_last_error(void);

/* Library version string. */
const char *rq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RQMC_H */
