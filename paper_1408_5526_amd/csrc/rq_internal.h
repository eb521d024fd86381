// rq_internal.h -- structures shared by the host side of the library and
// its kernels.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rq {

// Per-dimension constants (one entry per Halton base j).  The point index
// range of a replication is cut in segments of S consecutive indices
// (S a power of two); within a segment a lane only expands the low
// L = min{L : p^L >= S} base-p digits of its index, the rest comes from a
// per-(replication, segment, dimension) table built by the setup kernel.
struct alignas(16) BaseEnt {
    double pd;        // p as FP64
    double invp_up;   // 1/p rounded toward +inf (exact floor(v/p) for v < 2^31)
    double pDLd;      // p^{D-L} as FP64 (exact)
    double Pd;        // P = p^D as FP64 (exact, <= 2^53)
    uint64_t P;       // p^D
    uint64_t pDL;     // p^{D-L}
    uint32_t p;       // the prime
    uint32_t D;       // digits carried
    uint32_t L;       // low digits expanded per lane
    uint32_t pL;      // p^L (< 2^30)
    uint32_t perm_off;// offset of this base's permutation in the u16 table
    uint32_t pad0;
    double invP;      // RN(1/P)
};
static_assert(sizeof(BaseEnt) == 80, "BaseEnt layout");

// Start decomposition of (replication, segment, dimension): index
// base = (n + seg*S) mod P = hi * p^L + nlo.  A lane with local offset t
// forms v = nlo + t (< 2 p^L), carry c = [v >= p^L]; its point is
// R = rev_L(v - c p^L) * p^{D-L} + Rhi[c] with Rhi[c] the D-L digit
// reversal of (hi + c) mod p^{D-L}.
struct alignas(16) StartEnt {
    double rhi0;      // Rhi[0] (exact integer < 2^53)
    double drhi;      // Rhi[1] - Rhi[0] (exact)
    uint32_t nlo;
    uint32_t hz;      // bit c set: (hi + c) mod p^{D-L} == 0 (leading-zero rule)
    uint32_t pad0, pad1;
};
static_assert(sizeof(StartEnt) == 32, "StartEnt layout");

constexpr int kBlock = 256;          // threads per pricing block (4 waves)
constexpr int kWave = 64;

// Flags (mirror of the public ones).
constexpr int kStartZero = 1;
constexpr int kPermRandom = 2;
constexpr int kOutDigits = 4;
constexpr int kMcPhilox = 8;
constexpr int kLmmEuler = 16;
constexpr int kPermPerRep = 32;

// Arguments common to every kernel that generates points.
struct SeqGeom {
    const BaseEnt *base;     // [s]
    const StartEnt *starts;  // [M][n_seg][s]
    const uint16_t *perm;    // packed permutations or nullptr
    int64_t perm_stride;     // elements between replications' tables (0: shared by all)
    int s;
    int M;
    int n_seg;
    int perm_on;
    int mc;                  // 1: Philox4x64-10 pseudo-random points instead of Halton
    uint64_t seed;           // MC key word 0
    int64_t m_offset;        // MC key word 1 = m_offset + m
    int64_t N;
    int64_t S;               // segment length (power of two)
    int log2S;
};

struct SetupArgs {
    BaseEnt *base_dev;       // read
    StartEnt *starts;        // written [M][n_seg][s]
    const uint16_t *perm;
    int64_t perm_stride;     // as in SeqGeom
    uint64_t seed;
    int64_t m_offset;
    int s, M, n_seg;
    int64_t S;
    int flags;
};

// LIBOR model tables, per forward n = 1..n_fwd (row n-1), kFwdRow doubles:
//   [0..2] a_n            vol vector
//   [3..5] delta a_n
//   [6]    c_n = -delta |a_n|^2 / 2
//   [7]    L_n(0)
//   [8]    K_n (0 when there is no caplet)
//   [9]    1 if forward n carries a caplet, else 0
//   [10]   1 / (L_n(0) ln 2)
//   [11]   1 / sigma~_n, sigma~_n = max(sigma_n, 2^-60) (the adjoint's vega scale)
// followed by the FP32 rows, kRow32 floats per forward, log2 units:
//   [0..2] log2(e) a_n
//   [3..5] delta a_n
//   [6]    log2(e) c_n
//   [7]    kappa_n = 1 / (delta L_n(0))  (the drift factor is 1 / (1 + kappa_n 2^{-X_n}))
// Every table has kMaxFwd rows; the rows beyond n_fwd are zero.
constexpr int kFwdRow = 12;
constexpr int kRow32 = 8;
constexpr int kGrp = 4;   // forwards per branch-free group of the LIBOR kernel

// Adjoint table, kAdjRow entries per forward in the kernel's precision, the
// FP32 row's layout with a_n = sigma~_n b_n (b_n the unit loading row):
//   [0..2] log2(e) a_n     [3..5] delta a_n
//   [6]    log2(e) c_n = -log2(e) delta |a_n|^2 / 2
//   [7]    1 / (delta L_n(0))
// A zero sigma_n enters as sigma~_n = 2^-60: the increments it adds to the
// state and to w lie far below their rounding, and the vega it gives is the
// derivative at 2^-60, equal to the one at 0 up to O(2^-60).
constexpr int kAdjRow = 8;
constexpr double kMinSigma = 0x1p-60;

struct LmmArgs {
    SeqGeom g;
    const double *fwd;       // [n_fwd][kFwdRow]
    const float *fwd32;      // [n_fwd][kRow32]
    const void *adj;         // [n_fwd][kAdjRow] (FP32 or FP64) or nullptr
    void *wtop;              // adjoint: step-final w, kernel precision: batch [n_slots][n_fwd][d][64],
                             // single call [chunk][n_fwd][d][64]
    int n_slots;             // batch adjoint: blocks of the persistent grid
    void *xs;                // single-call adjoint: [chunk][NFC][64] final states (log2 units)
    int64_t task0;           // single-call adjoint: first task (m n_blk + blk) of this launch
    int64_t chunk;           // single-call adjoint: tasks of this launch
    double *partial_g;       // [M][n_blk][n_g] Greek partial sums or nullptr
    int n_g;                 // 2 n_fwd + 1
    double *partial;         // [M][n_blk][n_out]
    double *per_path;        // [M][N][n_out] or nullptr
    int n_fwd;
    int n_out;
    int n_blk;               // blocks per replication
    double delta, sqrt_delta, num0;   // num0 = 1 + delta L_0(0)
    int euler;               // pricing kernel only: plain Euler step instead of log-Euler
};

struct MbsArgs {
    SeqGeom g;
    const double *ck;        // [months+1]: c_k, then [months+1]: dc_k/di0
    double *partial;         // [M][n_blk][n_part] (PV, then dPV/di0 with Greeks)
    double *per_path;        // [M][N] or nullptr
    int months;
    int n_blk;
    int n_part;              // 1, or 2 with the tangent
    double i0, sig, K0, K1, K2, K3, K4, c, dc;   // dc = dc/di0
};

struct ReduceArgs {
    const double *partial;   // [M][n_blk][stride], outputs at [off, off + n_out)
    double *theta;           // [M][n_out]
    int M, n_blk, n_out;
    int stride, off;
    double Nd;               // N as FP64
};

struct FinalizeArgs {
    const double *theta;     // [M][n_out]
    double *mean, *sd, *se;  // [n_out] (any may be null)
    int M, n_out;
};

// Per-replication digit permutations: table[m][perm_off_j + a], one
// Fisher-Yates per (replication, base).
struct PermArgs {
    uint16_t *table;
    const BaseEnt *base;
    uint64_t seed;
    int64_t m_offset;
    int64_t stride;          // sum of the s primes
    int s, M;
};

// Launchers (each returns the hipError_t of its launch).
hipError_t launch_setup(const SetupArgs &a, hipStream_t st);
hipError_t launch_perm(const PermArgs &a, hipStream_t st);
hipError_t launch_sequence(const SeqGeom &g, int flags, void *out, hipStream_t st);
hipError_t launch_lmm(const LmmArgs &a, int n_factors, int fp32, hipStream_t st);
// part 1: forward halves of tasks [task0, task0 + chunk), storing w and the
// final states; part 2: their payoffs and reverse sweeps
hipError_t launch_lmm_adjoint(const LmmArgs &a, int n_factors, int fp32, int part, hipStream_t st);
constexpr int kAdjBlockHost = 64;    // paths per block (task) of the adjoint kernels (one wave)
constexpr int kAdjSlots = 2048;      // batch adjoint grid: 256 CUs x 8 resident waves
// Single-call adjoint: bytes of stored w and final states per launch pair,
// at most (the tasks are processed in chunks that fit), FP64-counted; the
// batch's window store likewise.  64 GiB of the 288 GB of HBM: fewer
// windows, so fewer phase boundaries where the persistent batch grid drains
// (-2.4% batch time against 16 GiB)
constexpr size_t kAdjStoreBytes = (size_t)64 << 30;
hipError_t launch_mbs(const MbsArgs &a, int fp32, hipStream_t st);   // n_part == 2: tangent
hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st);
hipError_t launch_inv_normal(int64_t n, const double *u, void *z, int fp32, hipStream_t st);

// Largest forward count of the compiled LIBOR kernels.
constexpr int kMaxFwd = 80;

// ---- batch of instruments (one persistent launch over all work items) ----
// A work item is one 64-path block of one replication of one instrument.
// Items are numbered instrument by instrument in the execution order;
// instrument k owns [item0[k], item0[k+1]).
constexpr int kInstLmm = 0;
constexpr int kInstMbs = 1;
// Greeks batch: per LIBOR work item, the stored step-final w and final
// states of its forward half ([kMaxFwd][3][64] then [kMaxFwd][64]), elements
constexpr int kBatchItemElems = kMaxFwd * 3 * kWave + kMaxFwd * kWave;

struct BatchInst {
    LmmArgs lmm;             // kind LMM: n_blk counts 64-path blocks
    MbsArgs mbs;             // kind MBS: n_blk counts 64-path blocks
    int kind;
    int n_factors;           // LMM
    int slot;                // index of the instrument in the caller's list
    int pad0;
};

struct BatchArgs {
    const BatchInst *inst;   // [n_inst], execution order
    const int64_t *item0;    // [n_inst + 1]
    int n_inst;
    int chunk;               // items taken per queue grab
    int64_t n_items;
    unsigned long long *queue;                  // next free item (zeroed by batch_init)
    unsigned long long *t_first, *t_last;       // [n_caller] s_memrealtime ticks, or nullptr
    int n_caller;
    void *store;             // Greeks: [w1 - w0][kBatchItemElems] kernel precision
    int64_t w0, w1;          // the items of this launch (a window of the execution order)
};

// Batched setup / reductions: argument arrays with an exclusive prefix of
// the per-entry unit counts (threads, blocks or outputs), prefix[n] = total.
struct BatchSetup {
    const SetupArgs *args;
    const int64_t *prefix;   // units = M * n_seg * s
    int n;
};
struct BatchReduce {
    const ReduceArgs *args;
    const int64_t *prefix;   // units = M (one block each)
    int n;
};
struct BatchFinalize {
    const FinalizeArgs *args;
    const int64_t *prefix;   // units = n_out (one thread each; args with no output pointer count 0)
    int n;
};

hipError_t launch_batch_init(unsigned long long *queue, unsigned long long *t_first, unsigned long long *t_last,
                             int n_caller, hipStream_t st);
hipError_t launch_batch_setup(const BatchSetup &b, int64_t total, hipStream_t st);
hipError_t launch_batch_reduce(const BatchReduce &b, int64_t blocks, hipStream_t st);
hipError_t launch_batch_finalize(const BatchFinalize &b, int64_t total, hipStream_t st);
// phase 0: whole items without Greeks; with Greeks phase 1 runs the LIBOR
// items' forward halves and the MBS items, phase 2 the LIBOR reverse halves
hipError_t launch_batch(const BatchArgs &b, int grid, int fp32, int greeks, int phase, hipStream_t st);
// Resident blocks per CU of the batch kernel for (fp32, greeks), from the
// occupancy calculator.
int batch_blocks_per_cu(int fp32, int greeks, int phase);

}  // namespace rq
