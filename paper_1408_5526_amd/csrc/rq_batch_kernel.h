// rq_batch_kernel.h -- one persistent launch over every work item of a
// batch of instruments (LIBOR books of 1..80 forwards and 1..3 factors, and
// MBS pools), in a fixed precision, with or without Greeks.
//
// Each block is one wave.  It takes `chunk` consecutive items at a time from
// an atomic queue (one vector atomic by lane 0) until the window [w0, w1)
// of items runs dry, so every wave reaches the exit.  With Greeks a window
// runs in two launches, as the single-call adjoint does: phase 1 the LIBOR
// items' forward halves (storing w and the final states in the item's slot
// of the window's store) and the whole MBS items, at four waves per SIMD in
// FP32; phase 2 the LIBOR items' payoffs and reverse sweeps, at two.  The instrument of an item is found by a
// binary search over item0 (wave-uniform scalar loads); its kind and factor
// count select the path code, so all branches are wave-uniform.  LIBOR
// items run the task of rq_lmm_adj.h at the full forward capacity (forwards
// beyond n_fwd are skipped by uniform branches); MBS items the task of
// rq_mbs.h.  Every item writes its own partial row, so results do not
// depend on which wave ran it: they are bit-identical for any chunk, grid
// or instrument order.  Per instrument, lane 0 records the earliest start
// and latest end (s_memrealtime ticks) of its items with atomic min/max.
#pragma once

#include "rq_lmm_adj.h"
#include "rq_mbs.h"

namespace rq {

// Waves per SIMD asked of the compiler: FP32 phase 1 (forward halves, the
// 24 lowest forwards' states in LDS, and MBS items) five (a few values
// spilled; 4% faster than four), FP32 phases 0 and 2 two (their payoff and
// adjoint state need the registers); FP64 one.
template <typename T, bool GREEKS, int PHASE>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? (PHASE == 1 ? 5 : 2) : 1)))
void batch_kernel(BatchArgs b)
{
    constexpr int part = PHASE == 1 ? kTaskFwd : PHASE == 2 ? kTaskRev : kTaskWhole;
    // vega rows (phase 2 in FP32 keeps VR of them in registers) and the drift
    // constants (every phase but FP64's phase 2, whose vega rows take the LDS)
    constexpr int VR = PHASE == 2 ? rev_reg_rows<kMaxFwd, T>() : 0;
    constexpr bool kC6 = !(PHASE == 2 && sizeof(T) == 8);
    __shared__ T vbar[kMaxFwd - VR][kWave];
    constexpr int XL = PHASE == 1 && sizeof(T) == 4 ? 24 : 0;   // forward states in LDS (phase 1)
    __shared__ T xl[XL > 0 ? XL : 1][kWave];
    __shared__ __align__(32) T c6s[kC6 ? kMaxFwd : 1];
    const int lane = threadIdx.x;
    const cptr<int64_t> item0 = as_const<int64_t>(b.item0);
    const cptr<BatchInst> inst = as_const<BatchInst>(b.inst);
#pragma unroll 1
    for (;;) {
        unsigned long long got = 0ull;
        if (lane == 0) got = atomicAdd(b.queue, (unsigned long long)b.chunk);
        // every lane is active here: the first active lane is lane 0
        const int64_t start = b.w0 + (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(got >> 32)) << 32) |
                                               (uint64_t)__builtin_amdgcn_readfirstlane((unsigned)got));
        if (start >= b.w1) break;
        const int64_t end = start + b.chunk < b.w1 ? start + b.chunk : b.w1;
#pragma unroll 1
        for (int64_t it = start; it < end; ++it) {
            int lo = 0, hi = b.n_inst;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (item0[mid] <= it) lo = mid;
                else hi = mid;
            }
            const int64_t local = it - item0[lo];
            const bool lmm = inst[lo].kind == kInstLmm;
            if (PHASE == 2 && !lmm) continue;   // MBS items are done in phase 1
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            if (lmm) {
                const LmmArgs a = load_uniform<LmmArgs>(&b.inst[lo].lmm);
                const int m = (int)(local / a.n_blk);
                const int blk = (int)(local - (int64_t)m * a.n_blk);
                T *slot = GREEKS ? (T *)b.store + (it - b.w0) * (int64_t)kBatchItemElems : nullptr;
                T *wt = GREEKS ? slot + lane : nullptr;
                T *xs = GREEKS ? slot + kMaxFwd * 3 * kWave + lane : nullptr;
                const int sel = inst[lo].n_factors * 2 + (a.g.mc ? 1 : 0);
                T *c6p = kC6 ? &c6s[0] : nullptr;
                switch (sel) {
                case 2: lmm_task<kMaxFwd, 1, T, GREEKS, false, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                case 3: lmm_task<kMaxFwd, 1, T, GREEKS, true, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                case 4: lmm_task<kMaxFwd, 2, T, GREEKS, false, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                case 5: lmm_task<kMaxFwd, 2, T, GREEKS, true, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                case 7: lmm_task<kMaxFwd, 3, T, GREEKS, true, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                default: lmm_task<kMaxFwd, 3, T, GREEKS, false, part, VR, XL>(a, m, blk, local, wt, vbar, xs, c6p, xl); break;
                }
            } else if (PHASE != 2) {
                const MbsArgs a = load_uniform<MbsArgs>(&b.inst[lo].mbs);
                const int m = (int)(local / a.n_blk);
                const int blk = (int)(local - (int64_t)m * a.n_blk);
                mbs_task<T, GREEKS>(a, m, blk, local);
            }
            const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
            const int slot = inst[lo].slot;
            if (lane == 0 && b.t_first) {
                atomicMin(b.t_first + slot, (unsigned long long)t0);
                atomicMax(b.t_last + slot, (unsigned long long)t1);
            }
        }
    }
}

template <typename T, bool GREEKS, int PHASE>
static hipError_t launch_batch_t(const BatchArgs &b, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((batch_kernel<T, GREEKS, PHASE>), dim3((unsigned)grid), dim3(kWave), 0, st, b);
    return hipGetLastError();
}

template <typename T, bool GREEKS, int PHASE>
static int batch_blocks_per_cu_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<T, GREEKS, PHASE>, kWave, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_batch_f32p(const BatchArgs &b, int grid, hipStream_t st);
hipError_t launch_batch_f32g(const BatchArgs &b, int grid, int phase, hipStream_t st);
hipError_t launch_batch_f64p(const BatchArgs &b, int grid, hipStream_t st);
hipError_t launch_batch_f64g(const BatchArgs &b, int grid, int phase, hipStream_t st);
int batch_occ_f32p();
int batch_occ_f32g(int phase);
int batch_occ_f64p();
int batch_occ_f64g(int phase);

}  // namespace rq
