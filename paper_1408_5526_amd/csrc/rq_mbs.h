// rq_mbs.h -- Caflisch mortgage-backed-security path, one path per lane.
//
// Model (MBS section), months k = 1..K, z_k = Phi^{-1}(x_{k-1}):
//   u_k = u_{k-1} / (1 + i_{k-1})            discount factor      (FP64,
//                                            Newton reciprocal)
//   i_k = K0 exp(sigma z_k) i_{k-1}          monthly rate, K0 = exp(-sigma^2/2)
//   w_k = K1 + K2 atan(K3 i_k + K4)          prepayment fraction
//   PV += u_k c r_k ((1 - w_k) + w_k c_k)    cash flow m_k, discounted (FP64)
//   r_{k+1} = r_k (1 - w_k)                  surviving fraction
// The FP32 form keeps i, w, r and the normal in FP32; u, the cash-flow
// product, PV and every reduction stay FP64.
//
// The tangent (GRAD) carries d/di0 of every path quantity alongside it:
// rates scale with i0 (di_k = i_k / i0), so di follows the same recursion;
//   du_k = (du_{k-1} - u_k di_{k-1}) / (1 + i_{k-1}),
//   dw_k = K2 K3 di_k / (1 + (K3 i_k + K4)^2),
//   dm_k = dc r A + c dr A + c r (dw (c_k - 1) + w dc_k),  A = (1-w) + w c_k,
//   dr_{k+1} = dr (1 - w) - r dw,
// with dc and dc_k the (host-computed) derivatives of the level payment and
// the annuity factors.  dPV/di0 is summed exactly like PV.
#pragma once

#include "rq_device.h"

namespace rq {

// PV (and dPV/di0 with GRAD) of path i of replication m: Halton point at
// index t of the segment whose start entries are st, or (MC) Philox point i.
template <typename T, bool PERM, bool GRAD>
__device__ __forceinline__ void mbs_path(const MbsArgs &a, const StartEnt *__restrict__ st, uint32_t t,
                                         int m, int64_t i, double &pv_out, double &dpv_out)
{
    McPath mc;
    const cptr<double> ck = as_const<double>(a.ck);
    const cptr<double> dck = ck + (a.months + 1);
    const T K0 = (T)a.K0, sig = (T)a.sig, K1 = (T)a.K1, K2 = (T)a.K2, K3 = (T)a.K3, K4 = (T)a.K4;
    double u = 1.0, pv = 0.0;
    T ir = (T)a.i0;
    T r = T(1);
    double du = 0.0, dpv = 0.0;
    T di = T(1), dr = T(0);
#pragma unroll 1
    for (int k = 1; k <= a.months; ++k) {
        const int j = k - 1;
        double x;
        if (a.g.mc) {
            x = mc.point(a.g.seed, (uint64_t)(a.g.m_offset + m), (uint64_t)i, j);
        } else {
            const PointCtx c = load_base_uniform(a.g.base, j);
            x = radinv_x<PERM, sizeof(T) == 8>(c, load_uniform<StartEnt>(st + j), t,
                                               a.g.perm + (size_t)m * a.g.perm_stride);
        }
        const T z = inv_normal(x, T(0));
        // 1 / (1 + i) by the Newton reciprocal (within an ulp or two of the
        // quotient): one reciprocal serves u and du; a rate beyond 2^1000
        // (an overflowing FP32 rate included) discounts to 0, as a division
        // would
        const double onei = 1.0 + (double)ir;
        const double ri = onei < 0x1p1000 ? recip64(onei) : 0.0;
        u = u * ri;
        if (GRAD) du = (du - u * (double)di) * ri;
        const T f = K0 * fexp(sig * z);
        ir = f * ir;
        const T arg = K3 * ir + K4;
        const T w = K1 + K2 * fatan(arg);
        const double wd = (double)w;
        const double A = (1.0 - wd) + wd * ck[k];
        pv += u * a.c * (double)r * A;
        if (GRAD) {
            di = f * di;
            const T dw = K2 * K3 * di / (T(1) + arg * arg);
            const double dA = (double)dw * (ck[k] - 1.0) + wd * dck[k];
            const double dm = a.dc * (double)r * A + a.c * (double)dr * A + a.c * (double)r * dA;
            dpv += du * (a.c * (double)r * A) + u * dm;
            dr = dr * (T(1) - w) - r * dw;
        }
        r = r * (T(1) - w);
    }
    pv_out = pv;
    dpv_out = dpv;
}

// One task of the batch kernel: the 64 paths of block `blk` (64-path blocks)
// of replication m; one partial row of n_part sums at task.
template <typename T, bool GRAD>
__device__ __forceinline__ void mbs_task(const MbsArgs &a, int m, int blk, int64_t task)
{
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blk * kWave + lane;
    const bool active = i < a.g.N;
    const int seg = (int)(((int64_t)blk * kWave) >> a.g.log2S);
    const uint32_t t = (uint32_t)(i - ((int64_t)seg << a.g.log2S));
    const StartEnt *__restrict__ st = a.g.starts + ((size_t)m * a.g.n_seg + seg) * a.g.s;
    double pv, dpv;
    if (a.g.perm_on) mbs_path<T, true, GRAD>(a, st, t, m, i, pv, dpv);
    else mbs_path<T, false, GRAD>(a, st, t, m, i, pv, dpv);
    pv = active ? pv : 0.0;
    dpv = active ? dpv : 0.0;
    if (a.per_path && active) a.per_path[(size_t)m * (size_t)a.g.N + (size_t)i] = pv;
    const double w0 = wave_sum(pv);
    const double w1 = GRAD ? wave_sum(dpv) : 0.0;
    if (lane == 0) {
        a.partial[(size_t)task * a.n_part] = w0;
        if (GRAD) a.partial[(size_t)task * a.n_part + 1] = w1;
    }
}

}  // namespace rq
