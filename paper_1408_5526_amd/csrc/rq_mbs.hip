// rq_mbs.hip -- Caflisch mortgage-backed-security pricing, one path per lane.
//
// Model (MBS section), months k = 1..K, z_k = Phi^{-1}(x_{k-1}):
//   u_k = u_{k-1} / (1 + i_{k-1})            discount factor      (FP64)
//   i_k = K0 exp(sigma z_k) i_{k-1}          monthly rate, K0 = exp(-sigma^2/2)
//   w_k = K1 + K2 atan(K3 i_k + K4)          prepayment fraction
//   PV += u_k c r_k ((1 - w_k) + w_k c_k)    cash flow m_k, discounted (FP64)
//   r_{k+1} = r_k (1 - w_k)                  surviving fraction
// The FP32 form keeps i, w, r and the normal in FP32; u, the cash-flow
// product, PV and every reduction stay FP64.
#include "rq_device.h"

namespace rq {

// The tangent (GRAD) carries d/di0 of every path quantity alongside it:
// rates scale with i0 (di_k = i_k / i0), so di follows the same recursion;
//   du_k = (du_{k-1} - u_k di_{k-1}) / (1 + i_{k-1}),
//   dw_k = K2 K3 di_k / (1 + (K3 i_k + K4)^2),
//   dm_k = dc r A + c dr A + c r (dw (c_k - 1) + w dc_k),  A = (1-w) + w c_k,
//   dr_{k+1} = dr (1 - w) - r dw,
// with dc and dc_k the (host-computed) derivatives of the level payment and
// the annuity factors.  dPV/di0 is summed exactly like PV.
template <typename T, bool PERM, bool GRAD>
__global__ __launch_bounds__(kBlock) void mbs_kernel(MbsArgs a)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int m = blockIdx.x / a.n_blk;
    const int blk = blockIdx.x - m * a.n_blk;
    const int64_t i = (int64_t)blk * kBlock + tid;
    const bool active = i < a.g.N;
    const int seg = (int)(((int64_t)blk * kBlock) >> a.g.log2S);
    const uint32_t t = (uint32_t)(i - ((int64_t)seg << a.g.log2S));
    const StartEnt *__restrict__ st = a.g.starts + ((size_t)m * a.g.n_seg + seg) * a.g.s;
    const double *__restrict__ ck = a.ck;
    const double *__restrict__ dck = a.ck + (a.months + 1);

    __shared__ double red[kBlock / kWave][2];

    const T K0 = (T)a.K0, sig = (T)a.sig, K1 = (T)a.K1, K2 = (T)a.K2, K3 = (T)a.K3, K4 = (T)a.K4;
    double u = 1.0, pv = 0.0;
    T ir = (T)a.i0;
    T r = T(1);
    double du = 0.0, dpv = 0.0;
    T di = T(1), dr = T(0);
#pragma unroll 1
    for (int k = 1; k <= a.months; ++k) {
        const int j = k - 1;
        const PointCtx c = load_base(a.g.base, j);
        const double x = radinv_x<PERM, sizeof(T) == 8>(c, st + j, t, a.g.perm);
        const T z = inv_normal(x, T(0));
        const double onei = 1.0 + (double)ir;
        u = u / onei;
        if (GRAD) du = (du - u * (double)di) / onei;
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
    pv = active ? pv : 0.0;
    dpv = active ? dpv : 0.0;
    if (a.per_path && active) a.per_path[(size_t)m * (size_t)a.g.N + (size_t)i] = pv;
    const double w0 = wave_sum(pv);
    const double w1 = GRAD ? wave_sum(dpv) : 0.0;
    if (lane == 0) {
        red[wave][0] = w0;
        red[wave][1] = w1;
    }
    __syncthreads();
    if (tid < a.n_part) {
        double s = red[0][tid];
        s += red[1][tid];
        s += red[2][tid];
        s += red[3][tid];
        a.partial[((size_t)m * a.n_blk + blk) * a.n_part + tid] = s;
    }
}

template <typename T, bool GRAD>
static void launch_mbs_t(const MbsArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    if (a.g.perm_on) hipLaunchKernelGGL((mbs_kernel<T, true, GRAD>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((mbs_kernel<T, false, GRAD>), grid, block, 0, st, a);
}

hipError_t launch_mbs(const MbsArgs &a, int fp32, hipStream_t st)
{
    const int64_t blocks = (int64_t)a.n_blk * a.g.M;
    const dim3 grid((unsigned)blocks), block(kBlock);
    const bool grad = a.n_part == 2;
    if (fp32) {
        if (grad) launch_mbs_t<float, true>(a, grid, block, st);
        else launch_mbs_t<float, false>(a, grid, block, st);
    } else {
        if (grad) launch_mbs_t<double, true>(a, grid, block, st);
        else launch_mbs_t<double, false>(a, grid, block, st);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions over blocks (theta) and over replications (RQ, sd, SE), each a
// fixed-order Neumaier sum, so results are bit-reproducible run to run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    const int m = blockIdx.x;
    for (int o = threadIdx.x; o < a.n_out; o += blockDim.x) {
        Acc acc{0.0, 0.0};
        const double *p = a.partial + (size_t)m * a.n_blk * a.stride + a.off + o;
        for (int b = 0; b < a.n_blk; ++b) acc_add(acc, p[(size_t)b * a.stride]);
        a.theta[(size_t)m * a.n_out + o] = (acc.s + acc.c) / a.Nd;
    }
}

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(a.M), dim3(128), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= a.n_out) return;
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

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((a.n_out + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Elementwise inverse normal (verification / utility entry).
template <typename T>
__global__ __launch_bounds__(256) void inv_normal_kernel(int64_t n, const double *__restrict__ u,
                                                         T *__restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = inv_normal(u[i], T(0));
}

hipError_t launch_inv_normal(int64_t n, const double *u, void *z, int fp32, hipStream_t st)
{
    const int64_t blocks = (n + 255) / 256;
    if (fp32)
        hipLaunchKernelGGL(inv_normal_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, n, u, (float *)z);
    else
        hipLaunchKernelGGL(inv_normal_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, n, u, (double *)z);
    return hipGetLastError();
}

}  // namespace rq
