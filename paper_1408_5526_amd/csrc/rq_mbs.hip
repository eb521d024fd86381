// rq_mbs.hip -- Caflisch mortgage-backed-security pricing kernel (the path
// itself is in rq_mbs.h), and the reductions shared by every entry point.
#include "rq_mbs.h"
#include "rq_reduce.h"

namespace rq {

// FP64: three waves per SIMD (167 VGPRs, no spills; left alone the compiler
// keeps the FP64 polynomial constants in 227 and runs two waves: -4%)
template <typename T, bool PERM, bool GRAD>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 1))) void mbs_kernel(MbsArgs a)
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

    __shared__ double red[kBlock / kWave][2];

    double pv, dpv;
    mbs_path<T, PERM, GRAD>(a, st, t, m, i, pv, dpv);
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
// Reductions (bodies in rq_reduce.h).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    reduce_one(a, blockIdx.x, threadIdx.x, blockDim.x);
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
    finalize_one(a, o);
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
