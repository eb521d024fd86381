// rq_batch.hip -- the small kernels around the batch launch: queue and
// timestamp initialisation, and the setup and reductions of every
// instrument of a batch in one launch each (entry found by binary search
// over the prefix of unit counts).
#include "rq_reduce.h"
#include "rq_setup.h"

namespace rq {

// largest e in [0, n) with prefix[e] <= u (prefix[0] = 0, prefix[n] = total)
__device__ __forceinline__ int find_entry(const int64_t *__restrict__ prefix, int n, int64_t u)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void batch_init_kernel(unsigned long long *queue, unsigned long long *t_first,
                                                         unsigned long long *t_last, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *queue = 0ull;
    if (i < n) {
        if (t_first) t_first[i] = ~0ull;
        if (t_last) t_last[i] = 0ull;
    }
}

hipError_t launch_batch_init(unsigned long long *queue, unsigned long long *t_first, unsigned long long *t_last,
                             int n_caller, hipStream_t st)
{
    const int n = n_caller > 1 ? n_caller : 1;
    hipLaunchKernelGGL(batch_init_kernel, dim3((n + 255) / 256), dim3(256), 0, st, queue, t_first, t_last,
                       n_caller);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void batch_setup_kernel(BatchSetup b, int64_t total)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= total) return;
    const int e = find_entry(b.prefix, b.n, u);
    setup_one(b.args[e], u - b.prefix[e]);
}

hipError_t launch_batch_setup(const BatchSetup &b, int64_t total, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_setup_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, b, total);
    return hipGetLastError();
}

__global__ __launch_bounds__(128) void batch_reduce_kernel(BatchReduce b)
{
    const int64_t u = blockIdx.x;
    const int e = find_entry(b.prefix, b.n, u);
    reduce_one(b.args[e], (int)(u - b.prefix[e]), threadIdx.x, blockDim.x);
}

hipError_t launch_batch_reduce(const BatchReduce &b, int64_t blocks, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_reduce_kernel, dim3((unsigned)blocks), dim3(128), 0, st, b);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void batch_finalize_kernel(BatchFinalize b, int64_t total)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= total) return;
    const int e = find_entry(b.prefix, b.n, u);
    finalize_one(b.args[e], (int)(u - b.prefix[e]));
}

hipError_t launch_batch_finalize(const BatchFinalize &b, int64_t total, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, b, total);
    return hipGetLastError();
}

}  // namespace rq

#include "rq_batch_kernel.h"

namespace rq {

hipError_t launch_batch(const BatchArgs &b, int grid, int fp32, int greeks, int phase, hipStream_t st)
{
    if (fp32) return greeks ? launch_batch_f32g(b, grid, phase, st) : launch_batch_f32p(b, grid, st);
    return greeks ? launch_batch_f64g(b, grid, phase, st) : launch_batch_f64p(b, grid, st);
}

int batch_blocks_per_cu(int fp32, int greeks, int phase)
{
    if (fp32) return greeks ? batch_occ_f32g(phase) : batch_occ_f32p();
    return greeks ? batch_occ_f64g(phase) : batch_occ_f64p();
}

}  // namespace rq
