// rq_setup.hip -- replication setup kernel (the per-entry work is in
// rq_setup.h) and the materialising sequence kernel.
#include "rq_setup.h"

namespace rq {

__global__ __launch_bounds__(256) void setup_kernel(SetupArgs a)
{
    const int64_t total = (int64_t)a.M * a.n_seg * a.s;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    setup_one(a, idx);
}

// Replication m draws its own permutation of every base: Fisher-Yates from
// the identity, step t = p-1..1 swapping sigma[t] and sigma[r], r uniform on
// [0, t] by rejection from the SplitMix64 stream seeded with output
// 2^62 + m_global of the seed's stream, counters 2^60 + (j 65536 + t) 64 + a.
// One thread per (replication, base); its table slice is private.
__global__ __launch_bounds__(256) void perm_kernel(PermArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.M * a.s) return;
    const int j = (int)(idx % a.s);
    const int64_t m = idx / a.s;
    const uint32_t p = a.base[j].p;
    uint16_t *sg = a.table + (size_t)m * a.stride + a.base[j].perm_off;
    const uint64_t sm = sm64_at(a.seed, (1ull << 62) + (uint64_t)(a.m_offset + m));
    for (uint32_t v = 0; v < p; ++v) sg[v] = (uint16_t)v;
    for (uint32_t t = p - 1; t >= 1; --t) {
        const uint64_t range = (uint64_t)t + 1;
        const uint64_t rem = (0ull - range) % range;
        const uint64_t ctr0 = (1ull << 60) + ((uint64_t)j * 65536ull + t) * 64ull;
        uint64_t r = 0;
        for (uint64_t at = 0; at < 64; ++at) {   // a draw is rejected with probability < 2^-48
            const uint64_t u = sm64_at(sm, ctr0 + at);
            if (rem == 0 || u < 0ull - rem) { r = u % range; break; }
        }
        const uint16_t tmp = sg[t];
        sg[t] = sg[r];
        sg[r] = tmp;
    }
}

hipError_t launch_perm(const PermArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.M * a.s;
    hipLaunchKernelGGL(perm_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_setup(const SetupArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.M * a.n_seg * a.s;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(setup_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sequence(): materialise x[m][i][j] (or the integers R).  A block (four
// waves) covers a tile of kTile = 64 consecutive points of one replication
// and all s dimensions, kDimChunk dimensions at a time.  In a chunk each
// wave takes every fourth dimension, so the dimension is wave-uniform: its
// base and start entries arrive as scalar loads, the digit loop runs the
// same trip count in every lane, and lane l computes point i0 + l.  The
// chunk goes through LDS ([point][dimension]; one buffer, which keeps eight
// blocks per CU: two buffers and one barrier per chunk instead of two ran
// 35% slower at four) and leaves as whole rows of
// kDimChunk values per point (256 contiguous bytes): 16 bytes per thread
// for a whole chunk of a whole tile when s is even and the output 16-byte
// aligned (then so is every row), else 8 bytes per thread.
// ---------------------------------------------------------------------------
constexpr int kTile = 64;
constexpr int kDimChunk = 32;

template <bool PERM, bool DIGITS>
__global__ __launch_bounds__(256) void sequence_kernel(SeqGeom g, int64_t tiles_per_m, void *out)
{
    __shared__ uint64_t tile[kTile][kDimChunk + 1];   // +1: the column writes fall on distinct banks
    const int64_t m = blockIdx.x / tiles_per_m;
    const int64_t tl = blockIdx.x - m * tiles_per_m;
    const int64_t i0 = tl * kTile;
    const int npts = (int)((g.N - i0) < kTile ? (g.N - i0) : kTile);
    const int seg = (int)(i0 >> g.log2S);                 // tiles never straddle segments
    const StartEnt *st = g.starts + ((size_t)m * g.n_seg + seg) * g.s;
    const uint32_t t0 = (uint32_t)(i0 - ((int64_t)seg << g.log2S));
    const int lane = threadIdx.x & (kWave - 1);
    // uniform over the wave: the dimension loop's entries then come by scalar
    // loads and its digit loop runs on scalar trip counts
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint16_t *perm = g.perm + (size_t)m * g.perm_stride;
    uint64_t *o = (uint64_t *)out + ((size_t)m * (size_t)g.N + (size_t)i0) * (size_t)g.s;
    const bool wide = npts == kTile && (g.s & 1) == 0 && ((uintptr_t)out & 15) == 0;
    for (int j0 = 0; j0 < g.s; j0 += kDimChunk) {
        const int nd = (g.s - j0) < kDimChunk ? (g.s - j0) : kDimChunk;
        for (int dj = wave; dj < nd; dj += 256 / kWave) {
            const int j = j0 + dj;
            const PointCtx c = load_base_uniform(g.base, j);
            const StartEnt e = load_uniform<StartEnt>(st + j);
            uint64_t v = 0;
            if (lane < npts) {
                const double R = radinv_R<PERM>(c, e, t0 + (uint32_t)lane, perm);
                v = DIGITS ? (uint64_t)R : __builtin_bit_cast(uint64_t, div_rn(R, c.Pd, c.invP));
            }
            tile[lane][dj] = v;
        }
        __syncthreads();
        if (wide && nd == kDimChunk) {
            // 16 threads per row, two dimensions each; 16 rows per pass.  The
            // points are written once and not read back by this kernel:
            // non-temporal stores (26% less time than plain ones at s = 240)
            const int c2 = (threadIdx.x & 15) * 2;
            int r = threadIdx.x >> 4;
            uint64_t *dst = o + (size_t)r * (size_t)g.s + (size_t)(j0 + c2);
            const size_t step = (size_t)16 * (size_t)g.s;
            for (; r < kTile; r += 16, dst += step) {
                typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
                const u64x2 v = {tile[r][c2], tile[r][c2 + 1]};
                __builtin_nontemporal_store(v, (u64x2 *)dst);
            }
        } else {
            const int cnt = npts * nd;
            for (int q = threadIdx.x; q < cnt; q += 256) {
                const int r = q / nd;
                const int cj = q - r * nd;
                __builtin_nontemporal_store(tile[r][cj], o + (size_t)r * (size_t)g.s + (size_t)(j0 + cj));
            }
        }
        __syncthreads();
    }
}

// Pseudo-random points (Philox4x64-10), one element per thread: the
// counter of an element is (j/4, i, 0, 0), so consecutive elements of a row
// come from one block of four words.
__global__ __launch_bounds__(256) void sequence_mc_kernel(SeqGeom g, int64_t tiles_per_m, void *out)
{
    const int64_t m = blockIdx.x / tiles_per_m;
    const int64_t tl = blockIdx.x - m * tiles_per_m;
    const int64_t i0 = tl * kTile;
    const int64_t npts = (g.N - i0) < kTile ? (g.N - i0) : kTile;
    const uint32_t nel = (uint32_t)(npts * g.s);
    const size_t obase = ((size_t)m * (size_t)g.N + (size_t)i0) * (size_t)g.s;
    for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
        const uint32_t ip = e / (uint32_t)g.s;
        const int j = (int)(e - ip * (uint32_t)g.s);
        uint64_t c[4] = {(uint64_t)(j >> 2), (uint64_t)(i0 + ip), 0ull, 0ull};
        philox4x64_10(c, g.seed, (uint64_t)(g.m_offset + m));
        const int q = j & 3;
        __builtin_nontemporal_store(u53(q == 0 ? c[0] : q == 1 ? c[1] : q == 2 ? c[2] : c[3]), (double *)out + obase + e);
    }
}

hipError_t launch_sequence(const SeqGeom &g, int flags, void *out, hipStream_t st)
{
    const int64_t tiles = (g.N + kTile - 1) / kTile;
    const int64_t blocks = tiles * g.M;
    const bool perm = g.perm_on != 0;   // one shared table or one per replication
    const bool dig = (flags & kOutDigits) != 0;
    auto k = g.mc ? sequence_mc_kernel
                  : perm ? (dig ? sequence_kernel<true, true> : sequence_kernel<true, false>)
                         : (dig ? sequence_kernel<false, true> : sequence_kernel<false, false>);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, st, g, tiles, out);
    return hipGetLastError();
}

}  // namespace rq
