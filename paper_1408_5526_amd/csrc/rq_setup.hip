// rq_setup.hip -- replication setup (random starts) and the materialising
// sequence kernel.
//
// Setup: one thread per (replication, index segment, dimension) draws the
// random start n uniform on [0, P) (Algorithm 3, step 1, with omega read to
// D base-p digits), shifts it by the segment origin and splits it into the
// low part the lanes expand and the digit-reversed high part (both carries).
#include "rq_device.h"

namespace rq {

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output k of the stream
// seeded with `seed` is mix64(seed + (k + 1) * 0x9e3779b97f4a7c15).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sm64_at(uint64_t seed, uint64_t k)
{
    return sm64_mix(seed + (k + 1ull) * 0x9e3779b97f4a7c15ull);
}

// D-L digit reversal of h (< p^{D-L}) with the leading-zero rule.
__device__ uint64_t reverse_high(uint64_t h, uint32_t p, uint32_t ndig, const uint16_t *sg)
{
    uint64_t R = 0;
    for (uint32_t t = 0; t < ndig; ++t) {
        const uint64_t q = h / p;
        const uint32_t a = (uint32_t)(h - q * p);
        uint64_t dig = a;
        if (sg) dig = (h == 0) ? 0 : sg[a];
        R = R * p + dig;
        h = q;
    }
    return R;
}

__global__ __launch_bounds__(256) void setup_kernel(SetupArgs a)
{
    const int64_t total = (int64_t)a.M * a.n_seg * a.s;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int j = (int)(idx % a.s);
    const int64_t rest = idx / a.s;
    const int seg = (int)(rest % a.n_seg);
    const int64_t m = rest / a.n_seg;
    const BaseEnt b = a.base_dev[j];

    uint64_t n = 0;
    if (!(a.flags & kStartZero)) {
        const uint64_t ctr0 = ((uint64_t)(a.m_offset + m) * 4096ull + (uint64_t)j) * 64ull;
        const uint64_t rem = (0ull - b.P) % b.P;      // 2^64 mod P
        for (uint64_t at = 0; at < 64; ++at) {
            const uint64_t u = sm64_at(a.seed, ctr0 + at);
            if (rem == 0 || u < 0ull - rem) { n = u % b.P; break; }
        }
    }
    uint64_t base = n + (uint64_t)seg * (uint64_t)a.S;   // seg*S < N <= P
    if (base >= b.P) base -= b.P;
    const uint64_t hi = base / b.pL;
    const uint32_t nlo = (uint32_t)(base - hi * b.pL);
    const uint16_t *sg = (a.flags & kPermRandom) ? a.perm + b.perm_off : nullptr;
    const uint32_t nd = b.D - b.L;
    uint64_t h0 = hi;
    uint64_t h1 = hi + 1;
    if (h1 >= b.pDL) h1 -= b.pDL;
    StartEnt e;
    const uint64_t r0 = reverse_high(h0, b.p, nd, sg);
    const uint64_t r1 = reverse_high(h1, b.p, nd, sg);
    e.rhi0 = (double)r0;
    e.drhi = (double)(int64_t)(r1 - r0);   // |r1 - r0| < 2^53: exact
    e.nlo = nlo;
    e.hz = (h0 == 0 ? 1u : 0u) | (h1 == 0 ? 2u : 0u);
    e.pad0 = e.pad1 = 0;
    a.starts[idx] = e;
}

hipError_t launch_setup(const SetupArgs &a, hipStream_t st)
{
    const int64_t total = (int64_t)a.M * a.n_seg * a.s;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(setup_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sequence(): materialise x[m][i][j] (or the integers R).  A block covers a
// tile of kTile consecutive points of one replication and all s dimensions;
// consecutive threads write consecutive elements, so stores coalesce.
// ---------------------------------------------------------------------------
constexpr int kTile = 64;

template <bool PERM, bool DIGITS>
__global__ __launch_bounds__(256) void sequence_kernel(SeqGeom g, int64_t tiles_per_m, void *out)
{
    const int64_t m = blockIdx.x / tiles_per_m;
    const int64_t tile = blockIdx.x - m * tiles_per_m;
    const int64_t i0 = tile * kTile;
    const int64_t npts = (g.N - i0) < kTile ? (g.N - i0) : kTile;
    const int seg = (int)(i0 >> g.log2S);                 // tiles never straddle segments
    const StartEnt *st = g.starts + ((size_t)m * g.n_seg + seg) * g.s;
    const uint32_t t0 = (uint32_t)(i0 - ((int64_t)seg << g.log2S));
    const uint32_t nel = (uint32_t)(npts * g.s);
    const size_t obase = ((size_t)m * (size_t)g.N + (size_t)i0) * (size_t)g.s;
    for (uint32_t e = threadIdx.x; e < nel; e += blockDim.x) {
        const uint32_t ip = e / (uint32_t)g.s;
        const int j = (int)(e - ip * (uint32_t)g.s);
        const PointCtx c = load_base(g.base, j);
        const double R = radinv_R<PERM>(c, st + j, t0 + ip, g.perm);
        if (DIGITS)
            ((uint64_t *)out)[obase + e] = (uint64_t)R;
        else
            ((double *)out)[obase + e] = R / c.Pd;
    }
}

hipError_t launch_sequence(const SeqGeom &g, int flags, void *out, hipStream_t st)
{
    const int64_t tiles = (g.N + kTile - 1) / kTile;
    const int64_t blocks = tiles * g.M;
    const bool perm = (flags & kPermRandom) != 0;
    const bool dig = (flags & kOutDigits) != 0;
    auto k = perm ? (dig ? sequence_kernel<true, true> : sequence_kernel<true, false>)
                  : (dig ? sequence_kernel<false, true> : sequence_kernel<false, false>);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, st, g, tiles, out);
    return hipGetLastError();
}

}  // namespace rq
