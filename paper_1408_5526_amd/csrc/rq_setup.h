// rq_setup.h -- replication setup (random starts), per start-table entry.
//
// One thread per (replication, index segment, dimension) draws the random
// start n uniform on [0, P) (Algorithm 3, step 1, with omega read to D
// base-p digits), shifts it by the segment origin and splits it into the
// low part the lanes expand and the digit-reversed high part (both carries).
#pragma once

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
__device__ __forceinline__ uint64_t reverse_high(uint64_t h, uint32_t p, uint32_t ndig, const uint16_t *sg)
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

// Entry idx of the start table, idx = (m * n_seg + seg) * s + j.
__device__ __forceinline__ void setup_one(const SetupArgs &a, int64_t idx)
{
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
    const uint16_t *sg = a.perm ? a.perm + (size_t)m * a.perm_stride + b.perm_off : nullptr;
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

}  // namespace rq
