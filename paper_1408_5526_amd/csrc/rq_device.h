// rq_device.h -- device building blocks shared by the pricing kernels:
// the in-register radical inverse, the inverse normal CDF, deterministic
// wave reductions and compensated accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rq_internal.h"

namespace rq {

// Read-only parameter tables are read through the constant address space:
// the kernel never writes them, so the compiler may use scalar loads even
// after the kernel has stored to global memory.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const void *p)
{
    return (cptr<T>)p;
}

// A wave-uniform struct read through the constant address space (scalar
// loads; the fields the caller never uses are not loaded).
template <typename S>
__device__ __forceinline__ S load_uniform(const void *p)
{
    static_assert(sizeof(S) % 4 == 0, "struct size must be a multiple of 4");
    const cptr<uint32_t> q = as_const<uint32_t>(p);
    uint32_t w[sizeof(S) / 4];
#pragma unroll
    for (unsigned i = 0; i < sizeof(S) / 4; ++i) w[i] = q[i];
    S out;
    __builtin_memcpy(&out, w, sizeof(S));
    return out;
}

// ---------------------------------------------------------------------------
// Radical inverse (eqs. (1)-(3)) of the index (n + i) mod P for one lane.
//
// The segment table holds the split of the replication's start; the lane
// expands only the L low base-p digits of v = nlo + t.  Digit extraction is
// exact FP64 arithmetic: for integers 0 <= v < 2^31 and p < 2^20,
// trunc(RN(v * RU(1/p))) == floor(v/p) (the rounded product never reaches
// the next integer because (p-1)/p + 2^-21 < 1 - 2^-23), the remainder
// fma(-q, p, v) is exact, and the Horner accumulation R = R*p + a stays an
// exact integer below 2^53.  The returned R is P * phi exactly; the point
// is RN(R / P) (div_rn below).
//
// With a digit permutation sigma (eq. (3)) digits above the top nonzero
// digit of the whole index stay 0: when the high part (hi + c) is zero
// (bit c of hz) the zero digits of v above its own top digit are leading
// zeros too; they are exactly the digits met once the remaining value is 0.
// ---------------------------------------------------------------------------
struct PointCtx {
    double pd, invp, pDLd, Pd, invP;
    uint32_t L, pL, perm_off;
};

__device__ __forceinline__ PointCtx load_base(const BaseEnt *__restrict__ base, int j)
{
    PointCtx c;
    const BaseEnt *b = base + j;
    c.pd = b->pd;
    c.invp = b->invp_up;
    c.pDLd = b->pDLd;
    c.Pd = b->Pd;
    c.invP = b->invP;
    c.L = b->L;
    c.pL = b->pL;
    c.perm_off = b->perm_off;
    return c;
}

// The same, for a dimension j shared by the whole wave (every pricing
// kernel: j is the time step's dimension): scalar loads through the constant
// address space, so the digit loop's trip count and constants arrive in
// scalar registers after a short scalar-cache round trip.
__device__ __forceinline__ PointCtx load_base_uniform(const BaseEnt *base, int j)
{
    const BaseEnt b = load_uniform<BaseEnt>(base + j);
    PointCtx c;
    c.pd = b.pd;
    c.invp = b.invp_up;
    c.pDLd = b.pDLd;
    c.Pd = b.Pd;
    c.invP = b.invP;
    c.L = b.L;
    c.pL = b.pL;
    c.perm_off = b.perm_off;
    return c;
}

// R of the lane's point as an exact FP64 integer.  The carry picks the high
// part as Rhi[0] + c (Rhi[1] - Rhi[0]): arithmetic on two scalars instead of
// a per-lane selected load.  Digits go two at a time to keep the loop free
// of register shuffles.
template <bool PERM>
__device__ __forceinline__ double radinv_R(const PointCtx &c, const StartEnt &e, uint32_t t,
                                           const uint16_t *__restrict__ perm)
{
    uint32_t vi = e.nlo + t;                  // < 2 p^L <= 2^31
    const bool carry = vi >= c.pL;
    vi -= carry ? c.pL : 0u;
    const double rhi = __builtin_fma(carry ? 1.0 : 0.0, e.drhi, e.rhi0);
    double v = (double)vi;
    double R = 0.0;
    if (!PERM && c.L == 2) {
        // two low digits (p^2 >= N, most dimensions): v < p^2, so v = q1 p + a1
        // with q1 = floor(v/p) < p, and the reversal is a1 p + q1, no loop
        const double q1 = __builtin_trunc(v * c.invp);
        R = __builtin_fma(__builtin_fma(-q1, c.pd, v), c.pd, q1);
    } else if (!PERM) {
        uint32_t q = 0;
        for (; q + 2 <= c.L; q += 2) {
            const double q1 = __builtin_trunc(v * c.invp);
            const double a1 = __builtin_fma(-q1, c.pd, v);
            const double q2 = __builtin_trunc(q1 * c.invp);
            const double a2 = __builtin_fma(-q2, c.pd, q1);
            R = __builtin_fma(__builtin_fma(R, c.pd, a1), c.pd, a2);
            v = q2;
        }
        if (q < c.L) {
            const double q1 = __builtin_trunc(v * c.invp);
            R = __builtin_fma(R, c.pd, __builtin_fma(-q1, c.pd, v));
        }
    } else {
        const bool hz = (e.hz >> (carry ? 1 : 0)) & 1u;
        const uint16_t *sg = perm + c.perm_off;
        for (uint32_t q = 0; q < c.L; ++q) {
            const double qt = __builtin_trunc(v * c.invp);
            const double a = __builtin_fma(-qt, c.pd, v);
            const double dig = (hz && v == 0.0) ? 0.0 : (double)sg[(int)a];
            R = __builtin_fma(R, c.pd, dig);
            v = qt;
        }
    }
    return __builtin_fma(R, c.pDLd, rhi);
}

// RN(a / b) for finite a >= 0 and b > 0 (no underflow or overflow on the
// way) given y = RN(1/b): q = RN(a y) is within an ulp of a / b, the
// remainder r = a - b q is exact (one FMA), and RN(q + r y) is the
// correctly rounded quotient (Markstein's theorem, as in Muller et al.,
// Handbook of Floating-Point Arithmetic, on division by FMA).  Three
// instructions instead of an IEEE division's ten; for b = P = p^D and
// integer 0 <= a < P it was also checked against division on the host for
// 4.1e9 quotients over the first 4096 primes, without a difference.
__device__ __forceinline__ double div_rn(double a, double b, double y)
{
    const double q = a * y;
    const double r = __builtin_fma(-q, b, a);
    return __builtin_fma(r, y, q);
}

// The point RN(R / P).  EXACT = false forms R * RN(1/P) instead, within
// two ulps of it (used where the point only feeds FP32 arithmetic).
template <bool PERM, bool EXACT = true>
__device__ __forceinline__ double radinv_x(const PointCtx &c, const StartEnt &e, uint32_t t,
                                           const uint16_t *__restrict__ perm)
{
    const double R = radinv_R<PERM>(c, e, t, perm);
    return EXACT ? div_rn(R, c.Pd, c.invP) : R * c.invP;
}

// ---------------------------------------------------------------------------
// Inverse standard normal CDF: Wichura, "Algorithm AS 241" (Applied
// Statistics 37, 1988), PPND16 rational approximations on three regions:
// |u - 1/2| <= 0.425; r = sqrt(-ln min(u,1-u)) <= 5; r > 5.  The fold
// min(u, 1-u) is formed in FP64 and clamped to 2^-64 (u = 0 occurs only for
// the index whose digits are all zero).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T as241_central(T q)
{
    const T r = T(0.180625) - q * q;
    T num = T(2.5090809287301226727e3);
    num = num * r + T(3.3430575583588128105e4);
    num = num * r + T(6.7265770927008700853e4);
    num = num * r + T(4.5921953931549871457e4);
    num = num * r + T(1.3731693765509461125e4);
    num = num * r + T(1.9715909503065514427e3);
    num = num * r + T(1.3314166789178437745e2);
    num = num * r + T(3.3871328727963666080e0);
    T den = T(5.2264952788528545610e3);
    den = den * r + T(2.8729085735721942674e4);
    den = den * r + T(3.9307895800092710610e4);
    den = den * r + T(2.1213794301586595867e4);
    den = den * r + T(5.3941960214247511077e3);
    den = den * r + T(6.8718700749205790830e2);
    den = den * r + T(4.2313330701600911252e1);
    den = den * r + T(1.0);
    return q * num / den;
}

template <typename T>
__device__ __forceinline__ T as241_tail(T r)   // r = sqrt(-ln u_folded)
{
    if (r <= T(5.0)) {
        r -= T(1.6);
        T num = T(7.74545014278341407640e-4);
        num = num * r + T(2.27238449892691845833e-2);
        num = num * r + T(2.41780725177450611770e-1);
        num = num * r + T(1.27045825245236838258e0);
        num = num * r + T(3.64784832476320460504e0);
        num = num * r + T(5.76949722146069140550e0);
        num = num * r + T(4.63033784615654529590e0);
        num = num * r + T(1.42343711074968357734e0);
        T den = T(1.05075007164441684324e-9);
        den = den * r + T(5.47593808499534494600e-4);
        den = den * r + T(1.51986665636164571966e-2);
        den = den * r + T(1.48103976427480074590e-1);
        den = den * r + T(6.89767334985100004550e-1);
        den = den * r + T(1.67638483018380384940e0);
        den = den * r + T(2.05319162663775882187e0);
        den = den * r + T(1.0);
        return num / den;
    }
    r -= T(5.0);
    T num = T(2.01033439929228813265e-7);
    num = num * r + T(2.71155556874348757815e-5);
    num = num * r + T(1.24266094738807843860e-3);
    num = num * r + T(2.65321895265761230930e-2);
    num = num * r + T(2.96560571828504891230e-1);
    num = num * r + T(1.78482653991729133580e0);
    num = num * r + T(5.46378491116411436990e0);
    num = num * r + T(6.65790464350110377720e0);
    T den = T(2.04426310338993978564e-15);
    den = den * r + T(1.42151175831644588870e-7);
    den = den * r + T(1.84631831751005468180e-5);
    den = den * r + T(7.86869131145613259100e-4);
    den = den * r + T(1.48753612908506148525e-2);
    den = den * r + T(1.36929880922735805310e-1);
    den = den * r + T(5.99832206555887937690e-1);
    den = den * r + T(1.0);
    return num / den;
}

__device__ __forceinline__ double inv_normal(double u, double)
{
    const double q = u - 0.5;
    if (fabs(q) <= 0.425) return as241_central<double>(q);
    double r = q < 0.0 ? u : 1.0 - u;
    r = fmax(r, 0x1p-64);
    const double z = as241_tail<double>(sqrt(-log(r)));
    return q < 0.0 ? -z : z;
}

// FP32 form (a fit of our own, generated by fit_inv_normal.py, after the
// shape of Giles 2011): x = 2u - 1, w = -ln(4u(1-u)),
//   Phi^{-1}(u) = x P(w - 2.5) for w < 5 (~99.7% of points), else
//   Phi^{-1}(u) = x Q(sqrt(w) - 3), down to the clamp u(1-u) >= 2^-64.
// u(1-u) and x are formed in FP64 from the FP64 point; the rest is FP32.
// Relative error ~1e-8 of the fits plus float rounding (~2e-7).  The tail
// branch runs only in waves that hold a tail point (~20% of waves).
__device__ __forceinline__ float inv_normal(double u, float)
{
    const double p = __builtin_fma(-u, u, u);   // u (1 - u), rounded once
    const float pf = fmaxf((float)p, 0x1p-64f);
    const float w = __builtin_fmaf(__builtin_amdgcn_logf(pf), -0.693147180559945309f,
                                   -1.38629436111989062f);   // -ln(4 p)
    const float x = (float)__builtin_fma(2.0, u, -1.0);
    float r;
    if (w < 5.0f) {
        const float t = w - 2.5f;
        r = -1.2261584636519274e-08f;
        r = __builtin_fmaf(r, t, 3.278690030583675e-08f);
        r = __builtin_fmaf(r, t, 6.569200650119456e-07f);
        r = __builtin_fmaf(r, t, -4.896187874692259e-06f);
        r = __builtin_fmaf(r, t, -7.0085679908515885e-06f);
        r = __builtin_fmaf(r, t, 0.0003087827062699944f);
        r = __builtin_fmaf(r, t, -0.0017716623842716217f);
        r = __builtin_fmaf(r, t, -0.0059077139012515545f);
        r = __builtin_fmaf(r, t, 0.3488020598888397f);
        r = __builtin_fmaf(r, t, 2.1233134269714355f);
    } else {
        const float t = __builtin_amdgcn_sqrtf(w) - 3.0f;   // v_sqrt_f32
        r = -3.145217988276272e-07f;
        r = __builtin_fmaf(r, t, 5.651296305586584e-06f);
        r = __builtin_fmaf(r, t, -4.1833809518720955e-05f);
        r = __builtin_fmaf(r, t, 0.00015798278036527336f);
        r = __builtin_fmaf(r, t, -0.00026979981339536607f);
        r = __builtin_fmaf(r, t, -0.00016467731620650738f);
        r = __builtin_fmaf(r, t, 0.001944091753102839f);
        r = __builtin_fmaf(r, t, -0.004991183523088694f);
        r = __builtin_fmaf(r, t, 0.008097918704152107f);
        r = __builtin_fmaf(r, t, -0.010832239873707294f);
        r = __builtin_fmaf(r, t, 0.013349912129342556f);
        r = __builtin_fmaf(r, t, 1.416584849357605f);
        r = __builtin_fmaf(r, t, 4.006434440612793f);
    }
    return x * r;
}

// ---------------------------------------------------------------------------
// Elementary functions of the path arithmetic in the two precisions.
// ---------------------------------------------------------------------------
// 2^x in FP64 for the adjoint's FP64 form (its drift factor and fixing
// values): with k = rint(x), 2^x = e^r 2^k, r = (x - k) ln 2 (x - k is exact
// and its product with RN(ln 2) is within an ulp of r, |r| <= ln2 / 2); e^r
// by the Taylor polynomial of degree 12 (truncation below 2^-53 relative)
// in Horner form.  Within about two ulps (checked against 50-digit values
// when the constants were chosen).  Arguments are clamped to [-1020, 1020],
// where 2^x stays a normal number.
__device__ __forceinline__ double exp2_f64(double x)
{
    x = __builtin_fmin(__builtin_fmax(x, -1020.0), 1020.0);
    const double k = __builtin_rint(x);
    const double r = (x - k) * 0x1.62e42fefa39efp-1;
    double p = 0x1.1eed8eff8d898p-29;   // 1/12!
    p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26);
    p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22);
    p = __builtin_fma(p, r, 0x1.71de3a556c734p-19);
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16);
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13);
    p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10);
    p = __builtin_fma(p, r, 0x1.1111111111111p-7);
    p = __builtin_fma(p, r, 0x1.5555555555555p-5);
    p = __builtin_fma(p, r, 0x1.5555555555555p-3);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(__builtin_fma(p, r, 1.0), (int)k);
}
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
// a / b as a * rcp(b): v_rcp_f32 is accurate to 1 ulp
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// 1 / x for a normal x well inside the FP64 range (the spot numeraire,
// 1..~1e3 here): v_rcp_f64 refined by two Newton steps r += r (1 - x r),
// each of which squares the relative error; the result is within an ulp or
// two of the correctly rounded reciprocal, in 5 instructions instead of the
// 10 of an IEEE division.
__device__ __forceinline__ double recip64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }   // v_exp_f32
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fatan(double x) { return atan(x); }
__device__ __forceinline__ float fatan(float x) { return atanf(x); }

// ---------------------------------------------------------------------------
// Deterministic reductions: butterfly over the 64 lanes (every lane ends with
// the same total, summed in a fixed order), Neumaier compensated sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum 16 per-lane values over the wave with a transpose butterfly: at each
// of the steps 32, 16, 8, 4 a lane keeps one half of its values, sends the
// other half to its partner and adds what it receives, so 16 outputs cost
// 8+4+2+1 exchanges plus two final ones instead of 16*6.  Afterwards lane l
// with (l & 3) == 0 holds the wave total of output (l >> 2) & 15.  The
// summation tree is fixed, so the result is deterministic.
__device__ __forceinline__ double wave_sum16(double (&v)[16], int lane)
{
    // The per-lane choice between v[q] and v[q+h] is a bitwise select under
    // a mask the optimizer cannot see through: written as a conditional it
    // becomes a lane-dependent index into the array, lowered to a compare
    // per element whose masks end up in (spilled) scalar registers.
    auto pick = [](uint32_t m, double a, double b) -> double {
        const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
        const uint32_t lo = ((uint32_t)ua & m) | ((uint32_t)ub & ~m);
        const uint32_t hi = ((uint32_t)(ua >> 32) & m) | ((uint32_t)(ub >> 32) & ~m);
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    };
    // The first two levels (partners 32 and 16 lanes away) use the gfx950
    // lane-swap instructions: swapping the upper half of v[q] with the lower
    // half of v[q + h] leaves every lane holding its own element and its
    // partner's, with no selects and no LDS traffic (FP64 addition is
    // commutative, so the sums are the same as with the exchange below).
    auto swap_add = [](double &x, double y, auto sw) {
        const uint64_t ux = __builtin_bit_cast(uint64_t, x), uy = __builtin_bit_cast(uint64_t, y);
        const auto lo = sw((uint32_t)ux, (uint32_t)uy);
        const auto hi = sw((uint32_t)(ux >> 32), (uint32_t)(uy >> 32));
        const double a = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
        const double b = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
        x = a + b;
    };
    auto sw32 = [](uint32_t a, uint32_t b) { return __builtin_amdgcn_permlane32_swap(a, b, false, false); };
    auto sw16 = [](uint32_t a, uint32_t b) { return __builtin_amdgcn_permlane16_swap(a, b, false, false); };
#pragma unroll
    for (int q = 0; q < 8; ++q) swap_add(v[q], v[q + 8], sw32);   // lanes >= 32 now hold outputs 8..15
#pragma unroll
    for (int q = 0; q < 4; ++q) swap_add(v[q], v[q + 4], sw16);   // odd rows of 16 hold outputs +4
#pragma unroll
    for (int h = 2, b = 8; h >= 1; h >>= 1, b >>= 1) {
        uint32_t up = (lane & b) ? ~0u : 0u;
        asm volatile("" : "+v"(up));
#pragma unroll
        for (int q = 0; q < h; ++q) {
            const double send = pick(up, v[q], v[q + h]);
            const double keep = pick(up, v[q + h], v[q]);
            v[q] = keep + __shfl_xor(send, b, kWave);
        }
    }
    double r = v[0];
    r += __shfl_xor(r, 2, kWave);
    r += __shfl_xor(r, 1, kWave);
    return r;
}

struct Acc {
    double s, c;
};

// ---------------------------------------------------------------------------
// Pseudo-random points (the comparison baseline): Philox4x64-10 (Salmon,
// Moraes, Dror & Shaw, SC'11).  A round maps the counter (c0, c1, c2, c3)
// under the key (k0, k1) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)), hi/lo the halves of the 128-bit product, then adds the Weyl
// constants to the key; ten rounds.  Coordinate j of point i of replication
// m_global is word (j mod 4) of the block at counter (j / 4, i, 0, 0) under
// key (seed, m_global), mapped to ((x >> 11) + 1/2) 2^-53 in (0, 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
        const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ double u53(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1p-53; }

// The pseudo-random coordinates of one path, one Philox block (four
// coordinates) at a time; j must be wave-uniform.
struct McPath {
    uint64_t w[4];
    int blk = -1;
    __device__ __forceinline__ double point(uint64_t seed, uint64_t m_global, uint64_t i, int j)
    {
        const int b = j >> 2;
        if (b != blk) {
            uint64_t c[4] = {(uint64_t)b, i, 0ull, 0ull};
            philox4x64_10(c, seed, m_global);
            w[0] = c[0];
            w[1] = c[1];
            w[2] = c[2];
            w[3] = c[3];
            blk = b;
        }
        const int q = j & 3;
        return u53(q == 0 ? w[0] : q == 1 ? w[1] : q == 2 ? w[2] : w[3]);
    }
};

// A wave-uniform value the compiler must treat as new at this point: loads
// and comparisons derived from it are not hoisted above it (out of a
// persistent loop), where they would stay live in scalar registers.
__device__ __forceinline__ int opaque_u(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}
template <typename T>
__device__ __forceinline__ cptr<T> opaque_u(cptr<T> p)
{
    uint64_t u = (uint64_t)p;
    asm volatile("" : "+s"(u));
    return (cptr<T>)u;
}

// LDS tables read inside a loop: lds_base gives the table's local address
// through an empty asm (call it inside the loop), so the reads below depend
// on the iteration and are not hoisted into registers as loop-invariant
// values; they stay ds_read instructions next to their use.
template <typename T>
using lds_ptr = const __attribute__((address_space(3))) T *;
template <typename T>
__device__ __forceinline__ lds_ptr<T> lds_base(const T *table)
{
    uint32_t u = (uint32_t)(uintptr_t)(lds_ptr<T>)table;
    asm volatile("" : "+v"(u));   // a vector register: the ds_read address operand
    return (lds_ptr<T>)(uintptr_t)u;
}
// Entries n0..n0+3 (n0 a multiple of 4, the table aligned to 4 entries) in
// one vector read.
template <typename T>
struct Quad {
    T v[4];
};
template <typename T>
__device__ __forceinline__ Quad<T> lds_quad(lds_ptr<T> table, int n0)
{
    typedef T vec4 __attribute__((ext_vector_type(4)));
    const vec4 x = *(const __attribute__((address_space(3))) vec4 *)(table + n0);
    return Quad<T>{{x[0], x[1], x[2], x[3]}};
}

__device__ __forceinline__ void acc_add(Acc &a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}

}  // namespace rq
