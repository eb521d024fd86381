// rq_cpu_alg2.cpp -- the recursive Halton generator (Algorithm 2) on the
// host, multi-core and SIMD: the paper's fastest CPU method as a baseline
// beside the GPU's counter-based generator.
//
// Exact integer partial sums.  For base p with D digits (p^D <= 2^53) the
// index idx has digits a_0 (least significant) .. a_{D-1}, and
//   R(idx) = sum_t sigma(a_t) p^{D-1-t}   over t up to the top nonzero digit
// (digits above it are leading zeros and stay unpermuted), x = RN(R / p^D).
// The low k digits (p^k >= 64) are split off: for the B = p^k consecutive
// indices sharing the block index h = idx / B, R = R_high(h) + T(a) with
// a = idx mod B, so a block is one add and one divide per point, in SIMD
// lanes.  Algorithm 2's recursion runs once per block, on the high digits:
// going from h to h + 1, trailing digits p - 1 wrap to 0 and the next digit
// goes up by one, and only those digits' terms of R_high change.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <omp.h>

#include "../../include/rqmc_cpu.h"

namespace {

thread_local std::string g_err;

rq_status fail(rq_status st, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

const std::vector<uint32_t> &prime_table()
{
    static const std::vector<uint32_t> tab = [] {
        std::vector<uint32_t> out;
        std::vector<char> comp(40001, 0);
        for (uint32_t q = 2; q <= 40000 && (int)out.size() < RQ_MAX_DIM; ++q) {
            if (comp[q]) continue;
            out.push_back(q);
            for (uint64_t r = (uint64_t)q * q; r <= 40000; r += q) comp[r] = 1;
        }
        return out;
    }();
    return tab;
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output k of the stream
// seeded with `seed`.
uint64_t splitmix(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// uniform on [0, range) by rejection from counters ctr0, ctr0 + 1, ...
// (64 attempts; 0 if every one is rejected)
uint64_t draw_below(uint64_t seed, uint64_t ctr0, uint64_t range)
{
    const uint64_t rem = (0ull - range) % range;
    for (uint64_t t = 0; t < 64; ++t) {
        const uint64_t u = splitmix(seed, ctr0 + t);
        if (rem == 0 || u < 0ull - rem) return u % range;
    }
    return 0;
}

// One base and its tables.
struct Base {
    uint32_t p = 0;
    int D = 0, k = 0;
    uint64_t P = 0, B = 0;
    double Pd = 0.0, w0d = 0.0;
    std::vector<uint64_t> w;    // w_t = p^{D-1-t}
    std::vector<uint32_t> sg;   // digit permutation (identity when none)
    std::vector<double> T;      // k > 1: T[a] for a < B, exact
};

void make_base(uint32_t p, const uint32_t *sigma, Base &b)
{
    b.p = p;
    b.D = 0;
    uint64_t P = 1;
    while (P <= (1ull << 53) / p) { P *= p; ++b.D; }
    b.P = P;
    b.Pd = (double)P;
    b.w.assign(b.D, 0);
    uint64_t wt = P / p;
    for (int t = 0; t < b.D; ++t) { b.w[t] = wt; wt /= p; }
    b.w0d = (double)b.w[0];
    b.sg.resize(p);
    for (uint32_t a = 0; a < p; ++a) b.sg[a] = sigma ? sigma[a] : a;
    b.k = 1;
    b.B = p;
    while (b.B < 64 && b.k + 1 < b.D) { b.B *= p; ++b.k; }
    b.T.clear();
    if (b.k > 1) {
        b.T.assign(b.B, 0.0);
        for (uint64_t a = 0; a < b.B; ++a) {
            uint64_t v = a, R = 0;
            for (int t = 0; t < b.k; ++t) {
                R += b.sg[v % p] * b.w[t];
                v /= p;
            }
            b.T[a] = (double)R;
        }
    }
}

// R of one index from its digits (the definition); leading zeros unpermuted.
uint64_t radinv_direct(const Base &b, uint64_t idx)
{
    uint64_t R = 0;
    for (int t = 0; t < b.D && idx != 0; ++t) {
        R += b.sg[idx % b.p] * b.w[t];
        idx /= b.p;
    }
    return R;
}

// Algorithm 2's state on the high digits (positions k..D-1) of the block
// index h: the digits, the position of the top nonzero one (-1: h = 0) and
// the exact partial sum of their terms.
struct High {
    uint32_t dig[64];
    int top;
    uint64_t R;
};

void high_init(const Base &b, uint64_t h, High &s)
{
    std::memset(s.dig, 0, sizeof s.dig);
    s.top = -1;
    s.R = 0;
    for (int t = b.k; t < b.D && h != 0; ++t) {
        s.dig[t] = (uint32_t)(h % b.p);
        if (s.dig[t]) s.top = t;
        h /= b.p;
    }
    for (int t = b.k; t <= s.top; ++t) s.R += b.sg[s.dig[t]] * b.w[t];
}

void high_next(const Base &b, High &s)
{
    int t = b.k;
    while (t < b.D && s.dig[t] == b.p - 1) {   // p - 1 -> 0; the digit stays significant
        s.R = s.R - b.sg[b.p - 1] * b.w[t] + b.sg[0] * b.w[t];
        s.dig[t] = 0;
        ++t;
    }
    if (t == b.D) {   // past p^D - 1: index 0, every digit a leading zero
        std::memset(s.dig, 0, sizeof s.dig);
        s.top = -1;
        s.R = 0;
        return;
    }
    if (t > s.top) {   // a leading zero becomes 1
        s.R += b.sg[1] * b.w[t];
        s.top = t;
    } else {
        s.R = s.R - b.sg[s.dig[t]] * b.w[t] + b.sg[s.dig[t] + 1] * b.w[t];
    }
    s.dig[t] += 1;
}

// A position in one base's index sequence: the block index's state and
// the offset a in the block (idx = h B + a).
struct Cursor {
    High hs;
    uint64_t a;
};

void cursor_init(const Base &b, uint64_t idx, Cursor &c)
{
    const uint64_t h = idx / b.B;
    c.a = idx - h * b.B;
    high_init(b, h, c.hs);
}

// The next `count` indices from the cursor, in order, per run inside one
// block: run(i, len, R_high as an exact double, a) for a block with h > 0,
// one(i, R) per index in block 0 (there every digit of the index may be a
// leading zero, so it goes by the definition).
template <typename Run, typename One>
void advance(const Base &b, Cursor &c, int64_t count, Run &&run, One &&one)
{
    for (int64_t i = 0; i < count;) {
        const int64_t len = std::min<int64_t>(count - i, (int64_t)(b.B - c.a));
        if (c.hs.top < 0) {
            for (int64_t r = 0; r < len; ++r) one(i + r, (double)radinv_direct(b, c.a + (uint64_t)r));
        } else {
            run(i, len, (double)c.hs.R, c.a);
        }
        i += len;
        c.a += (uint64_t)len;
        if (c.a == b.B) {
            c.a = 0;
            high_next(b, c.hs);
        }
    }
}

// x = (R_high + T(a)) / P over one block run, written with stride `ld`:
// T(a) = sigma(a) p^{D-1} for k = 1 (a product of exact integers below
// 2^53, so exact), the table for k > 1.  The sums are exact and the one
// division rounds to nearest, as in the definition.
inline void emit_run(const Base &b, double Rh, uint64_t a0, int64_t len, double *out, int64_t ld)
{
    const double Pd = b.Pd;
    if (b.k == 1) {
        const uint32_t *sg = b.sg.data() + a0;
        const double w0 = b.w0d;
#pragma omp simd
        for (int64_t r = 0; r < len; ++r) out[r * ld] = (Rh + (double)sg[r] * w0) / Pd;
    } else {
        const double *T = b.T.data() + a0;
#pragma omp simd
        for (int64_t r = 0; r < len; ++r) out[r * ld] = (Rh + T[r]) / Pd;
    }
}

}  // namespace

extern "C" {

const char *rq_cpu_last_error(void) { return g_err.c_str(); }

int rq_cpu_max_threads(void) { return omp_get_max_threads(); }

rq_status rq_cpu_alg2_run(uint32_t p, const int32_t *sigma, uint64_t n, int64_t count, uint64_t *out)
{
    if (p < 2 || p > 40000) return fail(RQ_EINVAL, "base %u outside [2, 40000]", p);
    for (uint32_t q = 2; (uint64_t)q * q <= p; ++q)
        if (p % q == 0) return fail(RQ_EINVAL, "base %u is not prime", p);
    if (count < 0) return fail(RQ_EINVAL, "count must be >= 0");
    if (count > 0 && !out) return fail(RQ_EINVAL, "out is NULL");
    std::vector<uint32_t> sg;
    if (sigma) {
        std::vector<char> seen(p, 0);
        for (uint32_t a = 0; a < p; ++a) {
            if (sigma[a] < 0 || (uint32_t)sigma[a] >= p || seen[sigma[a]])
                return fail(RQ_EINVAL, "sigma is not a permutation of 0..%u", p - 1);
            seen[sigma[a]] = 1;
            sg.push_back((uint32_t)sigma[a]);
        }
    }
    Base b;
    make_base(p, sigma ? sg.data() : nullptr, b);
    Cursor c;
    cursor_init(b, n % b.P, c);
    advance(
        b, c, count,
        [&](int64_t i, int64_t len, double Rh, uint64_t a0) {
            for (int64_t r = 0; r < len; ++r) {
                const double lo = b.k == 1 ? (double)b.sg[a0 + r] * b.w0d : b.T[a0 + r];
                out[i + r] = (uint64_t)(Rh + lo);
            }
        },
        [&](int64_t i, double R) { out[i] = (uint64_t)R; });
    return RQ_OK;
}

rq_status rq_cpu_sequence(int s, int64_t N, int M, uint64_t seed, int flags, int64_t m_offset, double *out,
                          int threads)
{
    if (s < 1) return fail(RQ_EINVAL, "s must be >= 1 (got %d)", s);
    if (N < 1) return fail(RQ_EINVAL, "N must be >= 1");
    if (M < 1) return fail(RQ_EINVAL, "M must be >= 1");
    if (m_offset < 0) return fail(RQ_EINVAL, "m_offset must be >= 0");
    if (!out) return fail(RQ_EINVAL, "out is NULL");
    if (threads < 0) return fail(RQ_EINVAL, "threads must be >= 0");
    if (flags & ~(RQ_START_ZERO | RQ_PERM_RANDOM))
        return fail(RQ_EUNSUPPORTED, "the CPU generator takes RQ_START_ZERO and RQ_PERM_RANDOM only");
    if (s > RQ_MAX_DIM) return fail(RQ_ERANGE, "s = %d beyond the %d supported bases", s, RQ_MAX_DIM);
    if (m_offset + (int64_t)M > RQ_MAX_REPLICATION) return fail(RQ_ERANGE, "m_offset + M beyond 2^40");
    const auto &pr = prime_table();
    std::vector<Base> bases(s);
    for (int j = 0; j < s; ++j) {
        const uint32_t p = pr[j];
        std::vector<uint32_t> sg;
        if (flags & RQ_PERM_RANDOM) {   // Fisher-Yates from the identity, counters 2^60 + (j 65536 + t) 64
            sg.resize(p);
            for (uint32_t a = 0; a < p; ++a) sg[a] = a;
            for (uint32_t t = p - 1; t >= 1; --t) {
                const uint64_t r = draw_below(seed, (1ull << 60) + ((uint64_t)j * 65536ull + t) * 64ull, t + 1ull);
                std::swap(sg[t], sg[r]);
            }
        }
        make_base(p, sg.empty() ? nullptr : sg.data(), bases[j]);
        if ((uint64_t)N > bases[j].P)
            return fail(RQ_ERANGE, "N = %lld exceeds P_%d (base %u)", (long long)N, j, p);
    }
    // starts n_j^m: (m_global 4096 + j) 64 + attempt
    std::vector<uint64_t> start((size_t)M * s, 0);
    if (!(flags & RQ_START_ZERO))
        for (int m = 0; m < M; ++m)
            for (int j = 0; j < s; ++j)
                start[(size_t)m * s + j] =
                    draw_below(seed, ((uint64_t)(m_offset + m) * 4096ull + (uint64_t)j) * 64ull, bases[j].P);
    // Work units: (replication, range of indices), a few per thread.  A unit
    // keeps one cursor per dimension and walks its range in tiles of 128
    // indices: each dimension writes its 128 points contiguously into a
    // scratch tile [s][128], which is then transposed into the rows of out
    // in 8 x 8 blocks (whole cache lines on both sides).
    constexpr int64_t kTile = 128;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
    const int64_t tiles = (N + kTile - 1) / kTile;
    const int64_t per_m = std::max<int64_t>(1, std::min<int64_t>(tiles, (4 * (int64_t)nt + M - 1) / M));
    const int64_t tiles_per_unit = (tiles + per_m - 1) / per_m;
    const int64_t units = (int64_t)M * per_m;
#pragma omp parallel num_threads(nt)
    {
        std::vector<Cursor> cur(s);
        std::vector<double> tile((size_t)s * kTile);
#pragma omp for schedule(dynamic, 1)
        for (int64_t u = 0; u < units; ++u) {
            const int m = (int)(u / per_m);
            const int64_t t0 = (u - (int64_t)m * per_m) * tiles_per_unit;
            const int64_t i_begin = t0 * kTile;
            const int64_t i_end = std::min<int64_t>(N, (t0 + tiles_per_unit) * kTile);
            if (i_begin >= i_end) continue;
            for (int j = 0; j < s; ++j) {
                uint64_t idx0 = start[(size_t)m * s + j] + (uint64_t)i_begin;   // < 2 P
                if (idx0 >= bases[j].P) idx0 -= bases[j].P;
                cursor_init(bases[j], idx0, cur[j]);
            }
            for (int64_t i0 = i_begin; i0 < i_end; i0 += kTile) {
                const int64_t cnt = std::min<int64_t>(kTile, i_end - i0);
                for (int j = 0; j < s; ++j) {
                    const Base &b = bases[j];
                    double *col = tile.data() + (size_t)j * kTile;
                    advance(
                        b, cur[j], cnt,
                        [&](int64_t i, int64_t len, double Rh, uint64_t a0) { emit_run(b, Rh, a0, len, col + i, 1); },
                        [&](int64_t i, double R) { col[i] = R / b.Pd; });
                }
                double *o = out + ((size_t)m * N + i0) * s;
                for (int64_t r0 = 0; r0 < cnt; r0 += 8) {
                    const int64_t rn = std::min<int64_t>(8, cnt - r0);
                    for (int j0 = 0; j0 < s; j0 += 8) {
                        const int jn = std::min(8, s - j0);
                        for (int64_t r = 0; r < rn; ++r)
                            for (int j = 0; j < jn; ++j)
                                o[(r0 + r) * s + j0 + j] = tile[(size_t)(j0 + j) * kTile + r0 + r];
                    }
                }
            }
        }
    }
    return RQ_OK;
}

}  // extern "C"
