// rq_abi.cpp -- the C ABI: argument validation, per-dimension tables,
// workspace layout and the launch sequence of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rqmc.h"
#include "rq_internal.h"

// Device scratch of rq_price_caplets_noalloc: one copy per GPU, held until
// the process ends.  Host code never passes this name to a kernel or a copy
// (on the host it is only a stand-in for the symbol); it uses the device
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = RQ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using rq::BaseEnt;
using rq::StartEnt;

thread_local std::string g_err;

rq_status fail(rq_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define RQ_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RQ_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

// The scratch array's device address per device, looked up once per device
// (with that device current) by the first no-allocation call on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

rq_status scratch_of_device(void *&ws, size_t &ws_bytes);

// Optional kernel timer (rq_timer_begin / rq_timer_end).
// The adjoint's store region per chunk (single calls) or window (batch),
// FP64-counted (rq_set_adjoint_store_limit).
std::atomic<size_t> g_adj_store_limit{rq::kAdjStoreBytes};

// Tag 0 brackets an entry point's whole main path (what rq_timer_end
// reports); tags 1 and 2 bracket the forward and reverse halves of the
// two-kernel adjoint inside it (rq_timer_part).
constexpr int kTimerTags = 3;
constexpr int kTimerPairsPerLaunch = 33;
struct KernelTimer {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<int> tag;         // per pair
    size_t used = 0;
    bool record_failed = false;   // a hipEventRecord failed: rq_timer_end reports it
    double part_ms[kTimerTags] = {};
    int part_n[kTimerTags] = {};
} g_timer;

struct TimedRegion {
    hipStream_t st;
    hipEvent_t stop = nullptr;
    explicit TimedRegion(hipStream_t s, int tag = 0) : st(s)
    {
        std::lock_guard<std::mutex> lk(g_timer.mu);
        if (g_timer.on && 2 * (g_timer.used + 1) <= g_timer.ev.size()) {
            if (hipEventRecord(g_timer.ev[2 * g_timer.used], st) != hipSuccess) g_timer.record_failed = true;
            stop = g_timer.ev[2 * g_timer.used + 1];
            g_timer.tag[g_timer.used] = tag;
            ++g_timer.used;
        }
    }
    ~TimedRegion()
    {
        if (stop && hipEventRecord(stop, st) != hipSuccess) {
            std::lock_guard<std::mutex> lk(g_timer.mu);
            g_timer.record_failed = true;
        }
    }
};

rq_status scratch_of_device(void *&ws, size_t &ws_bytes)
{
    int dev = -1;
    RQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RQ_EUNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RQ_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    ws = g_scratch_ptr[dev];
    ws_bytes = kScratchBytes;
    return RQ_OK;
}

// The first RQ_MAX_DIM primes (sieve of Eratosthenes).
const std::vector<uint32_t> &primes()
{
    static const std::vector<uint32_t> tab = [] {
        std::vector<uint32_t> out;
        const uint32_t lim = 40000;
        std::vector<char> comp(lim + 1, 0);
        for (uint32_t q = 2; q <= lim && (int)out.size() < RQ_MAX_DIM; ++q) {
            if (comp[q]) continue;
            out.push_back(q);
            for (uint64_t r = (uint64_t)q * q; r <= lim; r += q) comp[r] = 1;
        }
        return out;
    }();
    return tab;
}

constexpr uint64_t kTwo53 = 1ull << 53;
constexpr uint64_t kLowLimit = 1ull << 30;   // p^L must stay below 2^30 (v < 2^31)

uint64_t ipow(uint64_t p, uint32_t e)
{
    uint64_t r = 1;
    while (e--) r *= p;
    return r;
}

uint32_t digits_D(uint64_t p)
{
    uint32_t D = 0;
    uint64_t P = 1;
    while (P <= kTwo53 / p) { P *= p; ++D; }
    return D;
}

uint32_t low_digits(uint64_t p, int64_t S)
{
    uint32_t L = 1;
    uint64_t v = p;
    while ((int64_t)v < S) { v *= p; ++L; }
    return L;
}

// Geometry of the index range: segment length S (power of two, >= 256 so a
// block never straddles two segments) such that p_j^{L_j} < 2^30 for every
// dimension; S never exceeds the next power of two of N.
struct Geometry {
    int64_t S = 0;
    int log2S = 0;
    int n_seg = 0;
};

bool choose_geometry(int s, int64_t N, Geometry &g)
{
    const auto &pr = primes();
    int64_t S = 256;
    int lg = 8;
    while (S < N && S < (int64_t)kLowLimit) { S <<= 1; ++lg; }
    auto ok = [&](int64_t SS) {
        for (int j = 0; j < s; ++j) {
            uint64_t p = pr[j];
            if (ipow(p, low_digits(p, SS)) >= kLowLimit) return false;
        }
        return true;
    };
    while (S > 256 && !ok(S)) { S >>= 1; --lg; }
    if (!ok(S)) return false;
    g.S = S;
    g.log2S = lg;
    g.n_seg = (int)((N + S - 1) / S);
    return true;
}

// 1/p rounded toward +infinity.
double inv_up(uint64_t p)
{
    double r = 1.0 / (double)p;
    if (std::fma(r, (double)p, -1.0) < 0.0) r = std::nextafter(r, INFINITY);
    return r;
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), random access by counter.
uint64_t sm64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Uniform on [0, range) by rejection from counters ctr0, ctr0+1, ...
bool uniform_below(uint64_t seed, uint64_t ctr0, uint64_t range, uint64_t &out)
{
    const uint64_t rem = (0ull - range) % range;
    for (uint64_t a = 0; a < 64; ++a) {
        const uint64_t u = sm64_at(seed, ctr0 + a);
        if (rem == 0 || u < 0ull - rem) { out = u % range; return true; }
    }
    return false;
}

// Host tables of the point geometry: BaseEnt[s] followed (when permuted)
// by the packed u16 permutations.  Fisher-Yates per base from the
// identity: step t = p-1..1 swaps sigma[t] and sigma[r], r uniform on
// [0, t] with counters 2^60 + (j*65536 + t)*64 + attempt (t < p < 65536).
struct PointTables {
    std::vector<BaseEnt> base;
    std::vector<uint16_t> perm;
};

rq_status build_point_tables(int s, const Geometry &g, uint64_t seed, int flags, PointTables &t)
{
    const auto &pr = primes();
    t.base.resize(s);
    uint32_t off = 0;
    for (int j = 0; j < s; ++j) {
        const uint64_t p = pr[j];
        BaseEnt &b = t.base[j];
        std::memset(&b, 0, sizeof b);
        b.p = (uint32_t)p;
        b.D = digits_D(p);
        b.L = low_digits(p, g.S);
        b.pL = (uint32_t)ipow(p, b.L);
        b.P = ipow(p, b.D);
        b.pDL = ipow(p, b.D - b.L);
        b.pd = (double)p;
        b.invp_up = inv_up(p);
        b.pDLd = (double)b.pDL;
        b.Pd = (double)b.P;
        b.invP = 1.0 / b.Pd;
        b.perm_off = off;
        if (flags & (RQ_PERM_RANDOM | RQ_PERM_PER_REP)) off += (uint32_t)p;
    }
    if (flags & RQ_PERM_RANDOM) {
        t.perm.resize(off);
        for (int j = 0; j < s; ++j) {
            const uint32_t p = t.base[j].p;
            uint16_t *sg = t.perm.data() + t.base[j].perm_off;
            for (uint32_t a = 0; a < p; ++a) sg[a] = (uint16_t)a;
            for (uint32_t st = p - 1; st >= 1; --st) {
                uint64_t r;
                const uint64_t ctr = (1ull << 60) + ((uint64_t)j * 65536ull + st) * 64ull;
                if (!uniform_below(seed, ctr, (uint64_t)st + 1, r))
                    return fail(RQ_ERANGE, "permutation draw exhausted its attempts");
                std::swap(sg[st], sg[r]);
            }
        }
    }
    return RQ_OK;
}

// Workspace layout.  Region offsets are 256-byte aligned.  Per-replication
// permutations (rperm, [M][sum of the primes]) are generated on the device.
struct Layout {
    size_t base = 0, perm = 0, model = 0, starts = 0, rperm = 0, partial = 0, total = 0;
    size_t host_bytes = 0;   // bytes staged from the host (base | perm | model)
    int64_t perm_stride = 0; // per-replication table length (elements)
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout(int s, const Geometry &g, int M, int flags, size_t model_bytes, size_t partial_bytes)
{
    Layout L;
    const auto &pr = primes();
    size_t perm_elems = 0;
    if (flags & RQ_PERM_RANDOM)
        for (int j = 0; j < s; ++j) perm_elems += pr[j];
    L.base = 0;
    L.perm = al(sizeof(BaseEnt) * (size_t)s);
    L.model = L.perm + al(perm_elems * sizeof(uint16_t));
    L.host_bytes = L.model + model_bytes;
    L.starts = al(L.host_bytes);
    L.rperm = L.starts + al(sizeof(StartEnt) * (size_t)M * (size_t)g.n_seg * (size_t)s);
    size_t rperm_bytes = 0;
    if (flags & RQ_PERM_PER_REP) {
        for (int j = 0; j < s; ++j) L.perm_stride += pr[j];
        rperm_bytes = (size_t)M * (size_t)L.perm_stride * sizeof(uint16_t);
    }
    L.partial = L.rperm + al(rperm_bytes);
    L.total = L.partial + al(partial_bytes);
    return L;
}

rq_status check_common(int s, int64_t N, int M, int flags, int64_t m_offset, Geometry &g)
{
    if (s < 1) return fail(RQ_EINVAL, "s must be >= 1 (got %d)", s);
    if (N < 1) return fail(RQ_EINVAL, "N must be >= 1 (got %lld)", (long long)N);
    if (M < 1) return fail(RQ_EINVAL, "M must be >= 1 (got %d)", M);
    if (m_offset < 0) return fail(RQ_EINVAL, "m_offset must be >= 0");
    if (flags & ~(RQ_START_ZERO | RQ_PERM_RANDOM | RQ_OUT_DIGITS | RQ_MC_PHILOX | RQ_LMM_EULER | RQ_PERM_PER_REP))
        return fail(RQ_EINVAL, "unknown flag bits 0x%x", flags);
    const bool mc = (flags & RQ_MC_PHILOX) != 0;
    if (mc && (flags & (RQ_START_ZERO | RQ_PERM_RANDOM | RQ_OUT_DIGITS | RQ_PERM_PER_REP)))
        return fail(RQ_EINVAL, "RQ_MC_PHILOX excludes RQ_START_ZERO, RQ_PERM_RANDOM, RQ_PERM_PER_REP and RQ_OUT_DIGITS");
    if ((flags & RQ_PERM_RANDOM) && (flags & RQ_PERM_PER_REP))
        return fail(RQ_EINVAL, "RQ_PERM_RANDOM and RQ_PERM_PER_REP are alternatives");
    if (s > RQ_MAX_DIM) return fail(RQ_ERANGE, "s = %d beyond the %d supported bases", s, RQ_MAX_DIM);
    if (m_offset + (int64_t)M > RQ_MAX_REPLICATION)
        return fail(RQ_ERANGE, "m_offset + M beyond 2^40");
    const auto &pr = primes();
    for (int j = 0; j < s && !mc; ++j) {
        const uint64_t P = ipow(pr[j], digits_D(pr[j]));
        if ((uint64_t)N > P)
            return fail(RQ_ERANGE, "N = %lld exceeds P_%d = %llu (base %u)", (long long)N, j,
                        (unsigned long long)P, pr[j]);
    }
    if (!choose_geometry(s, N, g)) return fail(RQ_ERANGE, "no segment length fits s = %d", s);
    return RQ_OK;
}

rq_status check_ws(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws) return fail(RQ_EINVAL, "workspace pointer is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RQ_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(RQ_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return RQ_OK;
}

// Stage the host tables, then run the setup kernel.
rq_status stage_and_setup(const PointTables &pt, const std::vector<uint8_t> &model, const Layout &L,
                          const Geometry &g, int s, int M, uint64_t seed, int64_t m_offset,
                          int flags, uint8_t *ws, hipStream_t st)
{
    std::vector<uint8_t> host(L.host_bytes, 0);
    std::memcpy(host.data() + L.base, pt.base.data(), sizeof(BaseEnt) * pt.base.size());
    if (!pt.perm.empty())
        std::memcpy(host.data() + L.perm, pt.perm.data(), pt.perm.size() * sizeof(uint16_t));
    if (!model.empty()) std::memcpy(host.data() + L.model, model.data(), model.size());
    RQ_HIP(hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, st));
    rq::SetupArgs a;
    a.base_dev = reinterpret_cast<BaseEnt *>(ws + L.base);
    a.starts = reinterpret_cast<StartEnt *>(ws + L.starts);
    a.perm = (flags & RQ_PERM_RANDOM) ? reinterpret_cast<const uint16_t *>(ws + L.perm) : nullptr;
    a.perm_stride = 0;
    if (flags & RQ_PERM_PER_REP) {   // each replication's permutations, drawn on the device
        rq::PermArgs pa;
        pa.table = reinterpret_cast<uint16_t *>(ws + L.rperm);
        pa.base = reinterpret_cast<const BaseEnt *>(ws + L.base);
        pa.seed = seed;
        pa.m_offset = m_offset;
        pa.stride = L.perm_stride;
        pa.s = s;
        pa.M = M;
        RQ_HIP(rq::launch_perm(pa, st));
        a.perm = pa.table;
        a.perm_stride = L.perm_stride;
    }
    a.seed = seed;
    a.m_offset = m_offset;
    a.s = s;
    a.M = M;
    a.n_seg = g.n_seg;
    a.S = g.S;
    a.flags = flags;
    if (!(flags & RQ_MC_PHILOX)) RQ_HIP(rq::launch_setup(a, st));   // pseudo-random points need no starts
    return RQ_OK;
}

rq::SeqGeom seq_geom(const Layout &L, const Geometry &g, uint8_t *ws, int s, int M, int64_t N, int flags,
                     uint64_t seed, int64_t m_offset)
{
    rq::SeqGeom sg;
    sg.base = reinterpret_cast<const BaseEnt *>(ws + L.base);
    sg.starts = reinterpret_cast<const StartEnt *>(ws + L.starts);
    sg.perm = (flags & RQ_PERM_RANDOM) ? reinterpret_cast<const uint16_t *>(ws + L.perm) : nullptr;
    sg.perm_stride = 0;
    if (flags & RQ_PERM_PER_REP) {
        sg.perm = reinterpret_cast<const uint16_t *>(ws + L.rperm);
        sg.perm_stride = L.perm_stride;
    }
    sg.s = s;
    sg.M = M;
    sg.n_seg = g.n_seg;
    sg.perm_on = (flags & (RQ_PERM_RANDOM | RQ_PERM_PER_REP)) ? 1 : 0;
    sg.mc = (flags & RQ_MC_PHILOX) ? 1 : 0;
    sg.seed = seed;
    sg.m_offset = m_offset;
    sg.N = N;
    sg.S = g.S;
    sg.log2S = g.log2S;
    return sg;
}

// ---- LIBOR model -----------------------------------------------------------

rq_status check_lmm(const rq_lmm_model *m)
{
    if (!m) return fail(RQ_EINVAL, "model is NULL");
    if (!m->L0 || !m->sigma || !m->loadings || !m->strike)
        return fail(RQ_EINVAL, "model arrays must not be NULL");
    if (m->n_fwd < 1) return fail(RQ_EINVAL, "n_fwd must be >= 1");
    if (m->n_factors < 1) return fail(RQ_EINVAL, "n_factors must be >= 1");
    if (m->n_fwd > RQ_MAX_FWD) return fail(RQ_EUNSUPPORTED, "n_fwd = %d > %d", m->n_fwd, RQ_MAX_FWD);
    if (m->n_factors > RQ_MAX_FACTORS)
        return fail(RQ_EUNSUPPORTED, "n_factors = %d > %d", m->n_factors, RQ_MAX_FACTORS);
    if (!(m->delta > 0.0) || !std::isfinite(m->delta)) return fail(RQ_EINVAL, "delta must be > 0");
    for (int n = 0; n <= m->n_fwd; ++n)
        if (!(m->L0[n] > 0.0) || !std::isfinite(m->L0[n]))
            return fail(RQ_EINVAL, "L0[%d] = %g must be finite and > 0", n, m->L0[n]);
    for (int n = 1; n <= m->n_fwd; ++n)
        if (!(m->sigma[n] >= 0.0) || !std::isfinite(m->sigma[n]))
            return fail(RQ_EINVAL, "sigma[%d] = %g must be finite and >= 0", n, m->sigma[n]);
    for (int n = 0; n < m->n_fwd; ++n) {
        double q = 0.0;
        for (int f = 0; f < m->n_factors; ++f) {
            const double b = m->loadings[(size_t)n * m->n_factors + f];
            if (!std::isfinite(b)) return fail(RQ_EINVAL, "loadings[%d] not finite", n);
            q += b * b;
        }
        if (std::fabs(std::sqrt(q) - 1.0) > 1e-9)
            return fail(RQ_EINVAL, "loadings row %d has norm %.17g, must be 1", n, std::sqrt(q));
        const double K = m->strike[n];
        if (!std::isnan(K) && !std::isfinite(K)) return fail(RQ_EINVAL, "strike[%d] infinite", n);
    }
    return RQ_OK;
}

// Table rows: every table has kMaxFwd rows, the rows beyond n_fwd zero (the
// kernels read up to their compile-time capacity without per-forward
// guards).
int lmm_rows(int) { return rq::kMaxFwd; }

// kappa_n = 1 / (delta L_n(0)) in T, the drift factor's constant; held finite
// (a product with it then never forms 0 x inf)
template <typename T>
T inv_dl(double delta, double L0)
{
    return (T)std::min(1.0 / (delta * L0), (double)std::numeric_limits<T>::max());
}

// Forward tables: FP64 rows then FP32 rows (layout in rq_internal.h).
std::vector<uint8_t> lmm_table(const rq_lmm_model *m)
{
    const int nf = m->n_fwd, d = m->n_factors;
    const int nrow = lmm_rows(nf);
    const double log2e = 1.4426950408889634074;
    std::vector<double> t((size_t)nrow * rq::kFwdRow, 0.0);
    std::vector<float> f32((size_t)nrow * rq::kRow32, 0.0f);
    for (int n = 1; n <= nf; ++n) {
        double *r = &t[(size_t)(n - 1) * rq::kFwdRow];
        float *q = &f32[(size_t)(n - 1) * rq::kRow32];
        double an2 = 0.0;
        for (int f = 0; f < d; ++f) {
            const double a = m->sigma[n] * m->loadings[(size_t)(n - 1) * d + f];
            r[f] = a;
            r[3 + f] = m->delta * a;
            an2 += a * a;
            q[f] = (float)(log2e * a);
            q[3 + f] = (float)(m->delta * a);
        }
        r[6] = -0.5 * an2 * m->delta;
        r[7] = m->L0[n];
        const double K = m->strike[n - 1];
        r[8] = std::isnan(K) ? 0.0 : K;
        r[9] = std::isnan(K) ? 0.0 : 1.0;
        r[10] = 1.0 / (m->L0[n] * 0.69314718055994530942);
        r[11] = 1.0 / std::max(m->sigma[n], rq::kMinSigma);
        q[6] = (float)(log2e * r[6]);
        q[7] = inv_dl<float>(m->delta, m->L0[n]);
    }
    std::vector<uint8_t> out(t.size() * sizeof(double) + f32.size() * sizeof(float));
    std::memcpy(out.data(), t.data(), t.size() * sizeof(double));
    std::memcpy(out.data() + t.size() * sizeof(double), f32.data(), f32.size() * sizeof(float));
    return out;
}

int lmm_blocks(int64_t N) { return (int)((N + rq::kBlock - 1) / rq::kBlock); }
int adj_blocks(int64_t N) { return (int)((N + rq::kAdjBlockHost - 1) / rq::kAdjBlockHost); }

// Adjoint table (layout in rq_internal.h) in the kernel's precision.
template <typename T>
std::vector<uint8_t> adj_table(const rq_lmm_model *m)
{
    const int nf = m->n_fwd, d = m->n_factors;
    const double log2e = 1.4426950408889634074;
    std::vector<T> t((size_t)lmm_rows(nf) * rq::kAdjRow, T(0));
    for (int n = 1; n <= nf; ++n) {
        T *r = &t[(size_t)(n - 1) * rq::kAdjRow];
        const double sg = std::max(m->sigma[n], rq::kMinSigma);
        double a2 = 0.0;
        for (int f = 0; f < d; ++f) {
            const double a = sg * m->loadings[(size_t)(n - 1) * d + f];
            r[f] = (T)(log2e * a);
            r[3 + f] = (T)(m->delta * a);
            a2 += a * a;
        }
        r[6] = (T)(log2e * (-0.5 * a2 * m->delta));
        r[7] = inv_dl<T>(m->delta, m->L0[n]);
    }
    std::vector<uint8_t> out(t.size() * sizeof(T));
    std::memcpy(out.data(), t.data(), out.size());
    return out;
}

// ---- MBS model ---------------------------------------------------------------

rq_status check_mbs(const rq_mbs_params *p)
{
    if (!p) return fail(RQ_EINVAL, "params is NULL");
    if (p->months < 1) return fail(RQ_EINVAL, "months must be >= 1");
    if (p->months > RQ_MAX_MONTHS) return fail(RQ_ERANGE, "months = %d > %d", p->months, RQ_MAX_MONTHS);
    if (!(p->i0 > 0.0) || !std::isfinite(p->i0)) return fail(RQ_EINVAL, "i0 must be > 0");
    if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) return fail(RQ_EINVAL, "sigma must be >= 0");
    if (!std::isfinite(p->K1) || !std::isfinite(p->K2) || !std::isfinite(p->K3) || !std::isfinite(p->K4))
        return fail(RQ_EINVAL, "K1..K4 must be finite");
    return RQ_OK;
}

// c_k = sum_{j=0}^{K-k} (1+i0)^{-j} for k = 0..K (geometric series), then
// dc_k/di0 = sum_{j=1}^{K-k} -j (1+i0)^{-j-1}.
std::vector<uint8_t> mbs_table(const rq_mbs_params *p)
{
    const int K = p->months;
    std::vector<double> ck(2 * (size_t)(K + 1), 0.0);
    const double v = 1.0 / (1.0 + p->i0);
    // accumulate from the end: c_K = 1, c_k = 1 + v c_{k+1};
    // dc_K = 0, dc_k = v (dc_{k+1} - v c_{k+1})  (since dv/di0 = -v^2)
    ck[K] = 1.0;
    double *dck = ck.data() + (K + 1);
    dck[K] = 0.0;
    for (int k = K - 1; k >= 1; --k) {
        ck[k] = 1.0 + v * ck[k + 1];
        dck[k] = v * dck[k + 1] - v * v * ck[k + 1];
    }
    std::vector<uint8_t> out(ck.size() * sizeof(double));
    std::memcpy(out.data(), ck.data(), out.size());
    return out;
}

// Model scalars of the MBS kernel arguments: K0, the level payment c and
// its derivative dc/di0.
void mbs_scalars(const rq_mbs_params *params, rq::MbsArgs &a)
{
    a.i0 = params->i0;
    a.sig = params->sigma;
    a.K0 = std::exp(-0.5 * params->sigma * params->sigma);
    a.K1 = params->K1;
    a.K2 = params->K2;
    a.K3 = params->K3;
    a.K4 = params->K4;
    const double vK = std::pow(1.0 + params->i0, -(double)params->months);
    a.c = params->i0 / (1.0 - vK);
    // dc/di0 with dv/di0 = -K (1+i0)^{-K-1}
    const double dvK = -params->months * vK / (1.0 + params->i0);
    a.dc = ((1.0 - vK) + params->i0 * dvK) / ((1.0 - vK) * (1.0 - vK));
}

rq_status finish(const rq_result *out, const double *partial, int stride, int off, int M, int n_blk,
                 int n_out, int64_t N, hipStream_t st)
{
    rq::ReduceArgs r;
    r.partial = partial;
    r.theta = out->theta;
    r.M = M;
    r.n_blk = n_blk;
    r.n_out = n_out;
    r.stride = stride;
    r.off = off;
    r.Nd = (double)N;
    RQ_HIP(rq::launch_reduce(r, st));
    if (out->mean || out->sd || out->se) {
        rq::FinalizeArgs f;
        f.theta = out->theta;
        f.mean = out->mean;
        f.sd = out->sd;
        f.se = out->se;
        f.M = M;
        f.n_out = n_out;
        RQ_HIP(rq::launch_finalize(f, st));
    }
    return RQ_OK;
}

// ---- batch of instruments ------------------------------------------------------

// Per-instrument plan: validated shape, tables and workspace offsets.
struct InstPlan {
    int kind = 0, s = 0, D = 0, nf = 0, months = 0;
    int64_t N = 0;
    int M = 0;
    uint64_t seed = 0;
    int64_t m_offset = 0;
    int flags = 0;
    Geometry g;
    int n_blk = 0, n_out = 0, n_g = 0;   // n_g: Greek outputs per replication
    double cost = 0.0;
    size_t perm_elems = 0, model_bytes = 0, adj_off = 0;
    size_t o_base = 0, o_perm = 0, o_model = 0, o_starts = 0, o_part = 0, part_g = 0;
    int64_t setup_units = 0;
};

struct BatchPlan {
    std::vector<InstPlan> ip;   // caller order
    std::vector<int> order;     // execution position -> caller index
    int n_red = 0;              // reduce / finalize entries
    size_t o_inst = 0, o_item0 = 0, o_setup = 0, o_setup_pf = 0, o_red = 0, o_red_pf = 0, o_fin = 0,
           o_fin_pf = 0, o_queue = 0;
    size_t host_bytes = 0, o_store = 0, store_bytes = 0, total = 0;
    int64_t n_items = 0, setup_total = 0, red_blocks = 0;
    bool any_lmm = false;
};

constexpr int kBatchMaxInst = 1 << 16;

rq_status plan_batch(const rq_instrument *inst, int n_inst, rq_precision prec, bool greeks, int order,
                     BatchPlan &bp)
{
    if (!inst) return fail(RQ_EINVAL, "instrument list is NULL");
    if (n_inst < 1 || n_inst > kBatchMaxInst) return fail(RQ_ERANGE, "n_inst = %d outside [1, %d]", n_inst, kBatchMaxInst);
    if (prec != RQ_FP64 && prec != RQ_FP32) return fail(RQ_EINVAL, "unknown precision %d", (int)prec);
    if (order != RQ_ORDER_COST && order != RQ_ORDER_GIVEN) return fail(RQ_EINVAL, "unknown order %d", order);
    const auto &pr = primes();
    bp.ip.assign(n_inst, InstPlan());
    for (int k = 0; k < n_inst; ++k) {
        const rq_instrument &I = inst[k];
        InstPlan &p = bp.ip[k];
        rq_status st;
        p.kind = I.kind;
        p.N = I.N;
        p.M = I.M;
        p.seed = I.seed;
        p.m_offset = I.m_offset;
        p.flags = I.flags;
        if (I.flags & RQ_OUT_DIGITS) return fail(RQ_EINVAL, "instrument %d: RQ_OUT_DIGITS applies to rq_sequence only", k);
        if (I.flags & RQ_LMM_EULER)
            return fail(RQ_EUNSUPPORTED, "instrument %d: the batch runs the log-Euler scheme only", k);
        if (I.flags & RQ_PERM_PER_REP)
            return fail(RQ_EUNSUPPORTED, "instrument %d: the batch uses shared permutations only", k);
        if (I.kind == RQ_INST_LMM) {
            if ((st = check_lmm(I.lmm))) return fail(st, "instrument %d: %s", k, g_err.c_str());
            p.nf = I.lmm->n_fwd;
            p.D = I.lmm->n_factors;
            p.s = p.nf * p.D;
            p.n_out = p.nf + 1;
            p.n_g = greeks ? 2 * p.nf + 1 : 0;
            const double fs = 0.5 * p.nf * (p.nf + 1.0);
            p.cost = fs * (6.0 * p.D + 8.0) * (greeks ? 3.0 : 1.0) + p.s * 40.0;
            bp.any_lmm = true;
        } else if (I.kind == RQ_INST_MBS) {
            if ((st = check_mbs(I.mbs))) return fail(st, "instrument %d: %s", k, g_err.c_str());
            p.months = I.mbs->months;
            p.s = p.months;
            p.n_out = 1;
            p.n_g = greeks ? 1 : 0;
            p.cost = p.months * (greeks ? 110.0 : 80.0);
        } else {
            return fail(RQ_EINVAL, "instrument %d: unknown kind %d", k, I.kind);
        }
        if ((st = check_common(p.s, p.N, p.M, p.flags, p.m_offset, p.g)))
            return fail(st, "instrument %d: %s", k, g_err.c_str());
        p.n_blk = (int)((p.N + rq::kWave - 1) / rq::kWave);
        if ((int64_t)p.n_blk * p.M >= (1ll << 31)) return fail(RQ_ERANGE, "instrument %d: N*M too large", k);
        p.cost *= (double)p.N * (double)p.M;
        p.perm_elems = 0;
        if (p.flags & RQ_PERM_RANDOM)
            for (int j = 0; j < p.s; ++j) p.perm_elems += pr[j];
        if (p.kind == RQ_INST_LMM) {
            const size_t rows = (size_t)lmm_rows(p.nf);
            p.adj_off = rows * (rq::kFwdRow * sizeof(double) + rq::kRow32 * sizeof(float));
            p.model_bytes = p.adj_off + rows * rq::kAdjRow * (prec == RQ_FP32 ? sizeof(float) : sizeof(double));
        } else {
            p.model_bytes = 2 * (size_t)(p.months + 1) * sizeof(double);
        }
        p.setup_units = (p.flags & RQ_MC_PHILOX) ? 0 : (int64_t)p.M * p.g.n_seg * p.s;
    }
    bp.order.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) bp.order[k] = k;
    if (order == RQ_ORDER_COST)   // largest first (LPT); ties keep the caller's order
        std::stable_sort(bp.order.begin(), bp.order.end(),
                         [&](int x, int y) { return bp.ip[x].cost > bp.ip[y].cost; });
    // reduce / finalize entries: prices of every instrument, then Greeks
    bp.n_red = n_inst * (greeks ? 2 : 1);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += al(bytes); return at; };
    bp.o_inst = take(sizeof(rq::BatchInst) * n_inst);
    bp.o_item0 = take(sizeof(int64_t) * (n_inst + 1));
    bp.o_setup = take(sizeof(rq::SetupArgs) * n_inst);
    bp.o_setup_pf = take(sizeof(int64_t) * (n_inst + 1));
    bp.o_red = take(sizeof(rq::ReduceArgs) * bp.n_red);
    bp.o_red_pf = take(sizeof(int64_t) * (bp.n_red + 1));
    bp.o_fin = take(sizeof(rq::FinalizeArgs) * bp.n_red);
    bp.o_fin_pf = take(sizeof(int64_t) * (bp.n_red + 1));
    bp.o_queue = take(sizeof(unsigned long long));
    for (int k = 0; k < n_inst; ++k) {
        InstPlan &p = bp.ip[k];
        p.o_base = take(sizeof(BaseEnt) * (size_t)p.s);
        p.o_perm = take(p.perm_elems * sizeof(uint16_t));
        p.o_model = take(p.model_bytes);
    }
    bp.host_bytes = o;
    bp.n_items = 0;
    bp.setup_total = 0;
    bp.red_blocks = 0;
    for (int k = 0; k < n_inst; ++k) {
        InstPlan &p = bp.ip[k];
        p.o_starts = take(sizeof(StartEnt) * (size_t)p.setup_units);
        const size_t rows = (size_t)p.M * p.n_blk;
        if (p.kind == RQ_INST_LMM) {
            p.o_part = take(rows * (p.n_out + p.n_g) * sizeof(double));
            p.part_g = rows * p.n_out;   // Greek rows follow the price rows
        } else {
            p.o_part = take(rows * (greeks ? 2 : 1) * sizeof(double));
        }
        bp.n_items += (int64_t)rows;
        bp.setup_total += p.setup_units;
        bp.red_blocks += (int64_t)p.M * (greeks ? 2 : 1);
    }
    // Greeks: the window store, one slot per item of a window, FP64-counted
    // so that the size does not depend on the precision (FP32 windows hold
    // twice the items)
    bp.store_bytes = 0;
    if (greeks && bp.any_lmm) {
        const size_t per = (size_t)rq::kBatchItemElems * sizeof(double);
        const int64_t fit = std::max<int64_t>(1, (int64_t)(g_adj_store_limit.load() / per));
        bp.store_bytes = (size_t)std::min<int64_t>(bp.n_items, fit) * per;
    }
    bp.o_store = take(bp.store_bytes);
    bp.total = o;
    return RQ_OK;
}

int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

// ---- the autotuner's choices, kept per batch signature ---------------------
// The signature covers what decides the time of a batch: the precision, the
// Greeks, and per instrument its kind, shape (forwards and factors, or
// months), N, M and flags (FNV-1a over those fields).  rq_autotune_batch
// stores its choice here, and rq_price_batch without a tuning uses it.  With
// RQ_TUNING_CACHE naming a file, choices are appended to it and the file's
// lines ("signature chunk waves_per_cu order", hexadecimal signature) are
// read on first use, so that they outlive the process.
uint64_t batch_signature(const rq_instrument *inst, int n_inst, rq_precision prec, bool greeks)
{
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)(v >> (8 * b)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    };
    mix(prec);
    mix(greeks ? 1 : 0);
    mix(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const rq_instrument &I = inst[k];
        mix(I.kind);
        mix(I.N);
        mix(I.M);
        mix(I.flags);
        if (I.kind == RQ_INST_LMM && I.lmm) {
            mix(I.lmm->n_fwd);
            mix(I.lmm->n_factors);
        } else if (I.kind == RQ_INST_MBS && I.mbs) {
            mix(I.mbs->months);
        }
    }
    return h;
}

struct TuningCache {
    std::mutex mu;
    bool loaded = false;
    std::vector<std::pair<uint64_t, rq_tuning>> entries;
} g_tuning;

const char *tuning_file() { return std::getenv("RQ_TUNING_CACHE"); }

void tuning_load_locked()
{
    if (g_tuning.loaded) return;
    g_tuning.loaded = true;
    const char *path = tuning_file();
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    unsigned long long sig;
    int c, w, o;
    while (std::fscanf(f, "%llx %d %d %d", &sig, &c, &w, &o) == 4) {
        if (c < 0 || c > 4096 || w < 0 || w > 32 || (o != RQ_ORDER_COST && o != RQ_ORDER_GIVEN)) continue;
        g_tuning.entries.emplace_back((uint64_t)sig, rq_tuning{c, w, o});
    }
    std::fclose(f);
}

bool tuning_find(uint64_t sig, rq_tuning &out)
{
    std::lock_guard<std::mutex> lk(g_tuning.mu);
    tuning_load_locked();
    for (auto it = g_tuning.entries.rbegin(); it != g_tuning.entries.rend(); ++it)   // the latest wins
        if (it->first == sig) {
            out = it->second;
            return true;
        }
    return false;
}

void tuning_store(uint64_t sig, const rq_tuning &t)
{
    std::lock_guard<std::mutex> lk(g_tuning.mu);
    tuning_load_locked();
    g_tuning.entries.emplace_back(sig, t);
    const char *path = tuning_file();
    if (!path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {   // best effort: an unwritable file only loses persistence
        std::fprintf(f, "%016llx %d %d %d\n", (unsigned long long)sig, t.chunk, t.waves_per_cu, t.order);
        std::fclose(f);
    }
}

rq_status run_batch(const rq_instrument *inst, int n_inst, rq_precision prec, bool greeks, const rq_tuning *tuning,
                    const rq_result *outs, const rq_result *grads, uint64_t *t_first, uint64_t *t_last, void *ws,
                    size_t ws_bytes, hipStream_t st)
{
    rq_tuning tu{0, 0, RQ_ORDER_COST};
    rq_tuning cached;
    if (!tuning && inst && n_inst >= 1 && n_inst <= kBatchMaxInst &&
        tuning_find(batch_signature(inst, n_inst, prec, greeks), cached))
        tuning = &cached;
    if (tuning) {
        tu = *tuning;
        if (tu.chunk < 0 || tu.chunk > 4096) return fail(RQ_EINVAL, "tuning.chunk = %d outside [0, 4096]", tu.chunk);
        if (tu.waves_per_cu < 0 || tu.waves_per_cu > 32)
            return fail(RQ_EINVAL, "tuning.waves_per_cu = %d outside [0, 32]", tu.waves_per_cu);
    }
    BatchPlan bp;
    rq_status stt;
    if ((stt = plan_batch(inst, n_inst, prec, greeks, tu.order, bp))) return stt;
    if (!outs) return fail(RQ_EINVAL, "outs is NULL");
    if (greeks && !grads) return fail(RQ_EINVAL, "grads is NULL with Greeks requested");
    if ((t_first == nullptr) != (t_last == nullptr)) return fail(RQ_EINVAL, "t_first and t_last go together");
    for (int k = 0; k < n_inst; ++k) {
        if (!outs[k].theta) return fail(RQ_EINVAL, "outs[%d].theta is NULL", k);
        if (greeks && !grads[k].theta) return fail(RQ_EINVAL, "grads[%d].theta is NULL", k);
    }
    if ((stt = check_ws(ws, ws_bytes, bp.total))) return stt;
    const bool f32 = prec == RQ_FP32;
    const int cus = device_cus();
    if (cus <= 0) return fail(RQ_EHIP, "cannot query the device's compute units");
    // launches: without Greeks one (phase 0) over all items; with Greeks,
    // per window of items, phase 1 (LIBOR forward halves, MBS items) and, if
    // any LIBOR item, phase 2 (LIBOR reverse halves)
    const size_t elem = f32 ? sizeof(float) : sizeof(double);
    const int64_t window = (greeks && bp.any_lmm)
                               ? std::max<int64_t>(1, (int64_t)(bp.store_bytes / ((size_t)rq::kBatchItemElems * elem)))
                               : bp.n_items;
    std::vector<int> phases;
    if (!greeks) phases = {0};
    else if (bp.any_lmm) phases = {1, 2};
    else phases = {1};
    // blocks per CU: the tuning's value holds for the two-wave kernels
    // (phase 2, or phase 0); phase 1 runs twice as many where it fits
    int occ_of[3] = {0, 0, 0};
    for (int ph : phases) {
        occ_of[ph] = rq::batch_blocks_per_cu(f32, greeks, ph);
        if (occ_of[ph] <= 0) return fail(RQ_EHIP, "occupancy query of the batch kernel failed");
    }
    auto grid_of = [&](int ph, int64_t n_win) {
        int per_cu = occ_of[ph];
        if (tu.waves_per_cu > 0) per_cu = std::min(per_cu, tu.waves_per_cu * (ph == 1 ? 2 : 1));
        return std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, n_win));
    };
    auto chunk_of = [&](int64_t grid, int64_t n_win) {
        if (tu.chunk > 0) return tu.chunk;   // else about 16 grabs per block, at most 8 items a grab
        return (int)std::max<int64_t>(1, std::min<int64_t>(8, n_win / (grid * 16)));
    };

    uint8_t *w = (uint8_t *)ws;
    std::vector<uint8_t> host(bp.host_bytes, 0);
    auto *bi = reinterpret_cast<rq::BatchInst *>(host.data() + bp.o_inst);
    auto *item0 = reinterpret_cast<int64_t *>(host.data() + bp.o_item0);
    auto *sa = reinterpret_cast<rq::SetupArgs *>(host.data() + bp.o_setup);
    auto *spf = reinterpret_cast<int64_t *>(host.data() + bp.o_setup_pf);
    auto *ra = reinterpret_cast<rq::ReduceArgs *>(host.data() + bp.o_red);
    auto *rpf = reinterpret_cast<int64_t *>(host.data() + bp.o_red_pf);
    auto *fa = reinterpret_cast<rq::FinalizeArgs *>(host.data() + bp.o_fin);
    auto *fpf = reinterpret_cast<int64_t *>(host.data() + bp.o_fin_pf);
    int64_t items = 0, su = 0, rb = 0, fu = 0;
    for (int e = 0; e < n_inst; ++e) {
        const int k = bp.order[e];
        const InstPlan &p = bp.ip[k];
        const rq_instrument &I = inst[k];
        // host tables of this instrument
        PointTables pt;
        if ((stt = build_point_tables(p.s, p.g, p.seed, p.flags, pt))) return fail(stt, "instrument %d: %s", k, g_err.c_str());
        std::memcpy(host.data() + p.o_base, pt.base.data(), sizeof(BaseEnt) * pt.base.size());
        if (!pt.perm.empty()) std::memcpy(host.data() + p.o_perm, pt.perm.data(), pt.perm.size() * sizeof(uint16_t));
        std::vector<uint8_t> tab;
        if (p.kind == RQ_INST_LMM) {
            tab = lmm_table(I.lmm);
            tab.resize(p.adj_off, 0);
            std::vector<uint8_t> at = f32 ? adj_table<float>(I.lmm) : adj_table<double>(I.lmm);
            tab.insert(tab.end(), at.begin(), at.end());
        } else {
            tab = mbs_table(I.mbs);
        }
        std::memcpy(host.data() + p.o_model, tab.data(), std::min(tab.size(), p.model_bytes));
        // geometry of the points, shared by both kinds
        Layout L;
        L.base = p.o_base;
        L.perm = p.o_perm;
        L.model = p.o_model;
        L.starts = p.o_starts;
        L.partial = p.o_part;
        const rq::SeqGeom sg = seq_geom(L, p.g, w, p.s, p.M, p.N, p.flags, p.seed, p.m_offset);
        rq::BatchInst &d = bi[e];
        std::memset(&d, 0, sizeof d);
        d.kind = p.kind;
        d.n_factors = p.D;
        d.slot = k;
        double *part = reinterpret_cast<double *>(w + p.o_part);
        if (p.kind == RQ_INST_LMM) {
            rq::LmmArgs &a = d.lmm;
            a.g = sg;
            a.fwd = reinterpret_cast<const double *>(w + p.o_model);
            a.fwd32 = reinterpret_cast<const float *>(w + p.o_model + (size_t)lmm_rows(p.nf) * rq::kFwdRow * sizeof(double));
            a.adj = w + p.o_model + p.adj_off;
            a.wtop = nullptr;   // the batch kernel passes each item's slot of the window store
            a.xs = nullptr;
            a.task0 = 0;
            a.chunk = 0;
            a.n_slots = 0;
            a.partial = part;
            a.partial_g = greeks ? part + p.part_g : nullptr;
            a.n_g = p.n_g;
            a.per_path = nullptr;
            a.n_fwd = p.nf;
            a.n_out = p.n_out;
            a.n_blk = p.n_blk;
            a.delta = I.lmm->delta;
            a.sqrt_delta = std::sqrt(I.lmm->delta);
            a.num0 = 1.0 + I.lmm->delta * I.lmm->L0[0];
        } else {
            rq::MbsArgs &a = d.mbs;
            a.g = sg;
            a.ck = reinterpret_cast<const double *>(w + p.o_model);
            a.partial = part;
            a.per_path = nullptr;
            a.months = p.months;
            a.n_blk = p.n_blk;
            a.n_part = greeks ? 2 : 1;
            mbs_scalars(I.mbs, a);
        }
        item0[e] = items;
        items += (int64_t)p.M * p.n_blk;
        // setup of the start table
        rq::SetupArgs &s = sa[e];
        s.base_dev = reinterpret_cast<BaseEnt *>(w + p.o_base);
        s.starts = reinterpret_cast<StartEnt *>(w + p.o_starts);
        s.perm = (p.flags & RQ_PERM_RANDOM) ? reinterpret_cast<const uint16_t *>(w + p.o_perm) : nullptr;
        s.seed = p.seed;
        s.m_offset = p.m_offset;
        s.s = p.s;
        s.M = p.M;
        s.n_seg = p.g.n_seg;
        s.S = p.g.S;
        s.flags = p.flags;
        spf[e] = su;
        su += p.setup_units;
    }
    item0[n_inst] = items;
    spf[n_inst] = su;
    // reductions: prices (caller order), then Greeks
    for (int r = 0; r < bp.n_red; ++r) {
        const int k = r % n_inst;
        const bool gr = r >= n_inst;
        const InstPlan &p = bp.ip[k];
        const rq_result &res = gr ? grads[k] : outs[k];
        const double *part = reinterpret_cast<const double *>(w + p.o_part);
        rq::ReduceArgs &a = ra[r];
        a.theta = res.theta;
        a.M = p.M;
        a.n_blk = p.n_blk;
        a.Nd = (double)p.N;
        if (p.kind == RQ_INST_LMM) {
            a.partial = gr ? part + p.part_g : part;
            a.n_out = gr ? p.n_g : p.n_out;
            a.stride = a.n_out;
            a.off = 0;
        } else {
            a.partial = part;
            a.n_out = 1;
            a.stride = greeks ? 2 : 1;
            a.off = gr ? 1 : 0;
        }
        rpf[r] = rb;
        rb += p.M;
        rq::FinalizeArgs &f = fa[r];
        f.theta = res.theta;
        f.mean = res.mean;
        f.sd = res.sd;
        f.se = res.se;
        f.M = p.M;
        f.n_out = a.n_out;
        fpf[r] = fu;
        if (res.mean || res.sd || res.se) fu += a.n_out;
    }
    rpf[bp.n_red] = rb;
    fpf[bp.n_red] = fu;

    RQ_HIP(hipMemcpyAsync(w, host.data(), host.size(), hipMemcpyHostToDevice, st));
    rq::BatchSetup bs{reinterpret_cast<const rq::SetupArgs *>(w + bp.o_setup),
                      reinterpret_cast<const int64_t *>(w + bp.o_setup_pf), n_inst};
    RQ_HIP(rq::launch_batch_setup(bs, su, st));
    auto *queue = reinterpret_cast<unsigned long long *>(w + bp.o_queue);
    RQ_HIP(rq::launch_batch_init(queue, reinterpret_cast<unsigned long long *>(t_first),
                                 reinterpret_cast<unsigned long long *>(t_last), t_first ? n_inst : 0, st));
    rq::BatchArgs ba;
    ba.inst = reinterpret_cast<const rq::BatchInst *>(w + bp.o_inst);
    ba.item0 = reinterpret_cast<const int64_t *>(w + bp.o_item0);
    ba.n_inst = n_inst;
    ba.chunk = 1;
    ba.n_items = items;
    ba.queue = queue;
    ba.t_first = reinterpret_cast<unsigned long long *>(t_first);
    ba.t_last = reinterpret_cast<unsigned long long *>(t_last);
    ba.n_caller = n_inst;
    ba.store = bp.store_bytes ? (void *)(w + bp.o_store) : nullptr;
    // window cuts: whole instruments where they fit (so that an instrument's
    // two phases run in one window), an instrument larger than a window in
    // full windows of its own
    std::vector<int64_t> cuts{0};
    if (window < items) {
        int64_t start = 0;
        for (int e = 0; e < n_inst; ++e) {
            const int64_t a = item0[e], b = item0[e + 1];
            if (b - start <= window) continue;
            if (a > start) {
                cuts.push_back(a);
                start = a;
            }
            while (b - start > window) {
                start += window;
                cuts.push_back(start);
            }
        }
    }
    if (cuts.back() != items) cuts.push_back(items);
    {
        TimedRegion tr(st);
        for (size_t c = 0; c + 1 < cuts.size(); ++c) {
            const int64_t w0 = cuts[c];
            ba.w0 = w0;
            ba.w1 = cuts[c + 1];
            for (int ph : phases) {
                if (w0 > 0 || ph != phases[0])   // the queue restarts at the window's first item
                    RQ_HIP(rq::launch_batch_init(queue, nullptr, nullptr, 0, st));
                const int64_t grid = grid_of(ph, ba.w1 - ba.w0);
                ba.chunk = chunk_of(grid, ba.w1 - ba.w0);
                RQ_HIP(rq::launch_batch(ba, (int)grid, f32, greeks, ph, st));
            }
        }
    }
    rq::BatchReduce br{reinterpret_cast<const rq::ReduceArgs *>(w + bp.o_red),
                       reinterpret_cast<const int64_t *>(w + bp.o_red_pf), bp.n_red};
    RQ_HIP(rq::launch_batch_reduce(br, rb, st));
    rq::BatchFinalize bf{reinterpret_cast<const rq::FinalizeArgs *>(w + bp.o_fin),
                         reinterpret_cast<const int64_t *>(w + bp.o_fin_pf), bp.n_red};
    RQ_HIP(rq::launch_batch_finalize(bf, fu, st));
    return RQ_OK;
}

}  // namespace

// =============================================================================
extern "C" {

const char *rq_last_error(void) { return g_err.c_str(); }

const char *rq_version(void) { return "rqmc-mi355x 0.1 (gfx950)"; }

rq_status rq_inv_normal(int64_t n, const double *u, void *z, rq_precision prec, void *stream)
{
    if (n < 0) return fail(RQ_EINVAL, "n must be >= 0");
    if (n == 0) return RQ_OK;
    if (!u || !z) return fail(RQ_EINVAL, "u and z must not be NULL");
    if (prec != RQ_FP64 && prec != RQ_FP32) return fail(RQ_EINVAL, "unknown precision %d", (int)prec);
    if ((n + 255) / 256 >= (1ll << 31)) return fail(RQ_ERANGE, "n too large for one launch");
    RQ_HIP(rq::launch_inv_normal(n, u, z, prec == RQ_FP32, (hipStream_t)stream));
    return RQ_OK;
}

rq_status rq_timer_begin(int max_launches)
{
    if (max_launches < 1 || max_launches > 100000) return fail(RQ_EINVAL, "max_launches out of range");
    std::lock_guard<std::mutex> lk(g_timer.mu);
    if (g_timer.on) return fail(RQ_EINVAL, "timer already running");
    g_timer.ev.assign(2 * (size_t)max_launches * kTimerPairsPerLaunch, nullptr);
    g_timer.tag.assign((size_t)max_launches * kTimerPairsPerLaunch, 0);
    for (auto &e : g_timer.ev) {
        hipError_t h = hipEventCreate(&e);
        if (h != hipSuccess) {
            for (auto &x : g_timer.ev) if (x) (void)hipEventDestroy(x);
            g_timer.ev.clear();
            return fail(RQ_EHIP, "hipEventCreate failed: %s", hipGetErrorString(h));
        }
    }
    g_timer.used = 0;
    g_timer.record_failed = false;
    g_timer.on = true;
    return RQ_OK;
}

rq_status rq_timer_end(double *total_ms, int *n_launches)
{
    std::lock_guard<std::mutex> lk(g_timer.mu);
    if (!g_timer.on) return fail(RQ_EINVAL, "timer not running");
    g_timer.on = false;
    rq_status st = RQ_OK;
    for (int t = 0; t < kTimerTags; ++t) {
        g_timer.part_ms[t] = 0.0;
        g_timer.part_n[t] = 0;
    }
    for (size_t q = 0; q < g_timer.used; ++q) {
        float ms = 0.0f;
        hipError_t h = hipEventSynchronize(g_timer.ev[2 * q + 1]);
        if (h == hipSuccess) h = hipEventElapsedTime(&ms, g_timer.ev[2 * q], g_timer.ev[2 * q + 1]);
        if (h != hipSuccess && st == RQ_OK) st = fail(RQ_EHIP, "event timing failed: %s", hipGetErrorString(h));
        g_timer.part_ms[g_timer.tag[q]] += ms;
        ++g_timer.part_n[g_timer.tag[q]];
    }
    for (auto &e : g_timer.ev) (void)hipEventDestroy(e);
    g_timer.ev.clear();
    if (g_timer.record_failed && st == RQ_OK) st = fail(RQ_EHIP, "recording a timing event failed");
    if (total_ms) *total_ms = g_timer.part_ms[0];
    if (n_launches) *n_launches = g_timer.part_n[0];
    return st;
}

rq_status rq_timer_part(int part, double *total_ms, int *n_launches)
{
    std::lock_guard<std::mutex> lk(g_timer.mu);
    if (part < 1 || part >= kTimerTags) return fail(RQ_EINVAL, "part must be 1 or 2");
    if (g_timer.on) return fail(RQ_EINVAL, "timer still running");
    if (total_ms) *total_ms = g_timer.part_ms[part];
    if (n_launches) *n_launches = g_timer.part_n[part];
    return RQ_OK;
}

size_t rq_sequence_workspace(int s, int64_t N, int M, int flags)
{
    Geometry g;
    if (check_common(s, N, M, flags, 0, g) != RQ_OK) return 0;
    return layout(s, g, M, flags, 0, 0).total;
}

rq_status rq_sequence(int s, int64_t N, int M, uint64_t seed, int flags, int64_t m_offset, void *out,
                      void *ws, size_t ws_bytes, void *stream)
{
    Geometry g;
    if (flags & RQ_LMM_EULER) return fail(RQ_EINVAL, "RQ_LMM_EULER applies to rq_price_caplets only");
    rq_status stt = check_common(s, N, M, flags, m_offset, g);
    if (stt) return stt;
    if (!out) return fail(RQ_EINVAL, "out is NULL");
    const Layout L = layout(s, g, M, flags, 0, 0);
    if ((stt = check_ws(ws, ws_bytes, L.total))) return stt;
    PointTables pt;
    if ((stt = build_point_tables(s, g, seed, flags, pt))) return stt;
    hipStream_t st = (hipStream_t)stream;
    uint8_t *w = (uint8_t *)ws;
    if ((stt = stage_and_setup(pt, {}, L, g, s, M, seed, m_offset, flags, w, st))) return stt;
    {
        TimedRegion tr(st);
        RQ_HIP(rq::launch_sequence(seq_geom(L, g, w, s, M, N, flags, seed, m_offset), flags, out, st));
    }
    return RQ_OK;
}

// Single-call adjoint: per 64-path task, the stored step-final w
// ([n_fwd][d][64]) and final states ([NFC][64], NFC = n_fwd rounded up to 16)
// in elements; the store region holds a chunk of tasks, at most
// kAdjStoreBytes in FP64 (FP32 chunks are twice as many tasks).
static size_t adj_w_elems(const rq_lmm_model *model)
{
    return (size_t)model->n_fwd * model->n_factors * rq::kAdjBlockHost;
}
static size_t adj_task_elems(const rq_lmm_model *model)
{
    const int nfc = (model->n_fwd + 15) / 16 * 16;
    return adj_w_elems(model) + (size_t)nfc * rq::kAdjBlockHost;
}
static size_t adj_store_bytes(const rq_lmm_model *model, int64_t tasks, size_t limit)
{
    const size_t per = adj_task_elems(model) * sizeof(double);
    const int64_t fit = std::max<int64_t>(1, (int64_t)(limit / per));
    return (size_t)std::min<int64_t>(tasks, fit) * per;
}
static int64_t adj_chunk(const rq_lmm_model *model, int64_t tasks, size_t elem, size_t limit)
{
    const int64_t fit =
        std::max<int64_t>(1, (int64_t)(adj_store_bytes(model, tasks, limit) / (adj_task_elems(model) * elem)));
    const int64_t n_chunks = (tasks + fit - 1) / fit;
    return (tasks + n_chunks - 1) / n_chunks;   // equal chunks, the last one at most as large
}

// Model-region bytes and partial-region bytes of a LIBOR call; with Greeks
// the byte offset of the adjoint's store region inside the partial region.
static void caplet_sizes(const rq_lmm_model *model, int64_t N, int M, bool greeks, size_t store_limit, size_t &mb,
                         size_t &pb, int &n_blk, size_t *wtop_off = nullptr)
{
    const int rows = lmm_rows(model->n_fwd);
    const int n_out = model->n_fwd + 1;
    const int n_g = 2 * model->n_fwd + 1;
    mb = (size_t)rows * (rq::kFwdRow * sizeof(double) + rq::kRow32 * sizeof(float));
    if (greeks) {
        mb += (size_t)rows * rq::kAdjRow * sizeof(double);   // room for either precision
        n_blk = adj_blocks(N);
        pb = al((size_t)M * n_blk * (n_out + n_g) * sizeof(double));
        if (wtop_off) *wtop_off = pb;
        pb += adj_store_bytes(model, (int64_t)M * n_blk, store_limit) + 256;   // + room to align the state rows
    } else {
        n_blk = lmm_blocks(N);
        pb = (size_t)M * n_blk * n_out * sizeof(double);
    }
}

rq_status rq_set_adjoint_store_limit(size_t bytes)
{
    g_adj_store_limit.store(bytes ? bytes : rq::kAdjStoreBytes);
    return RQ_OK;
}

size_t rq_caplets_workspace(const rq_lmm_model *model, int64_t N, int M, int flags, rq_precision prec,
                            int with_greeks)
{
    if (check_lmm(model) != RQ_OK) return 0;
    Geometry g;
    const int s = model->n_fwd * model->n_factors;
    if (check_common(s, N, M, flags, 0, g) != RQ_OK) return 0;
    (void)prec;
    size_t mb, pb;
    int n_blk;
    caplet_sizes(model, N, M, with_greeks != 0, g_adj_store_limit.load(), mb, pb, n_blk);
    return layout(s, g, M, flags, mb, pb).total;
}

}  // extern "C"

namespace {

// The LIBOR entry point's body.  ws == nullptr selects the library's own
// scratch array of the current device (rq_price_caplets_noalloc): the store
// region of the adjoint is then cut to what fits beside the other regions.
rq_status price_caplets_impl(const rq_lmm_model *model, int64_t N, int M, uint64_t seed, int64_t m_offset,
                             int flags, rq_precision prec, const rq_result *out, const rq_result *grad,
                             double *per_path, void *ws, size_t ws_bytes, hipStream_t st)
{
    rq_status stt = check_lmm(model);
    if (stt) return stt;
    if (flags & RQ_OUT_DIGITS) return fail(RQ_EINVAL, "RQ_OUT_DIGITS applies to rq_sequence only");
    if ((flags & RQ_LMM_EULER) && grad)
        return fail(RQ_EUNSUPPORTED, "Greeks are computed for the log-Euler scheme only (RQ_LMM_EULER set)");
    if ((flags & RQ_LMM_EULER) && (flags & (RQ_PERM_RANDOM | RQ_PERM_PER_REP)))
        return fail(RQ_EUNSUPPORTED, "RQ_LMM_EULER is built for unpermuted Halton and Philox points");
    if (prec != RQ_FP64 && prec != RQ_FP32) return fail(RQ_EINVAL, "unknown precision %d", (int)prec);
    if (!out || !out->theta) return fail(RQ_EINVAL, "out->theta is NULL");
    if (grad && !grad->theta) return fail(RQ_EINVAL, "grad->theta is NULL");
    const int s = model->n_fwd * model->n_factors;
    Geometry g;
    if ((stt = check_common(s, N, M, flags, m_offset, g))) return stt;
    const bool greeks = grad != nullptr;
    size_t mb, pb, wtop_off = 0;
    int n_blk;
    size_t store_limit = g_adj_store_limit.load();
    const bool own = ws == nullptr;
    if (own) {
        if ((stt = scratch_of_device(ws, ws_bytes))) return stt;
        if (greeks) {   // the store region takes what the other regions leave
            caplet_sizes(model, N, M, true, 0, mb, pb, n_blk, &wtop_off);   // room for one task
            const size_t one = adj_task_elems(model) * sizeof(double);
            const size_t fixed = layout(s, g, M, flags, mb, pb - one).total;
            if (fixed + one > ws_bytes)
                return fail(RQ_ERANGE,
                            "rq_price_caplets_noalloc: %zu bytes of tables and partial sums plus %zu bytes per "
                            "stored 64-path task exceed the %zu-byte scratch array",
                            fixed, one, ws_bytes);
            store_limit = std::min(store_limit, (ws_bytes - fixed) / one * one);
        }
    }
    caplet_sizes(model, N, M, greeks, store_limit, mb, pb, n_blk, &wtop_off);
    const int n_out = model->n_fwd + 1;
    const int n_g = 2 * model->n_fwd + 1;
    if ((int64_t)n_blk * M >= (1ll << 31)) return fail(RQ_ERANGE, "N*M too large for one launch");
    std::vector<uint8_t> tab = lmm_table(model);
    const size_t adj_off = tab.size();
    if (greeks) {
        std::vector<uint8_t> at = prec == RQ_FP32 ? adj_table<float>(model) : adj_table<double>(model);
        tab.insert(tab.end(), at.begin(), at.end());
    }
    tab.resize(mb, 0);
    const Layout L = layout(s, g, M, flags, mb, pb);
    if (own && L.total > ws_bytes)
        return fail(RQ_ERANGE, "rq_price_caplets_noalloc: %zu bytes of tables and partial sums exceed the %zu-byte "
                               "scratch array", L.total, ws_bytes);
    if ((stt = check_ws(ws, ws_bytes, L.total))) return stt;
    PointTables pt;
    if ((stt = build_point_tables(s, g, seed, flags, pt))) return stt;
    uint8_t *w = (uint8_t *)ws;
    if ((stt = stage_and_setup(pt, tab, L, g, s, M, seed, m_offset, flags, w, st))) return stt;
    rq::LmmArgs a;
    a.g = seq_geom(L, g, w, s, M, N, flags, seed, m_offset);
    a.fwd = reinterpret_cast<const double *>(w + L.model);
    a.fwd32 = reinterpret_cast<const float *>(w + L.model + (size_t)lmm_rows(model->n_fwd) * rq::kFwdRow * sizeof(double));
    a.adj = greeks ? (const void *)(w + L.model + adj_off) : nullptr;
    const int64_t tasks = (int64_t)M * n_blk;
    const size_t elem = prec == RQ_FP32 ? sizeof(float) : sizeof(double);
    const int64_t chunk = greeks ? adj_chunk(model, tasks, elem, store_limit) : 0;
    a.wtop = greeks ? (void *)(w + L.partial + wtop_off) : nullptr;
    a.xs = greeks ? (void *)(w + L.partial + wtop_off + al((size_t)chunk * adj_w_elems(model) * elem)) : nullptr;
    a.n_slots = 0;
    a.task0 = 0;
    a.chunk = chunk;
    a.partial = reinterpret_cast<double *>(w + L.partial);
    a.partial_g = greeks ? a.partial + (size_t)M * n_blk * n_out : nullptr;
    a.n_g = n_g;
    a.per_path = per_path;
    a.n_fwd = model->n_fwd;
    a.n_out = n_out;
    a.n_blk = n_blk;
    a.delta = model->delta;
    a.sqrt_delta = std::sqrt(model->delta);
    a.num0 = 1.0 + model->delta * model->L0[0];
    a.euler = (flags & RQ_LMM_EULER) ? 1 : 0;
    {
        TimedRegion tr(st);
        if (greeks) {
            // chunks of tasks: the forward halves, then the reverse halves
            for (int64_t t0 = 0; t0 < tasks; t0 += chunk) {
                a.task0 = t0;
                a.chunk = std::min<int64_t>(chunk, tasks - t0);
                {
                    TimedRegion tf(st, 1);
                    RQ_HIP(rq::launch_lmm_adjoint(a, model->n_factors, prec == RQ_FP32, 1, st));
                }
                {
                    TimedRegion tv(st, 2);
                    RQ_HIP(rq::launch_lmm_adjoint(a, model->n_factors, prec == RQ_FP32, 2, st));
                }
            }
        } else {
            RQ_HIP(rq::launch_lmm(a, model->n_factors, prec == RQ_FP32, st));
        }
    }
    if ((stt = finish(out, a.partial, n_out, 0, M, n_blk, n_out, N, st))) return stt;
    if (greeks) return finish(grad, a.partial_g, n_g, 0, M, n_blk, n_g, N, st);
    return RQ_OK;
}

}  // namespace

extern "C" {

rq_status rq_price_caplets(const rq_lmm_model *model, int64_t N, int M, uint64_t seed, int64_t m_offset,
                           int flags, rq_precision prec, const rq_result *out, const rq_result *grad,
                           double *per_path, void *ws, size_t ws_bytes, void *stream)
{
    if (!ws) return fail(RQ_EINVAL, "workspace pointer is NULL");
    return price_caplets_impl(model, N, M, seed, m_offset, flags, prec, out, grad, per_path, ws, ws_bytes,
                              (hipStream_t)stream);
}

rq_status rq_price_caplets_noalloc(const rq_lmm_model *model, int64_t N, int M, uint64_t seed, int64_t m_offset,
                                   int flags, rq_precision prec, const rq_result *out, const rq_result *grad,
                                   double *per_path, void *stream)
{
    return price_caplets_impl(model, N, M, seed, m_offset, flags, prec, out, grad, per_path, nullptr, 0,
                              (hipStream_t)stream);
}

size_t rq_mbs_workspace(const rq_mbs_params *params, int64_t N, int M, int flags, rq_precision prec,
                        int with_greeks)
{
    if (check_mbs(params) != RQ_OK) return 0;
    Geometry g;
    if (check_common(params->months, N, M, flags, 0, g) != RQ_OK) return 0;
    (void)prec;
    const size_t mb = 2 * (size_t)(params->months + 1) * sizeof(double);
    const size_t pb = (size_t)M * lmm_blocks(N) * (with_greeks ? 2 : 1) * sizeof(double);
    return layout(params->months, g, M, flags, mb, pb).total;
}

rq_status rq_price_mbs(const rq_mbs_params *params, int64_t N, int M, uint64_t seed, int64_t m_offset,
                       int flags, rq_precision prec, const rq_result *out, const rq_result *grad,
                       double *per_path, void *ws, size_t ws_bytes, void *stream)
{
    rq_status stt = check_mbs(params);
    if (stt) return stt;
    if (flags & RQ_OUT_DIGITS) return fail(RQ_EINVAL, "RQ_OUT_DIGITS applies to rq_sequence only");
    if (flags & RQ_LMM_EULER) return fail(RQ_EINVAL, "RQ_LMM_EULER applies to rq_price_caplets only");
    if (prec != RQ_FP64 && prec != RQ_FP32) return fail(RQ_EINVAL, "unknown precision %d", (int)prec);
    if (!out || !out->theta) return fail(RQ_EINVAL, "out->theta is NULL");
    if (grad && !grad->theta) return fail(RQ_EINVAL, "grad->theta is NULL");
    const int s = params->months;
    Geometry g;
    if ((stt = check_common(s, N, M, flags, m_offset, g))) return stt;
    const int n_blk = lmm_blocks(N);
    const int n_part = grad ? 2 : 1;
    if ((int64_t)n_blk * M >= (1ll << 31)) return fail(RQ_ERANGE, "N*M too large for one launch");
    std::vector<uint8_t> tab = mbs_table(params);
    const Layout L = layout(s, g, M, flags, tab.size(), (size_t)M * n_blk * n_part * sizeof(double));
    if ((stt = check_ws(ws, ws_bytes, L.total))) return stt;
    PointTables pt;
    if ((stt = build_point_tables(s, g, seed, flags, pt))) return stt;
    hipStream_t st = (hipStream_t)stream;
    uint8_t *w = (uint8_t *)ws;
    if ((stt = stage_and_setup(pt, tab, L, g, s, M, seed, m_offset, flags, w, st))) return stt;
    rq::MbsArgs a;
    a.g = seq_geom(L, g, w, s, M, N, flags, seed, m_offset);
    a.ck = reinterpret_cast<const double *>(w + L.model);
    a.partial = reinterpret_cast<double *>(w + L.partial);
    a.per_path = per_path;
    a.months = params->months;
    a.n_blk = n_blk;
    a.n_part = n_part;
    mbs_scalars(params, a);
    {
        TimedRegion tr(st);
        RQ_HIP(rq::launch_mbs(a, prec == RQ_FP32, st));
    }
    if ((stt = finish(out, a.partial, n_part, 0, M, n_blk, 1, N, st))) return stt;
    if (grad) return finish(grad, a.partial, n_part, 1, M, n_blk, 1, N, st);
    return RQ_OK;
}

rq_status rq_lmm_pca_loadings(int n_fwd, int n_factors, double delta, double beta, double *out)
{
    if (n_fwd < 1 || n_fwd > RQ_MAX_FWD) return fail(RQ_ERANGE, "n_fwd = %d outside [1, %d]", n_fwd, RQ_MAX_FWD);
    if (n_factors < 1 || n_factors > RQ_MAX_FACTORS || n_factors > n_fwd)
        return fail(RQ_ERANGE, "n_factors = %d outside [1, min(%d, n_fwd)]", n_factors, RQ_MAX_FACTORS);
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(RQ_EINVAL, "delta must be > 0");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(RQ_EINVAL, "beta must be > 0");
    if (!out) return fail(RQ_EINVAL, "out is NULL");
    const int n = n_fwd;
    // rho_ij = exp(-beta |T_i - T_j|), T_i = (i+1) delta; cyclic Jacobi
    // rotations diagonalise it (A -> V^T A V, V accumulating the rotations)
    std::vector<double> A((size_t)n * n), V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        V[(size_t)i * n + i] = 1.0;
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = std::exp(-beta * delta * std::abs(i - j));
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
            for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        }
        if (off <= 1e-34 * diag) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                // rotation angle: tan(2 phi) = 2 a_pq / (a_qq - a_pp), |phi| <= pi/4
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::abs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
        }
    }
    // the n_factors largest eigenvalues, descending
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(),
              [&](int x, int y) { return A[(size_t)x * n + x] > A[(size_t)y * n + y]; });
    for (int f = 0; f < n_factors; ++f) {
        const int e = idx[f];
        const double lam = A[(size_t)e * n + e];
        if (!(lam > 0.0)) return fail(RQ_EINVAL, "correlation matrix is not positive definite");
        const double sg = V[e] < 0.0 ? -1.0 : 1.0;   // first component positive
        const double sl = std::sqrt(lam);
        for (int i = 0; i < n; ++i) out[(size_t)i * n_factors + f] = sg * V[(size_t)i * n + e] * sl;
    }
    for (int i = 0; i < n; ++i) {   // unit rows: forward i's total vol is sigma_i
        double r = 0.0;
        for (int f = 0; f < n_factors; ++f) r += out[(size_t)i * n_factors + f] * out[(size_t)i * n_factors + f];
        r = std::sqrt(r);
        for (int f = 0; f < n_factors; ++f) out[(size_t)i * n_factors + f] /= r;
    }
    return RQ_OK;
}

size_t rq_batch_workspace(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks)
{
    BatchPlan bp;
    if (plan_batch(inst, n_inst, prec, with_greeks != 0, RQ_ORDER_COST, bp) != RQ_OK) return 0;
    return bp.total;
}

rq_status rq_price_batch(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                         const rq_tuning *tuning, const rq_result *outs, const rq_result *grads, uint64_t *t_first,
                         uint64_t *t_last, void *ws, size_t ws_bytes, void *stream)
{
    return run_batch(inst, n_inst, prec, with_greeks != 0, tuning, outs, grads, t_first, t_last, ws, ws_bytes,
                     (hipStream_t)stream);
}

rq_status rq_autotune_batch(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                            const rq_result *outs, const rq_result *grads, rq_tuning *best, double *best_ms,
                            void *ws, size_t ws_bytes, void *stream)
{
    if (!best) return fail(RQ_EINVAL, "best is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool greeks = with_greeks != 0;
    {   // validate everything before the first launch
        BatchPlan bp;
        rq_status s0 = plan_batch(inst, n_inst, prec, greeks, RQ_ORDER_COST, bp);
        if (s0) return s0;
    }
    const int occ = rq::batch_blocks_per_cu(prec == RQ_FP32, greeks, greeks ? 2 : 0);
    if (occ <= 0) return fail(RQ_EHIP, "occupancy query of the batch kernel failed");
    // the automatic shape (chunk from each window's item count, every
    // resident block) in both orders, then the fixed shapes; cand[0], the
    // shape rq_price_batch takes without a tuning, is always a finalist, so
    // the choice is never slower than running untuned (up to timing noise)
    std::vector<rq_tuning> cand = {rq_tuning{0, 0, RQ_ORDER_COST}, rq_tuning{0, 0, RQ_ORDER_GIVEN}};
    const int chunks[] = {1, 2, 4, 8, 16};
    const int orders[] = {RQ_ORDER_COST, RQ_ORDER_GIVEN};
    std::vector<int> per_cu = {occ};
    if (occ > 1) per_cu.push_back(occ / 2);
    for (int o : orders)
        for (int pc : per_cu)
            for (int c : chunks) cand.push_back(rq_tuning{c, pc, o});
    // a large batch is screened on a probe of itself: every instrument with
    // its replications divided by a power of two (at least one), so that
    // the probe holds about 2^28 paths; the three fastest shapes on the
    // probe are then timed on the batch itself
    double paths = 0.0;
    for (int k = 0; k < n_inst; ++k) paths += (double)inst[k].N * (double)inst[k].M;
    int div = 1;
    while (paths / div > (double)(1 << 28) && div < 64) div *= 2;
    std::vector<rq_instrument> probe(inst, inst + n_inst);
    for (auto &I : probe) I.M = std::max(1, I.M / div);
    hipEvent_t e0, e1;
    RQ_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RQ_EHIP, "hipEventCreate failed");
    }
    auto time_one = [&](const rq_instrument *list, const rq_tuning &t, double &ms_out) -> rq_status {
        if (hipEventRecord(e0, st) != hipSuccess) return fail(RQ_EHIP, "hipEventRecord failed");
        rq_status r = run_batch(list, n_inst, prec, greeks, &t, outs, grads, nullptr, nullptr, ws, ws_bytes, st);
        if (r != RQ_OK) return r;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(RQ_EHIP, "timing the batch failed");
        ms_out = ms;
        return RQ_OK;
    };
    // one untimed run (first touch of the workspace, code load), then each
    // candidate once on the probe (the batch itself when div = 1)
    const rq_instrument *screen = div > 1 ? probe.data() : inst;
    std::vector<std::pair<double, int>> timed;
    double ms = 0.0;
    rq_status stt = run_batch(screen, n_inst, prec, greeks, &cand[0], outs, grads, nullptr, nullptr, ws, ws_bytes, st);
    for (size_t c = 0; stt == RQ_OK && c < cand.size(); ++c) {
        stt = time_one(screen, cand[c], ms);
        if (stt == RQ_OK) timed.emplace_back(ms, (int)c);
    }
    rq_tuning bt = cand[0];
    double bms = INFINITY;
    if (stt == RQ_OK) {
        std::stable_sort(timed.begin(), timed.end());
        if (div == 1) {
            bt = cand[timed[0].second];
            bms = timed[0].first;
        } else {
            // the finalists on the full batch, after one untimed full run:
            // the probe's three fastest and the automatic shape
            std::vector<int> fin;
            for (size_t r = 0; r < std::min<size_t>(3, timed.size()); ++r) fin.push_back(timed[r].second);
            if (std::find(fin.begin(), fin.end(), 0) == fin.end()) fin.push_back(0);
            stt = run_batch(inst, n_inst, prec, greeks, &cand[fin[0]], outs, grads, nullptr, nullptr, ws, ws_bytes,
                            st);
            for (size_t r = 0; stt == RQ_OK && r < fin.size(); ++r) {
                stt = time_one(inst, cand[fin[r]], ms);
                if (stt == RQ_OK && ms < bms) {
                    bms = ms;
                    bt = cand[fin[r]];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stt != RQ_OK) return stt;
    tuning_store(batch_signature(inst, n_inst, prec, greeks), bt);
    *best = bt;
    if (best_ms) *best_ms = bms;
    return RQ_OK;
}

rq_status rq_batch_tuning(const rq_instrument *inst, int n_inst, rq_precision prec, int with_greeks,
                          rq_tuning *out, int *from_autotuner)
{
    if (!out) return fail(RQ_EINVAL, "out is NULL");
    BatchPlan bp;
    rq_status s0 = plan_batch(inst, n_inst, prec, with_greeks != 0, RQ_ORDER_COST, bp);
    if (s0) return s0;
    rq_tuning t{0, 0, RQ_ORDER_COST};
    const bool hit = tuning_find(batch_signature(inst, n_inst, prec, with_greeks != 0), t);
    *out = hit ? t : rq_tuning{0, 0, RQ_ORDER_COST};
    if (from_autotuner) *from_autotuner = hit ? 1 : 0;
    return RQ_OK;
}

rq_status rq_realtime_hz(double *hz)
{
    if (!hz) return fail(RQ_EINVAL, "hz is NULL");
    int dev = 0, khz = 0;
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *hz = 1000.0 * (double)khz;
    return RQ_OK;
}

}  // extern "C"
